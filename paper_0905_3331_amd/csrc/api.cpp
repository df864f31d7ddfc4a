// api.cpp -- the extern "C" entry points declared in include/tmq.h.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "engine.h"
#include "lattice.h"

namespace tmq {
int solve_batch(Lattice *L, int n, const tmq_params *p, const tmq_solver_opts &o, const double *const *b,
                double *const *x, hipStream_t st, tmq_solve_info *info, const double *eps = nullptr);
int solve_full(Lattice *L, const tmq_params &p, const tmq_solver_opts &o, const FieldDesc &b, const FieldDesc &x,
               hipStream_t st, tmq_solve_info *info);
int solve_M(Lattice *L, const tmq_params &p, int sign, const tmq_solver_opts &o, const double2 *phi, double2 *psi,
            hipStream_t st, tmq_solve_info *info);
int solve_qhat_bicgstab(Lattice *L, const tmq_params &p, int sign, const tmq_solver_opts &o, const FieldDesc &fb,
                        const FieldDesc &fx, hipStream_t st, tmq_solve_info *info);
int solve_M_batch(Lattice *L, const tmq_params &p, int sign, const tmq_solver_opts &o, int nb, const double2 *const *phi,
                  double2 *const *psi, hipStream_t st, tmq_solve_info *info);
}  // namespace tmq

using namespace tmq;

namespace {

// Sets the lattice's device for the duration of a call and restores the caller's.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        hipGetDevice(&prev);
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) hipSetDevice(prev);
    }
};

int check_lat(tmq_lattice *lat, bool need_gauge)
{
    if (!lat || !lat->L) {
        set_error("NULL tmq_lattice");
        return TMQ_EINVAL;
    }
    if (need_gauge && !lat->L->gauge) {
        set_error("no gauge field loaded (call tmq_load_gauge first)");
        return TMQ_ESTATE;
    }
    return TMQ_OK;
}

int check_sign(int sign)
{
    if (sign != 1 && sign != -1) {
        set_error("sign must be +1 or -1");
        return TMQ_EINVAL;
    }
    return TMQ_OK;
}

int check_ptrs(const void *a, const void *b)
{
    if (!a || !b) {
        set_error("NULL field pointer");
        return TMQ_EINVAL;
    }
    return TMQ_OK;
}

// odd-site Qhat on device canonical buffers
int qhat_dev(Lattice *L, const tmq_params *p, int sign, int prec, const double *in, double *out, hipStream_t st)
{
    const long vh = L->g.vh;
    FieldDesc fi, fo, te;
    TMQ_TRY(work_field(L, "op_in", prec, vh, &fi));
    TMQ_TRY(work_field(L, "op_out", prec, vh, &fo));
    TMQ_TRY(work_field(L, "op_te", prec, vh, &te));
    const LinkDesc lk = lattice_links(L, link_fmt_for(L, prec, prec == TMQ_FP32 ? P32 : P16));
    TMQ_HIP(launch_from_canonical((const double2 *)in, fi, st));
    TMQ_TRY(apply_Qhat(L, make_op(L, p, 1), sign, fi, fo, te, lk, rhs_all(1), nullptr, nullptr, st));
    TMQ_HIP(launch_to_canonical(fo, (double2 *)out, st));
    return TMQ_OK;
}

int check_nd(const tmq_nd_params *p)
{
    if (!p) {
        set_error("NULL tmq_nd_params");
        return TMQ_EINVAL;
    }
    const double d = 1.0 + p->mubar_tilde * p->mubar_tilde - p->epsbar_tilde * p->epsbar_tilde;
    if (!std::isfinite(p->kappa) || !std::isfinite(p->mubar_tilde) || !std::isfinite(p->epsbar_tilde) ||
        !(d > 0.0)) {
        set_error("doublet parameters must be finite with 1 + mubar^2 - epsbar^2 > 0");
        return TMQ_EINVAL;
    }
    for (int mu = 0; mu < 4; mu++)
        if (!std::isfinite(p->theta[mu])) {
            set_error("theta must be finite");
            return TMQ_EINVAL;
        }
    return TMQ_OK;
}

// the one-flavour parameter record of a doublet (mu_tilde carries 2 kappa mubar)
tmq_params nd_base(const tmq_nd_params &p)
{
    tmq_params q{};
    q.kappa = p.kappa;
    q.mu_tilde = p.mubar_tilde;
    for (int mu = 0; mu < 4; mu++) q.theta[mu] = p.theta[mu];
    return q;
}

// doublet Qhat_h on device canonical buffers [2][V/2][12]
int qhat_nd_dev(Lattice *L, const tmq_nd_params &p, int sign, int prec, const double *in, double *out, hipStream_t st)
{
    const long n = 2 * L->g.vh;
    FieldDesc fi, fo, te;
    TMQ_TRY(work_field(L, "nd_in", prec, n, &fi));
    TMQ_TRY(work_field(L, "nd_out", prec, n, &fo));
    TMQ_TRY(work_field(L, "nd_te", prec, n, &te));
    const LinkDesc lk = lattice_links(L, link_fmt_for(L, prec, prec == TMQ_FP32 ? P32 : P16));
    const tmq_params q = nd_base(p);
    OpParams op = make_op(L, &q, 1);
    op.eps[0] = p.epsbar_tilde;
    op.nd = 1;
    TMQ_HIP(launch_from_canonical((const double2 *)in, fi, st));
    TMQ_TRY(apply_Qhat(L, op, sign, fi, fo, te, lk, rhs_all(1), nullptr, nullptr, st));
    TMQ_HIP(launch_to_canonical(fo, (double2 *)out, st));
    return TMQ_OK;
}

int copy_in(Lattice *L, int slot, const double *host, size_t bytes, double **dev)
{
    void *d = nullptr;
    TMQ_TRY(stage_buffer(L, slot, bytes, &d));
    TMQ_HIP(hipMemcpyAsync(d, host, bytes, hipMemcpyHostToDevice, L->own));
    *dev = (double *)d;
    return TMQ_OK;
}

}  // namespace

extern "C" {

const char *tmq_last_error(void) { return get_error(); }

const char *tmq_version(void) { return "tmq 0.1 (gfx950)"; }

int tmq_lattice_create(const int dims[4], int device, tmq_lattice **out)
{
    if (!out) {
        set_error("tmq_lattice_create: NULL out");
        return TMQ_EINVAL;
    }
    *out = nullptr;
    Lattice *L = nullptr;
    TMQ_TRY(lattice_create(dims, device, &L));
    tmq_lattice *h = new (std::nothrow) tmq_lattice{L};
    if (!h) {
        delete L;
        set_error("host allocation failed");
        return TMQ_ENOMEM;
    }
    *out = h;
    return TMQ_OK;
}

void tmq_lattice_destroy(tmq_lattice *lat)
{
    if (!lat) return;
    delete lat->L;
    delete lat;
}

int tmq_load_gauge_dev(tmq_lattice *lat, const double *U, void *stream)
{
    TMQ_TRY(check_lat(lat, false));
    TMQ_TRY(check_ptrs(U, U));
    DeviceGuard dg(lat->L->device);
    return lattice_load_gauge(lat->L, (const double2 *)U, (hipStream_t)stream);
}

int tmq_load_gauge(tmq_lattice *lat, const double *U)
{
    TMQ_TRY(check_lat(lat, false));
    TMQ_TRY(check_ptrs(U, U));
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    const size_t bytes = (size_t)2 * L->g.vh * 4 * 9 * 16;
    void *d = nullptr;
    TMQ_HIP(hipMalloc(&d, bytes));
    int s = TMQ_OK;
    if (hipMemcpyAsync(d, U, bytes, hipMemcpyHostToDevice, L->own) != hipSuccess) {
        set_error("tmq_load_gauge: host to device copy failed");
        s = TMQ_EDEVICE;
    }
    if (s == TMQ_OK) s = lattice_load_gauge(L, (const double2 *)d, L->own);
    hipStreamSynchronize(L->own);
    hipFree(d);
    return s;
}

int tmq_gauge_is_su3(const tmq_lattice *lat) { return lat && lat->L && lat->L->su3 ? 1 : 0; }

int tmq_apply_Qhat_dev(tmq_lattice *lat, const tmq_params *p, int sign, tmq_prec prec, const double *in,
                       double *out, void *stream)
{
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_params(p));
    TMQ_TRY(check_sign(sign));
    TMQ_TRY(check_prec(prec));
    TMQ_TRY(check_ptrs(in, out));
    DeviceGuard dg(lat->L->device);
    return qhat_dev(lat->L, p, sign, prec, in, out, (hipStream_t)stream);
}

int tmq_apply_Qhat_noalloc_dev(tmq_lattice *lat, const tmq_params *p, int sign, tmq_prec prec, const double *in,
                               double *out, void *stream)
{
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_params(p));
    TMQ_TRY(check_sign(sign));
    TMQ_TRY(check_prec(prec));
    TMQ_TRY(check_ptrs(in, out));
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    size_t cap = 0;
    char *base = (char *)noalloc_scratch(L->device, &cap);
    if (!base) {
        set_error("tmq_apply_Qhat_noalloc_dev: the device address of the fixed work space is unknown "
                  "(hipGetSymbolAddress failed when the lattice was created)");
        return TMQ_EDEVICE;
    }
    // the three work fields of qhat_dev, one after the other in the array
    const long vh = L->g.vh;
    size_t b0 = 0, b1 = 0, b2 = 0;
    const FieldDesc fi = field_at(base, prec, vh, &b0);
    const FieldDesc fo = field_at(base + b0, prec, vh, &b1);
    const FieldDesc te = field_at(base + b0 + b1, prec, vh, &b2);
    if (b0 + b1 + b2 > cap) {
        char msg[256];
        snprintf(msg, sizeof(msg),
                 "tmq_apply_Qhat_noalloc_dev: this lattice needs %zu bytes of work space in this precision, "
                 "above the fixed %zu (TMQ_NOALLOC_SCRATCH_BYTES)",
                 b0 + b1 + b2, cap);
        set_error(msg);
        return TMQ_EINVAL;
    }
    const hipStream_t st = (hipStream_t)stream;
    const LinkDesc lk = lattice_links(L, link_fmt_for(L, prec, prec == TMQ_FP32 ? P32 : P16));
    struct NoAllocScope {
        Lattice *L;
        ~NoAllocScope() { L->no_alloc = false; }
    } scope{L};
    L->no_alloc = true;
    TMQ_HIP(launch_from_canonical((const double2 *)in, fi, st));
    TMQ_TRY(apply_Qhat(L, make_op(L, p, 1), sign, fi, fo, te, lk, rhs_all(1), nullptr, nullptr, st));
    TMQ_HIP(launch_to_canonical(fo, (double2 *)out, st));
    return TMQ_OK;
}

int tmq_apply_Qhat(tmq_lattice *lat, const tmq_params *p, int sign, tmq_prec prec, const double *in, double *out)
{
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_params(p));
    TMQ_TRY(check_sign(sign));
    TMQ_TRY(check_prec(prec));
    TMQ_TRY(check_ptrs(in, out));
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    const size_t bytes = (size_t)L->g.vh * 12 * 16;
    double *din = nullptr, *dout = nullptr;
    TMQ_TRY(copy_in(L, 0, in, bytes, &din));
    void *d = nullptr;
    TMQ_TRY(stage_buffer(L, 1, bytes, &d));
    dout = (double *)d;
    TMQ_TRY(qhat_dev(L, p, sign, prec, din, dout, L->own));
    TMQ_HIP(hipMemcpyAsync(out, dout, bytes, hipMemcpyDeviceToHost, L->own));
    TMQ_HIP(hipStreamSynchronize(L->own));
    return TMQ_OK;
}

int tmq_apply_QhatQhat_dev(tmq_lattice *lat, const tmq_params *p, const double *in, double *out, void *stream)
{
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_params(p));
    TMQ_TRY(check_ptrs(in, out));
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    hipStream_t st = (hipStream_t)stream;
    const long vh = L->g.vh;
    FieldDesc fi, fo, te, to;
    TMQ_TRY(work_field(L, "op_in", P64, vh, &fi));
    TMQ_TRY(work_field(L, "op_out", P64, vh, &fo));
    TMQ_TRY(work_field(L, "op_te", P64, vh, &te));
    TMQ_TRY(work_field(L, "op_to", P64, vh, &to));
    TMQ_HIP(launch_from_canonical((const double2 *)in, fi, st));
    TMQ_TRY(apply_QhatQhat(L, make_op(L, p, 1), fi, fo, te, to, lattice_links(L, link_fmt_for(L, P64, P64)),
                           rhs_all(1), nullptr, nullptr, st));
    TMQ_HIP(launch_to_canonical(fo, (double2 *)out, st));
    return TMQ_OK;
}

int tmq_apply_Q_full_dev(tmq_lattice *lat, const tmq_params *p, int sign, const double *in, double *out,
                         void *stream)
{
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_params(p));
    TMQ_TRY(check_sign(sign));
    TMQ_TRY(check_ptrs(in, out));
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    hipStream_t st = (hipStream_t)stream;
    const long n = 2 * L->g.vh;
    FieldDesc fi, fo;
    TMQ_TRY(work_field(L, "full_in", P64, n, &fi));
    TMQ_TRY(work_field(L, "full_out", P64, n, &fo));
    TMQ_HIP(launch_full_from_canonical(L->g, (const double2 *)in, fi, st));
    TMQ_TRY(apply_Q_full(L, make_op(L, p, 1), sign, fi, fo, lattice_links(L, link_fmt_for(L, P64, P64)),
                         rhs_all(1), st));
    TMQ_HIP(launch_full_to_canonical(L->g, fo, (double2 *)out, st));
    return TMQ_OK;
}

int tmq_apply_Q_full(tmq_lattice *lat, const tmq_params *p, int sign, const double *in, double *out)
{
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_ptrs(in, out));
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    const size_t bytes = (size_t)2 * L->g.vh * 12 * 16;
    double *din = nullptr;
    TMQ_TRY(copy_in(L, 0, in, bytes, &din));
    void *d = nullptr;
    TMQ_TRY(stage_buffer(L, 1, bytes, &d));
    TMQ_TRY(tmq_apply_Q_full_dev(lat, p, sign, din, (double *)d, L->own));
    TMQ_HIP(hipMemcpyAsync(out, d, bytes, hipMemcpyDeviceToHost, L->own));
    TMQ_HIP(hipStreamSynchronize(L->own));
    return TMQ_OK;
}

int tmq_solve_batch_dev(tmq_lattice *lat, int nrhs, const tmq_params *p, const tmq_solver_opts *opts,
                        const double *const *b, double *const *x, void *stream, tmq_solve_info *info)
{
    if (info && nrhs > 0) memset(info, 0, sizeof(*info) * (size_t)nrhs);
    TMQ_TRY(check_lat(lat, true));
    if (nrhs < 1 || nrhs > TMQ_MAX_RHS || !p || !b || !x) {
        set_error("tmq_solve_batch: need 1 <= nrhs <= TMQ_MAX_RHS and non-NULL arrays");
        return TMQ_EINVAL;
    }
    for (int r = 0; r < nrhs; r++) {
        TMQ_TRY(check_params(&p[r]));
        TMQ_TRY(check_ptrs(b[r], x[r]));
        for (int mu = 0; mu < 4; mu++)
            if (p[r].theta[mu] != p[0].theta[mu]) {
                set_error("tmq_solve_batch: every right-hand side must have the same boundary phases");
                return TMQ_EINVAL;
            }
    }
    TMQ_TRY(check_opts(opts));
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    hipStream_t st = (hipStream_t)stream;
    return solve_batch(L, nrhs, p, *opts, b, x, st, info);
}

int tmq_solve_batch(tmq_lattice *lat, int nrhs, const tmq_params *p, const tmq_solver_opts *opts,
                    const double *const *b, double *const *x, tmq_solve_info *info)
{
    if (info && nrhs > 0) memset(info, 0, sizeof(*info) * (size_t)nrhs);
    TMQ_TRY(check_lat(lat, true));
    if (nrhs < 1 || nrhs > TMQ_MAX_RHS || !b || !x) {
        set_error("tmq_solve_batch: need 1 <= nrhs <= TMQ_MAX_RHS and non-NULL arrays");
        return TMQ_EINVAL;
    }
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    const auto t0 = std::chrono::steady_clock::now();
    const size_t bytes = (size_t)L->g.vh * 12 * 16;
    void *db = nullptr, *dx = nullptr;
    TMQ_TRY(stage_buffer(L, 0, bytes * nrhs, &db));
    TMQ_TRY(stage_buffer(L, 1, bytes * nrhs, &dx));
    std::vector<const double *> bp(nrhs);
    std::vector<double *> xp(nrhs);
    for (int r = 0; r < nrhs; r++) {
        TMQ_TRY(check_ptrs(b[r], x[r]));
        bp[r] = (const double *)((char *)db + bytes * r);
        xp[r] = (double *)((char *)dx + bytes * r);
        TMQ_HIP(hipMemcpyAsync((void *)bp[r], b[r], bytes, hipMemcpyHostToDevice, L->own));
    }
    const int s = tmq_solve_batch_dev(lat, nrhs, p, opts, bp.data(), xp.data(), L->own, info);
    if (s == TMQ_OK || s == TMQ_ENOCONV) {
        for (int r = 0; r < nrhs; r++) TMQ_HIP(hipMemcpyAsync(x[r], xp[r], bytes, hipMemcpyDeviceToHost, L->own));
        TMQ_HIP(hipStreamSynchronize(L->own));
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info)
        for (int r = 0; r < nrhs; r++) info[r].seconds = secs;
    return s;
}

int tmq_solve_dev(tmq_lattice *lat, const tmq_params *p, const tmq_solver_opts *opts, const double *b, double *x,
                  void *stream, tmq_solve_info *info)
{
    return tmq_solve_batch_dev(lat, 1, p, opts, &b, &x, stream, info);
}

int tmq_solve(tmq_lattice *lat, const tmq_params *p, const tmq_solver_opts *opts, const double *b, double *x,
              tmq_solve_info *info)
{
    return tmq_solve_batch(lat, 1, p, opts, &b, &x, info);
}

int tmq_solve_full_dev(tmq_lattice *lat, const tmq_params *p, const tmq_solver_opts *opts, const double *b,
                       double *x, void *stream, tmq_solve_info *info)
{
    if (info) memset(info, 0, sizeof(*info));
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_params(p));
    TMQ_TRY(check_opts(opts));
    TMQ_TRY(check_ptrs(b, x));
    if (opts->sloppy != TMQ_FP64) {
        set_error("tmq_solve_full_dev: only FP64 is provided for the full-lattice operator");
        return TMQ_EINVAL;
    }
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    hipStream_t st = (hipStream_t)stream;
    const long n = 2 * L->g.vh;
    FieldDesc fb, fx;
    TMQ_TRY(work_field(L, "full_b", P64, n, &fb));
    TMQ_TRY(work_field(L, "full_x", P64, n, &fx));
    TMQ_HIP(launch_full_from_canonical(L->g, (const double2 *)b, fb, st));
    const int s = solve_full(L, *p, *opts, fb, fx, st, info);
    if (s == TMQ_OK || s == TMQ_ENOCONV) {
        TMQ_HIP(launch_full_to_canonical(L->g, fx, (double2 *)x, st));
        TMQ_HIP(hipStreamSynchronize(st));
    }
    return s;
}

int tmq_solve_Qhat_dev(tmq_lattice *lat, const tmq_params *p, int sign, const tmq_solver_opts *opts, const double *b,
                       double *x, void *stream, tmq_solve_info *info)
{
    if (info) memset(info, 0, sizeof(*info));
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_params(p));
    TMQ_TRY(check_sign(sign));
    TMQ_TRY(check_opts(opts));
    TMQ_TRY(check_ptrs(b, x));
    if (opts->sloppy != TMQ_FP64) {
        set_error("tmq_solve_Qhat: BiCGstab runs in FP64 only (sloppy = TMQ_FP64)");
        return TMQ_EINVAL;
    }
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    hipStream_t st = (hipStream_t)stream;
    const long vh = L->g.vh;
    FieldDesc fb, fx;
    TMQ_TRY(work_field(L, "bq_b", P64, vh, &fb));
    TMQ_TRY(work_field(L, "bq_x", P64, vh, &fx));
    TMQ_HIP(launch_from_canonical((const double2 *)b, fb, st));
    const int s = solve_qhat_bicgstab(L, *p, sign, *opts, fb, fx, st, info);
    if (s == TMQ_OK || s == TMQ_ENOCONV) {
        TMQ_HIP(launch_to_canonical(fx, (double2 *)x, st));
        TMQ_HIP(hipStreamSynchronize(st));
    }
    return s;
}

int tmq_solve_Qhat(tmq_lattice *lat, const tmq_params *p, int sign, const tmq_solver_opts *opts, const double *b,
                   double *x, tmq_solve_info *info)
{
    if (info) memset(info, 0, sizeof(*info));
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_ptrs(b, x));
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    const size_t bytes = (size_t)L->g.vh * 12 * sizeof(double2);
    double *db = nullptr;
    TMQ_TRY(copy_in(L, 0, b, bytes, &db));
    void *dx = nullptr;
    TMQ_TRY(stage_buffer(L, 1, bytes, &dx));
    const int s = tmq_solve_Qhat_dev(lat, p, sign, opts, db, (double *)dx, L->own, info);
    if (s == TMQ_OK || s == TMQ_ENOCONV) {
        TMQ_HIP(hipMemcpyAsync(x, dx, bytes, hipMemcpyDeviceToHost, L->own));
        TMQ_HIP(hipStreamSynchronize(L->own));
    }
    return s;
}

int tmq_solve_M_dev(tmq_lattice *lat, const tmq_params *p, int sign, const tmq_solver_opts *opts, const double *phi,
                    double *psi, void *stream, tmq_solve_info *info)
{
    if (info) memset(info, 0, sizeof(*info));
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_params(p));
    TMQ_TRY(check_sign(sign));
    TMQ_TRY(check_opts(opts));
    TMQ_TRY(check_ptrs(phi, psi));
    if (phi == psi) {
        set_error("tmq_solve_M: phi and psi must not overlap");
        return TMQ_EINVAL;
    }
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    return solve_M(L, *p, sign, *opts, (const double2 *)phi, (double2 *)psi, (hipStream_t)stream, info);
}

int tmq_solve_M_batch_dev(tmq_lattice *lat, const tmq_params *p, int sign, const tmq_solver_opts *opts, int n,
                          const double *const *phi, double *const *psi, void *stream, tmq_solve_info *info)
{
    if (info && n > 0) memset(info, 0, sizeof(*info) * (size_t)n);
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_params(p));
    TMQ_TRY(check_sign(sign));
    TMQ_TRY(check_opts(opts));
    if (n < 1 || n > TMQ_MAX_RHS || !phi || !psi) {
        set_error("tmq_solve_M_batch: need 1 <= n <= TMQ_MAX_RHS and non-NULL arrays");
        return TMQ_EINVAL;
    }
    for (int r = 0; r < n; r++) {
        TMQ_TRY(check_ptrs(phi[r], psi[r]));
        for (int q = 0; q < n; q++)
            if (psi[r] == phi[q] || (q != r && psi[r] == psi[q])) {
                set_error("tmq_solve_M_batch: the psi buffers must not overlap one another or any phi");
                return TMQ_EINVAL;
            }
    }
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    return solve_M_batch(L, *p, sign, *opts, n, (const double2 *const *)phi, (double2 *const *)psi,
                         (hipStream_t)stream, info);
}

int tmq_solve_M(tmq_lattice *lat, const tmq_params *p, int sign, const tmq_solver_opts *opts, const double *phi,
                double *psi, tmq_solve_info *info)
{
    if (info) memset(info, 0, sizeof(*info));
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_ptrs(phi, psi));
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    const size_t bytes = (size_t)2 * L->g.vh * 12 * sizeof(double2);
    void *dphi = nullptr, *dpsi = nullptr;
    TMQ_TRY(stage_buffer(L, 0, bytes, &dphi));
    TMQ_TRY(stage_buffer(L, 1, bytes, &dpsi));
    TMQ_HIP(hipMemcpyAsync(dphi, phi, bytes, hipMemcpyHostToDevice, L->own));
    const int s = tmq_solve_M_dev(lat, p, sign, opts, (const double *)dphi, (double *)dpsi, L->own, info);
    if (s == TMQ_OK || s == TMQ_ENOCONV) {
        TMQ_HIP(hipMemcpyAsync(psi, dpsi, bytes, hipMemcpyDeviceToHost, L->own));
        TMQ_HIP(hipStreamSynchronize(L->own));
    }
    return s;
}

int tmq_apply_Qhat_nd_dev(tmq_lattice *lat, const tmq_nd_params *p, int sign, tmq_prec prec, const double *in,
                          double *out, void *stream)
{
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_nd(p));
    TMQ_TRY(check_sign(sign));
    TMQ_TRY(check_prec(prec));
    TMQ_TRY(check_ptrs(in, out));
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    return qhat_nd_dev(L, *p, sign, prec, in, out, (hipStream_t)stream);
}

int tmq_apply_Qhat_nd(tmq_lattice *lat, const tmq_nd_params *p, int sign, tmq_prec prec, const double *in,
                      double *out)
{
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_ptrs(in, out));
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    const size_t bytes = (size_t)2 * L->g.vh * 12 * sizeof(double2);
    double *din = nullptr;
    TMQ_TRY(copy_in(L, 0, in, bytes, &din));
    void *d = nullptr;
    TMQ_TRY(stage_buffer(L, 1, bytes, &d));
    TMQ_TRY(tmq_apply_Qhat_nd_dev(lat, p, sign, prec, din, (double *)d, L->own));
    TMQ_HIP(hipMemcpyAsync(out, d, bytes, hipMemcpyDeviceToHost, L->own));
    TMQ_HIP(hipStreamSynchronize(L->own));
    return TMQ_OK;
}

int tmq_solve_nd_batch_dev(tmq_lattice *lat, int n, const tmq_nd_params *p, const tmq_solver_opts *opts,
                           const double *const *b, double *const *x, void *stream, tmq_solve_info *info)
{
    if (info && n > 0) memset(info, 0, sizeof(*info) * (size_t)n);
    TMQ_TRY(check_lat(lat, true));
    if (n < 1 || n > TMQ_MAX_RHS / 2 || !p || !b || !x) {
        set_error("tmq_solve_nd_batch: need 1 <= n <= TMQ_MAX_RHS / 2 and non-NULL arrays");
        return TMQ_EINVAL;
    }
    std::vector<tmq_params> q((size_t)n);
    std::vector<double> eps((size_t)n);
    for (int r = 0; r < n; r++) {
        TMQ_TRY(check_nd(&p[r]));
        TMQ_TRY(check_ptrs(b[r], x[r]));
        for (int mu = 0; mu < 4; mu++)
            if (p[r].theta[mu] != p[0].theta[mu]) {
                set_error("tmq_solve_nd_batch: every doublet must have the same boundary phases");
                return TMQ_EINVAL;
            }
        q[r] = nd_base(p[r]);
        eps[r] = p[r].epsbar_tilde;
    }
    TMQ_TRY(check_opts(opts));
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    return solve_batch(L, n, q.data(), *opts, b, x, (hipStream_t)stream, info, eps.data());
}

int tmq_solve_nd_dev(tmq_lattice *lat, const tmq_nd_params *p, const tmq_solver_opts *opts, const double *b,
                     double *x, void *stream, tmq_solve_info *info)
{
    return tmq_solve_nd_batch_dev(lat, 1, p, opts, &b, &x, stream, info);
}

int tmq_solve_nd(tmq_lattice *lat, const tmq_nd_params *p, const tmq_solver_opts *opts, const double *b, double *x,
                 tmq_solve_info *info)
{
    if (info) memset(info, 0, sizeof(*info));
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_ptrs(b, x));
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    const size_t bytes = (size_t)2 * L->g.vh * 12 * sizeof(double2);
    double *db = nullptr;
    TMQ_TRY(copy_in(L, 0, b, bytes, &db));
    void *dx = nullptr;
    TMQ_TRY(stage_buffer(L, 1, bytes, &dx));
    const int s = tmq_solve_nd_dev(lat, p, opts, db, (double *)dx, L->own, info);
    if (s == TMQ_OK || s == TMQ_ENOCONV) {
        TMQ_HIP(hipMemcpyAsync(x, dx, bytes, hipMemcpyDeviceToHost, L->own));
        TMQ_HIP(hipStreamSynchronize(L->own));
    }
    return s;
}

// ---------------------------------------------------- solver consumers

namespace {

// sums of the bilinear partials per time slice, in a fixed order, shifted by t0
int ts_bilinear_host(Lattice *L, const double *psi, const SpinMat &m, int t0, double *out, hipStream_t st)
{
    const int nb = ts_bilinear_blocks(L->g), T = L->g.T;
    if ((long)nb * T > L->pstride * MAX_RHS) {
        set_error("internal: too many time-slice partial sums");
        return TMQ_EINVAL;
    }
    TMQ_HIP(launch_ts_bilinear(L->g, (const double2 *)psi, m, L->partial[0], L->partial[1], st));
    std::vector<double> re((size_t)nb * T), im((size_t)nb * T);
    TMQ_HIP(hipMemcpyAsync(re.data(), L->partial[0], sizeof(double) * re.size(), hipMemcpyDeviceToHost, st));
    TMQ_HIP(hipMemcpyAsync(im.data(), L->partial[1], sizeof(double) * im.size(), hipMemcpyDeviceToHost, st));
    TMQ_HIP(hipStreamSynchronize(st));
    for (int t = 0; t < T; t++) {
        const int ts = ((t0 + t) % T + T) % T;
        double a = 0.0, b = 0.0;
        for (int k = 0; k < nb; k++) a += re[(size_t)ts * nb + k], b += im[(size_t)ts * nb + k];
        out[2 * t] = a;
        out[2 * t + 1] = b;
    }
    return TMQ_OK;
}

}  // namespace

int tmq_timeslice_bilinear_dev(tmq_lattice *lat, const double *gamma, const double *psi, int t0, double *out,
                               void *stream)
{
    TMQ_TRY(check_lat(lat, false));
    if (!gamma || !psi || !out) {
        set_error("tmq_timeslice_bilinear: NULL argument");
        return TMQ_EINVAL;
    }
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    SpinMat m;
    for (int i = 0; i < 16; i++) m.m[i / 4][i % 4] = make_double2(gamma[2 * i], gamma[2 * i + 1]);
    return ts_bilinear_host(L, psi, m, t0, out, (hipStream_t)stream);
}

int tmq_pion_correlator_dev(tmq_lattice *lat, const tmq_params *p, const tmq_solver_opts *opts, const double *xi,
                            int t0, double *corr, double *phi, void *stream, tmq_solve_info *info)
{
    if (info) memset(info, 0, sizeof(*info));
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_ptrs(xi, corr));
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    hipStream_t st = (hipStream_t)stream;
    double *ph = phi;
    if (!ph) {
        void *w = nullptr;
        TMQ_TRY(stage_buffer(L, 1, (size_t)2 * L->g.vh * 12 * sizeof(double2), &w));
        ph = (double *)w;
    }
    const int s = tmq_solve_M_dev(lat, p, +1, opts, xi, ph, stream, info);
    if (s != TMQ_OK && s != TMQ_ENOCONV) return s;
    SpinMat one{};
    for (int i = 0; i < 4; i++) one.m[i][i] = make_double2(1.0, 0.0);
    std::vector<double> c((size_t)2 * L->g.T);
    TMQ_TRY(ts_bilinear_host(L, ph, one, t0, c.data(), st));
    for (int t = 0; t < L->g.T; t++) corr[t] = c[2 * t];
    return s;
}

int tmq_solve_force_dev(tmq_lattice *lat, const tmq_params *p, const tmq_solver_opts *opts, const double *phi,
                        double *X, double *Y, double *action, void *stream, tmq_solve_info *info)
{
    if (info) memset(info, 0, sizeof(*info));
    TMQ_TRY(check_lat(lat, true));
    TMQ_TRY(check_params(p));
    TMQ_TRY(check_opts(opts));
    TMQ_TRY(check_ptrs(phi, X));
    if (X == phi || (Y && (Y == phi || Y == X))) {
        set_error("tmq_solve_force: phi, X and Y must not overlap");
        return TMQ_EINVAL;
    }
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    hipStream_t st = (hipStream_t)stream;
    const int s = solve_batch(L, 1, p, *opts, &phi, &X, st, info);
    if (s != TMQ_OK && s != TMQ_ENOCONV) return s;
    if (Y) TMQ_TRY(qhat_dev(L, p, -1, P64, X, Y, st));
    if (action) {
        const long vh = L->g.vh;
        FieldDesc fp, fx;
        TMQ_TRY(work_field(L, "force_phi", P64, vh, &fp));
        TMQ_TRY(work_field(L, "force_x", P64, vh, &fx));
        TMQ_HIP(launch_from_canonical((const double2 *)phi, fp, st));
        TMQ_HIP(launch_from_canonical((const double2 *)X, fx, st));
        TMQ_HIP(launch_bi_dot(fp, fx, nullptr, L->partial[0], L->partial[1], L->partial[2], st));
        const int nb = blas_grid(vh);
        std::vector<double> re((size_t)nb);
        TMQ_HIP(hipMemcpyAsync(re.data(), L->partial[0], sizeof(double) * nb, hipMemcpyDeviceToHost, st));
        TMQ_HIP(hipStreamSynchronize(st));
        double a = 0.0;
        for (double v : re) a += v;
        *action = a;
    }
    return s;
}

int tmq_split_eo_dev(tmq_lattice *lat, const double *full, double *even, double *odd, void *stream)
{
    TMQ_TRY(check_lat(lat, false));
    if (!full || (!even && !odd)) {
        set_error("tmq_split_eo: NULL full field, or both outputs NULL");
        return TMQ_EINVAL;
    }
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    TMQ_HIP(launch_split_eo(L->g, (const double2 *)full, (double2 *)even, (double2 *)odd, (hipStream_t)stream));
    return TMQ_OK;
}

int tmq_merge_eo_dev(tmq_lattice *lat, const double *even, const double *odd, double *full, void *stream)
{
    TMQ_TRY(check_lat(lat, false));
    if (!full) {
        set_error("tmq_merge_eo: NULL full field");
        return TMQ_EINVAL;
    }
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    TMQ_HIP(launch_merge_eo(L->g, (const double2 *)even, (const double2 *)odd, (double2 *)full, (hipStream_t)stream));
    return TMQ_OK;
}

static int split_merge_host(tmq_lattice *lat, bool merge, const double *full_in, double *full_out, const double *ev_in,
                            const double *od_in, double *ev_out, double *od_out)
{
    TMQ_TRY(check_lat(lat, false));
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    const size_t half = (size_t)L->g.vh * 12 * sizeof(double2);
    void *df = nullptr, *dh = nullptr;
    TMQ_TRY(stage_buffer(L, 0, 2 * half, &df));
    TMQ_TRY(stage_buffer(L, 1, 2 * half, &dh));
    double2 *de = (double2 *)dh, *dodd = (double2 *)((char *)dh + half);
    hipStream_t st = L->own;
    if (merge) {
        if (ev_in) TMQ_HIP(hipMemcpyAsync(de, ev_in, half, hipMemcpyHostToDevice, st));
        if (od_in) TMQ_HIP(hipMemcpyAsync(dodd, od_in, half, hipMemcpyHostToDevice, st));
        TMQ_TRY(tmq_merge_eo_dev(lat, ev_in ? (double *)de : nullptr, od_in ? (double *)dodd : nullptr, (double *)df,
                                 st));
        TMQ_HIP(hipMemcpyAsync(full_out, df, 2 * half, hipMemcpyDeviceToHost, st));
    } else {
        TMQ_HIP(hipMemcpyAsync(df, full_in, 2 * half, hipMemcpyHostToDevice, st));
        TMQ_TRY(tmq_split_eo_dev(lat, (double *)df, ev_out ? (double *)de : nullptr, od_out ? (double *)dodd : nullptr,
                                 st));
        if (ev_out) TMQ_HIP(hipMemcpyAsync(ev_out, de, half, hipMemcpyDeviceToHost, st));
        if (od_out) TMQ_HIP(hipMemcpyAsync(od_out, dodd, half, hipMemcpyDeviceToHost, st));
    }
    TMQ_HIP(hipStreamSynchronize(st));
    return TMQ_OK;
}

int tmq_split_eo(tmq_lattice *lat, const double *full, double *even, double *odd)
{
    if (!full || (!even && !odd)) {
        set_error("tmq_split_eo: NULL full field, or both outputs NULL");
        return TMQ_EINVAL;
    }
    return split_merge_host(lat, false, full, nullptr, nullptr, nullptr, even, odd);
}

int tmq_merge_eo(tmq_lattice *lat, const double *even, const double *odd, double *full)
{
    if (!full) {
        set_error("tmq_merge_eo: NULL full field");
        return TMQ_EINVAL;
    }
    return split_merge_host(lat, true, nullptr, full, even, odd, nullptr, nullptr);
}

static void recycle_timed(Lattice *L)
{
    for (auto &t : L->timed) {
        L->event_pool.push_back(t.a);
        L->event_pool.push_back(t.b);
    }
    L->timed.clear();
}

int tmq_set_kernel_timing(tmq_lattice *lat, int on)
{
    TMQ_TRY(check_lat(lat, false));
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    TMQ_HIP(hipDeviceSynchronize());
    recycle_timed(L);
    L->timing = on != 0;
    return TMQ_OK;
}

int tmq_kernel_stats(tmq_lattice *lat, const char *family, int *launches, double *total_ms, double *bytes,
                     double *flops)
{
    TMQ_TRY(check_lat(lat, false));
    // family = base[:part]; base selects the spinor storage, part the epilogue
    std::string base = family ? family : "", part;
    const size_t colon = base.find(':');
    if (colon != std::string::npos) {
        part = base.substr(colon + 1);
        base = base.substr(0, colon);
    }
    int want = -2;  // -1: every hop launch
    if (base == "hop") want = -1;
    if (base == "hop64") want = P64;
    if (base == "hop32") want = P32;
    if (base == "hop16") want = P16;
    // 0 all, 1 the plain half-sweeps (K1, K2), 2 K1, 3 K2, 4 the fused CG and residual epilogues
    const int sel = part.empty() ? 0 : part == "pure" ? 1 : part == "k1" ? 2 : part == "k2" ? 3 : part == "fused" ? 4 : -1;
    if (want == -2 || sel < 0) {
        set_error("tmq_kernel_stats: unknown kernel family (hop, hop64, hop32, hop16, optionally :pure, :k1, :k2 "
                  "or :fused)");
        return TMQ_EINVAL;
    }
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    TMQ_HIP(hipDeviceSynchronize());
    double ms = 0, by = 0, fl = 0;
    int n = 0;
    for (auto &t : L->timed) {
        const int fam = t.prec == PB16 ? P16 : t.prec;
        if (want >= 0 && fam != want) continue;
        const bool fused = t.epi == EPI_K2_CG || t.epi == EPI_K2_RES;
        if ((sel == 1 && fused) || (sel == 2 && t.epi != EPI_K1) || (sel == 3 && t.epi != EPI_K2) ||
            (sel == 4 && !fused))
            continue;
        float e = 0.f;
        TMQ_HIP(hipEventElapsedTime(&e, t.a, t.b));
        ms += e;
        by += t.bytes;
        fl += t.flops;
        n++;
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms;
    if (bytes) *bytes = by;
    if (flops) *flops = fl;
    return TMQ_OK;
}

int tmq_stream_copy(int device, size_t bytes, int reps, double *gbps)
{
    if (bytes < 16 || reps < 1 || !gbps) {
        set_error("tmq_stream_copy: bytes >= 16, reps >= 1 and an output pointer are required");
        return TMQ_EINVAL;
    }
    bytes &= ~(size_t)15;
    DeviceGuard dg(device);
    if (!dg.ok) {
        set_error("tmq_stream_copy: no such HIP device");
        return TMQ_EDEVICE;
    }
    void *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int status = TMQ_OK;
    float ms = 0.f;
    if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
        set_error("tmq_stream_copy: allocation failed");
        status = TMQ_ENOMEM;
    } else if (hipMemset(a, 0, bytes) != hipSuccess ||
               hipEventCreateWithFlags(&e0, hipEventDisableSystemFence) != hipSuccess ||
               hipEventCreateWithFlags(&e1, hipEventDisableSystemFence) != hipSuccess ||
               launch_stream_copy(a, b, bytes, nullptr) != hipSuccess ||
               hipEventRecord(e0, nullptr) != hipSuccess) {
        set_error("tmq_stream_copy: HIP call failed");
        status = TMQ_EDEVICE;
    } else {
        for (int r = 0; r < reps && status == TMQ_OK; r++)
            if (launch_stream_copy(a, b, bytes, nullptr) != hipSuccess) status = TMQ_EDEVICE;
        if (status == TMQ_OK && (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            status = TMQ_EDEVICE;
        if (status != TMQ_OK) set_error("tmq_stream_copy: HIP call failed");
    }
    if (status == TMQ_OK) *gbps = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (a) hipFree(a);
    if (b) hipFree(b);
    return status;
}

int tmq_tuning_report(tmq_lattice *lat, char *buf, size_t len)
{
    TMQ_TRY(check_lat(lat, false));
    if (!buf || len == 0) {
        set_error("tmq_tuning_report: NULL buffer");
        return TMQ_EINVAL;
    }
    const std::string s = tuning_report(lat->L);
    snprintf(buf, len, "%s", s.c_str());
    return s.size() < len ? TMQ_OK : TMQ_EINVAL;
}

int tmq_encode_dev(tmq_lattice *lat, tmq_prec prec, long n_sites, const double *in, uint16_t *codes, float *scale,
                   void *stream)
{
    TMQ_TRY(check_lat(lat, false));
    if (prec != TMQ_FP16 && prec != TMQ_BF16) {
        set_error("tmq_encode_dev: prec must be TMQ_FP16 or TMQ_BF16");
        return TMQ_EINVAL;
    }
    if (n_sites < 0 || (n_sites > 0 && (!in || !codes || !scale))) {
        set_error("tmq_encode_dev: bad size or NULL pointer");
        return TMQ_EINVAL;
    }
    if (n_sites == 0) return TMQ_OK;
    Lattice *L = lat->L;
    DeviceGuard dg(L->device);
    hipStream_t st = (hipStream_t)stream;
    FieldDesc f;
    TMQ_TRY(work_field(L, "codec", prec, (n_sites + 7) / 8 * 8, &f));  // whole 8-site chunks
    f.n = n_sites;
    TMQ_HIP(launch_from_canonical((const double2 *)in, f, st));
    TMQ_HIP(launch_export_codes(f, codes, scale, st));
    return TMQ_OK;
}

int tmq_footprint_bytes(const int dims[4], const tmq_solver_opts *opts, int nrhs, size_t *out)
{
    if (!dims || !out || nrhs < 1) {
        set_error("tmq_footprint_bytes: bad argument");
        return TMQ_EINVAL;
    }
    for (int i = 0; i < 4; i++)
        if (dims[i] < 2 || dims[i] % 2) {
            set_error("tmq_footprint_bytes: every extent must be even and >= 2");
            return TMQ_EINVAL;
        }
    const long vh = (long)dims[0] * dims[1] * dims[2] * dims[3] / 2;
    // gauge copies: FP64 full + FP64, FP32, FP16 two-row, both parities, 4 directions
    size_t g = (size_t)8 * vh * (9 * 16 + 6 * 16 + 3 * 16 + 24);
    // work fields of one right-hand side in a CG engine
    const size_t per = engine_slot_bytes(vh, opts ? opts->sloppy : TMQ_FP64, opts ? opts->mode : 0);
    *out = g + per * (size_t)nrhs;
    return TMQ_OK;
}

}  // extern "C"
