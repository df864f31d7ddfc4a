// solver.cpp -- CG on Qhat^+ Qhat^- (even/odd) and on Q^+ Q^- (full lattice).
//
// Even/odd solves run on a CG engine of the lattice (engine.h): the batch's
// right-hand sides join the engine's slots together and step until every one
// has finished.  A single solve is the batch of one, and each right-hand side
// goes through exactly the same arithmetic whatever shares the batch, so a
// batched solution equals its solve alone bit for bit.
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <vector>

#include "engine.h"

namespace tmq {

// the lattice's engine for this inner precision and link format with at
// least n slots (grown by reallocation when a larger batch comes)
static int lattice_engine(Lattice *L, const tmq_solver_opts &o, int n, bool nd, Engine **out)
{
    const int sp = o.sloppy;
    const int lk = sp == P64 ? link_fmt_for(L, P64, P64) : link_fmt_for(L, sp, o.sloppy_link);
    for (size_t i = 0; i < L->engines.size(); i++) {
        Engine *E = L->engines[i];
        if (E->sloppy != sp || E->lks.fmt != lk || E->mode != o.mode || E->nd != nd) continue;
        if (E->cap >= n) {
            *out = E;
            return TMQ_OK;
        }
        delete E;
        L->engines.erase(L->engines.begin() + (long)i);
        break;
    }
    Engine *E = nullptr;
    TMQ_TRY(engine_create(L, sp, o.sloppy_link, o.mode, n, nullptr, &E, nd));
    L->engines.push_back(E);
    *out = E;
    return TMQ_OK;
}

// leaves the engine idle (every slot free, no stream) however the solve ends
struct EngineScope {
    Engine *E;
    ~EngineScope()
    {
        if (E->st) hipStreamSynchronize(E->st);
        E->st = nullptr;
        for (auto &s : E->slots) s = Engine::Slot{};
        E->body_pending = false;
    }
};

// eps != nullptr: the right-hand sides are flavour doublets with 2 kappa
// epsbar = eps[r] (and 2 kappa mubar = p[r].mu_tilde)
int solve_batch(Lattice *L, int n, const tmq_params *p, const tmq_solver_opts &o, const double *const *b,
                double *const *x, hipStream_t st, tmq_solve_info *info, const double *eps)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (o.mode == TMQ_MODE_BICGSTAB) {
        set_error("TMQ_MODE_BICGSTAB solves Qhat x = b (tmq_solve_Qhat) or M psi = phi (tmq_solve_M), "
                  "not the normal equations");
        return TMQ_EINVAL;
    }
    Engine *E = nullptr;
    TMQ_TRY(lattice_engine(L, o, n, eps != nullptr, &E));
    E->st = st;
    EngineScope scope{E};
    // TMQ_ENGINE_GRAPHS=1: run the iteration bodies as captured HIP graphs
    const char *eg = getenv("TMQ_ENGINE_GRAPHS");
    TMQ_TRY(engine_set_graphs(E, eg && eg[0] == '1'));
    for (int r = 0; r < n; r++) TMQ_TRY(engine_join(E, r, p[r], o, (const double2 *)b[r], eps ? eps[r] : 0.0));
    while (engine_running(E) > 0) {
        TMQ_TRY(engine_begin_step(E));
        TMQ_TRY(engine_end_step(E, nullptr));
    }
    int status = TMQ_OK;
    for (int r = 0; r < n; r++) {
        tmq_solve_info ir{};
        TMQ_TRY(engine_take(E, r, (double2 *)x[r], &ir));
        if (ir.status == TMQ_ENAN || (ir.status == TMQ_ENOCONV && status == TMQ_OK)) status = ir.status;
        if (info) info[r] = ir;
    }
    TMQ_HIP(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info)
        for (int r = 0; r < n; r++) info[r].seconds = secs;
    if (status == TMQ_ENAN) set_error("tmq_solve: non-finite value in CG");
    if (status == TMQ_ENOCONV) set_error("tmq_solve: max_iter reached before the tolerance");
    return status;
}

// the sum of nb per-block partials (device), on the host in a fixed order
static int field_norm2_partials(Lattice *, const double *partial, int nb, hipStream_t st, double *out)
{
    std::vector<double> part(nb);
    TMQ_HIP(hipMemcpyAsync(part.data(), partial, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    TMQ_HIP(hipStreamSynchronize(st));
    double s = 0.0;
    for (double x : part) s += x;
    *out = s;
    return TMQ_OK;
}

// |v|^2 of a one-RHS FP64 field, summed on the host in a fixed order
static int field_norm2(Lattice *L, const FieldDesc &v, hipStream_t st, double *out)
{
    TMQ_HIP(launch_norm2(v, rhs_all(1), L->partial[2], L->pstride, st));
    return field_norm2_partials(L, L->partial[2], blas_grid(v.n), st, out);
}

// ------------------------------------------------- BiCGstab on Qhat^{+-}

static int bicg_state(Lattice *L)
{
    if (L->bicg) return TMQ_OK;
    if (hipMalloc((void **)&L->bicg, sizeof(BicgScalars)) != hipSuccess) {
        L->bicg = nullptr;
        set_error("BiCGstab: device allocation of scalars failed");
        return TMQ_ENOMEM;
    }
    if (hipHostMalloc((void **)&L->bicg_ring, 2 * sizeof(BicgScalars), hipHostMallocMapped) != hipSuccess) {
        L->bicg_ring = nullptr;
        set_error("BiCGstab: pinned scalar allocation failed");
        return TMQ_ENOMEM;
    }
    TMQ_HIP(hipHostGetDevicePointer((void **)&L->bicg_ring_dev, L->bicg_ring, 0));
    for (auto &e : L->bicg_ev) TMQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return TMQ_OK;
}

// Solve Qhat^{sign} x = b (odd-site FP64 fields) by BiCGstab, x_0 = 0.  The
// host enqueues iteration k, then reads the scalars of iteration k - 1 (the
// device skips the work of an iteration once it has flagged the solve done).
// When the iterated residual meets the target, or the recursion breaks down
// (rho or omega zero), the FP64 true residual b - Qhat x is recomputed: the
// solve ends if it meets the target, else BiCGstab restarts from it.
int solve_qhat_bicgstab(Lattice *L, const tmq_params &p, int sign, const tmq_solver_opts &o, const FieldDesc &fb,
                        const FieldDesc &fx, hipStream_t st, tmq_solve_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const long vh = L->g.vh;
    TMQ_TRY(bicg_state(L));
    FieldDesc r, rh, pp, v, s, t, te;
    TMQ_TRY(work_field(L, "bi_r", P64, vh, &r));
    TMQ_TRY(work_field(L, "bi_rh", P64, vh, &rh));
    TMQ_TRY(work_field(L, "bi_p", P64, vh, &pp));
    TMQ_TRY(work_field(L, "bi_v", P64, vh, &v));
    TMQ_TRY(work_field(L, "bi_s", P64, vh, &s));
    TMQ_TRY(work_field(L, "bi_t", P64, vh, &t));
    TMQ_TRY(work_field(L, "bi_te", P64, vh, &te));
    const OpParams op = make_op(L, &p, 1);
    const RhsList one = rhs_all(1);
    const LinkDesc lk = lattice_links(L, link_fmt_for(L, P64, P64));
    double *P0 = L->partial[0], *P1 = L->partial[1], *P2 = L->partial[2];
    const int nparts = blas_grid(vh);
    const int max_iter = o.max_iter > 0 ? o.max_iter : 10000;
    const double tol2 = o.tol * o.tol;
    BicgScalars *S = L->bicg;

    BicgScalars init{};
    init.max_iter = max_iter;
    TMQ_HIP(hipStreamSynchronize(st));
    TMQ_HIP(hipMemcpy(S, &init, sizeof(BicgScalars), hipMemcpyHostToDevice));
    TMQ_HIP(launch_zero(fx, one, st));
    TMQ_HIP(launch_convert(fb, r, one, st));
    int status = TMQ_OK, truths = 0;
    double rr_true = 0.0;
    BicgScalars last{};
    for (int restart = 0;; restart++) {
        // rhat = r ; p = v = 0 ; rho = <rhat, r>
        TMQ_HIP(launch_convert(r, rh, one, st));
        TMQ_HIP(launch_zero(pp, one, st));
        TMQ_HIP(launch_zero(v, one, st));
        TMQ_HIP(launch_bi_dot(rh, r, nullptr, P0, P1, P2, st));
        TMQ_HIP(launch_bi_scalar(BI_START, P0, P1, P2, nparts, S, tol2, o.relative, nullptr, st));
        for (long k = 0;; k++) {
            TMQ_HIP(launch_bi_p(r, pp, v, S, st));
            TMQ_TRY(apply_Qhat(L, op, sign, pp, v, te, lk, one, nullptr, nullptr, st));
            TMQ_HIP(launch_bi_dot(rh, v, S, P0, P1, P2, st));
            TMQ_HIP(launch_bi_scalar(BI_ALPHA, P0, P1, P2, nparts, S, 0.0, 0, nullptr, st));
            TMQ_HIP(launch_bi_s(r, v, s, S, st));
            TMQ_TRY(apply_Qhat(L, op, sign, s, t, te, lk, one, nullptr, nullptr, st));
            TMQ_HIP(launch_bi_dot(t, s, S, P0, P1, P2, st));
            TMQ_HIP(launch_bi_scalar(BI_OMEGA, P0, P1, P2, nparts, S, 0.0, 0, nullptr, st));
            TMQ_HIP(launch_bi_xr(fx, pp, s, t, r, rh, S, P0, P1, P2, st));
            TMQ_HIP(launch_bi_scalar(BI_UPDATE, P0, P1, P2, nparts, S, 0.0, 0, L->bicg_ring_dev + (k & 1), st));
            TMQ_HIP(hipEventRecord(L->bicg_ev[k & 1], st));
            if (k == 0) continue;
            TMQ_HIP(hipEventSynchronize(L->bicg_ev[(k - 1) & 1]));
            const BicgScalars prev = L->bicg_ring[(k - 1) & 1];
            if (prev.done) break;
        }
        TMQ_HIP(hipStreamSynchronize(st));
        TMQ_HIP(hipMemcpy(&last, S, sizeof(BicgScalars), hipMemcpyDeviceToHost));
        if (last.nan) {
            status = TMQ_ENAN;
            break;
        }
        // the true residual r = b - Qhat x
        TMQ_TRY(apply_Qhat(L, op, sign, fx, t, te, lk, one, nullptr, nullptr, st));
        TMQ_HIP(launch_residual(fb, t, r, one, P2, L->pstride, st));
        TMQ_TRY(field_norm2_partials(L, P2, nparts, st, &rr_true));
        truths++;
        if (!std::isfinite(rr_true)) {
            status = TMQ_ENAN;
            break;
        }
        if (rr_true <= last.target) break;
        if (last.iter >= max_iter || restart >= 50) {
            status = TMQ_ENOCONV;
            break;
        }
        // restart from the true residual (S keeps |b|^2, the target and the count)
        BicgScalars keep = last;
        keep.restarts = restart + 1;
        keep.done = 0;
        TMQ_HIP(hipStreamSynchronize(st));
        TMQ_HIP(hipMemcpy(S, &keep, sizeof(BicgScalars), hipMemcpyHostToDevice));
    }
    TMQ_HIP(hipStreamSynchronize(st));
    if (info) {
        info->status = status;
        info->iters = last.iter;
        info->reliable_updates = truths;
        info->true_rel_residual = last.bb > 0 ? std::sqrt(rr_true / last.bb) : std::sqrt(rr_true);
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (status == TMQ_ENAN) set_error("BiCGstab: non-finite value");
    if (status == TMQ_ENOCONV) set_error("BiCGstab: tolerance not reached within max_iter");
    return status;
}

// ------------------------------------------- M psi = phi through even/odd



// Solve M^{sign} psi = phi (full lattice, canonical device buffers) with the
// even/odd factorisation of the inversion in App. B:
//   phi'_e = (M_ee)^-1 phi_e,  phi'_o = phi_o - M_oe (M_ee)^-1 phi_e,
//   psi_o  = (M_oo - M_oe (M_ee)^-1 M_eo)^-1 phi'_o,
//   psi_e  = phi'_e - (M_ee)^-1 M_eo psi_o = (M_ee)^-1 (phi_e + kappa H_eo psi_o),
// with M_ee = 1 + sign i mut g5, M_eo = -kappa H_eo, M_oe = -kappa H_oe.  The
// Schur complement is g5 Qhat^{sign} (eq. (eo4)), so psi_o solves
// Qhat^{sign} psi_o = g5 phi'_o: psi_o = Qhat^- A^-1 g5 phi'_o for sign +1
// and psi_o = A^-1 Qhat^+ g5 phi'_o for sign -1, A = Qhat^+ Qhat^- by CG.
// The residual phi - M psi is recomputed in FP64 on the full lattice; while
// it is above the tolerance the same steps solve for the correction.
// per-RHS |v|^2 of the RHS in rl of a batched FP64 field, summed on the host in a fixed order
static int field_norms(Lattice *L, const FieldDesc &v, const RhsList &rl, hipStream_t st, std::vector<double> &out)
{
    const int nb = blas_grid(v.n);
    TMQ_HIP(launch_norm2(v, rl, L->partial[2], L->pstride, st));
    std::vector<double> part((size_t)L->pstride * MAX_RHS);
    TMQ_HIP(hipMemcpyAsync(part.data(), L->partial[2], sizeof(double) * part.size(), hipMemcpyDeviceToHost, st));
    TMQ_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < rl.n; i++) {
        const int r = rl.idx[i];
        double s = 0.0;
        for (int k = 0; k < nb; k++) s += part[(size_t)r * L->pstride + k];
        out[r] = s;
    }
    return TMQ_OK;
}

static RhsList rhs_list(const std::vector<int> &idx)
{
    RhsList l;
    l.n = (int)idx.size();
    for (int i = 0; i < l.n; i++) l.idx[i] = (unsigned char)idx[i];
    return l;
}

int solve_M_batch(Lattice *L, const tmq_params &p, int sign, const tmq_solver_opts &o, int nb, const double2 *const *phi,
                  double2 *const *psi, hipStream_t st, tmq_solve_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const long vh = L->g.vh, n = 2 * vh;
    FieldDesc fphi, fpsi, fr, fd, fq, fg, te, to, wo, yo, bc, yc;
    TMQ_TRY(work_field(L, "m_phi", P64, n, &fphi, nb));  // g5 phi
    TMQ_TRY(work_field(L, "m_psi", P64, n, &fpsi, nb));
    TMQ_TRY(work_field(L, "m_r", P64, n, &fr, nb));      // source of the round (the residual)
    TMQ_TRY(work_field(L, "m_d", P64, n, &fd, nb));      // solution of the round
    TMQ_TRY(work_field(L, "m_q", P64, n, &fq, nb));
    TMQ_TRY(work_field(L, "m_g", P64, n, &fg, nb));
    TMQ_TRY(work_field(L, "m_te", P64, vh, &te, nb));
    TMQ_TRY(work_field(L, "m_to", P64, vh, &to, nb));
    TMQ_TRY(work_field(L, "m_wo", P64, vh, &wo, nb));
    TMQ_TRY(work_field(L, "m_yo", P64, vh, &yo, nb));
    TMQ_TRY(work_field(L, "m_bc", P64, vh, &bc, nb));  // canonical odd buffers (same size)
    TMQ_TRY(work_field(L, "m_yc", P64, vh, &yc, nb));
    const std::vector<tmq_params> pv((size_t)nb, p);
    const OpParams op = make_op(L, pv.data(), nb);
    const RhsList all = rhs_all(nb);
    const LinkDesc lk = lattice_links(L, link_fmt_for(L, P64, P64));
    const double m = sign * p.mu_tilde, c = 1.0 / (1.0 + m * m);
    const double2 mee_u = make_double2(c, -c * m), mee_d = make_double2(c, c * m);  // (M_ee)^-1
    const double2 g5_u = make_double2(1.0, 0.0), g5_d = make_double2(-1.0, 0.0);
    const int max_rounds = 4;

    for (int r = 0; r < nb; r++) TMQ_HIP(launch_full_from_canonical(L->g, phi[r], field_rhs(fr, r), st));
    TMQ_HIP(launch_twist(fr, fphi, all, g5_u, g5_d, st));
    TMQ_HIP(launch_zero(fpsi, all, st));
    std::vector<double> bb((size_t)nb), rr((size_t)nb), target((size_t)nb);
    std::vector<int> status((size_t)nb, TMQ_OK), iters((size_t)nb, 0), rus((size_t)nb, 0);
    TMQ_TRY(field_norms(L, fr, all, st, bb));
    std::vector<int> active;
    for (int r = 0; r < nb; r++) {
        target[r] = o.relative ? o.tol * o.tol * bb[r] : o.tol * o.tol;
        rr[r] = bb[r];
        if (rr[r] > target[r] && bb[r] > 0.0) active.push_back(r);
    }
    for (int round = 0; !active.empty() && round < max_rounds; round++) {
        const RhsList al = rhs_list(active);
        const FieldDesc re = field_sub(fr, 0, vh), ro = field_sub(fr, vh, vh);
        const FieldDesc de = field_sub(fd, 0, vh), dd = field_sub(fd, vh, vh);
        // phi'_o = r_o + kappa H_oe (M_ee)^-1 r_e
        TMQ_HIP(launch_twist(re, te, al, mee_u, mee_d, st));
        TMQ_TRY(hop(L, 1, te, ro, wo, lk, op, EPI_SRC, sign, al, nullptr, nullptr, st));
        // odd system: Qhat^{sign} d_o = g5 phi'_o
        TMQ_HIP(launch_twist(wo, to, al, g5_u, g5_d, st));
        if (o.mode == TMQ_MODE_BICGSTAB) {
            // BiCGstab on Qhat^{sign} itself, one right-hand side at a time
            for (int r : active) {
                tmq_solve_info ci{};
                const int cs = solve_qhat_bicgstab(L, p, sign, o, field_rhs(to, r), field_rhs(dd, r), st, &ci);
                iters[r] += ci.iters;
                rus[r] += ci.reliable_updates;
                if (cs != TMQ_OK && cs != TMQ_ENOCONV && cs != TMQ_ENAN) return cs;
                if (cs != TMQ_OK) status[r] = cs;
            }
        } else {
            // CG on Qhat^+ Qhat^- for all of them together
            if (sign < 0) TMQ_TRY(apply_Qhat(L, op, +1, to, wo, te, lk, al, nullptr, nullptr, st));
            const FieldDesc &src = sign < 0 ? wo : to;
            std::vector<const double *> bp;
            std::vector<double *> yp;
            std::vector<tmq_params> pa;
            for (int r : active) {
                TMQ_HIP(launch_to_canonical(field_rhs(src, r), (double2 *)field_rhs(bc, r).data, st));
                bp.push_back((const double *)field_rhs(bc, r).data);
                yp.push_back((double *)field_rhs(yc, r).data);
                pa.push_back(p);
            }
            std::vector<tmq_solve_info> ci(active.size());
            const int cs = solve_batch(L, (int)active.size(), pa.data(), o, bp.data(), yp.data(), st, ci.data(),
                                       nullptr);
            if (cs != TMQ_OK && cs != TMQ_ENOCONV && cs != TMQ_ENAN) return cs;
            for (size_t i = 0; i < active.size(); i++) {
                const int r = active[i];
                iters[r] += ci[i].iters;
                rus[r] += ci[i].reliable_updates;
                if (ci[i].status != TMQ_OK) status[r] = ci[i].status;
                TMQ_HIP(launch_from_canonical((const double2 *)field_rhs(yc, r).data, field_rhs(yo, r), st));
            }
            if (sign > 0)
                TMQ_TRY(apply_Qhat(L, op, -1, yo, dd, te, lk, al, nullptr, nullptr, st));
            else
                TMQ_HIP(launch_convert(yo, dd, al, st));
        }
        // d_e = (M_ee)^-1 (r_e + kappa H_eo d_o) ; psi += d
        TMQ_TRY(hop(L, 0, dd, re, de, lk, op, EPI_REC, sign, al, nullptr, nullptr, st));
        TMQ_HIP(launch_accumulate(fpsi, fd, al, st));
        // r = phi - M psi = g5 (g5 phi - Q psi)
        TMQ_TRY(apply_Q_full(L, op, sign, fpsi, fq, lk, al, st));
        TMQ_HIP(launch_residual(fphi, fq, fg, al, L->partial[2], L->pstride, st));
        TMQ_HIP(launch_twist(fg, fr, al, g5_u, g5_d, st));
        TMQ_TRY(field_norms(L, fr, al, st, rr));
        std::vector<int> next;
        for (int r : active)
            if (status[r] == TMQ_OK && rr[r] > target[r]) next.push_back(r);
        active.swap(next);
    }
    int worst = TMQ_OK;
    for (int r = 0; r < nb; r++) {
        if (!std::isfinite(rr[r])) status[r] = TMQ_ENAN;
        if (status[r] == TMQ_OK && rr[r] > target[r]) status[r] = TMQ_ENOCONV;
        if (status[r] == TMQ_ENAN || (status[r] == TMQ_ENOCONV && worst == TMQ_OK)) worst = status[r];
        TMQ_HIP(launch_full_to_canonical(L->g, field_rhs(fpsi, r), psi[r], st));
    }
    TMQ_HIP(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info)
        for (int r = 0; r < nb; r++) {
            info[r].status = status[r];
            info[r].iters = iters[r];
            info[r].reliable_updates = rus[r];
            info[r].true_rel_residual = bb[r] > 0 ? std::sqrt(rr[r] / bb[r]) : std::sqrt(rr[r]);
            info[r].seconds = secs;
        }
    if (worst == TMQ_ENAN) set_error("tmq_solve_M: non-finite value");
    if (worst == TMQ_ENOCONV) set_error("tmq_solve_M: tolerance not reached");
    return worst;
}

int solve_M(Lattice *L, const tmq_params &p, int sign, const tmq_solver_opts &o, const double2 *phi, double2 *psi,
            hipStream_t st, tmq_solve_info *info)
{
    return solve_M_batch(L, p, sign, o, 1, &phi, &psi, st, info);
}

// ------------------------------------------------------ full lattice CG

static int read_scalars(Lattice *L, int n, hipStream_t st, std::vector<CgScalars> &out)
{
    TMQ_HIP(hipStreamSynchronize(st));
    out.resize(n);
    TMQ_HIP(hipMemcpy(out.data(), L->scal, sizeof(CgScalars) * n, hipMemcpyDeviceToHost));
    return TMQ_OK;
}

// Small lattices are launch-latency bound (a 4^4 iteration is nine kernels
// of a few microseconds).  Tiny ones (at most SMALL_CG_MAX_SITES sites) run
// the whole CG in one workgroup (small_cg.hip); on the others up to
// GRAPH_MAX_SITES sites the iterations run as HIP graphs of CHUNK
// iterations each, captured once per solve, two graphs publishing their
// scalars to the two halves of the ring so that the host reads one chunk
// while the next runs.  Right-hand sides already converged skip their work
// inside a chunk, so the result equals that of single iterations.
constexpr int GRAPH_CHUNK = 4;
constexpr long GRAPH_MAX_SITES = 1L << 16;

int solve_full(Lattice *L, const tmq_params &p, const tmq_solver_opts &o, const FieldDesc &b, const FieldDesc &x,
               hipStream_t st, tmq_solve_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const long n = 2 * L->g.vh;
    FieldDesc r, pp, ap, t;
    TMQ_TRY(work_field(L, "fr", P64, n, &r));
    TMQ_TRY(work_field(L, "fp", P64, n, &pp));
    TMQ_TRY(work_field(L, "fap", P64, n, &ap));
    TMQ_TRY(work_field(L, "ft", P64, n, &t));
    const LinkDesc lk = lattice_links(L, link_fmt_for(L, P64, P64));
    const OpParams op = make_op(L, &p, 1);
    const RhsList one = rhs_all(1);
    const int max_iter = o.max_iter > 0 ? o.max_iter : 10000;
    CgScalars *S = L->scal;
    const double tol2 = o.tol * o.tol;
    const long ps = L->pstride;
    if (n <= SMALL_CG_MAX_SITES && !L->timing && !getenv("TMQ_NO_SMALL_CG")) {
        // the whole CG in one workgroup (small_cg.hip); called again from its
        // true residual if that has not met the target
        const FieldDesc f[6] = {b, x, r, pp, t, ap};
        TMQ_HIP(launch_zero(x, one, st));
        TMQ_HIP(hipMemsetAsync(S, 0, sizeof(CgScalars), st));
        std::vector<CgScalars> cur;
        for (int call = 0;; call++) {
            TMQ_HIP(launch_small_cg(L->g, f, lk, op, tol2, o.relative, max_iter, S, st));
            TMQ_TRY(read_scalars(L, 1, st, cur));
            if (cur[0].done || cur[0].nan || cur[0].iter >= max_iter || call >= 20) break;
        }
        int status = TMQ_OK;
        if (cur[0].nan) {
            status = TMQ_ENAN;
            set_error("tmq_solve_full: non-finite value in CG");
        } else if (!cur[0].done) {
            status = TMQ_ENOCONV;
            set_error("tmq_solve_full: max_iter reached before the tolerance");
        }
        if (info) {
            info->status = status;
            info->iters = cur[0].iter;
            info->reliable_updates = cur[0].reliable;
            info->true_rel_residual = cur[0].bb > 0 ? std::sqrt(cur[0].rr / cur[0].bb) : std::sqrt(cur[0].rr);
            info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        return status;
    }
    const bool graphs = n <= GRAPH_MAX_SITES && !L->timing && !getenv("TMQ_NO_GRAPH");
    if (graphs) {
        // graphs are captured on the lattice's own stream (never the null stream)
        TMQ_HIP(hipStreamSynchronize(st));
        st = L->own;
    }

    // t = Q^- in ; out = Q^+ t ; partial = |t|^2
    auto apply_A = [&](const FieldDesc &in, const FieldDesc &out, double *partial) -> int {
        TMQ_TRY(apply_Q_full(L, op, -1, in, t, lk, one, st));
        if (partial) TMQ_HIP(launch_norm2(t, one, partial, ps, st));
        TMQ_TRY(apply_Q_full(L, op, +1, t, out, lk, one, st));
        return TMQ_OK;
    };
    // one CG iteration publishing its scalars to ring slot `slot`
    auto iterate = [&](int slot) -> int {
        TMQ_TRY(apply_A(pp, ap, L->partial[0]));
        TMQ_HIP(launch_scalar(SC_ALPHA, one, L->partial[0], ps, blas_grid(n), S, 0, 0, true, nullptr, st));
        TMQ_HIP(launch_axpy_norm(x, pp, r, ap, one, S, L->partial[1], ps, true, st));
        TMQ_HIP(launch_scalar(SC_BETA, one, L->partial[1], ps, blas_grid(n), S, 0, 0, true,
                              L->ring_dev + (size_t)slot * MAX_RHS, st));
        TMQ_HIP(launch_xpay(r, pp, one, S, true, st));
        return TMQ_OK;
    };
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    struct GraphScope {
        hipGraph_t *g;
        hipGraphExec_t *e;
        ~GraphScope()
        {
            for (int i = 0; i < 2; i++) {
                if (e[i]) hipGraphExecDestroy(e[i]);
                if (g[i]) hipGraphDestroy(g[i]);
            }
        }
    } gscope{graph, exec};
    auto capture = [&]() -> int {
        for (int h = 0; h < 2; h++) {
            TMQ_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            int rc = TMQ_OK;
            for (int k = 0; k < GRAPH_CHUNK && rc == TMQ_OK; k++) rc = iterate(h * GRAPH_CHUNK + k);
            hipGraph_t gr = nullptr;
            const hipError_t ec = hipStreamEndCapture(st, &gr);
            graph[h] = gr;
            if (rc != TMQ_OK) return rc;
            TMQ_HIP(ec);
            TMQ_HIP(hipGraphInstantiate(&exec[h], graph[h], nullptr, nullptr, 0));
        }
        return TMQ_OK;
    };

    TMQ_HIP(launch_zero(x, one, st));
    TMQ_HIP(launch_convert(b, r, one, st));
    TMQ_HIP(launch_norm2(r, one, L->partial[1], ps, st));
    TMQ_HIP(launch_scalar(SC_INIT, one, L->partial[1], ps, blas_grid(n), S, tol2, o.relative, false, nullptr, st));
    TMQ_HIP(launch_convert(r, pp, one, st));
    std::vector<CgScalars> cur;
    TMQ_TRY(read_scalars(L, 1, st, cur));
    int enq = 0;
    while (!(cur[0].done && cur[0].last_true) && !cur[0].nan && enq < max_iter) {
        if (graphs) {
            // one plain iteration first (it tunes the kernels), then chunks of
            // GRAPH_CHUNK; the host checks chunk c - 1 while chunk c runs
            if (enq == 0) {
                TMQ_TRY(iterate(0));
                enq++;
            }
            if (!exec[0]) TMQ_TRY(capture());
            int c = 0;
            while (enq + GRAPH_CHUNK <= max_iter) {
                TMQ_HIP(hipGraphLaunch(exec[c & 1], st));
                TMQ_HIP(hipEventRecord(L->ring_ev[c & 1], st));
                enq += GRAPH_CHUNK;
                if (c > 0) {
                    const int h = (c - 1) & 1;
                    TMQ_HIP(hipEventSynchronize(L->ring_ev[h]));
                    const CgScalars pv = L->ring[(size_t)(h * GRAPH_CHUNK + GRAPH_CHUNK - 1) * MAX_RHS];
                    if (pv.done || pv.nan) break;
                }
                c++;
            }
            // the last iterations before max_iter, one at a time
            TMQ_TRY(read_scalars(L, 1, st, cur));
            while (!cur[0].done && !cur[0].nan && enq < max_iter) {
                TMQ_TRY(iterate(0));
                enq++;
                TMQ_TRY(read_scalars(L, 1, st, cur));
            }
        } else {
            while (enq < max_iter) {
                const int slot = enq % Lattice::RING;
                TMQ_TRY(iterate(slot));
                TMQ_HIP(hipEventRecord(L->ring_ev[slot], st));
                enq++;
                if (enq > 1) {
                    const int pslot = (enq - 2) % Lattice::RING;
                    TMQ_HIP(hipEventSynchronize(L->ring_ev[pslot]));
                    const CgScalars pv = L->ring[(size_t)pslot * MAX_RHS];
                    if (pv.done || pv.nan) break;
                }
            }
        }
        TMQ_TRY(read_scalars(L, 1, st, cur));
        if (cur[0].nan) break;
        // true residual r = b - A x
        TMQ_TRY(apply_A(x, ap, nullptr));
        TMQ_HIP(launch_residual(b, ap, r, one, L->partial[2], ps, st));
        TMQ_HIP(launch_scalar(SC_RELIABLE, one, L->partial[2], ps, blas_grid(n), S, tol2, o.relative, false, nullptr,
                              st));
        TMQ_TRY(read_scalars(L, 1, st, cur));
        if (cur[0].nan || cur[0].done || enq >= max_iter) break;
        TMQ_HIP(launch_xpay(r, pp, one, S, false, st));
    }
    int status = TMQ_OK;
    if (cur[0].nan) {
        status = TMQ_ENAN;
        set_error("tmq_solve_full: non-finite value in CG");
    } else if (!cur[0].done) {
        status = TMQ_ENOCONV;
        set_error("tmq_solve_full: max_iter reached before the tolerance");
    }
    if (info) {
        info->status = status;
        info->iters = cur[0].iter;
        info->reliable_updates = cur[0].reliable;
        info->true_rel_residual = cur[0].bb > 0 ? std::sqrt(cur[0].rr / cur[0].bb) : std::sqrt(cur[0].rr);
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

}  // namespace tmq
