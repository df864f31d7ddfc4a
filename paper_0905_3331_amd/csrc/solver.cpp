// solver.cpp -- CG on Qhat^+ Qhat^- (even/odd) and on Q^+ Q^- (full lattice).
//
// Textbook CG (Sec. 4.4) with every vector operation, inner product and
// scalar (alpha, beta, convergence) on the device: the host only enqueues
// work and reads one small scalar record per right-hand side and iteration,
// one iteration behind the device, so the GPU never waits for the host.
// Kernels skip the blocks of right-hand sides that are done.
//
// A batch of right-hand sides (each with its own kappa and mu, common
// boundary phases) advances in lock step through the same launches; one
// right-hand side alone is the batch of one and goes through exactly the same
// arithmetic, so a batched solution equals its solve alone bit for bit.
//
// Mixed precision (the paper's reduced-precision CG with a true-residual
// check, Sec. 4.4): the iteration runs with FP32 arithmetic on FP32/FP16/BF16
// spinors and reduced-precision two-row links, accumulating its correction
// in an FP32 vector x_s.  Whenever the iterated residual has fallen by delta
// relative to the largest residual since the last such step, a reliable
// update folds x_s into the FP64 solution x, recomputes r = b - A x with the
// FP64 operator, and continues the recursion from that true residual with the
// same search direction.  Convergence is only declared on a recomputed FP64
// true residual: when the iterated residual meets the tolerance, the next
// step is a reliable update.  The host reads the scalars one iteration late,
// so an update is triggered by the residual of the iteration before; this is
// a deterministic rule of its own.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "lattice.h"

namespace tmq {

struct SolveWork {
    FieldDesc b, x;          // FP64 odd
    FieldDesc r64, ax64;     // FP64 odd
    FieldDesc te64, to64;    // FP64 even / odd temporaries of A
    FieldDesc rs, ps, aps;   // sloppy odd
    FieldDesc tes, tos;      // sloppy even / odd temporaries
    FieldDesc xs;            // sloppy solution correction (FP32, or the FP64 x itself)
    LinkDesc lk64, lks;
    OpParams op;
    bool mixed;
};

static int reliable_update(Lattice *L, SolveWork &w, const RhsList &rl, const tmq_solver_opts &o, hipStream_t st,
                           CgScalars *publish)
{
    if (rl.n == 0) return TMQ_OK;
    if (w.mixed) TMQ_HIP(launch_accumulate(w.x, w.xs, rl, st));
    TMQ_TRY(apply_QhatQhat(L, w.op, w.x, w.ax64, w.te64, w.to64, w.lk64, rl, nullptr, nullptr, st));
    TMQ_HIP(launch_residual(w.b, w.ax64, w.r64, rl, L->partial[2], L->pstride, st));
    TMQ_HIP(launch_scalar(SC_RELIABLE, rl, L->partial[2], L->pstride, blas_grid(w.b.n), L->scal, o.tol * o.tol,
                          o.relative, false, publish, st));
    if (w.mixed) TMQ_HIP(launch_convert(w.r64, w.rs, rl, st));
    return TMQ_OK;
}

static int read_scalars(Lattice *L, int n, hipStream_t st, std::vector<CgScalars> &out)
{
    TMQ_HIP(hipStreamSynchronize(st));
    out.resize(n);
    TMQ_HIP(hipMemcpy(out.data(), L->scal, sizeof(CgScalars) * n, hipMemcpyDeviceToHost));
    return TMQ_OK;
}

// one CG iteration for the RHS of rl (done ones skip); scalars published to `publish`
static int cg_body(Lattice *L, SolveWork &w, const RhsList &rl, hipStream_t st, CgScalars *publish)
{
    CgScalars *S = L->scal;
    // t = Qhat^- p, <p, A p> = |t|^2 ; Ap = Qhat^+ t
    TMQ_TRY(apply_Qhat(L, w.op, -1, w.ps, w.tos, w.tes, w.lks, rl, L->partial[0], S, st));
    TMQ_HIP(launch_scalar(SC_ALPHA, rl, L->partial[0], L->pstride, L->hop_blocks_last, S, 0, 0, true, nullptr, st));
    TMQ_TRY(apply_Qhat(L, w.op, +1, w.tos, w.aps, w.tes, w.lks, rl, nullptr, S, st));
    // x_s += alpha p ; r -= alpha A p ; |r|^2 ; beta
    TMQ_HIP(launch_axpy_norm(w.xs, w.ps, w.rs, w.aps, rl, S, L->partial[1], L->pstride, true, st));
    TMQ_HIP(launch_scalar(SC_BETA, rl, L->partial[1], L->pstride, blas_grid(w.ps.n), S, 0, 0, true, publish, st));
    return TMQ_OK;
}

static RhsList make_list(const std::vector<int> &idx)
{
    RhsList l;
    l.n = (int)idx.size();
    for (int i = 0; i < l.n; i++) l.idx[i] = (unsigned char)idx[i];
    return l;
}

int solve_batch(Lattice *L, int n, const tmq_params *p, const tmq_solver_opts &o, const FieldDesc &b,
                const FieldDesc &x, hipStream_t st, tmq_solve_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const long vh = L->g.vh;
    SolveWork w{};
    w.b = b;
    w.x = x;
    w.mixed = o.sloppy != TMQ_FP64;
    w.op = make_op(L, p, n);
    w.lk64 = lattice_links(L, link_fmt_for(L, P64, P64));
    TMQ_TRY(work_field(L, "r64", P64, vh, &w.r64, n));
    TMQ_TRY(work_field(L, "ax64", P64, vh, &w.ax64, n));
    TMQ_TRY(work_field(L, "te64", P64, vh, &w.te64, n));
    TMQ_TRY(work_field(L, "to64", P64, vh, &w.to64, n));
    if (w.mixed) {
        const int sp = o.sloppy;
        w.lks = lattice_links(L, link_fmt_for(L, sp, o.sloppy_link));
        TMQ_TRY(work_field(L, "rs", sp, vh, &w.rs, n));
        TMQ_TRY(work_field(L, "ps", sp, vh, &w.ps, n));
        TMQ_TRY(work_field(L, "aps", sp, vh, &w.aps, n));
        TMQ_TRY(work_field(L, "tes", sp, vh, &w.tes, n));
        TMQ_TRY(work_field(L, "tos", sp, vh, &w.tos, n));
        TMQ_TRY(work_field(L, "xs", P32, vh, &w.xs, n));
    } else {
        w.lks = w.lk64;
        w.rs = w.r64;
        w.xs = w.x;
        TMQ_TRY(work_field(L, "ps64", P64, vh, &w.ps, n));
        TMQ_TRY(work_field(L, "aps64", P64, vh, &w.aps, n));
        w.tes = w.te64;
        w.tos = w.to64;
    }
    // default trigger: the FP32 recursion stays faithful over 4 decades, FP16 over
    // about 2, BF16 (8-bit mantissa) over a little more than 1
    const double delta = o.delta > 0.0 && o.delta < 1.0 ? o.delta
                         : o.sloppy == TMQ_FP32                ? 1e-4
                         : o.sloppy == TMQ_BF16                ? 0.05
                                                               : 0.02;
    const int max_iter = o.max_iter > 0 ? o.max_iter : 10000;
    CgScalars *S = L->scal;
    const RhsList all = rhs_all(n);

    // x = 0 ; r = b ; p = r ; bb = |b|^2
    TMQ_HIP(launch_zero(w.x, all, st));
    TMQ_HIP(launch_convert(w.b, w.r64, all, st));
    TMQ_HIP(launch_norm2(w.r64, all, L->partial[1], L->pstride, st));
    TMQ_HIP(launch_scalar(SC_INIT, all, L->partial[1], L->pstride, blas_grid(vh), S, o.tol * o.tol, o.relative, false,
                          nullptr, st));
    if (w.mixed) {
        TMQ_HIP(launch_convert(w.r64, w.rs, all, st));
        TMQ_HIP(launch_zero(w.xs, all, st));
    }
    TMQ_HIP(launch_convert(w.rs, w.ps, all, st));
    std::vector<CgScalars> cur;
    TMQ_TRY(read_scalars(L, n, st, cur));

    std::vector<int> act;  // RHS still iterating
    std::vector<double> maxr2(n);
    for (int r = 0; r < n; r++) {
        maxr2[r] = cur[r].rr;
        if (!(cur[r].done || cur[r].nan)) act.push_back(r);
    }

    int enq = 0;  // iteration bodies enqueued
    while (!act.empty() && enq < max_iter) {
        const int slot = enq % Lattice::RING;
        CgScalars *pub = L->ring_dev + (size_t)slot * MAX_RHS;
        const RhsList al = make_list(act);
        TMQ_TRY(cg_body(L, w, al, st, pub));
        // while the GPU runs this iteration, read the previous one's scalars
        std::vector<int> ru, keep;
        if (enq > 0) {
            const int ps = (enq - 1) % Lattice::RING;
            TMQ_HIP(hipEventSynchronize(L->ring_ev[ps]));
            const CgScalars *prev = L->ring + (size_t)ps * MAX_RHS;
            for (int r : act) {
                const CgScalars pv = prev[r];
                if (pv.nan || (pv.done && pv.last_true)) continue;  // finished: leaves the active set
                keep.push_back(r);
                if (pv.done) {  // iterated residual met the tolerance: check the true one
                    ru.push_back(r);
                    continue;
                }
                if (pv.last_true || pv.rr > maxr2[r]) maxr2[r] = pv.rr;
                if (w.mixed && pv.rr < delta * delta * maxr2[r]) ru.push_back(r);
            }
        } else {
            keep = act;
        }
        // a reliable update after this iteration republishes its RHS's scalars to the same slot
        TMQ_TRY(reliable_update(L, w, make_list(ru), o, st, pub));
        TMQ_HIP(launch_xpay(w.rs, w.ps, al, S, true, st));
        TMQ_HIP(hipEventRecord(L->ring_ev[slot], st));
        enq++;
        act = keep;
    }
    TMQ_TRY(read_scalars(L, n, st, cur));
    // stopped by max_iter before a true residual: fold in x_s and measure it
    std::vector<int> fin;
    for (int r = 0; r < n; r++)
        if (!cur[r].nan && !cur[r].last_true) fin.push_back(r);
    if (!fin.empty()) {
        TMQ_TRY(reliable_update(L, w, make_list(fin), o, st, nullptr));
        TMQ_TRY(read_scalars(L, n, st, cur));
    }
    int status = TMQ_OK;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int r = 0; r < n; r++) {
        int sr = TMQ_OK;
        if (cur[r].nan)
            sr = TMQ_ENAN;
        else if (!cur[r].done)
            sr = TMQ_ENOCONV;
        if (sr == TMQ_ENAN || (sr == TMQ_ENOCONV && status == TMQ_OK)) status = sr;
        if (info) {
            info[r].status = sr;
            info[r].iters = cur[r].iter;
            info[r].reliable_updates = cur[r].reliable;
            info[r].true_rel_residual = cur[r].bb > 0 ? std::sqrt(cur[r].rr / cur[r].bb) : std::sqrt(cur[r].rr);
            info[r].seconds = secs;
        }
    }
    if (status == TMQ_ENAN) set_error("tmq_solve: non-finite value in CG");
    if (status == TMQ_ENOCONV) set_error("tmq_solve: max_iter reached before the tolerance");
    return status;
}

// ------------------------------------------------------ full lattice CG

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

    // t = Q^- in ; out = Q^+ t ; partial = |t|^2
    auto apply_A = [&](const FieldDesc &in, const FieldDesc &out, double *partial) -> int {
        TMQ_TRY(apply_Q_full(L, op, -1, in, t, lk, one, st));
        if (partial) TMQ_HIP(launch_norm2(t, one, partial, ps, st));
        TMQ_TRY(apply_Q_full(L, op, +1, t, out, lk, one, st));
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
        while (enq < max_iter) {
            const int slot = enq % Lattice::RING;
            TMQ_TRY(apply_A(pp, ap, L->partial[0]));
            TMQ_HIP(launch_scalar(SC_ALPHA, one, L->partial[0], ps, blas_grid(n), S, 0, 0, true, nullptr, st));
            TMQ_HIP(launch_axpy_norm(x, pp, r, ap, one, S, L->partial[1], ps, true, st));
            TMQ_HIP(launch_scalar(SC_BETA, one, L->partial[1], ps, blas_grid(n), S, 0, 0, true,
                                  L->ring_dev + (size_t)slot * MAX_RHS, st));
            TMQ_HIP(launch_xpay(r, pp, one, S, true, st));
            TMQ_HIP(hipEventRecord(L->ring_ev[slot], st));
            enq++;
            if (enq > 1) {
                const int pslot = (enq - 2) % Lattice::RING;
                TMQ_HIP(hipEventSynchronize(L->ring_ev[pslot]));
                const CgScalars pv = L->ring[(size_t)pslot * MAX_RHS];
                if (pv.done || pv.nan) break;
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
