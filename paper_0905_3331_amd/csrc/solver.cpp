// solver.cpp -- CG on Qhat^+ Qhat^- (even/odd) and on Q^+ Q^- (full lattice).
//
// Textbook CG (Sec. 4.4) with every vector operation, inner product and
// scalar (alpha, beta, convergence) on the device: the host only enqueues
// work and reads one small scalar record per iteration, one iteration behind
// the device, so the GPU never waits for the host.  Kernels take a pointer to
// the device "done" flag and turn into no-ops once the solve has converged.
//
// Mixed precision (the paper's reduced-precision CG with a true-residual
// check, Sec. 4.4): the iteration runs with FP32 arithmetic on FP32/FP16/BF16
// spinors and reduced-precision two-row links, accumulating its correction
// in an FP32 vector x_s.  Whenever the iterated residual has fallen by delta
// relative to the largest residual since the last such step, a reliable
// update folds x_s into the FP64 solution x, recomputes r = b - A x with the
// FP64 operator, and restarts the recursion from that true residual while
// keeping the search direction.  Convergence is only declared on a
// recomputed FP64 true residual.  Because the host reads the scalars one
// iteration late, a reliable update is triggered by the residual of the
// iteration before; this is a deterministic rule of its own.
#include <chrono>
#include <cmath>
#include <cstring>

#include "lattice.h"

namespace tmq {

struct SolveWork {
    FieldDesc b, x;          // FP64 odd, caller's (device SoA)
    FieldDesc r64, ax64;     // FP64 odd
    FieldDesc te64, to64;    // FP64 even / odd temporaries of A
    FieldDesc rs, ps, aps;   // sloppy odd
    FieldDesc tes, tos;      // sloppy even / odd temporaries
    FieldDesc xs;            // sloppy solution correction (FP32 or the FP64 x itself)
    LinkDesc lk64, lks;
    bool mixed;
};

static int reliable_update(Lattice *L, const tmq_params &p, SolveWork &w, const tmq_solver_opts &o,
                           hipStream_t st, CgScalars *publish = nullptr)
{
    CgScalars *S = L->scal;
    if (w.mixed) TMQ_HIP(launch_accumulate(w.x, w.xs, st));
    TMQ_TRY(apply_QhatQhat(L, p, w.x, w.ax64, w.te64, w.to64, w.lk64, nullptr, nullptr, st));
    TMQ_HIP(launch_residual(w.b, w.ax64, w.r64, L->partial[2], st));
    TMQ_HIP(launch_scalar(SC_RELIABLE, L->partial[2], blas_grid(w.b.n), S, o.tol * o.tol, o.relative, nullptr, st,
                          publish));
    if (w.mixed) TMQ_HIP(launch_convert(w.r64, w.rs, st));
    return TMQ_OK;
}

static int read_scalars(Lattice *L, hipStream_t st, CgScalars *out)
{
    TMQ_HIP(hipMemcpyAsync(L->ring, L->scal, sizeof(CgScalars), hipMemcpyDeviceToHost, st));
    TMQ_HIP(hipStreamSynchronize(st));
    *out = L->ring[0];
    return TMQ_OK;
}

// body of one CG iteration; all kernels skip once S->done is set.  The scalars
// after the iteration are published to `publish` (host-mapped) unless a
// reliable update follows, which publishes them itself.
static int cg_body(Lattice *L, const tmq_params &p, SolveWork &w, hipStream_t st, CgScalars *publish)
{
    CgScalars *S = L->scal;
    const int *skip = &S->done;
    // t = Qhat^- p, <p, A p> = |t|^2 ; Ap = Qhat^+ t
    TMQ_TRY(apply_Qhat(L, p, -1, w.ps, w.tos, w.tes, w.lks, L->partial[0], skip, st));
    TMQ_HIP(launch_scalar(SC_ALPHA, L->partial[0], L->hop_blocks_last, S, 0, 0, skip, st));
    TMQ_TRY(apply_Qhat(L, p, +1, w.tos, w.aps, w.tes, w.lks, nullptr, skip, st));
    // x_s += alpha p ; r -= alpha A p ; |r|^2 ; beta
    TMQ_HIP(launch_axpy_norm(w.xs, w.ps, w.rs, w.aps, S, L->partial[1], skip, st));
    TMQ_HIP(launch_scalar(SC_BETA, L->partial[1], blas_grid(w.ps.n), S, 0, 0, skip, st, publish));
    return TMQ_OK;
}

int solve_eo(Lattice *L, const tmq_params &p, const tmq_solver_opts &o, const FieldDesc &b, const FieldDesc &x,
             hipStream_t st, tmq_solve_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    const long vh = L->g.vh;
    SolveWork w{};
    w.b = b;
    w.x = x;
    w.mixed = o.sloppy != TMQ_FP64;
    w.lk64 = lattice_links(L, link_fmt_for(L, P64, P64));
    TMQ_TRY(work_field(L, "r64", P64, vh, &w.r64));
    TMQ_TRY(work_field(L, "ax64", P64, vh, &w.ax64));
    TMQ_TRY(work_field(L, "te64", P64, vh, &w.te64));
    TMQ_TRY(work_field(L, "to64", P64, vh, &w.to64));
    if (w.mixed) {
        const int sp = o.sloppy;
        w.lks = lattice_links(L, link_fmt_for(L, sp, o.sloppy_link));
        TMQ_TRY(work_field(L, "rs", sp, vh, &w.rs));
        TMQ_TRY(work_field(L, "ps", sp, vh, &w.ps));
        TMQ_TRY(work_field(L, "aps", sp, vh, &w.aps));
        TMQ_TRY(work_field(L, "tes", sp, vh, &w.tes));
        TMQ_TRY(work_field(L, "tos", sp, vh, &w.tos));
        TMQ_TRY(work_field(L, "xs", P32, vh, &w.xs));
    } else {
        w.lks = w.lk64;
        w.rs = w.r64;
        w.xs = w.x;
        TMQ_TRY(work_field(L, "ps64", P64, vh, &w.ps));
        TMQ_TRY(work_field(L, "aps64", P64, vh, &w.aps));
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

    // x = 0 ; r = b ; p = r ; bb = |b|^2
    TMQ_HIP(launch_zero(w.x, st));
    TMQ_HIP(launch_convert(w.b, w.r64, st));
    TMQ_HIP(launch_norm2(w.r64, L->partial[1], st));
    TMQ_HIP(launch_scalar(SC_INIT, L->partial[1], blas_grid(vh), S, o.tol * o.tol, o.relative, nullptr, st));
    if (w.mixed) {
        TMQ_HIP(launch_convert(w.r64, w.rs, st));
        TMQ_HIP(launch_zero(w.xs, st));
    }
    TMQ_HIP(launch_convert(w.rs, w.ps, st));
    CgScalars cur{};
    TMQ_TRY(read_scalars(L, st, &cur));

    int status = TMQ_OK;
    int enq = 0;  // iteration bodies enqueued
    double maxr2 = cur.rr;
    while (!(cur.done && cur.last_true) && !cur.nan && enq < max_iter) {
        // lagged loop: enqueue body k, then read the scalars of iteration k - 1
        bool leave = false;
        int k0 = enq;
        while (!leave && enq < max_iter) {
            // enqueue iteration `enq` (its scalars go to ring slot `slot`), then,
            // while the GPU runs it, read the scalars of iteration enq - 1
            const int slot = enq % Lattice::RING;
            TMQ_TRY(cg_body(L, p, w, st, &L->ring_dev[slot]));
            bool ru = false;
            if (enq > k0) {
                const int ps = (enq - 1) % Lattice::RING;
                TMQ_HIP(hipEventSynchronize(L->ring_ev[ps]));
                const CgScalars prev = L->ring[ps];
                if (prev.nan || prev.done) leave = true;
                if (prev.last_true)
                    maxr2 = prev.rr;
                else if (prev.rr > maxr2)
                    maxr2 = prev.rr;
                ru = !leave && w.mixed && prev.rr < delta * delta * maxr2;
            }
            // a reliable update after this iteration republishes the scalars to the same slot
            if (ru) TMQ_TRY(reliable_update(L, p, w, o, st, &L->ring_dev[slot]));
            TMQ_HIP(launch_xpay(w.rs, w.ps, S, &S->done, st));
            TMQ_HIP(hipEventRecord(L->ring_ev[slot], st));
            enq++;
        }
        TMQ_TRY(read_scalars(L, st, &cur));
        if (cur.nan) break;
        if (cur.done && cur.last_true) break;
        // iterated residual converged (or iterations exhausted): check the FP64 true residual
        TMQ_TRY(reliable_update(L, p, w, o, st));
        TMQ_TRY(read_scalars(L, st, &cur));
        maxr2 = cur.rr;
        if (cur.nan || (cur.done && cur.last_true)) break;
        if (enq >= max_iter) break;
        // not yet: continue from the true residual with p = r + beta p
        TMQ_HIP(launch_xpay(w.rs, w.ps, S, nullptr, st));
    }
    if (!cur.nan && !cur.last_true) {
        // left on max_iter before a true residual: fold in x_s and measure it
        TMQ_TRY(reliable_update(L, p, w, o, st));
        TMQ_TRY(read_scalars(L, st, &cur));
    }
    if (cur.nan) {
        status = TMQ_ENAN;
        set_error("tmq_solve: non-finite value in CG");
    } else if (!cur.done) {
        status = TMQ_ENOCONV;
        set_error("tmq_solve: max_iter reached before the tolerance");
    }
    if (info) {
        info->status = status;
        info->iters = cur.iter;
        info->reliable_updates = cur.reliable;
        info->true_rel_residual = cur.bb > 0 ? std::sqrt(cur.rr / cur.bb) : std::sqrt(cur.rr);
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
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
    const int max_iter = o.max_iter > 0 ? o.max_iter : 10000;
    CgScalars *S = L->scal;
    const double tol2 = o.tol * o.tol;

    auto apply_A = [&](const FieldDesc &in, const FieldDesc &out, double *partial, const int *skip) -> int {
        // t = Q^- in ; out = Q^+ t ; partial = |t|^2
        (void)skip;
        TMQ_TRY(apply_Q_full(L, p, -1, in, t, lk, st));
        if (partial) TMQ_HIP(launch_norm2(t, partial, st));
        TMQ_TRY(apply_Q_full(L, p, +1, t, out, lk, st));
        return TMQ_OK;
    };

    TMQ_HIP(launch_zero(x, st));
    TMQ_HIP(launch_convert(b, r, st));
    TMQ_HIP(launch_norm2(r, L->partial[1], st));
    TMQ_HIP(launch_scalar(SC_INIT, L->partial[1], blas_grid(n), S, tol2, o.relative, nullptr, st));
    TMQ_HIP(launch_convert(r, pp, st));
    CgScalars cur{};
    TMQ_TRY(read_scalars(L, st, &cur));
    int enq = 0;
    while (!(cur.done && cur.last_true) && !cur.nan && enq < max_iter) {
        while (enq < max_iter) {
            TMQ_TRY(apply_A(pp, ap, L->partial[0], &S->done));
            TMQ_HIP(launch_scalar(SC_ALPHA, L->partial[0], blas_grid(n), S, 0, 0, &S->done, st));
            TMQ_HIP(launch_axpy_norm(x, pp, r, ap, S, L->partial[1], &S->done, st));
            TMQ_HIP(launch_scalar(SC_BETA, L->partial[1], blas_grid(n), S, 0, 0, &S->done, st));
            TMQ_HIP(launch_xpay(r, pp, S, &S->done, st));
            const int slot = enq % Lattice::RING;
            TMQ_HIP(hipMemcpyAsync(&L->ring[slot], S, sizeof(CgScalars), hipMemcpyDeviceToHost, st));
            TMQ_HIP(hipEventRecord(L->ring_ev[slot], st));
            if (enq > 0) {
                const int ps = (enq - 1) % Lattice::RING;
                TMQ_HIP(hipEventSynchronize(L->ring_ev[ps]));
                if (L->ring[ps].done || L->ring[ps].nan) {
                    enq++;
                    break;
                }
            }
            enq++;
        }
        TMQ_TRY(read_scalars(L, st, &cur));
        if (cur.nan) break;
        // true residual r = b - A x
        TMQ_TRY(apply_A(x, ap, nullptr, nullptr));
        TMQ_HIP(launch_residual(b, ap, r, L->partial[2], st));
        TMQ_HIP(launch_scalar(SC_RELIABLE, L->partial[2], blas_grid(n), S, tol2, o.relative, nullptr, st));
        TMQ_TRY(read_scalars(L, st, &cur));
        if (cur.nan || cur.done || enq >= max_iter) break;
        TMQ_HIP(launch_xpay(r, pp, S, nullptr, st));
    }
    int status = TMQ_OK;
    if (cur.nan) {
        status = TMQ_ENAN;
        set_error("tmq_solve_full: non-finite value in CG");
    } else if (!cur.done) {
        status = TMQ_ENOCONV;
        set_error("tmq_solve_full: max_iter reached before the tolerance");
    }
    if (info) {
        info->status = status;
        info->iters = cur.iter;
        info->reliable_updates = cur.reliable;
        info->true_rel_residual = cur.bb > 0 ? std::sqrt(cur.rr / cur.bb) : std::sqrt(cur.rr);
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

}  // namespace tmq
