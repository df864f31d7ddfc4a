// solver.cpp -- CG on Qhat^+ Qhat^- (even/odd) and on Q^+ Q^- (full lattice).
//
// Even/odd solves run on a CG engine of the lattice (engine.h): the batch's
// right-hand sides join the engine's slots together and step until every one
// has finished.  A single solve is the batch of one, and each right-hand side
// goes through exactly the same arithmetic whatever shares the batch, so a
// batched solution equals its solve alone bit for bit.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "engine.h"

namespace tmq {

// the lattice's engine for this inner precision and link format with at
// least n slots (grown by reallocation when a larger batch comes)
static int lattice_engine(Lattice *L, const tmq_solver_opts &o, int n, Engine **out)
{
    const int sp = o.sloppy;
    const int lk = sp == P64 ? link_fmt_for(L, P64, P64) : link_fmt_for(L, sp, o.sloppy_link);
    for (size_t i = 0; i < L->engines.size(); i++) {
        Engine *E = L->engines[i];
        if (E->sloppy != sp || E->lks.fmt != lk) continue;
        if (E->cap >= n) {
            *out = E;
            return TMQ_OK;
        }
        delete E;
        L->engines.erase(L->engines.begin() + (long)i);
        break;
    }
    Engine *E = nullptr;
    TMQ_TRY(engine_create(L, sp, o.sloppy_link, n, nullptr, &E));
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

int solve_batch(Lattice *L, int n, const tmq_params *p, const tmq_solver_opts &o, const double *const *b,
                double *const *x, hipStream_t st, tmq_solve_info *info)
{
    const auto t0 = std::chrono::steady_clock::now();
    Engine *E = nullptr;
    TMQ_TRY(lattice_engine(L, o, n, &E));
    E->st = st;
    EngineScope scope{E};
    for (int r = 0; r < n; r++) TMQ_TRY(engine_join(E, r, p[r], o, (const double2 *)b[r]));
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

// ------------------------------------------------------ full lattice CG

static int read_scalars(Lattice *L, int n, hipStream_t st, std::vector<CgScalars> &out)
{
    TMQ_HIP(hipStreamSynchronize(st));
    out.resize(n);
    TMQ_HIP(hipMemcpy(out.data(), L->scal, sizeof(CgScalars) * n, hipMemcpyDeviceToHost));
    return TMQ_OK;
}

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
