// engine.cpp -- CG engine with slots that join and leave (protocol in engine.h).
//
// The iteration is textbook CG on Qhat^+ Qhat^- (Sec. 4.4) with every vector
// operation, inner product and scalar on the device; the host reads one small
// scalar record per slot and step, one step behind the device.  Mixed
// precision follows the paper's reduced-precision CG with a true-residual
// check: the inner iteration runs on FP32/FP16/BF16 spinors with
// reduced-precision two-row links and accumulates its correction in an FP32
// vector x_s; a reliable update folds x_s into the FP64 solution x,
// recomputes r = b - A x with the FP64 operator and continues the recursion
// from that true residual with the same search direction.  Convergence is
// declared on a recomputed FP64 true residual only.
#include "engine.h"

#include <cmath>
#include <cstring>

namespace tmq {

size_t engine_slot_bytes(long vh, int sloppy, int mode, bool nd)
{
    if (nd) return engine_slot_bytes(2 * vh, sloppy, mode, false);
    // switch mode: b, x, r, t_e, t_o, p, A p in FP64 and p, A p, t_e, t_o reduced
    if (mode == TMQ_MODE_SWITCH)
        return 7 * field_bytes(P64, vh) + (sloppy == P64 ? 0 : 4 * field_bytes(sloppy, vh));
    // FP64: b, x, r, t_e, t_o, p ; mixed: b, x, r, t_e, t_o in FP64, four inner
    // vectors (r, p, t_e, t_o) and the FP32 x_s (A p never reaches memory: the
    // CG update is fused into the half-sweep that forms it)
    if (sloppy == P64) return 6 * field_bytes(P64, vh);
    return 5 * field_bytes(P64, vh) + 4 * field_bytes(sloppy, vh) + field_bytes(P32, vh);
}

size_t engine_bytes(const Lattice *L, int sloppy, int cap, int mode, bool nd)
{
    return (size_t)cap * engine_slot_bytes(L->g.vh, sloppy, mode, nd) + (size_t)cap * 3 * L->pstride * sizeof(double) +
           (size_t)cap * sizeof(CgScalars);
}

double engine_default_delta(int sloppy, int sloppy_link)
{
    // How far the reduced-precision recursion stays faithful to the true
    // residual, set by the coarser of spinor and link storage (measured on the
    // 32^3x64 workload): FP32 with FP32 links over 4 decades; with FP16 links
    // about 2; FP16 spinors a little over 2; BF16 (8-bit mantissa) a little
    // over 1.  A delta below that reach stalls the recursion (FP32 spinors
    // with FP16 links at 1e-4 took 765 iterations instead of 35).
    if (sloppy == P32) return sloppy_link == P32 ? 1e-4 : 0.01;
    return sloppy == PB16 ? 0.05 : 0.005;
}

Engine::~Engine()
{
    if (st) hipStreamSynchronize(st);
    for (auto &g : graph)
        if (g.exec) hipGraphExecDestroy(g.exec);
    if (cap_st) hipStreamDestroy(cap_st);
    for (auto &e : step_ev)
        if (e) hipEventDestroy(e);
    for (auto &f : fields) field_free(f);
    for (double *p : partial)
        if (p) hipFree(p);
    if (scal) hipFree(scal);
    if (ring) hipHostFree(ring);
}

int engine_create(Lattice *L, int sloppy, int sloppy_link, int mode, int cap, hipStream_t st, Engine **out,
                  bool nd)
{
    if (cap < 1 || cap > (nd ? MAX_RHS / 2 : MAX_RHS)) {
        set_error(nd ? "engine: capacity must be 1..32 doublets" : "engine: capacity must be 1..64");
        return TMQ_EINVAL;
    }
    Engine *E = new Engine();
    auto fail = [&](int code) {
        delete E;
        return code;
    };
    E->L = L;
    E->sloppy = sloppy;
    E->sloppy_link = sloppy_link;
    E->st = st;
    E->cap = cap;
    E->mode = mode;
    E->mixed = sloppy != P64 && mode == TMQ_MODE_RELIABLE;
    E->switching = sloppy != P64 && mode == TMQ_MODE_SWITCH;
    E->nd = nd;
    E->op.nd = nd ? 1 : 0;
    const long vh = nd ? 2 * L->g.vh : L->g.vh;
    E->n = vh;
    E->fields.reserve(16);
    auto field = [&](int prec, FieldDesc *d) -> int {
        E->fields.emplace_back();
        TMQ_TRY(field_alloc(E->fields.back(), prec, vh, cap));
        *d = E->fields.back().d;
        return TMQ_OK;
    };
    int s = TMQ_OK;
    for (FieldDesc *d : {&E->b, &E->x, &E->r64, &E->te64, &E->to64})
        if ((s = field(P64, d)) != TMQ_OK) return fail(s);
    E->lk64 = lattice_links(L, link_fmt_for(L, P64, P64));
    if (E->mixed) {
        E->lks = lattice_links(L, link_fmt_for(L, sloppy, sloppy_link));
        for (FieldDesc *d : {&E->rs, &E->ps, &E->tes, &E->tos})
            if ((s = field(sloppy, d)) != TMQ_OK) return fail(s);
        if ((s = field(P32, &E->xs)) != TMQ_OK) return fail(s);
    } else {
        E->lks = E->lk64;
        E->rs = E->r64;
        E->xs = E->x;
        E->tes = E->te64;
        E->tos = E->to64;
        if ((s = field(P64, &E->ps)) != TMQ_OK) return fail(s);
        if (E->switching) {
            E->lks = lattice_links(L, link_fmt_for(L, sloppy, sloppy_link));
            if ((s = field(P64, &E->ap64)) != TMQ_OK) return fail(s);
            for (FieldDesc *d : {&E->pss, &E->apss, &E->tes, &E->tos})
                if ((s = field(sloppy, d)) != TMQ_OK) return fail(s);
        }
    }
    for (auto &p : E->partial)
        if (hipMalloc((void **)&p, sizeof(double) * L->pstride * cap) != hipSuccess) {
            p = nullptr;
            set_error("engine: device allocation of partial sums failed");
            return fail(TMQ_ENOMEM);
        }
    if (hipMalloc((void **)&E->scal, sizeof(CgScalars) * cap) != hipSuccess) {
        E->scal = nullptr;
        set_error("engine: device allocation of scalars failed");
        return fail(TMQ_ENOMEM);
    }
    if (hipMemset(E->scal, 0, sizeof(CgScalars) * cap) != hipSuccess) {
        set_error("engine: clearing scalars failed");
        return fail(TMQ_EDEVICE);
    }
    if (hipHostMalloc((void **)&E->ring, sizeof(CgScalars) * cap * Lattice::RING, hipHostMallocMapped) !=
        hipSuccess) {
        E->ring = nullptr;
        set_error("engine: pinned scalar ring allocation failed");
        return fail(TMQ_ENOMEM);
    }
    if (hipHostGetDevicePointer((void **)&E->ring_dev, E->ring, 0) != hipSuccess) {
        set_error("engine: device view of the scalar ring failed");
        return fail(TMQ_EDEVICE);
    }
    E->step_ev.assign(Lattice::RING, nullptr);
    for (auto &e : E->step_ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            e = nullptr;
            set_error("engine: event creation failed");
            return fail(TMQ_EDEVICE);
        }
    E->slots.assign(cap, Engine::Slot{});
    E->bytes = engine_bytes(L, sloppy, cap, mode, nd);
    *out = E;
    return TMQ_OK;
}

static RhsList list_of(const std::vector<int> &idx)
{
    RhsList l;
    l.n = (int)idx.size();
    for (int i = 0; i < l.n; i++) l.idx[i] = (unsigned char)idx[i];
    return l;
}

int engine_free_slot(const Engine *E)
{
    for (int i = 0; i < E->cap; i++)
        if (E->slots[i].state == Engine::FREE) return i;
    return -1;
}

int engine_running(const Engine *E)
{
    int n = 0;
    for (auto &s : E->slots) n += s.state == Engine::RUNNING;
    return n;
}

int engine_occupied(const Engine *E)
{
    int n = 0;
    for (auto &s : E->slots) n += s.state != Engine::FREE;
    return n;
}

int engine_join(Engine *E, int slot, const tmq_params &p, const tmq_solver_opts &o, const double2 *b, double epsbar)
{
    if (slot < 0 || slot >= E->cap || E->slots[slot].state != Engine::FREE) {
        set_error("engine: slot is not free");
        return TMQ_EINVAL;
    }
    if (E->body_pending) {
        set_error("engine: join between begin_step and end_step");
        return TMQ_ESTATE;
    }
    Lattice *L = E->L;
    const OpParams pp = make_op(L, &p, 1);
    if (engine_occupied(E) == 0)
        memcpy(E->op.ph, pp.ph, sizeof(pp.ph));
    else if (memcmp(E->op.ph, pp.ph, sizeof(pp.ph)) != 0) {
        set_error("engine: theta differs from the right-hand sides in flight");
        return TMQ_EINVAL;
    }
    E->op.kappa[slot] = p.kappa;
    E->op.mut[slot] = p.mu_tilde;
    E->op.eps[slot] = E->nd ? epsbar : 0.0;
    Engine::Slot &s = E->slots[slot];
    s = Engine::Slot{};
    s.tol = o.tol;
    s.relative = o.relative;
    s.max_iter = o.max_iter > 0 ? o.max_iter : 10000;
    s.delta = o.delta > 0.0 && o.delta < 1.0 ? o.delta : engine_default_delta(E->sloppy, E->sloppy_link);

    // x = 0 ; r = b ; p = r ; bb = |b|^2
    const RhsList one = list_of({slot});
    hipStream_t st = E->st;
    TMQ_HIP(launch_from_canonical(b, field_rhs(E->b, slot), st));
    TMQ_HIP(launch_zero(E->x, one, st));
    TMQ_HIP(launch_convert(E->b, E->r64, one, st));
    TMQ_HIP(launch_norm2(E->r64, one, E->partial[1], L->pstride, st));
    TMQ_HIP(launch_scalar(SC_INIT, one, E->partial[1], L->pstride, blas_grid(E->n), E->scal, o.tol * o.tol,
                          o.relative, false, nullptr, st));
    if (E->mixed) {
        TMQ_HIP(launch_convert(E->r64, E->rs, one, st));
        TMQ_HIP(launch_zero(E->xs, one, st));
    }
    TMQ_HIP(launch_convert(E->rs, E->ps, one, st));
    s.state = Engine::RUNNING;
    s.joined_step = E->step_no;
    return TMQ_OK;
}

// slots whose body runs at the current step
static std::vector<int> body_slots(const Engine *E)
{
    std::vector<int> r;
    for (int i = 0; i < E->cap; i++) {
        const Engine::Slot &s = E->slots[i];
        if (s.state == Engine::RUNNING && E->step_no - s.joined_step < s.max_iter) r.push_back(i);
    }
    return r;
}

// switch mode, slots on the reduced-precision operator: the FP64 p is
// converted down, A p = Qhat^+ Qhat^- p applied in reduced precision and
// converted back, then the CG update in FP64
static int body_switched(Engine *E, const RhsList &al, CgScalars *pub)
{
    Lattice *L = E->L;
    hipStream_t st = E->st;
    CgScalars *S = E->scal;
    TMQ_HIP(launch_convert(E->ps, E->pss, al, st));
    TMQ_TRY(apply_Qhat(L, E->op, -1, E->pss, E->tos, E->tes, E->lks, al, E->partial[0], S, st));
    TMQ_HIP(launch_scalar(SC_ALPHA, al, E->partial[0], L->pstride, L->hop_blocks_last, S, 0, 0, true, nullptr, st));
    TMQ_TRY(apply_Qhat(L, E->op, +1, E->tos, E->apss, E->tes, E->lks, al, nullptr, S, st));
    TMQ_HIP(launch_convert(E->apss, E->ap64, al, st));
    TMQ_HIP(launch_axpy_norm(E->x, E->ps, E->r64, E->ap64, al, S, E->partial[1], L->pstride, true, st));
    TMQ_HIP(launch_scalar(SC_BETA, al, E->partial[1], L->pstride, blas_grid(E->n), S, 0, 0, true, pub, st));
    return TMQ_OK;
}

// the launches of one iteration body for the slots of `all` (the reduced
// precision or FP64 operator) and `sw` (switch mode, on the reduced
// operator), publishing their scalars to pub; every launch goes to st
static int enqueue_body(Engine *E, const std::vector<int> &all, const std::vector<int> &sw, CgScalars *pub,
                        hipStream_t st)
{
    Lattice *L = E->L;
    const RhsList al = list_of(all);
    CgScalars *S = E->scal;
    const hipStream_t keep = E->st;
    E->st = st;  // body_switched launches on E->st
    struct Restore {
        Engine *E;
        hipStream_t s;
        ~Restore() { E->st = s; }
    } restore{E, keep};
    if (!sw.empty()) TMQ_TRY(body_switched(E, list_of(sw), pub));
    if (al.n > 0 && E->switching) {
        // switch mode, slots still on the FP64 operator
        TMQ_TRY(apply_Qhat(L, E->op, -1, E->ps, E->to64, E->te64, E->lk64, al, E->partial[0], S, st));
        TMQ_HIP(launch_scalar(SC_ALPHA, al, E->partial[0], L->pstride, L->hop_blocks_last, S, 0, 0, true, nullptr,
                              st));
        CgFields cg;
        cg.r = E->r64;
        cg.p = E->ps;
        cg.x = E->x;
        TMQ_TRY(apply_Qhat_cg(L, E->op, E->to64, E->te64, E->lk64, al, cg, E->partial[1], S, st));
        TMQ_HIP(launch_scalar(SC_BETA, al, E->partial[1], L->pstride, L->hop_blocks_last, S, 0, 0, true, pub, st));
    } else if (al.n > 0) {
        // t = Qhat^- p, <p, A p> = |t|^2 ; A p = Qhat^+ t
        TMQ_TRY(apply_Qhat(L, E->op, -1, E->ps, E->tos, E->tes, E->lks, al, E->partial[0], S, st));
        TMQ_HIP(launch_scalar(SC_ALPHA, al, E->partial[0], L->pstride, L->hop_blocks_last, S, 0, 0, true, nullptr,
                              st));
        // A p = Qhat^+ t fused with x_s += alpha p ; r -= alpha A p ; |r|^2 ; then beta
        CgFields cg;
        cg.r = E->rs;
        cg.p = E->ps;
        cg.x = E->xs;
        TMQ_TRY(apply_Qhat_cg(L, E->op, E->tos, E->tes, E->lks, al, cg, E->partial[1], S, st));
        TMQ_HIP(launch_scalar(SC_BETA, al, E->partial[1], L->pstride, L->hop_blocks_last, S, 0, 0, true, pub, st));
    }
    return TMQ_OK;
}

int engine_set_graphs(Engine *E, bool on)
{
    if (on && !E->cap_st)
        if (hipStreamCreateWithFlags(&E->cap_st, hipStreamNonBlocking) != hipSuccess) {
            E->cap_st = nullptr;
            set_error("engine: capture stream creation failed");
            return TMQ_EDEVICE;
        }
    E->graphs = on;
    return TMQ_OK;
}

int engine_begin_step(Engine *E)
{
    if (E->body_pending) return TMQ_OK;
    Lattice *L = E->L;
    std::vector<int> all = body_slots(E), sw;
    if (E->switching) {
        std::vector<int> keep;
        for (int r : all) (E->slots[r].switched ? sw : keep).push_back(r);
        all.swap(keep);
    }
    const int ring = (int)(E->step_no % Lattice::RING);
    CgScalars *pub = E->ring_dev + (size_t)ring * E->cap;
    if (!E->graphs || L->timing || (all.empty() && sw.empty())) {
        TMQ_TRY(enqueue_body(E, all, sw, pub, E->st));
        E->body_pending = true;
        return TMQ_OK;
    }
    // what the body's launches depend on besides the engine's fixed buffers
    std::vector<double> key;
    key.push_back((double)all.size());
    for (int r : all) key.insert(key.end(), {(double)r, E->op.kappa[r], E->op.mut[r], E->op.eps[r]});
    key.push_back((double)sw.size());
    for (int r : sw) key.insert(key.end(), {(double)r, E->op.kappa[r], E->op.mut[r], E->op.eps[r]});
    for (int mu = 0; mu < 4; mu++) key.insert(key.end(), {E->op.ph[mu][0], E->op.ph[mu][1]});
    Engine::StepGraph &gr = E->graph[ring];
    if (!(gr.exec && gr.key == key)) {
        if (key != E->last_eager_key) {
            // first time for this body: plain launches (tunes any new launch shape)
            TMQ_TRY(enqueue_body(E, all, sw, pub, E->st));
            E->last_eager_key = key;
            E->body_pending = true;
            return TMQ_OK;
        }
        if (gr.exec) hipGraphExecDestroy(gr.exec);
        gr.exec = nullptr;
        hipGraph_t g = nullptr;
        TMQ_HIP(hipStreamBeginCapture(E->cap_st, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue_body(E, all, sw, pub, E->cap_st);
        const hipError_t ec = hipStreamEndCapture(E->cap_st, &g);
        if (rc != TMQ_OK) {
            if (g) hipGraphDestroy(g);
            return rc;
        }
        TMQ_HIP(ec);
        const hipError_t ei = hipGraphInstantiate(&gr.exec, g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        TMQ_HIP(ei);
        gr.key = key;
        E->graph_captures++;
    }
    TMQ_HIP(hipGraphLaunch(gr.exec, E->st));
    E->graph_launches++;
    E->body_pending = true;
    return TMQ_OK;
}

bool engine_ready(Engine *E)
{
    if (E->step_no == 0) return true;
    return hipEventQuery(E->step_ev[(E->step_no - 1) % Lattice::RING]) == hipSuccess;
}

// x += x_s ; r = b - A x (FP64) ; the slot's scalars continue from |r|^2
static int reliable_update(Engine *E, const RhsList &rl, CgScalars *publish)
{
    if (rl.n == 0) return TMQ_OK;
    Lattice *L = E->L;
    hipStream_t st = E->st;
    if (E->mixed) TMQ_HIP(launch_accumulate(E->x, E->xs, rl, st));
    TMQ_TRY(residual_QhatQhat(L, E->op, E->x, E->b, E->r64, E->te64, E->to64, E->lk64, rl, E->partial[2], st));
    TMQ_HIP(launch_scalar(SC_RELIABLE, rl, E->partial[2], L->pstride, L->hop_blocks_last, E->scal, 0.0, 0, false,
                          publish, st));
    if (E->mixed) TMQ_HIP(launch_convert(E->r64, E->rs, rl, st));
    return TMQ_OK;
}

static void finish(Engine::Slot &sl, const CgScalars &pv, int r, std::vector<int> *finished)
{
    sl.state = Engine::FINISHED;
    sl.last = pv;
    sl.status = pv.nan ? TMQ_ENAN : pv.done ? TMQ_OK : TMQ_ENOCONV;
    if (finished) finished->push_back(r);
}

int engine_end_step(Engine *E, std::vector<int> *finished)
{
    if (!E->body_pending) TMQ_TRY(engine_begin_step(E));
    const long s = E->step_no;
    const int cur = (int)(s % Lattice::RING);
    CgScalars *pub = E->ring_dev + (size_t)cur * E->cap;
    const std::vector<int> in_body = body_slots(E);
    std::vector<int> ru;
    if (s > 0) {
        const int prev_slot = (int)((s - 1) % Lattice::RING);
        TMQ_HIP(hipEventSynchronize(E->step_ev[prev_slot]));
        const CgScalars *prev = E->ring + (size_t)prev_slot * E->cap;
        for (int r = 0; r < E->cap; r++) {
            Engine::Slot &sl = E->slots[r];
            if (sl.state != Engine::RUNNING) continue;
            const long k = s - sl.joined_step;
            if (k < 1) continue;  // its first body is this step's: no scalars yet
            const CgScalars pv = prev[r];
            if (k == 1) sl.maxr2 = pv.bb;  // |r_0|^2
            if (pv.nan || (pv.done && pv.last_true)) {
                finish(sl, pv, r, finished);
                continue;
            }
            if (k >= sl.max_iter) {  // no more bodies: end on a true residual
                if (pv.last_true)
                    finish(sl, pv, r, finished);
                else
                    ru.push_back(r);
                continue;
            }
            if (pv.done) {  // iterated residual met the target: check the true one
                ru.push_back(r);
                continue;
            }
            if (pv.last_true || pv.rr > sl.maxr2) sl.maxr2 = pv.rr;
            if (E->mixed && pv.rr < sl.delta * sl.delta * sl.maxr2) ru.push_back(r);
            // switch mode: the reduced-precision operator once |r| / |b| < sqrt(tol)
            if (E->switching && !sl.switched && pv.rr < sl.tol * (sl.relative ? pv.bb : 1.0)) sl.switched = true;
        }
    }
    // reliable updates after this step's body publish to the same ring entry
    TMQ_TRY(reliable_update(E, list_of(ru), pub));
    if (!in_body.empty()) TMQ_HIP(launch_xpay(E->rs, E->ps, list_of(in_body), E->scal, true, E->st));
    TMQ_HIP(hipEventRecord(E->step_ev[cur], E->st));
    E->step_no++;
    E->body_pending = false;
    return TMQ_OK;
}

int engine_take(Engine *E, int slot, double2 *x, tmq_solve_info *info)
{
    if (slot < 0 || slot >= E->cap || E->slots[slot].state != Engine::FINISHED) {
        set_error("engine: slot has not finished");
        return TMQ_ESTATE;
    }
    Engine::Slot &sl = E->slots[slot];
    if (x) TMQ_HIP(launch_to_canonical(field_rhs(E->x, slot), x, E->st));
    if (info) {
        const CgScalars &c = sl.last;
        info->status = sl.status;
        info->iters = c.iter;
        info->reliable_updates = c.reliable;
        info->true_rel_residual = c.bb > 0 ? std::sqrt(c.rr / c.bb) : std::sqrt(c.rr);
    }
    sl = Engine::Slot{};
    return TMQ_OK;
}

}  // namespace tmq
