// engine.h -- the CG engine: right-hand sides in slots that join and leave.
//
// An engine owns batch work fields with `cap` slots on one lattice, for one
// inner precision.  A right-hand side occupies a slot from join() until it
// has finished and been taken; every step advances all occupied slots by one
// CG iteration (Sec. 4.4) in shared launches.  The decisions per slot (when
// to recompute the true residual, when to stop) depend only on that slot's
// own scalars and on the number of steps since it joined, so a right-hand
// side computes the same numbers whatever the other slots hold.
//
// A step has two halves, so that the GPU never waits for the host:
//   begin_step()  enqueue the iteration body for the slots still iterating;
//   end_step()    read the scalars the previous step published (waiting for
//                 them if needed), decide per slot, enqueue the reliable
//                 updates and p = r + beta p, record the step's event.
// join() and take() are called between end_step() and the next begin_step().
//
// Per slot, with k = steps since the slot joined (its first body is step 0):
//   bodies run for k = 0 .. max_iter-1; at step k >= 1 the scalars of step
//   k-1 decide: non-finite -> finished (ENAN); a true residual below the
//   target -> finished; an iterated residual below the target -> reliable
//   update (true residual) now; mixed precision and the iterated residual
//   below delta^2 times the largest since the last true one -> reliable
//   update.  At k = max_iter a solution that has no true residual yet gets
//   one, and the slot finishes one step later (ENOCONV unless converged).
//
// Switch mode (the paper's reduced-precision CG, Sec. 4.4): the vectors stay
// in FP64 and a slot's operator is FP64 until its iterated residual is below
// sqrt(tol) relative (rr < tol * bb), then the reduced-precision operator
// (its input converted down, its output converted back); the switch decided at
// step k takes effect at step k+1.  No delta updates; the true-residual check
// at convergence is the same.
#pragma once
#include <vector>

#include "lattice.h"

namespace tmq {

struct Engine {
    Lattice *L = nullptr;
    int sloppy = P64;       // inner spinor precision (P64: plain FP64 CG)
    int sloppy_link = P32;  // inner link precision (mixed only)
    int mode = 0;           // TMQ_MODE_RELIABLE or TMQ_MODE_SWITCH
    hipStream_t st = nullptr;
    int cap = 0;
    bool mixed = false;     // reliable-update mode with a reduced inner precision
    bool switching = false; // switch mode with a reduced operator precision
    bool nd = false;        // slots hold flavour doublets (eq. (Dh)), op.nd set
    long n = 0;             // sites of a slot's fields: V/2, or 2 V/2 for doublets

    std::vector<Field> fields;
    FieldDesc b, x, r64, te64, to64, rs, ps, tes, tos, xs;
    FieldDesc ap64, pss, apss;  // switch mode: FP64 A p, reduced-precision p and A p
    LinkDesc lk64{}, lks{};
    OpParams op{};
    double *partial[3] = {nullptr, nullptr, nullptr};  // per slot at + slot * L->pstride
    CgScalars *scal = nullptr;                         // device, cap entries
    CgScalars *ring = nullptr, *ring_dev = nullptr;    // pinned, RING x cap entries
    std::vector<hipEvent_t> step_ev;                   // RING events
    size_t bytes = 0;                                  // device memory held

    enum SlotState { FREE = 0, RUNNING = 1, FINISHED = 2 };
    struct Slot {
        int state = FREE;
        long joined_step = 0;  // step whose body is the slot's first
        double maxr2 = 0.0;    // largest |r|^2 since the last true residual
        double tol = 0.0, delta = 0.0;
        int relative = 1, max_iter = 0;
        bool switched = false;  // switch mode: reduced-precision operator in use
        CgScalars last{};      // scalars at finish
        int status = TMQ_OK;
    };
    std::vector<Slot> slots;

    long step_no = 0;           // steps begun
    bool body_pending = false;  // begin_step() done, end_step() not yet

    // HIP graphs of the iteration body (engine_set_graphs): one per scalar
    // ring entry, keyed by the body's slot lists and their parameters; a key
    // is captured only after it ran once without a graph (so every launch
    // shape it needs has been tuned)
    struct StepGraph {
        std::vector<double> key;
        hipGraphExec_t exec = nullptr;
    };
    bool graphs = false;
    hipStream_t cap_st = nullptr;  // capture stream (default priority)
    StepGraph graph[Lattice::RING];
    std::vector<double> last_eager_key;
    long graph_launches = 0, graph_captures = 0;

    Engine() = default;
    Engine(const Engine &) = delete;
    Engine &operator=(const Engine &) = delete;
    ~Engine();
};

// Bytes of device memory one slot holds (work fields of one right-hand side).
size_t engine_slot_bytes(long vh, int sloppy, int mode = 0, bool nd = false);
// Bytes an engine of cap slots holds in total.
size_t engine_bytes(const Lattice *L, int sloppy, int cap, int mode = 0, bool nd = false);

// Allocate an engine with cap slots (1..MAX_RHS, 1..MAX_RHS/2 for doublets)
// on L for the inner precision (sloppy, sloppy_link) and mode of the options;
// commands go to stream st.  nd: every slot is a flavour doublet (fields of
// 2 V/2 sites, upper flavour first) and the operator that of eq. (Dh).
int engine_create(Lattice *L, int sloppy, int sloppy_link, int mode, int cap, hipStream_t st, Engine **out,
                  bool nd = false);
// Default delta of reliable updates for an inner spinor and link precision.
double engine_default_delta(int sloppy, int sloppy_link);

// Put right-hand side b (device, canonical odd-site complex128 [V/2][12];
// [2][V/2][12] for doublets) into free slot `slot` and enqueue its
// initialisation.  Boundary phases are common to the engine: theta must equal
// that of the slots already running.  tol, relative, max_iter and delta of o
// apply to this slot; epsbar (2 kappa epsbar) only to doublets, whose p.mu_tilde
// is 2 kappa mubar.
int engine_join(Engine *E, int slot, const tmq_params &p, const tmq_solver_opts &o, const double2 *b,
                double epsbar = 0.0);
int engine_free_slot(const Engine *E);  // a free slot, or -1
int engine_begin_step(Engine *E);
// Run the iteration bodies as captured HIP graphs (on) or as plain launches.
int engine_set_graphs(Engine *E, bool on);
// True when the scalars end_step() reads are on the host (never blocks).
bool engine_ready(Engine *E);
// Blocks until ready, then decides; `finished` receives the slots that ended.
int engine_end_step(Engine *E, std::vector<int> *finished);
// Slots running (joined and not finished).
int engine_running(const Engine *E);
int engine_occupied(const Engine *E);
// Enqueue the canonical copy of a finished slot's solution into x (device,
// may be nullptr), fill info (seconds untouched) and free the slot.
int engine_take(Engine *E, int slot, double2 *x, tmq_solve_info *info);

}  // namespace tmq
