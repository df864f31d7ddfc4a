// lattice.h -- the lattice object behind the C ABI: device memory, resident
// gauge copies, operator application and solver work space.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <string>
#include <vector>

#include "../../include/tmq.h"
#include "kernels.h"

namespace tmq {

struct Engine;

// thread-local error message behind tmq_last_error()
void set_error(const std::string &msg);
const char *get_error();

#define TMQ_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ::tmq::set_error(std::string(#call) + ": " + hipGetErrorString(e_));        \
            return TMQ_EDEVICE;                                                         \
        }                                                                               \
    } while (0)

#define TMQ_TRY(expr)                 \
    do {                              \
        int s_ = (expr);              \
        if (s_ != TMQ_OK) return s_;  \
    } while (0)

// one device field with its own allocation
struct Field {
    FieldDesc d;
    void *mem = nullptr;
    float *scale = nullptr;
};

int field_alloc(Field &f, int prec, long n, int nrhs = 1);
// a one-RHS field of n sites placed at mem (16-bit scales after the codes,
// 256-byte aligned); *bytes receives the bytes it occupies from mem
FieldDesc field_at(void *mem, int prec, long n, size_t *bytes);
void field_free(Field &f);
size_t field_bytes(int prec, long n);

struct TimedLaunch {
    hipEvent_t a, b;
    double bytes, flops;
    int prec;  // spinor storage of the launch
    int nrhs;  // right-hand sides in the launch
    int epi;   // epilogue (HopEpi)
};

struct Lattice {
    int device = 0;
    int dims[4] = {0, 0, 0, 0};
    Geom g{};
    hipStream_t own = nullptr;  // stream of the host-pointer calls

    bool gauge = false;
    bool su3 = false;
    double su3_dev = 0.0;
    double2 *u64f = nullptr, *u64r = nullptr;
    float4 *u32r = nullptr;
    uint4 *u16a = nullptr;
    uint2 *u16b = nullptr;
    float2 *u32f = nullptr;  // FP32 full links, built only for fields that fail the SU(3) check

    // reductions and solver scalars: partial sums of RHS r at partial[k] + r * pstride
    double *partial[3] = {nullptr, nullptr, nullptr};
    long pstride = 0;
    CgScalars *scal = nullptr;      // device, MAX_RHS entries
    CgScalars *ring = nullptr;      // pinned host-mapped, RING slots of MAX_RHS entries (host view)
    CgScalars *ring_dev = nullptr;  // device view of the same slots
    hipEvent_t ring_ev[8] = {};
    static constexpr int RING = 8;

    // CG engines of the even/odd solves, one per inner precision and link format
    std::vector<Engine *> engines;

    // BiCGstab scalars (device) and their published copies (pinned, 2 entries)
    BicgScalars *bicg = nullptr;
    BicgScalars *bicg_ring = nullptr, *bicg_ring_dev = nullptr;
    hipEvent_t bicg_ev[2] = {};

    // named work fields, grown on demand
    std::vector<std::pair<std::string, Field>> work;

    // canonical staging buffers for host calls
    void *stage[2] = {nullptr, nullptr};
    size_t stage_bytes[2] = {0, 0};

    // autotuned hop variant per key = spinor precision * N_LINK_FMT + link format; -1 = not tuned yet
    static constexpr int NKEY = 4 * N_LINK_FMT;
    int hop_variant[NKEY];
    float hop_tune_us[NKEY][HOP_VARIANTS];
    int forced_variant = -1;  // TMQ_HOP_VARIANT in the environment
    int forced_cap = -1;      // TMQ_HOP_CAP in the environment
    int forced_rpl = 0;       // TMQ_HOP_RPL in the environment (RHS per lane of batched hops)
    // blocks-per-CU cap tuned for that variant (0: none; see launch_hop's lds)
    int hop_occ[NKEY];
    float hop_occ_us[NKEY][6];
    int lds_per_cu = 65536;
    int lds_per_block = 65536;  // largest LDS reservation of one block
    // autotuned launch shape of batched hops, per (spinor precision, link
    // format) key and power-of-two batch size class
    struct BatchTune {
        int key, cls;
        HopTune tu;
        int cap = 0;                              // blocks-per-CU cap of tu (0: none)
        std::vector<std::array<float, 3>> tried;  // (RHS per lane, group, us per launch)
        float cap_us[6] = {-1.f, -1.f, -1.f, -1.f, -1.f, -1.f};  // the chosen shape per cap
    };
    std::vector<BatchTune> hop_batch;
    int hop_blocks_last = 0;  // blocks (partial sums) of the last hop launch

    // set for the duration of an allocation-free call: hop launches neither
    // tune (an untuned format runs variant 0) nor record timing events
    bool no_alloc = false;

    // kernel timing
    bool timing = false;
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;

    ~Lattice();
};

int lattice_create(const int dims[4], int device, Lattice **out);
// device address of the allocation-free work space (noalloc.hip)
hipError_t noalloc_scratch_init(int device);
void *noalloc_scratch(int device, size_t *bytes);
int lattice_load_gauge(Lattice *L, const double2 *U_dev, hipStream_t st);
LinkDesc lattice_links(const Lattice *L, int fmt);
// link format used for a spinor precision (sloppy_link: P32 or P16 for the inner
// links); the full-link formats when the loaded field is not SU(3)
int link_fmt_for(const Lattice *L, int prec, int sloppy_link);

// a work field of the given role, precision, site count and RHS count (allocated once, reused)
int work_field(Lattice *L, const char *role, int prec, long n, FieldDesc *out, int nrhs = 1);
int stage_buffer(Lattice *L, int slot, size_t bytes, void **out);

// operator parameters of a batch (theta of p[0] for all; kappa, mut per RHS)
OpParams make_op(const Lattice *L, const tmq_params *p, int n);

// one hop half-sweep through the autotuner and the timing hook
int hop(Lattice *L, int out_par, const FieldDesc &in, const FieldDesc &self, const FieldDesc &out,
        const LinkDesc &lk, const OpParams &op, int epi, int sign, const RhsList &rl, double *partial,
        const CgScalars *scal, hipStream_t st, const CgFields *cg = nullptr);

// Qhat^{sign} in -> out (odd fields), tmp_e an even work field; partial: |out|^2 per block
int apply_Qhat(Lattice *L, const OpParams &op, int sign, const FieldDesc &in, const FieldDesc &out,
               const FieldDesc &tmp_e, const LinkDesc &lk, const RhsList &rl, double *partial,
               const CgScalars *scal, hipStream_t st);
// Qhat^+ applied to in (odd), fused with the CG update of the vectors of cg
// (r -= alpha Qhat^+ in ; x += alpha p, alpha from scal); partial: |r|^2 per block
int apply_Qhat_cg(Lattice *L, const OpParams &op, const FieldDesc &in, const FieldDesc &tmp_e, const LinkDesc &lk,
                  const RhsList &rl, const CgFields &cg, double *partial, const CgScalars *scal, hipStream_t st);
// r = b - Qhat^+ Qhat^- x (FP64 or any one format) with |r|^2 per block in partial
int residual_QhatQhat(Lattice *L, const OpParams &op, const FieldDesc &x, const FieldDesc &b, const FieldDesc &r,
                      const FieldDesc &tmp_e, const FieldDesc &tmp_o, const LinkDesc &lk, const RhsList &rl,
                      double *partial, hipStream_t st);
// Qhat^+ Qhat^- in -> out; partial receives |Qhat^- in|^2 per block
int apply_QhatQhat(Lattice *L, const OpParams &op, const FieldDesc &in, const FieldDesc &out,
                   const FieldDesc &tmp_e, const FieldDesc &tmp_o, const LinkDesc &lk, const RhsList &rl,
                   double *partial, const CgScalars *scal, hipStream_t st);
// full-lattice Q^{sign} on stacked (even, odd) fields
int apply_Q_full(Lattice *L, const OpParams &op, int sign, const FieldDesc &in, const FieldDesc &out,
                 const LinkDesc &lk, const RhsList &rl, hipStream_t st);

// algorithmic bytes of one hop half-sweep per output site for nrhs RHS
// (links once, spinors per RHS)
double hop_bytes_per_site(int prec, int link_fmt, bool self, int nrhs = 1);

int check_params(const tmq_params *p);
int check_prec(int prec);
int check_opts(const tmq_solver_opts *o);
std::string tuning_report(const Lattice *L);

}  // namespace tmq

struct tmq_lattice {
    tmq::Lattice *L;
};
