// kernels.h -- host-side declarations of the device kernels' launch wrappers.
//
// Host code (the lattice object, the solvers, the C ABI) is format-agnostic:
// it passes FieldDesc / LinkDesc descriptors and the wrappers dispatch to the
// template instantiations in hop.hip, blas.hip and codec.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tmq {

enum Prec { P64 = 0, P32 = 1, P16 = 2, PB16 = 3 };  // same values as tmq_prec
enum LinkFmt { LK64F = 0, LK64R = 1, LK32R = 2, LK16R = 3 };

// Lattice geometry.  Extents (T, LZ, LY, LX) all even; V/2 sites per parity,
// eo index h = site >> 1 with site = ((t*LZ + z)*LY + y)*LX + x.
struct Geom {
    int T, LZ, LY, LX;
    int XH;   // LX / 2
    long vh;  // V / 2
};

// A spinor field of n sites (one parity, or both parities stacked: even sites
// 0..V/2-1, odd sites V/2..V-1) in the 8-site chunked layout of fields.h.
struct FieldDesc {
    int prec = P64;
    void *data = nullptr;   // element type by prec: double2, float4, uint4
    float *scale = nullptr; // FP32 per-site scale of 16-bit formats
    long n = 0;             // number of sites (a multiple of 8)
};

// sub-view starting at site `off` (a multiple of 8), n sites
FieldDesc field_sub(const FieldDesc &f, long off, long n);
size_t field_elem_bytes(int prec);
int field_blocks(int prec);  // component blocks per site: 12, 6, 3, 3

struct LinkDesc {
    int fmt = LK64F;
    const void *a = nullptr;  // main array
    const void *b = nullptr;  // second array (LK16R)
    long vh = 0;              // sites per parity
};

// Epilogue of a hop half-sweep at output site h (spin s; u = upper spins 0,1,
// d = lower spins 2,3):  out_s = A_{u|d} * self_s + B_{u|d} * (sum of hops)_s.
struct HopCoef {
    double ph[4][2];  // e^{i theta_mu pi / L_mu} (re, im), mu = t, x, y, z
    double A[2][2];   // (re, im) for upper, lower
    double B[2][2];
};

// Device scalars of a CG solve (one struct per right-hand side).
struct CgScalars {
    double rr;       // current ||r||^2 (iterated, or true after a reliable update)
    double rr_prev;  // ||r||^2 at the start of the last iteration
    double pAp;      // <p, A p> = ||Qhat^- p||^2
    double alpha, beta;
    double bb;       // ||b||^2
    double target;   // stop when rr < target
    int iter;        // iterations done
    int done;        // 1 once rr < target or nan (kernels given a skip pointer then do nothing)
    int nan;         // 1 once a non-finite scalar appeared
    int reliable;    // number of true-residual recomputations
    int last_true;   // 1 if rr is a recomputed true residual
    int pad;
};

constexpr int HOP_BLOCK = 256;
constexpr int BLAS_BLOCK = 256;
constexpr int RED_MAX_BLOCKS = 1 << 16;

int hop_grid(long n);
int blas_grid(long n);

// hop half-sweep: out(h) over the n sites of parity out_par; `in` holds parity
// 1 - out_par; `self` (may have data == nullptr) holds parity out_par.
// partial != nullptr: per-block sums of |out|^2 written to partial[0..hop_grid(n)).
// skip != nullptr: the launch does nothing when *skip != 0.
// hop kernel variants (see hop.hip): 0 plain order, 1 XCD slabs, 2 slabs +
// scheduling barriers, 3/4 as 2 with >= 2/3 waves per SIMD, 5 plain order with
// barriers and >= 2 waves; every variant loads links non-temporally.  Slab
// variants need LZ >= 8.
constexpr int HOP_VARIANTS = 6;
bool hop_variant_valid(const Geom &g, int v);
// blocks (= per-block partial sums written with NORM) of a launch of variant v
int hop_grid_variant(const Geom &g, int v);
hipError_t launch_hop(const Geom &g, int out_par, const FieldDesc &in, const FieldDesc &self,
                      const FieldDesc &out, const LinkDesc &lk, const HopCoef &c, double *partial,
                      const int *skip, int variant, hipStream_t st);

// BLAS-1 over the sites of the given views; every launch with `partial` writes
// blas_grid(n) per-block sums.  Scalars come from device memory.
hipError_t launch_norm2(const FieldDesc &v, double *partial, hipStream_t st);
hipError_t launch_convert(const FieldDesc &in, const FieldDesc &out, hipStream_t st);
hipError_t launch_zero(const FieldDesc &v, hipStream_t st);
// x += alpha p ; r -= alpha ap ; partial |r|^2   (alpha = s->alpha)
hipError_t launch_axpy_norm(const FieldDesc &x, const FieldDesc &p, const FieldDesc &r,
                            const FieldDesc &ap, const CgScalars *s, double *partial,
                            const int *skip, hipStream_t st);
// p = r + beta p   (beta = s->beta)
hipError_t launch_xpay(const FieldDesc &r, const FieldDesc &p, const CgScalars *s, const int *skip,
                       hipStream_t st);
// r = b - ax (FP64 views), partial |r|^2
hipError_t launch_residual(const FieldDesc &b, const FieldDesc &ax, const FieldDesc &r,
                           double *partial, hipStream_t st);
// x64 += xs ; xs = 0
hipError_t launch_accumulate(const FieldDesc &x64, const FieldDesc &xs, hipStream_t st);
// y = a x + y with a host scalar (FP64 views)
hipError_t launch_axpy_host(double a, const FieldDesc &x, const FieldDesc &y, hipStream_t st);

// scalar kernels (one block): deterministic sums of the partials
enum ScalarOp {
    SC_INIT = 0,     // bb = rr = sum ; target = tol2 * (relative ? bb : 1) ; counters cleared
    SC_ALPHA = 1,    // pAp = sum ; alpha = rr / pAp
    SC_BETA = 2,     // rr_prev = rr ; rr = sum ; beta = rr / rr_prev ; iter++ ; done = rr < target
    SC_RELIABLE = 3  // rr = sum (true residual) ; beta = rr / rr_prev ; done = rr < target
};
hipError_t launch_scalar(int op, const double *partial, int n, CgScalars *s, double tol2, int relative,
                         const int *skip, hipStream_t st, CgScalars *publish = nullptr);
// b = a, bytes / 16 lanes of 16 bytes (bandwidth calibration)
hipError_t launch_stream_copy(const void *src, void *dst, size_t bytes, hipStream_t st);
// out[0] = deterministic sum of partial[0..n)
hipError_t launch_sum(const double *partial, int n, double *out, hipStream_t st);

// codec: canonical complex128 [site][12] <-> device format
// odd-site fields: canonical k-th site -> view site k
hipError_t launch_from_canonical(const double2 *in, const FieldDesc &out, hipStream_t st);
hipError_t launch_to_canonical(const FieldDesc &in, double2 *out, hipStream_t st);
// full-lattice fields: canonical site s of parity p -> stacked view site p * V/2 + (s >> 1)
hipError_t launch_full_from_canonical(const Geom &g, const double2 *in, const FieldDesc &out, hipStream_t st);
hipError_t launch_full_to_canonical(const Geom &g, const FieldDesc &in, double2 *out, hipStream_t st);
// export 16-bit codes of a field in canonical [site][24] order plus scales
hipError_t launch_export_codes(const FieldDesc &in, uint16_t *codes, float *scale, hipStream_t st);

// gauge ingest from canonical complex128 [site][mu][3][3]: writes the enabled
// formats (null pointers skip) and per-block maxima of |U U^+ - 1| and |det U - 1|
struct GaugeOut {
    double2 *full64;  // LK64F
    double2 *row64;   // LK64R
    float4 *row32;    // LK32R
    uint4 *row16a;    // LK16R
    uint2 *row16b;
};
hipError_t launch_gauge_ingest(const Geom &g, const double2 *U, const GaugeOut &o, double *partial_max,
                               hipStream_t st);
hipError_t launch_max(const double *partial, int n, double *out, hipStream_t st);

}  // namespace tmq
