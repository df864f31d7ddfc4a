// kernels.h -- host-side declarations of the device kernels' launch wrappers.
//
// Host code (the lattice object, the solvers, the C ABI) is format-agnostic:
// it passes FieldDesc / LinkDesc descriptors and the wrappers dispatch to the
// template instantiations in hop.hip, blas.hip and codec.hip.
//
// Every vector kernel works on a batch of right-hand sides (RHS): a field
// holds nrhs fields of n sites each, and a launch covers the RHS named in an
// RhsList.  One block handles one RHS, so per-RHS scalars, "done" flags and
// partial sums stay separate, and each RHS is computed exactly as if it were
// alone (a single solve is the batch of one).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fastdiv.h"

namespace tmq {

enum Prec { P64 = 0, P32 = 1, P16 = 2, PB16 = 3 };  // same values as tmq_prec
// LK32F: FP32 full 3x3 links, the reduced-precision copy of a gauge field
// that is not SU(3) (two-row storage rebuilds row 2 assuming SU(3))
enum LinkFmt { LK64F = 0, LK64R = 1, LK32R = 2, LK16R = 3, LK32F = 4 };
constexpr int N_LINK_FMT = 8;  // stride of the (spinor precision, link format) tuning keys

constexpr int MAX_RHS = 64;

// Lattice geometry.  Extents (T, LZ, LY, LX) all even; V/2 sites per parity,
// eo index h = site >> 1 with site = ((t*LZ + z)*LY + y)*LX + x.
struct Geom {
    int T, LZ, LY, LX;
    int XH;   // LX / 2
    long vh;  // V / 2
};

// A batch of spinor fields, each of n sites (one parity, or both parities
// stacked: even sites 0..V/2-1, odd sites V/2..V-1) in the 8-site chunked
// layout of fields.h; RHS r starts rhs_elems elements (and rhs_sites scales)
// after RHS 0.
struct FieldDesc {
    int prec = P64;
    void *data = nullptr;   // element type by prec: double2, float4, uint4
    float *scale = nullptr; // FP32 per-site scale of 16-bit formats
    long n = 0;             // sites per RHS (a multiple of 8)
    int nrhs = 1;
    long rhs_elems = 0;
    long rhs_sites = 0;
};

// sub-view starting at site `off` (a multiple of 8), n sites, every RHS
FieldDesc field_sub(const FieldDesc &f, long off, long n);
// the single field of RHS r
FieldDesc field_rhs(const FieldDesc &f, int r);
size_t field_elem_bytes(int prec);
int field_blocks(int prec);  // component blocks per site: 12, 6, 3, 3

// The RHS a launch covers (indices into the batch).
struct RhsList {
    int n = 0;
    unsigned char idx[MAX_RHS];
};
RhsList rhs_all(int n);

struct LinkDesc {
    int fmt = LK64F;
    const void *a = nullptr;  // main array
    const void *b = nullptr;  // second array (LK16R)
    long vh = 0;              // sites per parity
};

// Operator parameters of a launch: boundary phases common to the batch,
// kappa and mut = 2 kappa mu per RHS (indexed by the batch index).
//
// nd = 1: the flavour doublet of eq. (Dh) (mut is 2 kappa mubar, eps is
// 2 kappa epsbar).  A doublet field is one field of twice the sites, the
// upper flavour's sites first; doublet d of a batch has its parameters at
// index d.  Host wrappers present the launch to the kernel as a batch of
// single-flavour fields in which doublet d is the pair 2d, 2d + 1.
struct OpParams {
    double ph[4][2];  // e^{i theta_mu pi / L_mu} (re, im), mu = t, x, y, z
    double kappa[MAX_RHS];
    double mut[MAX_RHS];
    double eps[MAX_RHS];
    int nd = 0;
};

// Epilogue of a hop half-sweep at output site h (spin s; upper = spins 0,1
// where gamma_5 = +1, lower = spins 2,3), with sigma = sign of Qhat^{+-}:
//   EPI_K1   out = kappa^2/(1+mut^2) (1 - sigma i mut g5) acc              (eq. (eo3))
//   EPI_K2   out = g5 [(1 + sigma i mut g5) self - acc]                    (eq. (eo4))
//   EPI_FULL out = g5 [(1 + sigma i mut g5) self - kappa acc]              (eq. (eo1))
//   EPI_SRC  out = self + kappa acc                                       (even/odd source, App. B)
//   EPI_REC  out = (1 - sigma i mut g5)/(1+mut^2) (self + kappa acc)      (even-site solution, App. B)
//   EPI_K2_CG  as EPI_K2, then the CG update with the RHS's alpha (device
//              scalars): r -= alpha out ; x += alpha p ; norm of the new r; out is
//              not stored
//   EPI_K2_RES as EPI_K2, then r = b - out (the true residual) with its norm;
//              out is not stored
// For a doublet (OpParams::nd) a lane pair holds the two flavours (f, f') of
// a site and, with A = 1 + sigma i mubar g5 tau^3 + epsbar tau^1 the site term
// and d = 1 + mubar^2 - epsbar^2,
//   EPI_K1   out = kappa^2 / d (1 - sigma i mubar g5 tau^3 - epsbar tau^1) acc
//   EPI_K2   out = g5 [A self - acc]
// and the fused epilogues as above, per flavour, with the doublet's scalars;
// the norm is over both flavours.  Other epilogues are refused.
enum HopEpi { EPI_K1 = 0, EPI_K2 = 1, EPI_FULL = 2, EPI_K2_CG = 3, EPI_K2_RES = 4, EPI_SRC = 5, EPI_REC = 6 };

// Vectors of the fused epilogues: r and p in the hop's spinor format (p is b
// for EPI_K2_RES), x in FP32 (FP64 for an FP64 hop).
struct CgFields {
    FieldDesc r, p, x;
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
    int done;        // 1 once rr < target or nan (kernels told to skip done RHS then do nothing)
    int nan;         // 1 once a non-finite scalar appeared
    int reliable;    // number of true-residual recomputations
    int last_true;   // 1 if rr is a recomputed true residual
    int pad;
};

constexpr int HOP_BLOCK = 256;
constexpr int BLAS_BLOCK = 256;

int hop_grid(long n);
int blas_grid(long n);

// hop kernel variants (see hop.hip): 0 plain order, 1 z-slabs per XCD, 2
// z-slabs + scheduling barriers, 3 t-slabs per XCD, 4 t-slabs + barriers.
// z-slabs need LZ >= 8, t-slabs T >= 8.  Links are loaded non-temporally in
// single-RHS launches and cached in batched ones.
enum HopOrder { ORD_PLAIN = 0, ORD_ZSLAB = 1, ORD_TSLAB = 2 };
constexpr int HOP_VARIANTS = 5;
bool hop_variant_valid(const Geom &g, int v);
// whether the (spinor precision, link format) pairing has every variant; the
// others always run variant 0 whatever HopTune asks for
bool hop_all_variants(int prec, int link_fmt);
// blocks per RHS (= per-block partial sums written with a norm) of variant v;
// lanes_per_site = 2 for doublets in the general kernel (a lane pair per site)
int hop_grid_variant(const Geom &g, int v, int lanes_per_site = 1);

// bit mu set when the boundary phase of direction mu is not 1
inline int hop_phase_mask(const OpParams &op)
{
    int m = 0;
    for (int mu = 0; mu < 4; mu++)
        if (op.ph[mu][0] != 1.0 || op.ph[mu][1] != 0.0) m |= 1 << mu;
    return m;
}
// whether a launch of 16-bit spinors on FP16 two-row links runs in the 16-bit
// kernel (hop16_kernel): 32-bit offsets (V/2 < 2^26) and a boundary phase in
// time only, or none
inline bool hop16_ok(const Geom &g, int phase_mask) { return g.vh < (1L << 26) && (phase_mask == 0 || phase_mask == 1); }
// lanes per site of a doublet launch: 1 in the 16-bit kernel (both flavours
// in a lane), 2 in the general kernel (a lane pair)
inline int hop_nd_lanes(const Geom &g, int prec, int link_fmt, const OpParams &op)
{
    return (prec == P16 || prec == PB16) && link_fmt == LK16R && hop16_ok(g, hop_phase_mask(op)) ? 1 : 2;
}

// Hop half-sweep: out(h) over the V/2 sites of parity out_par for every RHS
// of rl; `in` holds parity 1 - out_par; `self` (data may be nullptr unless
// the epilogue needs it) holds parity out_par.  partial != nullptr: per-block
// sums of |out|^2 at partial[r * pstride + block].  scal != nullptr: blocks of
// RHS r with scal[r].done set do nothing.
// Launch shape of a hop half-sweep, chosen by the autotuner.
struct HopTune {
    int variant = 0;   // block order (see above)
    int group = 0;     // RHS per L2 group of a batched launch (0: sized from the L2 capacity)
    int rpl = 1;       // RHS per lane in a batched launch: 1 or 2 (FP32-arithmetic formats)
    unsigned lds = 0;  // LDS bytes reserved per block (unused by the kernel; a value above
                       // the CU's LDS / (c + 1) caps the blocks resident per CU at c)
};
hipError_t launch_hop(const Geom &g, int out_par, const FieldDesc &in, const FieldDesc &self,
                      const FieldDesc &out, const LinkDesc &lk, const OpParams &op, int epi, int sign,
                      const RhsList &rl, double *partial, long pstride, const CgScalars *scal, const HopTune &tu,
                      hipStream_t st, const CgFields *cg = nullptr);

// Vector kernels over the n sites of each RHS of rl.  Reductions write
// blas_grid(n) per-block sums at partial[r * pstride + block]; scalars come
// from scal[r]; skip_done: blocks of RHS with scal[r].done do nothing.
hipError_t launch_norm2(const FieldDesc &v, const RhsList &rl, double *partial, long pstride, hipStream_t st);
hipError_t launch_convert(const FieldDesc &in, const FieldDesc &out, const RhsList &rl, hipStream_t st);
hipError_t launch_zero(const FieldDesc &v, const RhsList &rl, hipStream_t st);
// x += alpha p ; r -= alpha ap ; partial |r|^2
hipError_t launch_axpy_norm(const FieldDesc &x, const FieldDesc &p, const FieldDesc &r, const FieldDesc &ap,
                            const RhsList &rl, const CgScalars *scal, double *partial, long pstride,
                            bool skip_done, hipStream_t st);
// p = r + beta p
hipError_t launch_xpay(const FieldDesc &r, const FieldDesc &p, const RhsList &rl, const CgScalars *scal,
                       bool skip_done, hipStream_t st);
// r = b - ax (FP64), partial |r|^2
hipError_t launch_residual(const FieldDesc &b, const FieldDesc &ax, const FieldDesc &r, const RhsList &rl,
                           double *partial, long pstride, hipStream_t st);
// out = cu in (spins 0, 1), cd in (spins 2, 3); FP64 fields
hipError_t launch_twist(const FieldDesc &in, const FieldDesc &out, const RhsList &rl, double2 cu, double2 cd,
                        hipStream_t st);
// x64 += xs ; xs = 0
hipError_t launch_accumulate(const FieldDesc &x64, const FieldDesc &xs, const RhsList &rl, hipStream_t st);

// Scalar kernels (one block per RHS): deterministic sums of nparts partials.
enum ScalarOp {
    SC_INIT = 0,     // bb = rr = sum ; target = tol2 * (relative ? bb : 1) ; counters cleared
    SC_ALPHA = 1,    // pAp = sum ; alpha = rr / pAp
    SC_BETA = 2,     // rr_prev = rr ; rr = sum ; beta = rr / rr_prev ; iter++ ; done = rr < target
    SC_RELIABLE = 3  // rr = sum (true residual) ; beta = rr / rr_prev ; done = rr < target
};
// publish != nullptr: the scalars of RHS r are finally copied to publish[r]
// (host-mapped memory), also when the block is skipped.
hipError_t launch_scalar(int op, const RhsList &rl, const double *partial, long pstride, int nparts,
                         CgScalars *scal, double tol2, int relative, bool skip_done, CgScalars *publish,
                         hipStream_t st);
// out[0] = deterministic maximum of partial[0..n)
hipError_t launch_max(const double *partial, int n, double *out, hipStream_t st);
// b = a, bytes / 16 lanes of 16 bytes (bandwidth calibration)
hipError_t launch_stream_copy(const void *src, void *dst, size_t bytes, hipStream_t st);

// BiCGstab on one odd-site system (FP64, RHS 0 of each field), scalars on
// the device; every kernel does nothing once `done` is set (see bicgstab.hip)
struct BicgScalars {
    double rho[2], alpha[2], omega[2], beta[2];  // complex (re, im)
    double rr, bb, target;
    int iter, restarts, done, nan, breakdown;
    int max_iter;  // done once iter reaches it (set by the host before the start)
};
enum BicgOp {
    BI_START = 0,  // r = rhat: sums <rhat, r>, |r|^2 ; alpha = omega = 1, beta = 0
    BI_ALPHA = 1,  // sum <rhat, v> ; alpha = rho / <rhat, v>
    BI_OMEGA = 2,  // sums <t, s>, |t|^2 ; omega = <t, s> / |t|^2
    BI_UPDATE = 3  // sums <rhat, r>, |r|^2 of the new r ; beta = (rho' / rho)(alpha / omega) ; done
};
// <a, b> -> p0 (re), p1 (im); |a|^2 -> p2, one partial per block (blas_grid(n))
hipError_t launch_bi_dot(const FieldDesc &a, const FieldDesc &b, const BicgScalars *sc, double *p0, double *p1,
                         double *p2, hipStream_t st);
// p = r + beta (p - omega v)
hipError_t launch_bi_p(const FieldDesc &r, const FieldDesc &p, const FieldDesc &v, const BicgScalars *sc,
                       hipStream_t st);
// s = r - alpha v
hipError_t launch_bi_s(const FieldDesc &r, const FieldDesc &v, const FieldDesc &s, const BicgScalars *sc,
                       hipStream_t st);
// x += alpha p + omega s ; r = s - omega t ; <rhat, r> -> p0, p1 ; |r|^2 -> p2
hipError_t launch_bi_xr(const FieldDesc &x, const FieldDesc &p, const FieldDesc &s, const FieldDesc &t,
                        const FieldDesc &r, const FieldDesc &rhat, const BicgScalars *sc, double *p0, double *p1,
                        double *p2, hipStream_t st);
// one scalar step (BicgOp) from nparts partials of p0, p1, p2; publish: copy of the scalars
hipError_t launch_bi_scalar(int op, const double *p0, const double *p1, const double *p2, int nparts,
                            BicgScalars *s, double tol2, int relative, BicgScalars *publish, hipStream_t st);

// the whole full-lattice FP64 CG on Q^+ Q^- of a tiny lattice in one
// workgroup (small_cg.hip): f = {b, x, r, p, t, ap}, stacked full fields;
// continues from x and the counters in *sc (zeroed before the first call),
// ends with the true residual in sc->rr and sc->done set if it met the target
constexpr long SMALL_CG_MAX_SITES = 1024;
hipError_t launch_small_cg(const Geom &g, const FieldDesc *f, const LinkDesc &lk, const OpParams &op, double tol2,
                           int relative, int max_iter, CgScalars *sc, hipStream_t st);

// a 4x4 complex spin matrix (row-major)
struct SpinMat {
    double2 m[4][4];
};
// per time slice t and block b of it: partial sums of psi^+ Gamma psi over the
// slice's sites (psi canonical full-lattice complex128 [V][12]) at
// pre / pim[t * ts_bilinear_blocks(g) + b]
int ts_bilinear_blocks(const Geom &g);
hipError_t launch_ts_bilinear(const Geom &g, const double2 *psi, const SpinMat &m, double *pre, double *pim,
                              hipStream_t st);

// codec: canonical complex128 [site][12] <-> one device field (RHS 0 of the view)
hipError_t launch_from_canonical(const double2 *in, const FieldDesc &out, hipStream_t st);
hipError_t launch_to_canonical(const FieldDesc &in, double2 *out, hipStream_t st);
// full-lattice fields: canonical site s of parity p -> stacked view site p * V/2 + (s >> 1)
hipError_t launch_full_from_canonical(const Geom &g, const double2 *in, const FieldDesc &out, hipStream_t st);
hipError_t launch_full_to_canonical(const Geom &g, const FieldDesc &in, double2 *out, hipStream_t st);
// canonical full field (complex128 [V][12], lexicographic sites) <-> canonical
// even and odd fields ([V/2][12], eo index = site >> 1); split skips a null
// parity, merge writes zeros for one
hipError_t launch_split_eo(const Geom &g, const double2 *full, double2 *even, double2 *odd, hipStream_t st);
hipError_t launch_merge_eo(const Geom &g, const double2 *even, const double2 *odd, double2 *full, hipStream_t st);
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
    float2 *full32;   // LK32F
};
hipError_t launch_gauge_ingest(const Geom &g, const double2 *U, const GaugeOut &o, double *partial_max,
                               hipStream_t st);

}  // namespace tmq
