// views.h -- device views of the host-side field and link descriptors.
#pragma once
#include "fields.h"
#include "kernels.h"

namespace tmq {

template <class SP>
inline SP make_sp(const FieldDesc &f);
template <>
inline SpF64 make_sp<SpF64>(const FieldDesc &f) { return SpF64{(double2 *)f.data}; }
template <>
inline SpF32 make_sp<SpF32>(const FieldDesc &f) { return SpF32{(float4 *)f.data}; }
template <>
inline SpH16 make_sp<SpH16>(const FieldDesc &f) { return SpH16{(uint4 *)f.data, f.scale}; }
template <>
inline SpB16 make_sp<SpB16>(const FieldDesc &f) { return SpB16{(uint4 *)f.data, f.scale}; }

template <class LK>
inline LK make_lk(const LinkDesc &l);
template <>
inline L64F make_lk<L64F>(const LinkDesc &l) { return L64F{(const double2 *)l.a, l.vh}; }
template <>
inline L64R make_lk<L64R>(const LinkDesc &l) { return L64R{(const double2 *)l.a, l.vh}; }
template <>
inline L32R make_lk<L32R>(const LinkDesc &l) { return L32R{(const float4 *)l.a, l.vh}; }
template <>
inline L16R make_lk<L16R>(const LinkDesc &l) { return L16R{(const uint4 *)l.a, (const uint2 *)l.b, l.vh}; }
template <>
inline L32F make_lk<L32F>(const LinkDesc &l) { return L32F{(const float2 *)l.a, l.vh}; }

// the view of RHS r of a batch (elems / sites: offsets of RHS r)
__device__ __forceinline__ SpF64 rhs_view(const SpF64 &v, long elems, long) { return SpF64{v.p + elems}; }
__device__ __forceinline__ SpF32 rhs_view(const SpF32 &v, long elems, long) { return SpF32{v.p + elems}; }
template <bool BF>
__device__ __forceinline__ Sp16<BF> rhs_view(const Sp16<BF> &v, long elems, long sites)
{
    return Sp16<BF>{v.p + elems, v.scale + sites};
}

// a batched field argument: RHS 0 view plus the per-RHS offsets
template <class SP>
struct BatchView {
    SP v;
    long rhs_elems, rhs_sites;
    __device__ __forceinline__ SP at(int r) const { return rhs_view(v, r * rhs_elems, r * rhs_sites); }
};
template <class SP>
inline BatchView<SP> make_bv(const FieldDesc &f)
{
    return BatchView<SP>{make_sp<SP>(f), f.rhs_elems, f.rhs_sites};
}

// dispatch a statement over the four spinor formats (F is the format type)
#define TMQ_DISPATCH_SP(prec, F, ...)                      \
    switch (prec) {                                        \
    case P64: { using F = SpF64; __VA_ARGS__; } break;     \
    case P32: { using F = SpF32; __VA_ARGS__; } break;     \
    case P16: { using F = SpH16; __VA_ARGS__; } break;     \
    case PB16: { using F = SpB16; __VA_ARGS__; } break;    \
    default: return hipErrorInvalidValue;                  \
    }

}  // namespace tmq
