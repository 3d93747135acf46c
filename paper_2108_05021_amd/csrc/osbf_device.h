// Device-side helpers shared by the one-sided box filter kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace osbf {

// Storage types of the iterate.  Arithmetic is always FP32; the iterate is
// rounded to the storage type (round to nearest even) after every sweep, also
// inside a launch that fuses several sweeps, so results do not depend on how
// sweeps are grouped into launches.
enum : int { DT_F32 = 0, DT_F16 = 1, DT_BF16 = 2 };

template <int DT> struct Storage;

// Raw buffer resource over `bytes` bytes from `base`: loads and stores then
// take a 32-bit lane offset and a scalar (row) offset, so a row walk needs no
// 64-bit vector address arithmetic.  Word 3 is the gfx9-family format word.
using BufRsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ BufRsrc buf_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

// Besides cvt/load/pack/round, each storage type has buffer forms: load_raw
// returns the stored bits in an FP32 register (the value itself for F32),
// from_raw converts them, store rounds and writes one element.  bits rounds
// a value to the storage type and keeps the result in the form store_bits
// writes without converting again (for a value that is only stored).
template <> struct Storage<DT_F32> {
    using T = float;
    static __device__ __forceinline__ float cvt(T v) { return v; }
    static __device__ __forceinline__ float load(const T *p, size_t i) { return p[i]; }
    static __device__ __forceinline__ T pack(float v) { return v; }
    static __device__ __forceinline__ float round(float v) { return v; }
    static __device__ __forceinline__ float load_raw(BufRsrc r, int voff, int soff) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
    }
    static __device__ __forceinline__ float from_raw(float v) { return v; }
    static __device__ __forceinline__ void store(BufRsrc r, int voff, int soff, float v) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, voff, soff, 0);
    }
    static __device__ __forceinline__ float bits(float v) { return v; }
    static __device__ __forceinline__ void store_bits(BufRsrc r, int voff, int soff, float b) { store(r, voff, soff, b); }
};

template <> struct Storage<DT_F16> {
    using T = _Float16;
    static __device__ __forceinline__ float cvt(T v) { return (float)v; }
    static __device__ __forceinline__ float load(const T *p, size_t i) { return (float)p[i]; }
    // The FP32 value is made opaque before the conversion, so the compiler
    // cannot fuse the FMA that produced it with the conversion (a single
    // rounding straight to F16 can differ by one ulp from rounding the FP32
    // result); every kernel then rounds the same FP32 value.
    static __device__ __forceinline__ T pack(float v) {
        asm("" : "+v"(v));
        return (T)v;
    }
    static __device__ __forceinline__ float round(float v) { return (float)pack(v); }
    static __device__ __forceinline__ float load_raw(BufRsrc r, int voff, int soff) {
        return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
    }
    static __device__ __forceinline__ float from_raw(float v) {
        return (float)__builtin_bit_cast(_Float16, (uint16_t)__float_as_uint(v));
    }
    static __device__ __forceinline__ void store(BufRsrc r, int voff, int soff, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, pack(v)), r, voff, soff, 0);
    }
    // the F16 bits in the low half
    static __device__ __forceinline__ float bits(float v) {
        return __uint_as_float((uint32_t)__builtin_bit_cast(uint16_t, pack(v)));
    }
    static __device__ __forceinline__ void store_bits(BufRsrc r, int voff, int soff, float b) {
        __builtin_amdgcn_raw_buffer_store_b16((uint16_t)__float_as_uint(b), r, voff, soff, 0);
    }
};

template <> struct Storage<DT_BF16> {
    using T = uint16_t;
    static __device__ __forceinline__ float cvt(T v) { return __uint_as_float(((uint32_t)v) << 16); }
    static __device__ __forceinline__ float load(const T *p, size_t i) { return cvt(p[i]); }
    // Round to nearest even on the upper 16 bits (inputs are finite).
    static __device__ __forceinline__ T pack(float v) {
        uint32_t u = __float_as_uint(v);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return (T)(u >> 16);
    }
    static __device__ __forceinline__ float round(float v) {
        return __uint_as_float(((uint32_t)pack(v)) << 16);
    }
    static __device__ __forceinline__ float load_raw(BufRsrc r, int voff, int soff) {
        return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
    }
    static __device__ __forceinline__ float from_raw(float v) { return __uint_as_float(__float_as_uint(v) << 16); }
    static __device__ __forceinline__ void store(BufRsrc r, int voff, int soff, float v) {
        __builtin_amdgcn_raw_buffer_store_b16(pack(v), r, voff, soff, 0);
    }
    // the rounded BF16 in the high half (the low half is not cleared)
    static __device__ __forceinline__ float bits(float v) {
        uint32_t u = __float_as_uint(v);
        return __uint_as_float(u + 0x7FFFu + ((u >> 16) & 1u));
    }
    static __device__ __forceinline__ void store_bits(BufRsrc r, int voff, int soff, float b) {
        __builtin_amdgcn_raw_buffer_store_b16((uint16_t)(__float_as_uint(b) >> 16), r, voff, soff, 0);
    }
};

// Scaled distances e_i = |w_i S_i - N c| (N times |mean_i - c|, Alg. 2) and the
// tie-ordered argmin.  `d` holds the signed w_i S_i - N c for the windows in the
// order R, L, D, U, SE, SW, NE, NW.  A balanced tournament in which the left
// (lower-numbered) entrant wins ties returns the lowest-numbered minimum.
struct Pick {
    float d;   // signed scaled difference of the winner
    int idx;   // window index of the winner
};

__device__ __forceinline__ void duel(float &da, int &ia, float db, int ib) {
    bool b_wins = fabsf(db) < fabsf(da);
    da = b_wins ? db : da;
    ia = b_wins ? ib : ia;
}

template <bool WANT_IDX>
__device__ __forceinline__ Pick select8(const float d[8]) {
    float a0 = d[0], a1 = d[2], a2 = d[4], a3 = d[6];
    int i0 = 0, i1 = 2, i2 = 4, i3 = 6;
    if (WANT_IDX) {
        duel(a0, i0, d[1], 1); duel(a1, i1, d[3], 3);
        duel(a2, i2, d[5], 5); duel(a3, i3, d[7], 7);
        duel(a0, i0, a1, i1);  duel(a2, i2, a3, i3);
        duel(a0, i0, a2, i2);
        return Pick{a0, i0};
    } else {
        // the four first-round comparisons are independent; evaluating them
        // before any select lets them share the issue slots of the selects
        const bool c0 = fabsf(d[1]) < fabsf(a0), c1 = fabsf(d[3]) < fabsf(a1);
        const bool c2 = fabsf(d[5]) < fabsf(a2), c3 = fabsf(d[7]) < fabsf(a3);
        a0 = c0 ? d[1] : a0;
        a1 = c1 ? d[3] : a1;
        a2 = c2 ? d[5] : a2;
        a3 = c3 ? d[7] : a3;
        const bool c4 = fabsf(a1) < fabsf(a0), c5 = fabsf(a3) < fabsf(a2);
        a0 = c4 ? a1 : a0;
        a2 = c5 ? a3 : a2;
        a0 = fabsf(a2) < fabsf(a0) ? a2 : a0;
        return Pick{a0, 0};
    }
}

// Wave priority (0 lowest .. 3) for the phases of the streaming kernels'
// steps.  The phases that end in a barrier (the staging of a step's rows
// with the loads and stores it issues, and the row pass between the two
// barriers) gate every wave of the workgroup, while the evaluation after the
// second barrier is VALU work that can fill the issue slots other
// workgroups leave; letting the gating phases issue first (1 for the
// staging, 2 for the row pass, 0 for the evaluation) shortened the forward
// bench step by 1.6-2.4% and the batched rounds by 2% on MI355X; in the
// tiled kernels (phases A and B before their barriers, C after) small images
// ran 1-7% faster, in the volume filter 5-14%; the streaming adjoint gained
// with another order (its VALU-heavy phase lowest), and the fused two-sweep,
// box and Gaussian kernels showed no gain.  Priorities change the order in
// which waves issue, never what they compute.
template <int P>
__device__ __forceinline__ void wave_priority() { __builtin_amdgcn_s_setprio(P); }

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// f(integral_constant<int, I>) for I = I0 .. N-1, unrolled at compile time
// (register arrays indexed by I stay in registers).
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// XCD-aware tile order: the 8 XCDs take workgroups round-robin, so linear
// workgroup b runs on XCD b % 8.  Give each XCD a contiguous run of tiles so
// neighbouring tiles (which share halo rows) hit the same L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int xcd = b & 7, idx = b >> 3;
    const int q = n >> 3, rem = n & 7;
    return xcd * q + min(xcd, rem) + idx;
}

}  // namespace osbf
