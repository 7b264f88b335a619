// Device helpers shared by the HIP translation units of libpairhmm.
// Internal; every function is inline.  Each translation unit that includes
// this header defines its own __constant__ Phred table `c_prob` first.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ph_internal.h"

namespace ph {

// ---------------------------------------------------------------------------
// lane shifts inside groups of P lanes: lane t receives lane t-1's value,
// the first lane of each group receives 0.  Groups of 4 and 8 lanes shift
// inside 16-lane rows like groups of 16: their first lanes other than lanes
// 0, 16, 32, 48 receive the previous group's last lane; callers clear that
// value or give it a zero coefficient (see the forward sweep's first row).
// ---------------------------------------------------------------------------
template <int P>
__device__ __forceinline__ uint32_t shift_up_zero(uint32_t v)
{
    int x = (int)v;
    if constexpr (P == 4 || P == 8 || P == 16) {
        x = __builtin_amdgcn_mov_dpp(x, 0x111 /* row_shr:1 */, 0xf, 0xf, true);
    } else if constexpr (P == 64) {
        x = __builtin_amdgcn_mov_dpp(x, 0x138 /* wave_shr:1 */, 0xf, 0xf, true);
    } else {
        static_assert(P == 32, "lane groups of 4, 8, 16, 32 or 64");
        // lanes 16 and 48 take lane 15 / 47 from the previous 16-lane row,
        // the rest shift inside their row; lanes 0 and 32 keep 0.
        int t = __builtin_amdgcn_update_dpp(0, x, 0x142 /* row_bcast:15 */, 0xa, 0x1, false);
        x = __builtin_amdgcn_update_dpp(t, x, 0x111 /* row_shr:1 */, 0xf, 0xf, false);
    }
    return (uint32_t)x;
}

template <int P>
__device__ __forceinline__ float shift_up(float v)
{
    return __builtin_bit_cast(float, shift_up_zero<P>(__builtin_bit_cast(uint32_t, v)));
}

template <int P>
__device__ __forceinline__ double shift_up(double v)
{
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = shift_up_zero<P>((uint32_t)u);
    uint32_t hi = shift_up_zero<P>((uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// The same shift for groups of 16, 32 or 64 lanes, with the group's first
// lane keeping `old` instead of taking 0 (the DPP move leaves a lane whose
// source lies outside the group unwritten).
template <int P>
__device__ __forceinline__ uint32_t shift_up_or(uint32_t old, uint32_t v)
{
    int x = (int)v, o = (int)old;
    if constexpr (P == 16) {
        x = __builtin_amdgcn_update_dpp(o, x, 0x111 /* row_shr:1 */, 0xf, 0xf, false);
    } else if constexpr (P == 64) {
        x = __builtin_amdgcn_update_dpp(o, x, 0x138 /* wave_shr:1 */, 0xf, 0xf, false);
    } else {
        static_assert(P == 32, "lane groups of 16, 32 or 64");
        int t = __builtin_amdgcn_update_dpp(o, x, 0x142 /* row_bcast:15 */, 0xa, 0x1, false);
        x = __builtin_amdgcn_update_dpp(t, x, 0x111 /* row_shr:1 */, 0xf, 0xf, false);
    }
    return (uint32_t)x;
}

template <int P>
__device__ __forceinline__ float shift_up_or(float old, float v)
{
    return __builtin_bit_cast(float, shift_up_or<P>(__builtin_bit_cast(uint32_t, old), __builtin_bit_cast(uint32_t, v)));
}

template <int P>
__device__ __forceinline__ double shift_up_or(double old, double v)
{
    const uint64_t o = __builtin_bit_cast(uint64_t, old), u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = shift_up_or<P>((uint32_t)o, (uint32_t)u);
    const uint32_t hi = shift_up_or<P>((uint32_t)(o >> 32), (uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <typename T>
struct Range;
template <>
struct Range<float> {
    static constexpr int kExp = 120;
};
template <>
struct Range<double> {
    static constexpr int kExp = 1020;
};


// lane shifts inside groups of P lanes the other way: lane t receives lane
// t+1's value, the last lane of each group receives 0.
template <int P>
__device__ __forceinline__ uint32_t shift_down_zero(uint32_t v)
{
    int x = (int)v;
    if constexpr (P == 16) {
        x = __builtin_amdgcn_mov_dpp(x, 0x101 /* row_shl:1 */, 0xf, 0xf, true);
    } else {
        static_assert(P == 32 || P == 64, "lane groups of 16, 32 or 64");
        x = __builtin_amdgcn_mov_dpp(x, 0x130 /* wave_shl:1 */, 0xf, 0xf, true);
        if constexpr (P == 32) {
            // lane 31 took lane 32's value across the group boundary
            if ((threadIdx.x & 31) == 31) x = 0;
        }
    }
    return (uint32_t)x;
}

template <int P>
__device__ __forceinline__ float shift_down(float v)
{
    return __builtin_bit_cast(float, shift_down_zero<P>(__builtin_bit_cast(uint32_t, v)));
}

template <int P>
__device__ __forceinline__ double shift_down(double v)
{
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = shift_down_zero<P>((uint32_t)u);
    uint32_t hi = shift_down_zero<P>((uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Work cursor of a persistent loop: lane 0 takes the next index, every lane
// reads it back with v_readlane, so the loop condition is wave-uniform and
// the control flow stays reducible.
__device__ __forceinline__ int next_tile(int32_t *cursor)
{
    int t = 0;
    if (threadIdx.x == 0) t = atomicAdd(cursor, 1);
    return __builtin_amdgcn_readlane(t, 0);
}

// Parameters of one read row in linear space.  Phred mode decodes the
// quality bytes through the FP64 table; explicit mode reads the row's
// exponentiated parameters, written once per call by k_prep_params.
struct RowPar {
    double a, b, d, e, z, lm, lx;
};

__device__ __forceinline__ RowPar load_row(const DevProblem &pb, const double *lin, int64_t pos,
                                          const double *c_prob)
{
    RowPar r;
    if (lin) {
        const double *p = lin + pos * 8;
        r.a = p[0];
        r.b = p[1];
        r.d = p[2];
        r.e = p[3];
        r.z = p[4];
        r.lm = p[5];
        r.lx = p[6];
    } else {
        const double Q = c_prob[pb.bq[pos]];
        r.d = c_prob[pb.iq[pos]];
        r.z = c_prob[pb.dq[pos]];
        r.e = c_prob[pb.gq[pos]];
        r.a = 1.0 - r.d - r.z;
        r.b = 1.0 - r.e;
        r.lm = 1.0 - Q;
        r.lx = Q / 3.0;
    }
    return r;
}

__device__ __forceinline__ double load_beta(const DevProblem &pb, const double *lin, int64_t pos,
                                           const double *c_prob)
{
    if (lin) return lin[pos * 8 + 1];
    return 1.0 - c_prob[pb.gq[pos]];
}

__device__ __forceinline__ uint32_t clamp_code(uint32_t c) { return c > 4u ? 4u : c; }

}  // namespace ph
