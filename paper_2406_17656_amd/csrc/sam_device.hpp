// sam_device.hpp -- device helpers shared by the gfx950 kernels of the SAM
// library: wave64 group reductions built on DPP row/quad permutations, the
// per-context status word, and small integer utilities.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace samk {

constexpr int kWave = 64;

// Status codes (same numeric values as sam_status in include/sam.h).
constexpr int kStRank = 5;
constexpr int kStNonfinite = 6;
constexpr int kStIndex = 3;
constexpr int kStUnsupported = 8;

// The status word keeps the earliest failing column: (col << 8) | code,
// reduced with atomicMin.  0x7fff... means "no failure".
__device__ inline void report(unsigned long long* status, int col, int code) {
    unsigned long long v = ((unsigned long long)(unsigned)col << 8) | (unsigned)code;
    atomicMin(status, v);
}

// ---------------------------------------------------------------------------
// DPP lane exchanges inside a wave64.  Controls (GCN/CDNA DPP encoding):
//   quad_perm [1,0,3,2] = 0xB1   (xor 1)
//   quad_perm [2,3,0,1] = 0x4E   (xor 2)
//   row_half_mirror     = 0x141  (lane i <-> 7-i inside each 8-lane half row)
//   row_mirror          = 0x140  (lane i <-> 15-i inside each 16-lane row)
// After the quad stages every lane of a quad holds the quad value, so a
// mirror stage pairs each lane with one holding the other half's value; the
// resulting sums are identical in every lane of the group (a + b == b + a).
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ inline int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}

template <int CTRL>
__device__ inline float dpp(float v) {
    return __int_as_float(dpp_i32<CTRL>(__float_as_int(v)));
}

template <int CTRL>
__device__ inline double dpp(double v) {
    int2 p = *reinterpret_cast<int2*>(&v);
    int2 q;
    q.x = dpp_i32<CTRL>(p.x);
    q.y = dpp_i32<CTRL>(p.y);
    return *reinterpret_cast<double*>(&q);
}

// xor-8 exchange inside 32-lane halves (ds_swizzle bitmask mode:
// and_mask = 0x1F, or_mask = 0, xor_mask = 0x08): the LDS pipe's form of the
// last exchange of a 16-lane sum.
__device__ inline float xor8(float v) {
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x201F));
}
// xor-16 exchange inside 32-lane halves (ds_swizzle bitmask mode:
// and_mask = 0x1F, or_mask = 0, xor_mask = 0x10).
__device__ inline float xor16(float v) {
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
}
__device__ inline double xor16(double v) {
    int2 p = *reinterpret_cast<int2*>(&v);
    int2 q;
    q.x = __builtin_amdgcn_ds_swizzle(p.x, 0x401F);
    q.y = __builtin_amdgcn_ds_swizzle(p.y, 0x401F);
    return *reinterpret_cast<double*>(&q);
}
__device__ inline float xor32(float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute((int)((threadIdx.x ^ 32) << 2), __float_as_int(v)));
}
__device__ inline double xor32(double v) {
    int2 p = *reinterpret_cast<int2*>(&v);
    int2 q;
    int a = (int)((threadIdx.x ^ 32) << 2);
    q.x = __builtin_amdgcn_ds_bpermute(a, p.x);
    q.y = __builtin_amdgcn_ds_bpermute(a, p.y);
    return *reinterpret_cast<double*>(&q);
}

// Sum over the G consecutive lanes of a group (G in 1,2,4,...,64); every
// lane of the group receives the same value.
template <int G, typename T>
__device__ inline T group_sum(T v) {
    if constexpr (G >= 2) v += dpp<0xB1>(v);
    if constexpr (G >= 4) v += dpp<0x4E>(v);
    if constexpr (G >= 8) v += dpp<0x141>(v);
    if constexpr (G >= 16) v += dpp<0x140>(v);
    if constexpr (G >= 32) v += xor16(v);
    if constexpr (G >= 64) v += xor32(v);
    return v;
}

// group_sum for FP32 with the exchange between the two 8-lane halves of a
// 16-lane group taken through the LDS pipe (ds_swizzle) instead of a DPP move
// and an add on the VALU: for kernels whose VALU is saturated and whose sums
// are not on the critical path.  The result equals group_sum's (each lane
// adds the same two half sums).
template <int G>
__device__ inline float group_sum_x(float v) {
    if constexpr (G == 16) {
        v += dpp<0xB1>(v);
        v += dpp<0x4E>(v);
        v += dpp<0x141>(v);
        return v + xor8(v);
    } else {
        return group_sum<G>(v);
    }
}

template <int G, typename T>
__device__ inline T group_max(T v) {
    if constexpr (G >= 2) v = fmax(v, dpp<0xB1>(v));
    if constexpr (G >= 4) v = fmax(v, dpp<0x4E>(v));
    if constexpr (G >= 8) v = fmax(v, dpp<0x141>(v));
    if constexpr (G >= 16) v = fmax(v, dpp<0x140>(v));
    if constexpr (G >= 32) v = fmax(v, xor16(v));
    if constexpr (G >= 64) v = fmax(v, xor32(v));
    return v;
}

// Value of lane `src` (0 <= src < G) of the caller's group, in every lane of
// the group: the other lanes contribute an exact zero to a group sum.
template <int G, typename T>
__device__ inline T group_bcast(T v, int g, int src) {
    // groups of 2 or 4 lanes: one quad_perm move; src is a constant once the
    // caller's loop is unrolled, so the switch folds away
    if constexpr (G == 1) {
        return v;
    } else if constexpr (G == 2) {
        return (src & 1) ? dpp<0xF5>(v) : dpp<0xA0>(v);  // [1,1,3,3] / [0,0,2,2]
    } else if constexpr (G == 4) {
        switch (src & 3) {
            case 0: return dpp<0x00>(v);  // [0,0,0,0]
            case 1: return dpp<0x55>(v);  // [1,1,1,1]
            case 2: return dpp<0xAA>(v);  // [2,2,2,2]
            default: return dpp<0xFF>(v); // [3,3,3,3]
        }
    } else {
        return group_sum<G>(g == src ? v : T(0));
    }
}

__device__ inline int wave_lane() { return (int)(threadIdx.x & 63); }

// Wave-level barrier for LDS traffic that stays inside one wavefront.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ inline bool finite_val(T x) { return isfinite(x); }

}  // namespace samk
