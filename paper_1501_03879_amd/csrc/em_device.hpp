// Device helpers shared by the EM-ADMM kernels (gfx950, wave64).
//
// Cross-lane sums use the CDNA4 lane-swap instructions
//   v_permlane32_swap_b32 X, Y : X <- [X.lo32, Y.lo32], Y <- [X.hi32, Y.hi32]
//   v_permlane16_swap_b32 X, Y : X <- [X.r0, Y.r0, X.r2, Y.r2], Y <- [X.r1, Y.r1, X.r3, Y.r3]
// (r = 16-lane row) followed by DPP butterflies inside a row.  Summation
// order is fixed, so every result is bit-reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace emx {

__device__ __forceinline__ float swap32_sum(float x, float y) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

__device__ __forceinline__ float swap16_sum(float x, float y) {
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}

// Sum over the 16 lanes of each row; every lane of the row receives it.
__device__ __forceinline__ float row_sum16(float x) {
    x += dpp<0xB1>(x);   // quad_perm [1,0,3,2]: lane ^ 1
    x += dpp<0x4E>(x);   // quad_perm [2,3,0,1]: lane ^ 2
    x += dpp<0x141>(x);  // row_half_mirror: pairs the two quads of each half-row
    x += dpp<0x140>(x);  // row_mirror: pairs the two half-rows
    return x;
}

// Sum over all 64 lanes; every lane receives it.
__device__ __forceinline__ float wave_sum(float x) {
    x = swap32_sum(x, x);
    x = swap16_sum(x, x);
    return row_sum16(x);
}

__device__ __forceinline__ float row_max16(float x) {
    x = fmaxf(x, dpp<0xB1>(x));
    x = fmaxf(x, dpp<0x4E>(x));
    x = fmaxf(x, dpp<0x141>(x));
    x = fmaxf(x, dpp<0x140>(x));
    return x;
}

__device__ __forceinline__ float wave_max(float x) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    x = fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
    auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    x = fmaxf(__uint_as_float(q[0]), __uint_as_float(q[1]));
    return row_max16(x);
}

// Reduce-scatter of V per-lane values over the 64 lanes of a wave.
//
// After the call, for slot j < H2 and row r = lane / 16, out[j] holds (on all
// 16 lanes of row r) the wave-wide sum of input coordinate
//     rs_coord<V>(r, j) = j + (r & 1) * H2 + (r >> 1) * H1,
// valid when rs_valid<V>(r, j); other (row, slot) pairs hold 0.
// Cost: H1 + H2 swaps and adds, then 4 DPP adds per output slot.
template <int V>
struct RS {
    static constexpr int H1 = (V + 1) / 2;
    static constexpr int H2 = (H1 + 1) / 2;
    static __host__ __device__ constexpr bool valid(int r, int j) {
        return (j + (r & 1) * H2 < H1) && (j + (r & 1) * H2 + (r >> 1) * H1 < V);
    }
    static __host__ __device__ constexpr int coord(int r, int j) {
        return j + (r & 1) * H2 + (r >> 1) * H1;
    }
    // inverse map: coordinate c -> row and slot
    static __host__ __device__ constexpr int row_of(int c) {
        return (c < H1) ? (c < H2 ? 0 : 1) : ((c - H1) < H2 ? 2 : 3);
    }
    static __host__ __device__ constexpr int slot_of(int c) {
        return (c < H1) ? (c < H2 ? c : c - H2) : ((c - H1) < H2 ? c - H1 : c - H1 - H2);
    }
};

template <int V>
__device__ __forceinline__ void reduce_scatter(const float (&x)[V], float (&out)[RS<V>::H2]) {
    constexpr int H1 = RS<V>::H1, H2 = RS<V>::H2;
    float t[H1];
#pragma unroll
    for (int j = 0; j < H1; ++j) t[j] = swap32_sum(x[j], (j + H1 < V) ? x[j + H1] : 0.0f);
#pragma unroll
    for (int j = 0; j < H2; ++j) out[j] = swap16_sum(t[j], (j + H2 < H1) ? t[j + H2] : 0.0f);
#pragma unroll
    for (int j = 0; j < H2; ++j) out[j] = row_sum16(out[j]);
}

// Full reduce-scatter of V <= 64 per-lane values over the 64 lanes: six
// halving stages (lane bit 5, 4: permlane32/16 swaps; bits 3, 2, 1, 0: DPP
// row_ror:8, row_half_mirror, quad_perm with selects).  Stage s keeps
// K_{s+1} = ceil(K_s / 2) values per lane: lanes whose stage bit is clear keep
// indices [0, K_{s+1}), the others [K_{s+1}, 2 K_{s+1}).  Afterwards every lane
// holds one wave-wide total, for coordinate RSF<V>::coord(lane) when
// RSF<V>::valid(lane); each valid coordinate is held by exactly one lane and
// the other lanes return 0.
template <int V>
struct RSF {
    static_assert(V >= 1 && V <= 64, "RSF: 1..64 values");
    static __host__ __device__ constexpr int K(int s) {
        int k = V;
        for (int i = 0; i < s; ++i) k = (k + 1) / 2;
        return k;
    }
    static __host__ __device__ constexpr int coord(int lane) {
        int c = 0;
        for (int s = 0; s < 6; ++s)
            if (lane & (32 >> s)) c += K(s + 1);
        return c;
    }
    static __host__ __device__ constexpr bool valid(int lane) {
        // the index a lane holds after stage s must be below K_{s+1}; at
        // every stage the upper lanes hold index + K_{s+1} of the K_s inputs
        int idx = 0;
        for (int s = 5; s >= 0; --s) {
            if (lane & (32 >> s)) idx += K(s + 1);
            if (idx >= K(s)) return false;
        }
        return true;
    }
    // bit l set when lane l holds a coordinate
    static __host__ __device__ constexpr uint64_t mask() {
        uint64_t m = 0;
        for (int l = 0; l < 64; ++l)
            if (valid(l)) m |= (uint64_t)1 << l;
        return m;
    }
    // the lane that holds coordinate c
    static __host__ __device__ constexpr int lane_of(int c) {
        for (int l = 0; l < 64; ++l)
            if (valid(l) && coord(l) == c) return l;
        return -1;
    }
};

template <int CTRL>
__device__ __forceinline__ float rs_dpp_stage(float lo, float hi, bool upper) {
    const float send = upper ? lo : hi;
    const float keep = upper ? hi : lo;
    return keep + dpp<CTRL>(send);
}

// One DPP stage of reduce_scatter_full for slot i: with an upper half
// (i + K < Kprev) the lanes exchange halves; without one the stage is a plain
// butterfly, which gives a valid lane the same sum (lo + partner's lo) and
// the lanes above it, which hold no coordinate, the same value instead of 0.
template <int CTRL, bool HALVES>
__device__ __forceinline__ float rs_dpp_slot(float lo, float hi, bool upper) {
    if constexpr (HALVES) return rs_dpp_stage<CTRL>(lo, hi, upper);
    else return lo + dpp<CTRL>(lo);
}

// `own` = RSF<V>::valid(lane): lanes that hold no coordinate return 0.
template <int V>
__device__ __forceinline__ float reduce_scatter_full(const float (&x)[V], int lane, bool own) {
    using R = RSF<V>;
    constexpr int K1 = R::K(1), K2 = R::K(2), K3 = R::K(3), K4 = R::K(4), K5 = R::K(5);
    float a[K1];
#pragma unroll
    for (int i = 0; i < K1; ++i) a[i] = swap32_sum(x[i], (i + K1 < V) ? x[i + K1] : 0.0f);
    float b[K2];
#pragma unroll
    for (int i = 0; i < K2; ++i) b[i] = swap16_sum(a[i], (i + K2 < K1) ? a[i + K2] : 0.0f);
    const bool u8 = lane & 8, u4 = lane & 4, u2 = lane & 2, u1 = lane & 1;
    float c[K3];
#pragma unroll
    for (int i = 0; i < K3; ++i)   // row_ror:8
        c[i] = (i + K3 < K2) ? rs_dpp_slot<0x128, true>(b[i], b[(i + K3) % K2], u8)
                             : rs_dpp_slot<0x128, false>(b[i], 0.0f, u8);
    float d[K4];
#pragma unroll
    for (int i = 0; i < K4; ++i)   // row_half_mirror
        d[i] = (i + K4 < K3) ? rs_dpp_slot<0x141, true>(c[i], c[(i + K4) % K3], u4)
                             : rs_dpp_slot<0x141, false>(c[i], 0.0f, u4);
    float e[K5];
#pragma unroll
    for (int i = 0; i < K5; ++i)   // lane ^ 2
        e[i] = (i + K5 < K4) ? rs_dpp_slot<0x4E, true>(d[i], d[(i + K5) % K4], u2)
                             : rs_dpp_slot<0x4E, false>(d[i], 0.0f, u2);
    const float r = (1 < K5) ? rs_dpp_slot<0xB1, true>(e[0], e[1 % K5], u1)   // lane ^ 1
                             : rs_dpp_slot<0xB1, false>(e[0], 0.0f, u1);
    return own ? r : 0.0f;
}

// Reads a wave-uniform float held by lane `lane` of a VGPR into an SGPR.
__device__ __forceinline__ float readlane(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ __forceinline__ float readfirstlane(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Marks a wave-uniform condition as such, so the compiler branches on it
// with scalar branches instead of exec masks (which would keep both sides'
// register state alive).
__device__ __forceinline__ bool uniform(bool b) { return __builtin_amdgcn_readfirstlane((int)b) != 0; }

// Shrink factor of the block soft-threshold (closed-form prox of
// lambda ||x - a||): x = v - s (v - a) with s = min(lambda, nu) / nu and
// nu = ||v - a||, i.e. s = min(1, lambda / nu).  s = 1 (x = a) whenever
// nu <= lambda; lambda = 0 gives s = 0 (x = v).  lambda >= 0.  Callers start
// their sums of squares at kNu2Floor, so nu2 > 0 and rsq stays finite
// (nu = 0 then gives s = 1 for lambda > 0, as the exact formula's limit).
constexpr float kNu2Floor = 1e-30f;
__device__ __forceinline__ float shrink(float nu2, float lambda) {
    return fminf(1.0f, lambda * __builtin_amdgcn_rsqf(nu2));
}

__device__ __forceinline__ float clampf(float x, float lo, float hi) {
    return fminf(fmaxf(x, lo), hi);
}

// Symmetric (edge-repeating) reflection into [0, N), then clamped so that
// positions the solver never reads still address valid memory.
__device__ __forceinline__ int reflect_idx(int i, int N) {
    i = (i < 0) ? (-i - 1) : i;
    i = (i >= N) ? (2 * N - i - 1) : i;
    return min(max(i, 0), N - 1);
}

}  // namespace emx
