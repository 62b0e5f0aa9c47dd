// Voxel-state storage formats.  Arithmetic is always FP32 in registers; these codecs convert on
// load and store (round to nearest, ties to even, for every 16-bit format).
//
//   MRH_STORE_F32   D float (m)             W uint32          S2 float (m^2)          12 B / voxel
//   MRH_STORE_F16   D half of D / tau       W uint16 (satur.) V half of S2 / (W tau^2)  6 B / voxel
//   MRH_STORE_BF16  D bfloat16 of D / tau   W half (satur.)   V half of S2 / (W tau^2)  6 B / voxel
//
// The 16-bit formats keep the per-voxel variance sigma^2 = S2 / W normalised by tau^2 rather than
// S2 itself: sigma^2 / tau^2 stays in [0, 4] whatever the weight, so it neither overflows half
// nor needs rescaling after a merge multiplies W.
#pragma once

#include <hip/hip_fp16.h>

#include <cstring>

#include "mrh_internal.h"

namespace mrh {

// float -> bfloat16, round to nearest even: the hardware conversion of gfx950 (v_cvt_pk_bf16_f32)
__device__ inline uint16_t f32_to_bf16(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }

__host__ __device__ inline float bf16_to_f32(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float x;
    __builtin_memcpy(&x, &u, 4);
    return x;
}

__device__ inline uint16_t f32_to_f16(float x) { return __half_as_ushort(__float2half_rn(x)); }
__device__ inline float f16_to_f32(uint16_t h) { return __half2float(__ushort_as_half(h)); }

// The same conversions on the host (clang's _Float16 rounds to nearest even; bfloat16 by integer
// rounding to nearest even, NaN kept NaN).
inline float h_f16(uint16_t b) {
    _Float16 x;
    std::memcpy(&x, &b, 2);
    return (float)x;
}
inline uint16_t h_to_f16(float f) {
    const _Float16 x = (_Float16)f;
    uint16_t b;
    std::memcpy(&b, &x, 2);
    return b;
}
inline float h_bf16(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}
inline uint16_t h_to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN stays NaN
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <int ST>
struct Store;

template <>
struct Store<MRH_STORE_F32> {
    static constexpr int kBytes = 12;
    __device__ static inline void get(const DevMap& m, int lvl, size_t i, float& D, uint32_t& W, float& S2) {
        D = static_cast<const float*>(m.D[lvl])[i];
        W = static_cast<const uint32_t*>(m.W[lvl])[i];
        S2 = static_cast<const float*>(m.S2[lvl])[i];
    }
    __device__ static inline void put(const DevMap& m, int lvl, size_t i, float D, uint32_t W, float S2) {
        static_cast<float*>(m.D[lvl])[i] = D;
        static_cast<uint32_t*>(m.W[lvl])[i] = W;
        static_cast<float*>(m.S2[lvl])[i] = S2;
    }
    __device__ static inline void round(const DevMap&, float&, uint32_t&, float&) {}
    __device__ static inline float getD(const DevMap& m, int lvl, size_t i) {
        return static_cast<const float*>(m.D[lvl])[i];
    }
    __device__ static inline uint32_t getW(const DevMap& m, int lvl, size_t i) {
        return static_cast<const uint32_t*>(m.W[lvl])[i];
    }
    // the weights of 8 consecutive level-0 voxels starting at base (a multiple of 8)
    __device__ static inline void getW8(const DevMap& m, size_t base, uint32_t W[8]) {
        const uint4* wp = reinterpret_cast<const uint4*>(static_cast<const uint32_t*>(m.W[0]) + base);
        const uint4 w0 = wp[0], w1 = wp[1];
        W[0] = w0.x, W[1] = w0.y, W[2] = w0.z, W[3] = w0.w, W[4] = w1.x, W[5] = w1.y, W[6] = w1.z, W[7] = w1.w;
    }
    // 8 consecutive level-0 voxels starting at base (a multiple of 8)
    __device__ static inline void get8(const DevMap& m, size_t base, float D[8], uint32_t W[8], float S2[8]) {
        const float4* dp = reinterpret_cast<const float4*>(static_cast<const float*>(m.D[0]) + base);
        const uint4* wp = reinterpret_cast<const uint4*>(static_cast<const uint32_t*>(m.W[0]) + base);
        const float4* sp = reinterpret_cast<const float4*>(static_cast<const float*>(m.S2[0]) + base);
        const float4 d0 = dp[0], d1 = dp[1], s0 = sp[0], s1 = sp[1];
        const uint4 w0 = wp[0], w1 = wp[1];
        D[0] = d0.x, D[1] = d0.y, D[2] = d0.z, D[3] = d0.w, D[4] = d1.x, D[5] = d1.y, D[6] = d1.z, D[7] = d1.w;
        S2[0] = s0.x, S2[1] = s0.y, S2[2] = s0.z, S2[3] = s0.w, S2[4] = s1.x, S2[5] = s1.y, S2[6] = s1.z, S2[7] = s1.w;
        W[0] = w0.x, W[1] = w0.y, W[2] = w0.z, W[3] = w0.w, W[4] = w1.x, W[5] = w1.y, W[6] = w1.z, W[7] = w1.w;
    }
    __device__ static inline void put8(const DevMap& m, size_t base, const float D[8], const uint32_t W[8],
                                       const float S2[8]) {
        float4* dp = reinterpret_cast<float4*>(static_cast<float*>(m.D[0]) + base);
        uint4* wp = reinterpret_cast<uint4*>(static_cast<uint32_t*>(m.W[0]) + base);
        float4* sp = reinterpret_cast<float4*>(static_cast<float*>(m.S2[0]) + base);
        dp[0] = make_float4(D[0], D[1], D[2], D[3]);
        dp[1] = make_float4(D[4], D[5], D[6], D[7]);
        wp[0] = make_uint4(W[0], W[1], W[2], W[3]);
        wp[1] = make_uint4(W[4], W[5], W[6], W[7]);
        sp[0] = make_float4(S2[0], S2[1], S2[2], S2[3]);
        sp[1] = make_float4(S2[4], S2[5], S2[6], S2[7]);
    }
};

// shared by the two 16-bit formats: D codec and W codec differ, the variance plane is half
template <int ST>
struct Store16 {
    static constexpr int kBytes = 6;
    __device__ static inline float decD(const DevMap& m, uint16_t b) {
        return (ST == MRH_STORE_F16 ? f16_to_f32(b) : bf16_to_f32(b)) * m.tau_f;
    }
    __device__ static inline uint16_t encD(const DevMap& m, float D) {
        const float x = D * m.inv_tau_f;
        return ST == MRH_STORE_F16 ? f32_to_f16(x) : f32_to_bf16(x);
    }
    __device__ static inline uint32_t decW(uint16_t b) {
        return ST == MRH_STORE_F16 ? (uint32_t)b : (uint32_t)f16_to_f32(b);
    }
    // u16 saturates at 65535; the half weight saturates at 65504, the largest finite half (a larger
    // W would round to infinity, whose conversion back to an integer is undefined).  A half weight
    // is exact up to 2048; above that it rounds to the nearest representable value (spacing 2 up
    // to 4096, 4 up to 8192, ...), so a single +1 observation of a voxel with W >= 2048 can leave
    // the stored weight unchanged while D and S2 still move.
    __device__ static inline uint16_t encW(uint32_t W) {
        return ST == MRH_STORE_F16 ? (uint16_t)(W < 65535u ? W : 65535u)
                                   : f32_to_f16((float)(W < 65504u ? W : 65504u));
    }
    __device__ static inline float decS2(const DevMap& m, uint16_t v, uint32_t W) {
        return f16_to_f32(v) * (float)W * m.tau2_f;
    }
    // S2 / (W tau^2) through the hardware reciprocal: the product of W and tau^2 (1/2 ulp), the
    // reciprocal (1 ulp) and the final product (1/2 ulp) keep the FP32 quotient within 2^-22 relative
    // of the exact one, against the 2^-11 relative half-ulp of the FP16 value it is rounded to
    // (an IEEE divide costs about ten instructions and this is done for every stored voxel).
    __device__ static inline uint16_t encS2(const DevMap& m, float S2, uint32_t W) {
        return f32_to_f16(W > 0 ? S2 * __builtin_amdgcn_rcpf((float)W * m.tau2_f) : 0.f);
    }
    // the values a store followed by a load gives back
    __device__ static inline void round(const DevMap& m, float& D, uint32_t& W, float& S2) {
        W = decW(encW(W));
        D = decD(m, encD(m, D));
        S2 = decS2(m, encS2(m, S2, W), W);
    }
    __device__ static inline void get(const DevMap& m, int lvl, size_t i, float& D, uint32_t& W, float& S2) {
        W = decW(static_cast<const uint16_t*>(m.W[lvl])[i]);
        D = decD(m, static_cast<const uint16_t*>(m.D[lvl])[i]);
        S2 = decS2(m, static_cast<const uint16_t*>(m.S2[lvl])[i], W);
    }
    __device__ static inline void put(const DevMap& m, int lvl, size_t i, float D, uint32_t W, float S2) {
        const uint16_t wb = encW(W);
        static_cast<uint16_t*>(m.D[lvl])[i] = encD(m, D);
        static_cast<uint16_t*>(m.W[lvl])[i] = wb;
        static_cast<uint16_t*>(m.S2[lvl])[i] = encS2(m, S2, decW(wb));
    }
    __device__ static inline float getD(const DevMap& m, int lvl, size_t i) {
        return decD(m, static_cast<const uint16_t*>(m.D[lvl])[i]);
    }
    __device__ static inline uint32_t getW(const DevMap& m, int lvl, size_t i) {
        return decW(static_cast<const uint16_t*>(m.W[lvl])[i]);
    }
    __device__ static inline void unpack8(uint4 v, uint16_t o[8]) {
        o[0] = (uint16_t)v.x, o[1] = (uint16_t)(v.x >> 16), o[2] = (uint16_t)v.y, o[3] = (uint16_t)(v.y >> 16);
        o[4] = (uint16_t)v.z, o[5] = (uint16_t)(v.z >> 16), o[6] = (uint16_t)v.w, o[7] = (uint16_t)(v.w >> 16);
    }
    __device__ static inline uint4 pack8(const uint16_t o[8]) {
        return make_uint4((uint32_t)o[0] | ((uint32_t)o[1] << 16), (uint32_t)o[2] | ((uint32_t)o[3] << 16),
                          (uint32_t)o[4] | ((uint32_t)o[5] << 16), (uint32_t)o[6] | ((uint32_t)o[7] << 16));
    }
    __device__ static inline void getW8(const DevMap& m, size_t base, uint32_t W[8]) {
        uint16_t wb[8];
        unpack8(*reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(m.W[0]) + base), wb);
        for (int q = 0; q < 8; ++q) W[q] = decW(wb[q]);
    }
    __device__ static inline void get8(const DevMap& m, size_t base, float D[8], uint32_t W[8], float S2[8]) {
        const uint4 d = *reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(m.D[0]) + base);
        const uint4 w = *reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(m.W[0]) + base);
        const uint4 s = *reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(m.S2[0]) + base);
        uint16_t db[8], wb[8], sb[8];
        unpack8(d, db);
        unpack8(w, wb);
        unpack8(s, sb);
        for (int q = 0; q < 8; ++q) {
            W[q] = decW(wb[q]);
            D[q] = decD(m, db[q]);
            S2[q] = decS2(m, sb[q], W[q]);
        }
    }
    __device__ static inline void put8(const DevMap& m, size_t base, const float D[8], const uint32_t W[8],
                                       const float S2[8]) {
        uint16_t db[8], wb[8], sb[8];
        for (int q = 0; q < 8; ++q) {
            wb[q] = encW(W[q]);
            db[q] = encD(m, D[q]);
            sb[q] = encS2(m, S2[q], decW(wb[q]));
        }
        *reinterpret_cast<uint4*>(static_cast<uint16_t*>(m.D[0]) + base) = pack8(db);
        *reinterpret_cast<uint4*>(static_cast<uint16_t*>(m.W[0]) + base) = pack8(wb);
        *reinterpret_cast<uint4*>(static_cast<uint16_t*>(m.S2[0]) + base) = pack8(sb);
    }
};

template <>
struct Store<MRH_STORE_F16> : Store16<MRH_STORE_F16> {};
template <>
struct Store<MRH_STORE_BF16> : Store16<MRH_STORE_BF16> {};

// host: bytes per voxel of each plane
__host__ __device__ inline int plane_bytes(int storage) { return storage == MRH_STORE_F32 ? 4 : 2; }

}  // namespace mrh
