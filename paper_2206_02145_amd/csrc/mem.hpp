// mem.hpp -- population planes accessed through buffer descriptors.
//
// A population array is q planes of N values. Each plane gets its own buffer descriptor (base
// address in SGPRs, extent = one plane), and a lane addresses a node with one 32-bit byte offset
// shared by every plane: the address arithmetic of the up to 33 loads and stores of a node costs
// one VGPR, and an offset outside the plane reads 0 / drops the store instead of touching other
// memory.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <type_traits>

namespace lbcg {

constexpr int BUF_RSRC_WORD3 = 0x00020000;  // raw (untyped) buffer, gfx9 family

template <typename T> struct BufOps;
// AUX: cache-policy bits of the access (0 = default; 2 = non-temporal / streaming).
// off: per-lane byte offset (VGPR); soff: byte offset shared by the wavefront (SGPR).
template <> struct BufOps<float> {
    template <int AUX = 0>
    __device__ static inline float ld(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff = 0) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, AUX));
    }
    template <int AUX = 0>
    __device__ static inline void st(__amdgpu_buffer_rsrc_t r, unsigned off, float v, unsigned soff = 0) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, soff, AUX);
    }
};
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
template <> struct BufOps<double> {
    template <int AUX = 0>
    __device__ static inline double ld(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff = 0) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, AUX));
    }
    template <int AUX = 0>
    __device__ static inline void st(__amdgpu_buffer_rsrc_t r, unsigned off, double v, unsigned soff = 0) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, soff, AUX);
    }
};
template <> struct BufOps<__half> {
    template <int AUX = 0>
    __device__ static inline __half ld(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff = 0) {
        return __builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, AUX));
    }
    template <int AUX = 0>
    __device__ static inline void st(__amdgpu_buffer_rsrc_t r, unsigned off, __half v, unsigned soff = 0) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, off, soff, AUX);
    }
};

// q planes of N values of storage type T; loads convert to the compute type R. Stores use the
// cache-policy bits AUX, loads LAUX, except for the first KC planes, which keep the default policy
// for both (the plane index is a compile-time constant after unrolling, so the choice folds away).
template <typename T, int AUX = 0, int LAUX = 0, int KC = 0> struct Planes {
    const char* base;
    unsigned plane_bytes;  // N * sizeof(T), < 2^32

    __device__ __forceinline__ Planes(const void* p, long long N)
        : base(static_cast<const char*>(p)), plane_bytes((unsigned)(N * (long long)sizeof(T))) {}
    __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(int a) const {
        return __builtin_amdgcn_make_buffer_rsrc((void*)(base + (size_t)a * plane_bytes), (short)0,
                                                 (int)plane_bytes, BUF_RSRC_WORD3);
    }
    __device__ __forceinline__ T raw_ld(int a, unsigned off, unsigned soff) const {
        if (a < KC) return BufOps<T>::template ld<0>(rsrc(a), off, soff);
        return BufOps<T>::template ld<LAUX>(rsrc(a), off, soff);
    }
    __device__ __forceinline__ void raw_st(int a, unsigned off, T v, unsigned soff) const {
        if (a < KC) BufOps<T>::template st<0>(rsrc(a), off, v, soff);
        else BufOps<T>::template st<AUX>(rsrc(a), off, v, soff);
    }
    template <typename R> __device__ __forceinline__ R ld(int a, unsigned node) const {
        if constexpr (std::is_same<T, __half>::value)
            return (R)__half2float(raw_ld(a, node * 2u, 0));
        else
            return (R)raw_ld(a, node * (unsigned)sizeof(T), 0);
    }
    template <typename R> __device__ __forceinline__ void st(int a, unsigned node, R v) const {
        if constexpr (std::is_same<T, __half>::value)
            raw_st(a, node * 2u, __float2half_rn((float)v), 0);
        else
            raw_st(a, node * (unsigned)sizeof(T), (T)v, 0);
    }
    // Node row + col where `row` is the same for the whole wavefront: it travels in the scalar
    // offset of the buffer instruction, and the lane supplies only its column.
    template <typename R> __device__ __forceinline__ R ldr(int a, unsigned row, unsigned col) const {
        constexpr unsigned B = sizeof(T);
        if constexpr (std::is_same<T, __half>::value)
            return (R)__half2float(raw_ld(a, col * B, row * B));
        else
            return (R)raw_ld(a, col * B, row * B);
    }
    template <typename R> __device__ __forceinline__ void str(int a, unsigned row, unsigned col, R v) const {
        constexpr unsigned B = sizeof(T);
        if constexpr (std::is_same<T, __half>::value)
            raw_st(a, col * B, __float2half_rn((float)v), row * B);
        else
            raw_st(a, col * B, (T)v, row * B);
    }
};

}  // namespace lbcg
