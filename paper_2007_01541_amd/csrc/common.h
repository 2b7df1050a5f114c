// Definitions shared by the device kernels: panel geometry, the 16x16x4
// MFMA operand and accumulator layouts, compile-time loops, vector types.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>

namespace wcs {
namespace dev {

constexpr int NB = 64;        // panel width
constexpr int EA_COLS = 8;    // update-matrix columns per extend-add task
constexpr int THREADS = 256;

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Operand layout of both 16x16x4 forms: lane l supplies A(l%16, l/16) and
// B(l/16, l%16).  The accumulator layout differs: element e of lane l holds
// C(4*(l/16) + e, l%16) for f32 and C(4*e + l/16, l%16) for f64.
template <> struct Mfma<float> {
    typedef floatx4 V;
    static __device__ __forceinline__ int row(int kq, int e) { return 4 * kq + e; }
    static __device__ __forceinline__ V mma(float a, float b, V c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<double> {
    typedef doublex4 V;
    static __device__ __forceinline__ int row(int kq, int e) { return 4 * e + kq; }
    static __device__ __forceinline__ V mma(double a, double b, V c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// ---------------------------------------------------------------- utilities

// compile-time loop: fn(integral_constant<int, I>) for I = B, B + S, ... < E
template <int B, int E, int S, typename Fn> __device__ __forceinline__ void static_for(Fn &&fn)
{
    if constexpr (B < E) {
        fn(std::integral_constant<int, B>());
        static_for<B + S, E, S>(fn);
    }
}

// four consecutive elements as one vector access (16 bytes FP32, 32 bytes FP64)
template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef float4 type; };
template <> struct Vec4<double> { typedef double4 type; };

// leading dimension of an m x m front (m rounded up to 8 elements)
__device__ __forceinline__ int front_ld(int m) { return (m + 7) & ~7; }
}  // namespace dev
}  // namespace wcs
