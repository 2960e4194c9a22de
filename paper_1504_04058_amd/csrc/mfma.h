// Complex products on the matrix cores (CDNA 16x16x4 FP32 / FP64
// instructions), shared by the 2D sweep steps and the 3D factor and solves.
#pragma once

#include <hip/hip_runtime.h>

#include "asp_internal.h"

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// 16x16x4 matrix-core product-accumulate: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; element v (0..3) of the result in lane l is entry
// (row(l, v), l % 16) of the 16 x 16 product.  The FP32 instruction stacks the
// four elements of a lane (rows 4 (l / 16) + v), the FP64 one interleaves them
// (rows l / 16 + 4 v).
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
    using V = f32x4;
    __device__ static __forceinline__ V mac(float a, float b, V c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};
template <>
struct Mfma<double> {
    using V = f64x4;
    __device__ static __forceinline__ V mac(double a, double b, V c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};

// complex 16 x 16 accumulator (real and imaginary planes)
template <typename T>
struct CTile {
    typename Mfma<T>::V re, im;
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            re[v] = T(0);
            im[v] = T(0);
        }
    }
};

// c += a b with complex operands split into four real products
template <typename T>
__device__ __forceinline__ void cmac(CTile<T>& c, cplx<T> a, cplx<T> b) {
    c.re = Mfma<T>::mac(a.x, b.x, c.re);
    c.re = Mfma<T>::mac(-a.y, b.y, c.re);
    c.im = Mfma<T>::mac(a.x, b.y, c.im);
    c.im = Mfma<T>::mac(a.y, b.x, c.im);
}

