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


// Real-split bf16 products: x = hi + lo with hi = bf16(x), lo = bf16(x - hi),
// and x y ~ hi hi + hi lo + lo hi accumulated in FP32 on the 16x16x32 bf16
// instruction (lane l supplies A[l % 16][8 (l / 16) .. 8 (l / 16) + 7] and
// B[8 (l / 16) .. + 7][l % 16]; the result has the layout of Mfma<float>).
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf16x8 neg8(bf16x8 x) {
    s16x8 b = __builtin_bit_cast(s16x8, x);
#pragma unroll
    for (int j = 0; j < 8; ++j) b[j] = (short)(b[j] ^ (short)0x8000);
    return __builtin_bit_cast(bf16x8, b);
}

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// c += x*y with x = xh + xl, y = yh + yl, dropping xl*yl
__device__ __forceinline__ f32x4 split_mac(bf16x8 xh, bf16x8 xl, bf16x8 yh, bf16x8 yl, f32x4 c) {
    c = mfma_bf16(xl, yh, c);
    c = mfma_bf16(xh, yl, c);
    return mfma_bf16(xh, yh, c);
}

// hi / lo planes of eight FP32 values
__device__ __forceinline__ void split8(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const __bf16 h = (__bf16)x[j];
        hi[j] = h;
        lo[j] = (__bf16)(x[j] - (float)h);
    }
}

// complex 16 x 16 tile += A B, the operands given as eight complex FP32
// values per lane (re / im), each real product split hi / lo
__device__ __forceinline__ void cmac_split(CTile<float>& c, const float (&ar)[8], const float (&ai)[8],
                                           const float (&br)[8], const float (&bi)[8]) {
    bf16x8 arh, arl, aih, ail, brh, brl, bih, bil;
    split8(ar, arh, arl);
    split8(ai, aih, ail);
    split8(br, brh, brl);
    split8(bi, bih, bil);
    c.re = split_mac(arh, arl, brh, brl, c.re);
    c.re = split_mac(aih, ail, neg8(bih), neg8(bil), c.re);
    c.im = split_mac(arh, arl, bih, bil, c.im);
    c.im = split_mac(aih, ail, brh, brl, c.im);
}
