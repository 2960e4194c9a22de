// Complex-double kernels outside the layer solves: the symmetric-form PML
// stencil of eq. (2D) / eq. (3D) and the batched vector operations of GMRES
// (multi-dot products, multi-axpy with the norm of the result, scaling).
// Every per-right-hand-side reduction runs in a fixed order that does not
// depend on how many right-hand sides share the launch.
#include "asp_internal.h"

namespace {

constexpr int BS = 256;
constexpr int CHUNK = 8;   // Krylov vectors per multi-dot / multi-axpy pass

// y = A x for the symmetric form.  2D: a thread walks SEG2 consecutive lines
// i2 at one i1, keeping x on lines i2-1, i2, i2+1 in registers (each value is
// read from memory once; the i1 neighbours come from the cache).  The stencil
// coefficients are formed from the 1D PML tables and omega^2/c^2:
//   coupling along axis a at the half line t+1/2:  s(t+1/2) / (h^2 prod_{b != a} s(i_b))
//   diagonal: -(sum of the couplings) + omega^2 / (c^2 prod_b s(i_b))
constexpr int SEG2 = 8;

__global__ __launch_bounds__(BS) void stencil2d_kernel(const zd* __restrict__ x,
                                                     zd* __restrict__ y,
                                                     const int* __restrict__ act,
                                                     AxisTables ax,
                                                     const double* __restrict__ ksq, int n,
                                                     long long N) {
    const int i1 = blockIdx.x * BS + threadIdx.x;
    const int i2a = blockIdx.y * SEG2;
    if (i1 >= n) return;
    const int rhs = act ? act[blockIdx.z] : (int)blockIdx.z;
    const zd* xr = x + (long long)rhs * N;
    zd* yr = y + (long long)rhs * N;
    const zd sh_e = ax.sh[i1 + 1], sh_w = ax.sh[i1], is2_1 = ax.inv_sh2[i1], is_1 = ax.inv_s[i1];
    zd xm = (i2a > 0) ? xr[(long long)(i2a - 1) * n + i1] : mk(0.0, 0.0);
    zd xc = xr[(long long)i2a * n + i1];
    const int i2e = min(i2a + SEG2, n);
    for (int i2 = i2a; i2 < i2e; ++i2) {
        const long long idx = (long long)i2 * n + i1;
        const zd xp = (i2 + 1 < n) ? xr[idx + n] : mk(0.0, 0.0);
        const zd ce = sh_e * ax.inv_sh2[i2];
        const zd cw = sh_w * ax.inv_sh2[i2];
        const zd cn = ax.sh[i2 + 1] * is2_1;
        const zd cs = ax.sh[i2] * is2_1;
        const zd dg = (ksq[idx] * is_1) * ax.inv_s[i2] - (ce + cw + cn + cs);
        zd acc = dg * xc;
        if (i1 + 1 < n) acc = cfma(ce, xr[idx + 1], acc);
        if (i1 > 0) acc = cfma(cw, xr[idx - 1], acc);
        if (i2 + 1 < n) acc = cfma(cn, xp, acc);
        if (i2 > 0) acc = cfma(cs, xm, acc);
        yr[idx] = acc;
        xm = xc;
        xc = xp;
    }
}

__global__ __launch_bounds__(BS) void stencil3d_kernel(const zd* __restrict__ x,
                                                     zd* __restrict__ y,
                                                     const int* __restrict__ act,
                                                     AxisTables ax,
                                                     const double* __restrict__ ksq, int n,
                                                     long long N, int nz) {
    const int i1 = blockIdx.x * BS + threadIdx.x;
    const int i2 = blockIdx.y;
    const int i3 = blockIdx.z % nz;
    if (i1 >= n) return;
    const int slot = blockIdx.z / nz;
    const int rhs = act ? act[slot] : slot;
    const long long nn = (long long)n * n;
    const long long idx = (long long)i3 * nn + (long long)i2 * n + i1;
    const zd s23 = ax.inv_sh2[i2] * ax.inv_s[i3];   // 1/(h^2 s2 s3)
    const zd s13 = ax.inv_sh2[i1] * ax.inv_s[i3];
    const zd s12 = ax.inv_sh2[i1] * ax.inv_s[i2];
    const zd c1p = ax.sh[i1 + 1] * s23, c1m = ax.sh[i1] * s23;
    const zd c2p = ax.sh[i2 + 1] * s13, c2m = ax.sh[i2] * s13;
    const zd c3p = ax.sh[i3 + 1] * s12, c3m = ax.sh[i3] * s12;
    const zd dg = ((ksq[idx] * ax.inv_s[i1]) * ax.inv_s[i2]) * ax.inv_s[i3] -
                  (c1p + c1m + c2p + c2m + c3p + c3m);
    const zd* xr = x + (long long)rhs * N;
    zd acc = dg * xr[idx];
    if (i1 + 1 < n) acc = cfma(c1p, xr[idx + 1], acc);
    if (i1 > 0) acc = cfma(c1m, xr[idx - 1], acc);
    if (i2 + 1 < n) acc = cfma(c2p, xr[idx + n], acc);
    if (i2 > 0) acc = cfma(c2m, xr[idx - n], acc);
    if (i3 + 1 < n) acc = cfma(c3p, xr[idx + nn], acc);
    if (i3 > 0) acc = cfma(c3m, xr[idx - nn], acc);
    y[(long long)rhs * N + idx] = acc;
}

// b = f / prod_k s_k(i_k)
__global__ void scale_by_s_kernel(const zd* __restrict__ f, zd* __restrict__ b, AxisTables ax,
                                  int n, int dim, long long N) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N) return;
    const long long o = (long long)blockIdx.y * N + idx;
    long long t = idx;
    zd sc = mk(1.0, 0.0);
    for (int a = 0; a < dim; ++a) {
        sc = sc * ax.inv_s[t % n];
        t /= n;
    }
    b[o] = f[o] * sc;
}

// fixed-order tree reduction of BS values per lane slot
template <int NV>
__device__ __forceinline__ void block_reduce(zd (&v)[NV], zd* sh) {
    const int t = threadIdx.x;
    for (int k = 0; k < NV; ++k) sh[k * BS + t] = v[k];
    __syncthreads();
    for (int s = BS / 2; s > 0; s >>= 1) {
        if (t < s)
            for (int k = 0; k < NV; ++k) sh[k * BS + t] = sh[k * BS + t] + sh[k * BS + t + s];
        __syncthreads();
    }
    for (int k = 0; k < NV; ++k) v[k] = sh[k * BS];
}

__global__ __launch_bounds__(BS) void multidot_kernel(const zd* __restrict__ V, long long vstride,
                                                    int i0, int ni, const zd* __restrict__ w,
                                                    long long N, const int* __restrict__ act,
                                                    zd* __restrict__ partial) {
    __shared__ zd sh[CHUNK * BS];
    const int rhs = act ? act[blockIdx.y] : (int)blockIdx.y;
    const int nblk = gridDim.x;
    zd acc[CHUNK];
    for (int k = 0; k < CHUNK; ++k) acc[k] = mk(0.0, 0.0);
    const zd* wr = w + (long long)rhs * N;
    for (long long idx = (long long)blockIdx.x * BS + threadIdx.x; idx < N;
         idx += (long long)nblk * BS) {
        const zd wv = wr[idx];
#pragma unroll
        for (int k = 0; k < CHUNK; ++k)
            if (k < ni) acc[k] = cfma_conj(V[(long long)(i0 + k) * vstride + (long long)rhs * N + idx], wv, acc[k]);
    }
    block_reduce<CHUNK>(acc, sh);
    // the sums sit in sh[k BS] for every thread (read from LDS: indexing the
    // register array by thread would put it in scratch memory)
    if (threadIdx.x < CHUNK)
        partial[((long long)rhs * nblk + blockIdx.x) * CHUNK + threadIdx.x] = sh[threadIdx.x * BS];
}

__global__ __launch_bounds__(64) void reduce_kernel(const zd* __restrict__ partial, int nblk,
                                                  int ni, const int* __restrict__ act,
                                                  zd* __restrict__ out, int out_stride) {
    __shared__ zd sh[CHUNK][64];
    const int rhs = act ? act[blockIdx.x] : (int)blockIdx.x;
    const int t = threadIdx.x;
    zd acc[CHUNK];
    for (int k = 0; k < CHUNK; ++k) acc[k] = mk(0.0, 0.0);
    for (int b = t; b < nblk; b += 64)
        for (int k = 0; k < CHUNK; ++k)
            acc[k] = acc[k] + partial[((long long)rhs * nblk + b) * CHUNK + k];
    for (int k = 0; k < CHUNK; ++k) sh[k][t] = acc[k];
    __syncthreads();
    for (int s = 32; s > 0; s >>= 1) {
        if (t < s)
            for (int k = 0; k < CHUNK; ++k) sh[k][t] = sh[k][t] + sh[k][t + s];
        __syncthreads();
    }
    if (t < ni) out[(long long)rhs * out_stride + t] = sh[t][0];
}

__global__ __launch_bounds__(BS) void axpy_multi_kernel(const zd* __restrict__ V, long long vstride,
                                                      int i0, int ni, const zd* __restrict__ coef,
                                                      int coef_stride, zd* __restrict__ w,
                                                      long long N, const int* __restrict__ act,
                                                      zd* __restrict__ norm_partial) {
    __shared__ zd sh[BS];
    const int rhs = act ? act[blockIdx.y] : (int)blockIdx.y;
    const int nblk = gridDim.x;
    zd cf[CHUNK];
    for (int k = 0; k < CHUNK; ++k)
        cf[k] = (k < ni) ? coef[(long long)rhs * coef_stride + i0 + k] : mk(0.0, 0.0);
    zd* wr = w + (long long)rhs * N;
    double nrm = 0.0;
    // a zero coefficient skips its vector (it may be unset, even NaN): every
    // vector is loaded (index clamped to a valid one) and the skip is a select,
    // so that the CHUNK loads of an element are in flight together instead of
    // each waiting under its own branch
    bool use[CHUNK];
    const zd* vp[CHUNK];
#pragma unroll
    for (int k = 0; k < CHUNK; ++k) {
        use[k] = k < ni && (cf[k].x != 0.0 || cf[k].y != 0.0);
        vp[k] = V + (long long)(i0 + (k < ni ? k : 0)) * vstride + (long long)rhs * N;
    }
    for (long long idx = (long long)blockIdx.x * BS + threadIdx.x; idx < N;
         idx += (long long)nblk * BS) {
        zd x[CHUNK];
#pragma unroll
        for (int k = 0; k < CHUNK; ++k) x[k] = vp[k][idx];
        zd v = wr[idx];
#pragma unroll
        for (int k = 0; k < CHUNK; ++k) v = csel(use[k], v - cf[k] * x[k], v);
        wr[idx] = v;
        nrm += abs2(v);
    }
    if (norm_partial) {
        zd r[1] = {mk(nrm, 0.0)};
        block_reduce<1>(r, sh);
        if (threadIdx.x == 0)
            norm_partial[((long long)rhs * nblk + blockIdx.x) * CHUNK] = r[0];
    }
}

// ----------------------------------------------------------------------------
// Fused classical Gram-Schmidt passes over the basis v_0 .. v_{nv-1} (nv <=
// CGS_MAXV), one right-hand side per grid row:
//   CGS_DOT:         p_k = sum conj(v_k) w
//   CGS_UPD_DOT_NRM: w -= sum_k c_k v_k, then p_k = sum conj(v_k) w and
//                    p_nv = |w|^2   (one read of V)
// Each thread walks its elements with a fixed stride; the per-block sums are
// reduced through a fixed butterfly inside each wavefront and a fixed order
// across the four wavefronts, so results do not depend on the other
// right-hand sides.
// ----------------------------------------------------------------------------
constexpr int CGS_DOT = 0, CGS_UPD_DOT_NRM = 1;

template <int NV, int MODE>
__global__ __launch_bounds__(BS) void cgs_kernel(const zd* __restrict__ V, long long vstride,
                                                const zd* __restrict__ coef, int coef_stride,
                                                zd* __restrict__ w, long long N,
                                                const int* __restrict__ act,
                                                zd* __restrict__ partial) {
    constexpr int NO = (MODE == CGS_UPD_DOT_NRM) ? NV + 1 : NV;   // sums per block
    static_assert(NO <= CGS_SLOTS, "partial sums per block");
    __shared__ zd red[BS / 64][NO];
    const int rhs = act ? act[blockIdx.y] : (int)blockIdx.y;
    const int nblk = gridDim.x;
    const zd* vr = V + (long long)rhs * N;
    zd* wr = w + (long long)rhs * N;
    zd cf[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k)
        cf[k] = (MODE == CGS_DOT) ? mk(0.0, 0.0) : coef[(long long)rhs * coef_stride + k];
    zd acc[NO];
#pragma unroll
    for (int k = 0; k < NO; ++k) acc[k] = mk(0.0, 0.0);
    for (long long idx = (long long)blockIdx.x * BS + threadIdx.x; idx < N;
         idx += (long long)nblk * BS) {
        zd x = wr[idx];
        zd vv[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) vv[k] = vr[(long long)k * vstride + idx];
        if (MODE != CGS_DOT) {
#pragma unroll
            for (int k = 0; k < NV; ++k) x = x - cf[k] * vv[k];
            wr[idx] = x;
        }
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] = cfma_conj(vv[k], x, acc[k]);
        if constexpr (MODE == CGS_UPD_DOT_NRM) acc[NV].x += abs2(x);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            acc[k].x += __shfl_xor(acc[k].x, o);
            acc[k].y += __shfl_xor(acc[k].y, o);
        }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < NO; ++k) red[wv][k] = acc[k];
    __syncthreads();
    if (threadIdx.x < NO) {
        zd t = red[0][threadIdx.x];
#pragma unroll
        for (int q = 1; q < BS / 64; ++q) t = t + red[q][threadIdx.x];
        partial[((long long)rhs * nblk + blockIdx.x) * CGS_SLOTS + threadIdx.x] = t;
    }
}

// out[rhs][k] = sum over blocks of partial[rhs][b][k], k < nv, in block order
__global__ __launch_bounds__(64) void cgs_reduce_kernel(const zd* __restrict__ partial, int nblk,
                                                      int nv, const int* __restrict__ act,
                                                      zd* __restrict__ out, int out_stride) {
    __shared__ zd sh[CGS_SLOTS][65];
    const int rhs = act ? act[blockIdx.x] : (int)blockIdx.x;
    const int t = threadIdx.x;
    for (int k = 0; k < nv; ++k) {
        zd a = mk(0.0, 0.0);
        for (int b = t; b < nblk; b += 64) a = a + partial[((long long)rhs * nblk + b) * CGS_SLOTS + k];
        sh[k][t] = a;
    }
    __syncthreads();
    if (t < nv) {
        zd a = sh[t][0];
        for (int q = 1; q < 64; ++q) a = a + sh[t][q];
        out[(long long)rhs * out_stride + t] = a;
    }
}

// The second Gram-Schmidt pass from the Gram matrix of the basis.  For the
// basis V = [v_0 .. v_j] with G = V^H V, the second pass's coefficients
// V^H (w - V h1) equal h1 - G h1; with unit vectors that is -E h1, E the
// off-diagonal part of G, whose entries are dot products of stored basis
// vectors (small, computed directly, so no cancellation).  The second pass
// then needs no read of V: w -= V (h1 + h2) in one pass, whose dots with V
// give the next column of E.  Per right-hand side: column j of E (upper
// triangle, E[i][j] = conj(v_i) . v_j) from the previous pass's dots d and the
// scale 1/beta that made v_j = w / beta; then h2 = -E h1 and c = h1 + h2.
// One workgroup per right-hand side, every sum in a fixed order.
__global__ __launch_bounds__(64) void gram_kernel(zd* __restrict__ small, int small_stride, int off_h1,
                                                 int off_h2, int off_coef, int off_d,
                                                 const zd* __restrict__ scal, zd* __restrict__ E,
                                                 int j, const int* __restrict__ act) {
    const int rhs = act ? act[blockIdx.x] : (int)blockIdx.x;
    zd* sm = small + (long long)rhs * small_stride;
    zd* Er = E + (long long)rhs * CGS_MAXV * CGS_MAXV;
    const int t = threadIdx.x;
    if (j >= 1 && t < j) Er[t * CGS_MAXV + j] = scal[rhs].x * sm[off_d + t];
    __syncthreads();
    if (t <= j) {
        zd acc = mk(0.0, 0.0);
        for (int k = 0; k <= j; ++k) {
            if (k == t) continue;
            // E[t][k] for k > t; the Hermitian mirror conj(E[k][t]) below
            acc = k > t ? cfma(Er[t * CGS_MAXV + k], sm[off_h1 + k], acc)
                        : cfma_conj(Er[k * CGS_MAXV + t], sm[off_h1 + k], acc);
        }
        const zd h2 = mk(-acc.x, -acc.y);
        sm[off_h2 + t] = h2;
        sm[off_coef + t] = sm[off_h1 + t] + h2;
    }
}

__global__ void scale_vec_kernel(const zd* __restrict__ w, zd* __restrict__ v,
                                 const zd* __restrict__ scal, long long N,
                                 const int* __restrict__ act) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N) return;
    const int rhs = act ? act[blockIdx.y] : (int)blockIdx.y;
    const long long o = (long long)rhs * N + idx;
    v[o] = w[o] * scal[rhs];
}

// out = b - out (out holds A x), partial sums of |out|^2
__global__ __launch_bounds__(BS) void residual_kernel(const zd* __restrict__ b, zd* __restrict__ out,
                                                    long long N, const int* __restrict__ act,
                                                    zd* __restrict__ norm_partial) {
    __shared__ zd sh[BS];
    const int rhs = act ? act[blockIdx.y] : (int)blockIdx.y;
    const int nblk = gridDim.x;
    double nrm = 0.0;
    for (long long idx = (long long)blockIdx.x * BS + threadIdx.x; idx < N;
         idx += (long long)nblk * BS) {
        const long long o = (long long)rhs * N + idx;
        const zd v = b[o] - out[o];
        out[o] = v;
        nrm += abs2(v);
    }
    zd r[1] = {mk(nrm, 0.0)};
    block_reduce<1>(r, sh);
    if (threadIdx.x == 0) norm_partial[((long long)rhs * nblk + blockIdx.x) * CHUNK] = r[0];
}

// partial sums of |v|^2 (the layout of residual_kernel's)
__global__ __launch_bounds__(BS) void norm_kernel(const zd* __restrict__ v, long long N,
                                                const int* __restrict__ act,
                                                zd* __restrict__ norm_partial) {
    __shared__ zd sh[BS];
    const int rhs = act ? act[blockIdx.y] : (int)blockIdx.y;
    const int nblk = gridDim.x;
    const zd* vr = v + (long long)rhs * N;
    double nrm = 0.0;
    for (long long idx = (long long)blockIdx.x * BS + threadIdx.x; idx < N;
         idx += (long long)nblk * BS)
        nrm += abs2(vr[idx]);
    zd r[1] = {mk(nrm, 0.0)};
    block_reduce<1>(r, sh);
    if (threadIdx.x == 0) norm_partial[((long long)rhs * nblk + blockIdx.x) * CHUNK] = r[0];
}

AxisTables axis_of(const asp_plan* P) {
    return AxisTables{P->d_axis, P->d_axis + (P->n + 1), P->d_axis + (2 * P->n + 1)};
}

}  // namespace

int krylov_blocks(long long N) {
    long long b = (N + BS * 4 - 1) / (BS * 4);
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

hipError_t launch_stencil(const asp_plan* P, const zd* x, zd* y, const int* act, int nact,
                          hipStream_t st) {
    if (nact <= 0) return hipSuccess;
    const int n = P->n;
    if (P->dim == 2) {
        dim3 grid((n + BS - 1) / BS, (n + SEG2 - 1) / SEG2, nact);
        hipLaunchKernelGGL(stencil2d_kernel, grid, dim3(BS), 0, st, x, y, act, axis_of(P), P->d_ksq,
                           n, P->N);
    } else {
        dim3 grid((n + BS - 1) / BS, n, (unsigned)n * nact);
        hipLaunchKernelGGL(stencil3d_kernel, grid, dim3(BS), 0, st, x, y, act, axis_of(P), P->d_ksq,
                           n, P->N, n);
    }
    return hipGetLastError();
}

hipError_t launch_residual(const asp_plan* P, const zd* b, const zd* x, zd* out, const int* act,
                           int nact, zd* red, int* nblk_out, hipStream_t st) {
    hipError_t e = launch_stencil(P, x, out, act, nact, st);
    if (e != hipSuccess) return e;
    const int nblk = krylov_blocks(P->N);
    *nblk_out = nblk;
    hipLaunchKernelGGL(residual_kernel, dim3(nblk, nact), dim3(BS), 0, st, b, out, P->N, act, red);
    return hipGetLastError();
}

hipError_t launch_scale_by_s(const asp_plan* P, const zd* f, zd* b, int nrhs, hipStream_t st) {
    dim3 grid((unsigned)((P->N + 255) / 256), nrhs);
    hipLaunchKernelGGL(scale_by_s_kernel, grid, dim3(256), 0, st, f, b, axis_of(P), P->n, P->dim,
                       P->N);
    return hipGetLastError();
}

hipError_t launch_norms(const zd* v, long long N, const int* act, int nact, zd* partial,
                        hipStream_t st) {
    hipLaunchKernelGGL(norm_kernel, dim3(krylov_blocks(N), nact), dim3(BS), 0, st, v, N, act, partial);
    return hipGetLastError();
}

hipError_t launch_multidot(const zd* V, long long vstride, int i0, int i1, const zd* w,
                           long long N, const int* act, int nact, zd* partial, hipStream_t st) {
    if (i1 - i0 > CHUNK || i1 <= i0) return hipErrorInvalidValue;   // one chunk per call
    const int nblk = krylov_blocks(N);
    hipLaunchKernelGGL(multidot_kernel, dim3(nblk, nact), dim3(BS), 0, st, V, vstride, i0,
                       i1 - i0, w, N, act, partial);
    return hipGetLastError();
}

hipError_t launch_reduce(const zd* partial, int nblk, int ni, const int* act, int nact, zd* out,
                         int out_stride, hipStream_t st) {
    hipLaunchKernelGGL(reduce_kernel, dim3(nact), dim3(64), 0, st, partial, nblk, ni, act, out,
                       out_stride);
    return hipGetLastError();
}

hipError_t launch_axpy_multi(const zd* V, long long vstride, int i0, int i1, const zd* coef,
                             int coef_stride, zd* w, long long N, const int* act, int nact,
                             zd* norm_partial, hipStream_t st) {
    if (i1 - i0 > CHUNK || i1 < i0) return hipErrorInvalidValue;
    const int nblk = krylov_blocks(N);
    hipLaunchKernelGGL(axpy_multi_kernel, dim3(nblk, nact), dim3(BS), 0, st, V, vstride, i0,
                       i1 - i0, coef, coef_stride, w, N, act, norm_partial);
    return hipGetLastError();
}

int cgs_blocks(long long N) {
    long long b = (N + BS * 16 - 1) / (BS * 16);
    if (b < 1) b = 1;
    if (b > 256) b = 256;
    return (int)b;
}

template <int MODE>
static hipError_t launch_cgs_mode(int nv, const zd* V, long long vstride, const zd* coef,
                                  int coef_stride, zd* w, long long N, const int* act, int nact,
                                  zd* partial, hipStream_t st) {
    dim3 grid(cgs_blocks(N), nact);
    switch (nv) {
#define ASP_CGS_CASE(K)                                                                        \
    case K:                                                                                    \
        hipLaunchKernelGGL((cgs_kernel<K, MODE>), grid, dim3(BS), 0, st, V, vstride, coef,     \
                           coef_stride, w, N, act, partial);                                   \
        break;
        ASP_CGS_CASE(1) ASP_CGS_CASE(2) ASP_CGS_CASE(3) ASP_CGS_CASE(4) ASP_CGS_CASE(5)
        ASP_CGS_CASE(6) ASP_CGS_CASE(7) ASP_CGS_CASE(8) ASP_CGS_CASE(9) ASP_CGS_CASE(10)
        ASP_CGS_CASE(11) ASP_CGS_CASE(12) ASP_CGS_CASE(13) ASP_CGS_CASE(14) ASP_CGS_CASE(15)
        ASP_CGS_CASE(16) ASP_CGS_CASE(17) ASP_CGS_CASE(18) ASP_CGS_CASE(19) ASP_CGS_CASE(20)
        ASP_CGS_CASE(21) ASP_CGS_CASE(22) ASP_CGS_CASE(23) ASP_CGS_CASE(24)
#undef ASP_CGS_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cgs(int mode, int nv, const zd* V, long long vstride, const zd* coef,
                      int coef_stride, zd* w, long long N, const int* act, int nact, zd* partial,
                      hipStream_t st) {
    static_assert(CGS_MAXV == 24, "one kernel instance per basis size");
    if (nv < 1 || nv > CGS_MAXV) return hipErrorInvalidValue;
    if (mode == CGS_DOT)
        return launch_cgs_mode<CGS_DOT>(nv, V, vstride, coef, coef_stride, w, N, act, nact,
                                        partial, st);
    return launch_cgs_mode<CGS_UPD_DOT_NRM>(nv, V, vstride, coef, coef_stride, w, N, act, nact,
                                            partial, st);
}

hipError_t launch_cgs_reduce(const zd* partial, int nblk, int nv, const int* act, int nact,
                             zd* out, int out_stride, hipStream_t st) {
    if (nv < 1 || nv > CGS_SLOTS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(cgs_reduce_kernel, dim3(nact), dim3(64), 0, st, partial, nblk, nv, act,
                       out, out_stride);
    return hipGetLastError();
}

hipError_t launch_gram(zd* small, int small_stride, int off_h1, int off_h2, int off_coef, int off_d,
                       const zd* scal, zd* E, int j, const int* act, int nact, hipStream_t st) {
    if (j < 0 || j >= CGS_MAXV) return hipErrorInvalidValue;
    hipLaunchKernelGGL(gram_kernel, dim3(nact), dim3(64), 0, st, small, small_stride, off_h1, off_h2,
                       off_coef, off_d, scal, E, j, act);
    return hipGetLastError();
}

hipError_t launch_scale_vec(const zd* w, zd* v, const zd* scal, long long N, const int* act,
                            int nact, hipStream_t st) {
    dim3 grid((unsigned)((N + 255) / 256), nact);
    hipLaunchKernelGGL(scale_vec_kernel, grid, dim3(256), 0, st, w, v, scal, N, act);
    return hipGetLastError();
}
