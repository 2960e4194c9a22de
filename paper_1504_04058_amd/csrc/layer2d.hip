// 2D auxiliary problems H^M_q, H^R_p, H^L_p (Section 3.1): factorization
// (Algorithm 1) and batched solves (the G~ operators used by Algorithm 2).
//
// Each 2D auxiliary problem lives on the n x L grid (i1 = 1..n, L sweep lines).
// Grouping the unknowns with the sweep axis fastest (Section 3.1: "grouping the
// elements along dimension 2 first and then dimension 1") makes H block
// tridiagonal in i1 with L x L blocks:
//   D_k      tridiagonal: the sweep-axis couplings s(lo+j+1/2)/(s1(k) h^2) and the diagonal,
//   E_k      diagonal coupling of block k to k+1: s1(k+1/2) / (s(lo+j) h^2),
// in the symmetric form.  The block recurrence S_1 = D_1,
// S_k = D_k - E_{k-1} S_{k-1}^-1 E_{k-1} is the banded LU of the paper in block
// form; the factor keeps S_k^-1 for every k.  A solve is the forward sweep
// y_k = S_k^-1 (g_k - E_{k-1} y_{k-1}) and the backward sweep
// v_k = y_k - S_k^-1 E_k v_{k+1}.
#include "asp_internal.h"

namespace {

constexpr int WAVE = 64;
constexpr int MAXL = 32;

// ----------------------------------------------------------------------------
// factorization: one wavefront per auxiliary problem, the current L x L block
// in LDS; S_k is inverted in place by Gauss-Jordan elimination with partial
// pivoting inside the block.  Arithmetic in double; the stored factor is
// rounded to TS.
// ----------------------------------------------------------------------------
template <typename TS>
__global__ __launch_bounds__(WAVE) void factor2d_kernel(const SubDesc* __restrict__ desc,
                                                      AxisTables ax,
                                                      const zd* __restrict__ subtab,
                                                      const double* __restrict__ ksq, int n,
                                                      cplx<TS>* __restrict__ fac,
                                                      int* __restrict__ flag) {
    __shared__ zd M[MAXL][MAXL + 1];
    __shared__ zd col[MAXL];
    __shared__ int piv[MAXL];

    const SubDesc d = desc[blockIdx.x];
    const int L = d.L;
    const int lane = threadIdx.x;
    const zd* tab = subtab + d.tab_off;
    const zd* ssh = tab;                // s at half lines lo-1/2 .. hi+1/2
    const zd* sinv2 = tab + L + 1;      // 1/(s h^2) on lines lo..hi
    const zd* sinv = tab + 2 * L + 1;   // 1/s on lines lo..hi
    const int Q = d.Q, U = d.U;
    bool bad = false;

    for (int k = 1; k <= n; ++k) {
        const zd sh_m = ax.sh[k - 1];   // s1 at k - 1/2
        const zd sh_p = ax.sh[k];       // s1 at k + 1/2
        const zd is2k = ax.inv_sh2[k - 1];
        const zd isk = ax.inv_s[k - 1];
        // S_k = D_k - E_{k-1} S_{k-1}^-1 E_{k-1}, in place over S_{k-1}^-1
        for (int e = lane; e < L * L; e += WAVE) {
            const int i = e / L, j = e % L;
            zd v = mk(0.0, 0.0);
            if (k > 1) {
                const zd ei = sh_m * sinv2[i];
                const zd ej = sh_m * sinv2[j];
                v = -(ei * M[i][j] * ej);
            }
            if (i == j) {
                const zd lap1 = (sh_p + sh_m) * sinv2[i];
                const zd lap2 = (ssh[i + 1] + ssh[i]) * is2k;
                const zd mass = (ksq[(long long)(k - 1) + (long long)n * (d.lo + i - 1)] * isk) * sinv[i];
                v = v + mass - lap1 - lap2;
            } else if (j == i + 1) {
                v = v + ssh[i + 1] * is2k;
            } else if (j == i - 1) {
                v = v + ssh[i] * is2k;
            }
            M[i][j] = v;
        }
        __syncthreads();
        // in-place inverse
        for (int kk = 0; kk < L; ++kk) {
            double a = -1.0;
            int ip = lane;
            if (lane >= kk && lane < L) a = abs2(M[lane][kk]);
            for (int off = 32; off > 0; off >>= 1) {
                const double ao = __shfl_xor(a, off);
                const int io = __shfl_xor(ip, off);
                if (ao > a || (ao == a && io < ip)) {
                    a = ao;
                    ip = io;
                }
            }
            if (lane == 0) piv[kk] = ip;
            if (ip != kk && lane < L) {
                const zd t = M[kk][lane];
                M[kk][lane] = M[ip][lane];
                M[ip][lane] = t;
            }
            __syncthreads();
            const zd pv = M[kk][kk];
            const double pa = abs2(pv);
            if (!(pa > 0.0) || !isfinite(pa)) bad = true;
            const zd inv = cinv(pv);
            if (lane < L) col[lane] = M[lane][kk];
            __syncthreads();
            if (lane < L) M[kk][lane] = (lane == kk) ? inv : M[kk][lane] * inv;
            __syncthreads();
            for (int e = lane; e < L * L; e += WAVE) {
                const int i = e / L, j = e % L;
                if (i == kk) continue;
                if (j == kk)
                    M[i][j] = -(col[i] * inv);
                else
                    M[i][j] = M[i][j] - col[i] * M[kk][j];
            }
            __syncthreads();
        }
        for (int kk = L - 1; kk >= 0; --kk) {
            const int p = piv[kk];
            if (p != kk && lane < L) {
                const zd t = M[lane][kk];
                M[lane][kk] = M[lane][p];
                M[lane][p] = t;
            }
            __syncthreads();
        }
        // store S_k^-1 in the solve layout
        cplx<TS>* out = fac + d.fac_off + (long long)(k - 1) * WAVE * U;
        const int i = lane / Q, q = lane % Q;
        for (int u = 0; u < U; ++u) {
            const int j = q + Q * u;
            const zd v = (i < L && j < L) ? M[i][j] : mk(0.0, 0.0);
            out[u * WAVE + lane] = ccast<TS>(v);
        }
        __syncthreads();
    }
    if (bad && lane == 0) *flag = 1;
}

// ----------------------------------------------------------------------------
// batched solves: one wavefront per (auxiliary problem, right-hand side).
// Lane l = Q*i + q owns row i of the L x L block products and the column group
// q; a step is a row-split matrix-vector product followed by a reduction over
// the Q lanes of a row.  The vector entering each step goes through LDS.
// ----------------------------------------------------------------------------
struct SolveArgs {
    const SubDesc* desc;
    const int* jobs;
    int njobs;
    const int* act;
    int nact;
    const void* fac;
    AxisTables ax;
    const zd* subtab;
    SolveIO io;
    void* y;
    long long y_per_wave;
    int n;
    long long N;
};

template <typename T>
__device__ __forceinline__ cplx<T> shfl_xor_c(cplx<T> v, int m) {
    return mk<T>(__shfl_xor(v.x, m), __shfl_xor(v.y, m));
}

template <typename T, int Q>
__global__ __launch_bounds__(WAVE) void solve2d_kernel(SolveArgs a) {
    constexpr int R = WAVE / Q;
    constexpr int UMAX = R / Q;
    __shared__ cplx<T> tb[2][MAXL];

    // XCD-aware order: consecutive work items (the right-hand sides of one
    // problem) land on the same XCD so that they share its L2 copy of the factor.
    const int B = a.njobs * a.nact;
    const int per = (B + 7) / 8;
    const int w = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (w >= B) return;
    const int jl = w / a.nact;
    const int rhs = a.act ? a.act[w % a.nact] : (w % a.nact);
    const SubDesc d = a.desc[a.jobs[jl]];
    const int L = d.L, U = d.U, n = a.n;
    const long long N = a.N;
    const int lane = threadIdx.x, i = lane / Q, q = lane % Q;
    const bool rowlane = (q == 0) && (i < L);
    const cplx<T>* F = reinterpret_cast<const cplx<T>*>(a.fac) + d.fac_off;
    const zd* tab = a.subtab + d.tab_off;
    const cplx<T> sinv2_i = (i < L) ? ccast<T>(tab[L + 1 + i]) : mk<T>(0, 0);
    cplx<T>* Y = reinterpret_cast<cplx<T>*>(a.y) + (long long)w * a.y_per_wave;
    const long long base = (long long)rhs * N;

    // right-hand side data
    const zd* src_r = a.io.r;
    const zd* b2 = (d.kind == ASP_SUB_R) ? a.io.bR : a.io.bL;
    const int grow = (d.kind == ASP_SUB_R) ? 0 : L - 1;         // row carrying the data
    const zd coupl = (d.kind == ASP_SUB_R) ? tab[0] : tab[L];   // s at lo-1/2 or hi+1/2
    const int line_i = d.lo + i;
    const bool in_X = (line_i >= d.xs) && (line_i <= d.xe);

    cplx<T> A[UMAX], An[UMAX];
#pragma unroll
    for (int u = 0; u < UMAX; ++u)
        A[u] = (u < U) ? F[u * WAVE + lane] : mk<T>(0, 0);

    // forward sweep
    cplx<T> yk = mk<T>(0, 0);
    for (int k = 1; k <= n; ++k) {
        if (k < n) {
            const cplx<T>* Fk = F + (long long)k * WAVE * U;
#pragma unroll
            for (int u = 0; u < UMAX; ++u)
                An[u] = (u < U) ? Fk[u * WAVE + lane] : mk<T>(0, 0);
        }
        if (rowlane) {
            cplx<T> g = mk<T>(0, 0);
            const long long off = base + (k - 1);
            if (d.kind == ASP_SUB_M) {
                if (in_X) g = ccast<T>(src_r[off + (long long)n * (line_i - 1)]);
            } else if (i == grow) {
                const long long o2 = off + (long long)n * (d.src_line - 1);
                zd wv = a.io.bU[o2];
                if (b2) wv = wv + b2[o2];
                g = ccast<T>(-(wv * (coupl * a.ax.inv_sh2[k - 1])));
            }
            if (k > 1) g = g - (ccast<T>(a.ax.sh[k - 1]) * sinv2_i) * yk;
            tb[k & 1][i] = g;
        }
        __syncthreads();
        cplx<T> acc = mk<T>(0, 0);
#pragma unroll
        for (int u = 0; u < UMAX; ++u) {
            const int j = q + Q * u;
            if (u < U && j < L) acc = cfma(A[u], tb[k & 1][j], acc);
        }
        if (Q >= 2) acc = acc + shfl_xor_c(acc, 1);
        if (Q >= 4) acc = acc + shfl_xor_c(acc, 2);
        yk = acc;
        if (rowlane) Y[(long long)(k - 1) * L + i] = yk;
#pragma unroll
        for (int u = 0; u < UMAX; ++u) A[u] = An[u];
    }

    // backward sweep; v_n = y_n
    zd* out = (d.kind == ASP_SUB_M) ? a.io.U : (d.kind == ASP_SUB_R ? a.io.AR : a.io.CL);
    cplx<T> vk = yk;
    if (rowlane && in_X) out[base + (n - 1) + (long long)n * (line_i - 1)] = ccast<double>(vk);
    {
        const cplx<T>* Fk = F + (long long)(n - 2) * WAVE * U;
        if (n >= 2) {
#pragma unroll
            for (int u = 0; u < UMAX; ++u)
                A[u] = (u < U) ? Fk[u * WAVE + lane] : mk<T>(0, 0);
        }
    }
    for (int k = n - 1; k >= 1; --k) {
        if (k > 1) {
            const cplx<T>* Fk = F + (long long)(k - 2) * WAVE * U;
#pragma unroll
            for (int u = 0; u < UMAX; ++u)
                An[u] = (u < U) ? Fk[u * WAVE + lane] : mk<T>(0, 0);
        }
        cplx<T> ykk = mk<T>(0, 0);
        if (rowlane) {
            ykk = Y[(long long)(k - 1) * L + i];
            tb[k & 1][i] = (ccast<T>(a.ax.sh[k]) * sinv2_i) * vk;
        }
        __syncthreads();
        cplx<T> acc = mk<T>(0, 0);
#pragma unroll
        for (int u = 0; u < UMAX; ++u) {
            const int j = q + Q * u;
            if (u < U && j < L) acc = cfma(A[u], tb[k & 1][j], acc);
        }
        if (Q >= 2) acc = acc + shfl_xor_c(acc, 1);
        if (Q >= 4) acc = acc + shfl_xor_c(acc, 2);
        vk = ykk - acc;
        if (rowlane && in_X) out[base + (k - 1) + (long long)n * (line_i - 1)] = ccast<double>(vk);
#pragma unroll
        for (int u = 0; u < UMAX; ++u) A[u] = An[u];
    }
}

__global__ void combine_kernel(const zd* __restrict__ U, const zd* __restrict__ AR,
                               const zd* __restrict__ CL, zd* __restrict__ z,
                               const int* __restrict__ act, long long N, long long S,
                               int line_R, int line_L) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N) return;
    const int rhs = act ? act[blockIdx.y] : (int)blockIdx.y;
    const long long o = (long long)rhs * N + idx;
    const long long line = idx / S + 1;
    zd v = U[o];
    if (AR && line >= line_R) v = v + AR[o];
    if (CL && line <= line_L) v = v + CL[o];
    z[o] = v;
}

}  // namespace

hipError_t launch_factor2d(const asp_plan* P, hipStream_t st) {
    const int nsub = (int)P->subs.size();
    AxisTables ax{P->d_axis, P->d_axis + (P->n + 1), P->d_axis + (2 * P->n + 1)};
    if (P->prec == ASP_PREC_FP32)
        hipLaunchKernelGGL(factor2d_kernel<float>, dim3(nsub), dim3(WAVE), 0, st, P->d_desc, ax,
                           P->d_subtab, P->d_ksq, P->n, reinterpret_cast<zf*>(P->d_fac),
                           P->d_flag);
    else
        hipLaunchKernelGGL(factor2d_kernel<double>, dim3(nsub), dim3(WAVE), 0, st, P->d_desc,
                           ax, P->d_subtab, P->d_ksq, P->n, reinterpret_cast<zd*>(P->d_fac),
                           P->d_flag);
    return hipGetLastError();
}

hipError_t launch_solve2d(const asp_plan* P, int job0, int njobs, bool rl, const int* act,
                          int nact, const SolveIO& io, hipStream_t st) {
    if (njobs <= 0 || nact <= 0) return hipSuccess;
    SolveArgs a;
    a.desc = P->d_desc;
    a.jobs = P->d_jobs + job0;
    a.njobs = njobs;
    a.act = act;
    a.nact = nact;
    a.fac = P->d_fac;
    a.ax = AxisTables{P->d_axis, P->d_axis + (P->n + 1), P->d_axis + (2 * P->n + 1)};
    a.subtab = P->d_subtab;
    a.io = io;
    a.y = P->d_y;
    a.y_per_wave = P->y_per_wave;
    a.n = P->n;
    a.N = P->N;
    // every job of one launch shares its Q (M jobs: Q_M; R/L jobs: Q_RL)
    const int Q = rl ? P->Q_RL : P->Q_M;
    const long long B = (long long)njobs * nact;
    const int blocks = (int)(((B + 7) / 8) * 8);
    const bool f32 = (P->prec == ASP_PREC_FP32);
    if (Q == 4) {
        if (f32)
            hipLaunchKernelGGL((solve2d_kernel<float, 4>), dim3(blocks), dim3(WAVE), 0, st, a);
        else
            hipLaunchKernelGGL((solve2d_kernel<double, 4>), dim3(blocks), dim3(WAVE), 0, st, a);
    } else {
        if (f32)
            hipLaunchKernelGGL((solve2d_kernel<float, 2>), dim3(blocks), dim3(WAVE), 0, st, a);
        else
            hipLaunchKernelGGL((solve2d_kernel<double, 2>), dim3(blocks), dim3(WAVE), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_combine(const asp_plan* P, const zd* U, const zd* AR, const zd* CL, zd* z,
                          const int* act, int nact, hipStream_t st) {
    if (nact <= 0) return hipSuccess;
    const int line_R = (P->m > 1) ? P->X[1][0] : P->n + 1;
    const int line_L = (P->m > 1) ? P->X[P->m - 2][1] : 0;
    const unsigned bx = 256;
    dim3 grid((unsigned)((P->N + bx - 1) / bx), (unsigned)nact);
    hipLaunchKernelGGL(combine_kernel, grid, dim3(bx), 0, st, U, P->m > 1 ? AR : nullptr,
                       P->m > 1 ? CL : nullptr, z, act, P->N, P->S, line_R, line_L);
    return hipGetLastError();
}
