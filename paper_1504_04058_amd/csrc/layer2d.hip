// 2D auxiliary problems H^M_q, H^R_p, H^L_p (Section 3.1): factorization
// (Algorithm 1), batched solves (the G~ operators of Algorithm 2) and the
// dense boundary-to-boundary maps used by the sweeps.
//
// Each 2D auxiliary problem lives on the n x L grid (i1 = 1..n, L sweep lines).
// Grouping the unknowns with the sweep axis fastest (Section 3.1: the quasi-1D
// subproblems reordered into a banded system) makes H block tridiagonal in i1
// with L x L blocks:
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
// batched solves: one wavefront per (auxiliary problem, group of RW
// right-hand sides).  Lane l = Q*i + q owns row i of the L x L block products
// and the column group q (columns q, q+Q, ...); a step is a row-split
// matrix-vector product for each of the RW right-hand sides followed by a
// reduction over the Q lanes of a row.  The vectors entering each step go
// through LDS, stored per column group so each lane reads them contiguously.
// ----------------------------------------------------------------------------
struct SolveArgs {
    const SubDesc* desc;
    const int* jobs;
    int njobs;
    const int* act;      // right-hand-side ids (NULL: 0..nact-1)
    int nact;
    int in_mode, out_mode;
    const void* fac;
    AxisTables ax;
    const zd* subtab;
    const zd* r;         // IN_GRID: grid vectors
    const zd* W;         // IN_BOUNDARY: boundary data per (problem, rhs)
    int w_rhs;           // right-hand-side stride of W (in n-vectors)
    zd* out;             // OUT_GRID_*: grid vectors
    const zd* Ugrid;     // OUT_GRID_ADD_U / ACC: u~_{p,p}
    void* Tout;          // OUT_LINE: boundary-to-boundary maps
    void* y;
    long long y_per_wave;
    int n;
    long long N;
};

template <typename T>
__device__ __forceinline__ cplx<T> shfl_xor_c(cplx<T> v, int m) {
    return mk<T>(__shfl_xor(v.x, m), __shfl_xor(v.y, m));
}

template <typename T, int Q, int RW>
__global__ __launch_bounds__(WAVE) void solve2d_kernel(SolveArgs a) {
    constexpr int R = WAVE / Q;
    constexpr int UMAX = R / Q;
    __shared__ cplx<T> tb[2][RW][Q][UMAX];

    // XCD-aware order: consecutive work items (the right-hand-side groups of one
    // problem) land on the same XCD so that they share its L2 copy of the factor.
    const int ngroups = (a.nact + RW - 1) / RW;
    const int B = a.njobs * ngroups;
    const int per = (B + 7) / 8;
    const int w = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (w >= B) return;
    const int jl = w / ngroups, grp = w % ngroups;
    const SubDesc d = a.desc[a.jobs[jl]];
    const int L = d.L, U = d.U, n = a.n;
    const long long N = a.N;
    const int lane = threadIdx.x, i = lane / Q, q = lane % Q;
    const bool rowlane = (q == 0) && (i < L);
    const cplx<T>* F = reinterpret_cast<const cplx<T>*>(a.fac) + d.fac_off;
    const zd* tab = a.subtab + d.tab_off;
    const cplx<T> sinv2_i = (i < L) ? ccast<T>(tab[L + 1 + i]) : mk<T>(0, 0);
    cplx<T>* Y = reinterpret_cast<cplx<T>*>(a.y) + (long long)w * a.y_per_wave;

    int slot[RW];
    bool valid[RW];
    long long base[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        slot[r] = grp * RW + r;
        valid[r] = slot[r] < a.nact;
        const int id = valid[r] ? (a.act ? a.act[slot[r]] : slot[r]) : 0;
        base[r] = (long long)id * N;
        if (a.in_mode == IN_BOUNDARY)   // W row of this problem and rhs
            base[r] = ((long long)d.wrow * a.w_rhs + id) * n;
    }
    // slots of tb past row L are read (against zero factor entries) but never
    // written: clear them once so that no stale LDS value can reach the sums
    for (int e = lane; e < 2 * RW * Q * UMAX; e += WAVE) (&tb[0][0][0][0])[e] = mk<T>(0, 0);
    __syncthreads();
    const int grow = (d.kind == ASP_SUB_R) ? 0 : L - 1;          // row carrying boundary data
    const zd coupl = (d.kind == ASP_SUB_R) ? tab[0] : tab[L];    // s at lo-1/2 or hi+1/2
    const int line_i = d.lo + i;
    const bool in_X = (line_i >= d.xs) && (line_i <= d.xe);
    const int tq = i % Q, tu = i / Q;   // where row i's entry sits in tb

    cplx<T> A[UMAX], An[UMAX];
#pragma unroll
    for (int u = 0; u < UMAX; ++u)
        A[u] = (u < U) ? F[u * WAVE + lane] : mk<T>(0, 0);

    // forward sweep
    cplx<T> yk[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) yk[r] = mk<T>(0, 0);
    for (int k = 1; k <= n; ++k) {
        const int buf = k & 1;
        if (k < n) {
            const cplx<T>* Fk = F + (long long)k * WAVE * U;
#pragma unroll
            for (int u = 0; u < UMAX; ++u)
                An[u] = (u < U) ? Fk[u * WAVE + lane] : mk<T>(0, 0);
        }
        if (rowlane) {
            const cplx<T> e = ccast<T>(a.ax.sh[k - 1]) * sinv2_i;    // E_{k-1}, row i
            zd cin = mk(0.0, 0.0);
            if (a.in_mode != IN_GRID && i == grow) cin = -(coupl * a.ax.inv_sh2[k - 1]);
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                cplx<T> g = mk<T>(0, 0);
                if (a.in_mode == IN_GRID) {
                    if (in_X) g = ccast<T>(a.r[base[r] + (k - 1) + (long long)n * (line_i - 1)]);
                } else if (i == grow) {
                    if (a.in_mode == IN_BOUNDARY)
                        g = ccast<T>(a.W[base[r] + (k - 1)] * cin);
                    else if (slot[r] == k - 1)   // IN_UNIT: unit data at i1 = slot + 1
                        g = ccast<T>(cin);
                }
                if (k > 1) g = g - e * yk[r];
                tb[buf][r][tq][tu] = g;
            }
        }
        __syncthreads();
        cplx<T> acc[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            acc[r] = mk<T>(0, 0);
#pragma unroll
            for (int u = 0; u < UMAX; ++u)
                if (u < U) acc[r] = cfma(A[u], tb[buf][r][q][u], acc[r]);
            if (Q >= 2) acc[r] = acc[r] + shfl_xor_c(acc[r], 1);
            if (Q >= 4) acc[r] = acc[r] + shfl_xor_c(acc[r], 2);
            yk[r] = acc[r];
        }
        if (rowlane) {
            cplx<T>* Yk = Y + ((long long)(k - 1) * L + i) * RW;
#pragma unroll
            for (int r = 0; r < RW; ++r) Yk[r] = yk[r];
        }
#pragma unroll
        for (int u = 0; u < UMAX; ++u) A[u] = An[u];
    }

    // backward sweep; v_n = y_n
    const int jout = (d.kind == ASP_SUB_R) ? (d.xe - d.lo) : (d.xs - d.lo);   // OUT_LINE row
    auto emit = [&](int k, const cplx<T>* v) {
        if (!rowlane) return;
        if (a.out_mode == OUT_LINE) {
            if (i != jout) return;
            cplx<T>* Tp = reinterpret_cast<cplx<T>*>(a.Tout) + d.tr_off;
#pragma unroll
            for (int r = 0; r < RW; ++r)
                if (valid[r]) Tp[(long long)slot[r] * n + (k - 1)] = v[r];
            return;
        }
        if (!in_X) return;
        const long long off = (k - 1) + (long long)n * (line_i - 1);
        const bool set_u = (a.out_mode == OUT_GRID_ADD_U) ||
                           (a.out_mode == OUT_GRID_ACC && d.kind == ASP_SUB_L && d.p == 1);
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            if (!valid[r]) continue;
            const long long o = (long long)(a.act ? a.act[slot[r]] : slot[r]) * N + off;
            zd val = ccast<double>(v[r]);
            if (set_u) val = val + a.Ugrid[o];
            else if (a.out_mode == OUT_GRID_ACC) val = val + a.out[o];
            a.out[o] = val;
        }
    };
    cplx<T> vk[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) vk[r] = yk[r];
    emit(n, vk);
    if (n >= 2) {
        const cplx<T>* Fk = F + (long long)(n - 2) * WAVE * U;
#pragma unroll
        for (int u = 0; u < UMAX; ++u)
            A[u] = (u < U) ? Fk[u * WAVE + lane] : mk<T>(0, 0);
    }
    for (int k = n - 1; k >= 1; --k) {
        const int buf = k & 1;
        if (k > 1) {
            const cplx<T>* Fk = F + (long long)(k - 2) * WAVE * U;
#pragma unroll
            for (int u = 0; u < UMAX; ++u)
                An[u] = (u < U) ? Fk[u * WAVE + lane] : mk<T>(0, 0);
        }
        cplx<T> ykk[RW];
        if (rowlane) {
            const cplx<T> e = ccast<T>(a.ax.sh[k]) * sinv2_i;        // E_k, row i
            const cplx<T>* Yk = Y + ((long long)(k - 1) * L + i) * RW;
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                ykk[r] = Yk[r];
                tb[buf][r][tq][tu] = e * vk[r];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            cplx<T> acc = mk<T>(0, 0);
#pragma unroll
            for (int u = 0; u < UMAX; ++u)
                if (u < U) acc = cfma(A[u], tb[buf][r][q][u], acc);
            if (Q >= 2) acc = acc + shfl_xor_c(acc, 1);
            if (Q >= 4) acc = acc + shfl_xor_c(acc, 2);
            vk[r] = rowlane ? ykk[r] - acc : acc;
        }
        emit(k, vk);
#pragma unroll
        for (int u = 0; u < UMAX; ++u) A[u] = An[u];
    }
}

// ----------------------------------------------------------------------------
// one step of the two boundary-value sweeps of Algorithm 2, with the
// boundary-to-boundary maps T (column c holds the outgoing line produced by
// unit data at i1 = c + 1):
//   right-going: W^R_{p+1} = T^R_p W^R_p + u~_{p,p} on the last line of X_p
//   left-going:  W^L_{p-1} = T^L_p W^L_p + u~_{p,p} on the first line of X_p
// blockIdx.z selects the sweep; a block computes 64 outputs i1 for a group of
// right-hand sides, reading W in chunks of 64 columns through LDS.
// ----------------------------------------------------------------------------
struct SweepArgs {
    const void* T;
    long long t_off[2];      // map of the problem stepped from (R, L)
    const zd* W;
    long long w_in[2];       // offsets (in n-vectors * w_rhs) of the input rows
    zd* Wout;
    long long w_out[2];
    int line[2];             // line of u~_{p,p} added (last of X_p / first of X_p)
    const zd* Ugrid;
    const int* act;
    int nact;
    int w_rhs;
    int n;
    long long N;
};

constexpr int SW_ROWS = 64;
constexpr int SW_RG = 4;       // right-hand-side lanes per block
constexpr int SW_RPT = 2;      // right-hand sides per thread
constexpr int SW_KC = 64;      // columns per LDS chunk

template <typename T>
__global__ __launch_bounds__(256) void sweep_step_kernel(SweepArgs a) {
    __shared__ cplx<T> Ws[SW_KC][SW_RG * SW_RPT];
    const int side = blockIdx.z;
    const int n = a.n;
    const int tid = threadIdx.x;
    const int k = blockIdx.x * SW_ROWS + (tid % SW_ROWS);
    const int rg = tid / SW_ROWS;
    const int r0 = blockIdx.y * SW_RG * SW_RPT;
    const cplx<T>* Tm = reinterpret_cast<const cplx<T>*>(a.T) + a.t_off[side];
    const zd* Win = a.W + a.w_in[side];
    cplx<T> acc[SW_RPT];
#pragma unroll
    for (int j = 0; j < SW_RPT; ++j) acc[j] = mk<T>(0, 0);
    for (int c0 = 0; c0 < n; c0 += SW_KC) {
        __syncthreads();
        for (int e = tid; e < SW_KC * SW_RG * SW_RPT; e += 256) {
            const int cc = e % SW_KC, rr = e / SW_KC;
            const int slot = r0 + rr;
            cplx<T> v = mk<T>(0, 0);
            if (c0 + cc < n && slot < a.nact) {
                const int id = a.act ? a.act[slot] : slot;
                v = ccast<T>(Win[(long long)id * n + c0 + cc]);
            }
            Ws[cc][rr] = v;
        }
        __syncthreads();
        if (k < n) {
            const int cmax = (n - c0 < SW_KC) ? n - c0 : SW_KC;
            for (int cc = 0; cc < cmax; ++cc) {
                const cplx<T> t = Tm[(long long)(c0 + cc) * n + k];
#pragma unroll
                for (int j = 0; j < SW_RPT; ++j) acc[j] = cfma(t, Ws[cc][rg * SW_RPT + j], acc[j]);
            }
        }
    }
    if (k >= n) return;
#pragma unroll
    for (int j = 0; j < SW_RPT; ++j) {
        const int slot = r0 + rg * SW_RPT + j;
        if (slot >= a.nact) continue;
        const int id = a.act ? a.act[slot] : slot;
        const zd u = a.Ugrid[(long long)id * a.N + (long long)n * (a.line[side] - 1) + k];
        a.Wout[a.w_out[side] + (long long)id * n + k] = ccast<double>(acc[j]) + u;
    }
}

// W rows of the first sweep step: u~_{1,1} on the last line of X_1 (right-going)
// and u~_{m,m} on the first line of X_m (left-going)
__global__ void sweep_seed_kernel(const zd* __restrict__ Ugrid, zd* __restrict__ W,
                                  long long outR, long long outL, int lineR, int lineL,
                                  const int* __restrict__ act, int n, long long N) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int id = act ? act[blockIdx.y] : (int)blockIdx.y;
    const long long u = (long long)id * N + k;
    W[outR + (long long)id * n + k] = Ugrid[u + (long long)n * (lineR - 1)];
    W[outL + (long long)id * n + k] = Ugrid[u + (long long)n * (lineL - 1)];
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

template <int Q, int RW>
static hipError_t launch_solve_q(const asp_plan* P, const SolveArgs& a, int blocks, hipStream_t st) {
    if (P->prec == ASP_PREC_FP32)
        hipLaunchKernelGGL((solve2d_kernel<float, Q, RW>), dim3(blocks), dim3(WAVE), 0, st, a);
    else
        hipLaunchKernelGGL((solve2d_kernel<double, Q, RW>), dim3(blocks), dim3(WAVE), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_solve2d(const asp_plan* P, const SolveLaunch& L, hipStream_t st) {
    if (L.njobs <= 0 || L.nact <= 0) return hipSuccess;
    SolveArgs a;
    a.desc = P->d_desc;
    a.jobs = P->d_jobs + L.job0;
    a.njobs = L.njobs;
    a.act = L.act;
    a.nact = L.nact;
    a.in_mode = L.in_mode;
    a.out_mode = L.out_mode;
    a.fac = P->d_fac;
    a.ax = AxisTables{P->d_axis, P->d_axis + (P->n + 1), P->d_axis + (2 * P->n + 1)};
    a.subtab = P->d_subtab;
    a.r = L.r;
    a.W = L.W;
    a.w_rhs = L.w_rhs;
    a.out = L.out;
    a.Ugrid = L.Ugrid;
    a.Tout = P->d_T;
    a.y = P->d_y;
    a.y_per_wave = P->y_per_wave;
    a.n = P->n;
    a.N = P->N;
    const int ngroups = (L.nact + SOLVE_RW - 1) / SOLVE_RW;
    const long long B = (long long)L.njobs * ngroups;
    if (B * a.y_per_wave > P->y_waves * P->y_per_wave) return hipErrorInvalidValue;   // scratch too small
    const int blocks = (int)(((B + 7) / 8) * 8);
    const int Q = L.rl ? P->Q_RL : P->Q_M;   // every job of one launch shares its Q
    if (Q == 4) return launch_solve_q<4, SOLVE_RW>(P, a, blocks, st);
    return launch_solve_q<2, SOLVE_RW>(P, a, blocks, st);
}

hipError_t launch_sweep_seed(const asp_plan* P, zd* W, long long outR, long long outL,
                             const int* act, int nact, hipStream_t st) {
    if (nact <= 0) return hipSuccess;
    const int lineR = P->X[0][1];
    const int lineL = P->X[P->m - 1][0];
    dim3 grid((P->n + 255) / 256, nact);
    hipLaunchKernelGGL(sweep_seed_kernel, grid, dim3(256), 0, st, P->d_U, W, outR, outL, lineR,
                       lineL, act, P->n, P->N);
    return hipGetLastError();
}

hipError_t launch_sweep_step(const asp_plan* P, int t, zd* W, int w_rhs, const int* act, int nact,
                             hipStream_t st) {
    // step t moves the right-going sweep from layer p = t+1 to p+1 and the
    // left-going sweep from layer p' = m-t to p'-1
    const int m = P->m;
    const int pR = t + 1, pL = m - t;
    SweepArgs a;
    a.T = P->d_T;
    a.t_off[0] = P->subs[P->idx_R(pR)].tr_off;
    a.t_off[1] = P->subs[P->idx_L(pL)].tr_off;
    a.W = W;
    a.Wout = W;
    a.w_in[0] = (long long)P->wrow(P->idx_R(pR)) * w_rhs * P->n;
    a.w_in[1] = (long long)P->wrow(P->idx_L(pL)) * w_rhs * P->n;
    a.w_out[0] = (long long)P->wrow(P->idx_R(pR + 1)) * w_rhs * P->n;
    a.w_out[1] = (long long)P->wrow(P->idx_L(pL - 1)) * w_rhs * P->n;
    a.line[0] = P->X[pR - 1][1];
    a.line[1] = P->X[pL - 1][0];
    a.Ugrid = P->d_U;
    a.act = act;
    a.nact = nact;
    a.w_rhs = w_rhs;
    a.n = P->n;
    a.N = P->N;
    dim3 grid((P->n + SW_ROWS - 1) / SW_ROWS, (nact + SW_RG * SW_RPT - 1) / (SW_RG * SW_RPT), 2);
    if (P->prec == ASP_PREC_FP32)
        hipLaunchKernelGGL(sweep_step_kernel<float>, grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(sweep_step_kernel<double>, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}
