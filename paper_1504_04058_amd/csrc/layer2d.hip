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
#include "mfma.h"

namespace {

constexpr int WAVE = 64;
constexpr int MAXL = 32;

// ----------------------------------------------------------------------------
// factorization: one wavefront per auxiliary problem.  Lane (j, h) holds rows
// 16h .. 16h+15 of column j of the current block in registers; S_k is formed
// from S_{k-1}^-1 in place and inverted by Gauss-Jordan elimination without
// pivoting (at a few points per wavelength the blocks are close to diagonally
// dominant; a zero or non-finite pivot is reported as a breakdown).  The pivot
// row and column pass through LDS, double-buffered: one wave barrier per
// pivot.  Arithmetic in double; the stored factor is rounded to TS.
// ----------------------------------------------------------------------------
template <typename TS>
__global__ __launch_bounds__(WAVE) void factor2d_kernel(const SubDesc* __restrict__ desc,
                                                      AxisTables ax,
                                                      const zd* __restrict__ subtab,
                                                      const double* __restrict__ ksq, int n,
                                                      cplx<TS>* __restrict__ fac,
                                                      int* __restrict__ flag) {
    __shared__ zd rowbuf[2][MAXL];
    __shared__ zd colbuf[2][MAXL];

    const SubDesc d = desc[blockIdx.x];
    const int L = d.L;
    const int lane = threadIdx.x;
    const int j = lane & 31, h = lane >> 5;
    const bool cj = j < L;
    const zd* tab = subtab + d.tab_off;
    const zd* ssh = tab;                // s at half lines lo-1/2 .. hi+1/2
    const zd* sinv2 = tab + L + 1;      // 1/(s h^2) on lines lo..hi
    const zd* sinv = tab + 2 * L + 1;   // 1/s on lines lo..hi
    const int LR = d.LR;
    const zd sj = cj ? sinv2[j] : mk(0.0, 0.0);
    bool bad = false;
    zd v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = mk(0.0, 0.0);

    for (int k = 1; k <= n; ++k) {
        const zd sh_m = ax.sh[k - 1];   // s1 at k - 1/2
        const zd sh_p = ax.sh[k];       // s1 at k + 1/2
        const zd is2k = ax.inv_sh2[k - 1];
        const zd isk = ax.inv_s[k - 1];
        // S_k = D_k - E_{k-1} S_{k-1}^-1 E_{k-1} over S_{k-1}^-1; identity padding
        const zd ej = sh_m * sj;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int i = 16 * h + q;
            zd val = mk(0.0, 0.0);
            if (i < L && cj) {
                if (k > 1) val = -((sh_m * sinv2[i]) * v[q] * ej);
                if (i == j) {
                    const zd lap1 = (sh_p + sh_m) * sinv2[i];
                    const zd lap2 = (ssh[i + 1] + ssh[i]) * is2k;
                    const zd mass =
                        (ksq[(long long)(k - 1) + (long long)n * (d.lo + i - 1)] * isk) * sinv[i];
                    val = val + mass - lap1 - lap2;
                } else if (j == i + 1) {
                    val = val + ssh[i + 1] * is2k;
                } else if (j == i - 1) {
                    val = val + ssh[i] * is2k;
                }
            } else if (i == j) {
                val = mk(1.0, 0.0);
            }
            v[q] = val;
        }
        // in-place inverse
        for (int kk = 0; kk < L; ++kk) {
            const int b = kk & 1;
            if (h == (kk >> 4)) {
                // select by value: a pointer into v would move it to scratch memory
                zd pr = v[0];
#pragma unroll
                for (int q = 1; q < 16; ++q) {
                    const bool hit = q == (kk & 15);
                    pr.x = hit ? v[q].x : pr.x;
                    pr.y = hit ? v[q].y : pr.y;
                }
                rowbuf[b][j] = pr;
            }
            if (j == kk)
#pragma unroll
                for (int q = 0; q < 16; ++q) colbuf[b][16 * h + q] = v[q];
            __syncthreads();
            const zd p = colbuf[b][kk];
            const double pa = abs2(p);
            if (!(pa > 1e-300) || !isfinite(pa)) bad = true;
            const zd pinv = cinv(p);
            const zd rp = rowbuf[b][j] * pinv;            // A[kk][j] / p
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int i = 16 * h + q;
                const zd ci = colbuf[b][i];                // A[i][kk]
                zd x = v[q] - ci * rp;
                if (i == kk) x = rp;
                if (j == kk) x = (i == kk) ? pinv : -(ci * pinv);
                v[q] = x;
            }
        }
        // store S_k^-1 column-major with leading dimension LR (rows past L zero)
        if (cj) {
            cplx<TS>* out = fac + d.fac_off + (long long)(k - 1) * L * LR + (long long)j * LR;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int i = 16 * h + q;
                if (i < LR) out[i] = ccast<TS>(i < L ? v[q] : mk(0.0, 0.0));
            }
        }
    }
    if (bad) *flag = 1;
}

// ----------------------------------------------------------------------------
// batched solves: one 1024-thread workgroup per (auxiliary problem, chunk of
// 1024 / LR right-hand sides); thread (row, rhs) owns one row of one
// right-hand side.  The L x L block S_k^-1 of each step is loaded once into an
// LDS ring (the load of block k+1 overlaps step k) and shared by all
// right-hand sides of the chunk; each thread forms its step input, writes it
// to LDS and, after the barrier, computes its row of the block product.
// ----------------------------------------------------------------------------
struct SolveArgs {
    const SubDesc* desc;
    const int* jobs;
    int njobs;
    const int* act;      // right-hand-side ids (NULL: 0..nact-1)
    int nact;
    int in_mode, out_mode;
    int out_mode_L;      // L problems of a launch with both kinds: their own output
    zd* out_L;
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
    long long y_per_wave;   // scratch entries per workgroup
    int n;
    long long N;
};

constexpr int SB = 1024;       // threads per solve workgroup (16 wavefronts)

template <typename T, int LR>
__global__ __launch_bounds__(SB) void solve2d_kernel(SolveArgs a) {
    constexpr int RG = 1, RPT = 1;          // one row of one right-hand side per thread
    constexpr int NRG = LR / RG;            // row groups
    constexpr int SRB = SB / NRG;           // right-hand sides per workgroup
    constexpr int FMAX = 32 * LR;           // largest block (L <= 32)
    constexpr int FPT = (FMAX + SB - 1) / SB;
    __shared__ cplx<T> Fs[2][FMAX];
    __shared__ cplx<T> tb[2][SRB][LR];

    // XCD-aware order: the chunks of one problem are consecutive work items
    const int nchunk = (a.nact + SRB - 1) / SRB;
    const int B = a.njobs * nchunk;
    const int per = (B + 7) / 8;
    const int w = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (w >= B) return;
    const int jl = w / nchunk, ch = w % nchunk;
    const SubDesc d = a.desc[a.jobs[jl]];
    const int L = d.L, n = a.n;
    const long long N = a.N;
    const int tid = threadIdx.x;
    const int rgi = tid % NRG, cgi = tid / NRG;
    const int i0 = rgi * RG;
    const cplx<T>* F = reinterpret_cast<const cplx<T>*>(a.fac) + d.fac_off;
    const int FS = L * LR;                  // entries of one block
    const zd* tab = a.subtab + d.tab_off;
    cplx<T>* Y = reinterpret_cast<cplx<T>*>(a.y) + (long long)w * a.y_per_wave;

    int slot[RPT];
    bool valid[RPT];
    long long base[RPT];
    int rid[RPT];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int r = cgi * RPT + j;
        slot[j] = ch * SRB + r;
        valid[j] = slot[j] < a.nact;
        rid[j] = valid[j] ? (a.act ? a.act[slot[j]] : slot[j]) : 0;
        base[j] = (a.in_mode == IN_BOUNDARY) ? ((long long)d.wrow * a.w_rhs + rid[j]) * n
                                             : (long long)rid[j] * N;
    }
    bool rowv[RG];
    bool in_X[RG];
    int line[RG];
    int lclamp[RG];   // line clamped to the grid, for unconditional loads
    cplx<T> sinv2[RG];
#pragma unroll
    for (int q = 0; q < RG; ++q) {
        const int i = i0 + q;
        rowv[q] = i < L;
        line[q] = d.lo + i;
        lclamp[q] = min(line[q], n);
        in_X[q] = rowv[q] && line[q] >= d.xs && line[q] <= d.xe;
        sinv2[q] = rowv[q] ? ccast<T>(tab[L + 1 + i]) : mk<T>(0, 0);
    }
    const int grow = (d.kind == ASP_SUB_R) ? 0 : L - 1;          // row carrying boundary data
    const zd coupl = (d.kind == ASP_SUB_R) ? tab[0] : tab[L];    // s at lo-1/2 or hi+1/2

    // rows past L are read against zero factor entries but never written, and
    // the factor columns past L are read against zero vectors: clear both once
    for (int e = tid; e < 2 * SRB * LR; e += SB) (&tb[0][0][0])[e] = mk<T>(0, 0);
    for (int e = tid; e < 2 * FMAX; e += SB) (&Fs[0][0])[e] = mk<T>(0, 0);
    __syncthreads();   // the first stash writes entries another thread cleared
    const int LP = (L + 3) & ~3;
    cplx<T> pf[FPT];
    // loads below are unconditional (from clamped, always valid addresses) and
    // their values selected where used: a load under a divergent branch makes
    // the compiler wait for every earlier load at the branch join
    auto fetch = [&](int blk) {
        const cplx<T>* Fk = F + (long long)blk * FS;
#pragma unroll
        for (int u = 0; u < FPT; ++u) pf[u] = Fk[min(tid + u * SB, FS - 1)];
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int u = 0; u < FPT; ++u) {
            const int e = tid + u * SB;
            if (e < FS) Fs[buf][e] = pf[u];
        }
    };
    // block product of rows i0.. for the chunk's vectors in tb[buf] with Fs[fb]
    auto product = [&](int fb, int buf, cplx<T> (&acc)[RG][RPT]) {
#pragma unroll
        for (int q = 0; q < RG; ++q)
#pragma unroll
            for (int j = 0; j < RPT; ++j) acc[q][j] = mk<T>(0, 0);
        // columns L..LP-1 of the ring and of tb are zero, so the loop runs to a
        // multiple of 4 and unrolls
#pragma unroll 4
        for (int c = 0; c < LP; ++c) {
            cplx<T> f[RG], t[RPT];
#pragma unroll
            for (int q = 0; q < RG; ++q) f[q] = Fs[fb][c * LR + i0 + q];
#pragma unroll
            for (int j = 0; j < RPT; ++j) t[j] = tb[buf][cgi * RPT + j][c];
#pragma unroll
            for (int q = 0; q < RG; ++q)
#pragma unroll
                for (int j = 0; j < RPT; ++j) acc[q][j] = cfma(f[q], t[j], acc[q][j]);
        }
    };

    // raw data entering step k (complex128), for rows i0.. and the chunk's
    // right-hand sides: read one step ahead, before the factor block, so that
    // waiting for it never waits for the block
    // one source pointer per (row, rhs): grid data (IN_GRID), boundary data
    // (IN_BOUNDARY, the same for every row) or a dummy valid address (IN_UNIT);
    // stride 1 along i1, 0 for the dummy
    const zd* inp[RG][RPT];
    const int ink = (a.in_mode == IN_UNIT) ? 0 : 1;
#pragma unroll
    for (int q = 0; q < RG; ++q)
#pragma unroll
        for (int j = 0; j < RPT; ++j)
            inp[q][j] = (a.in_mode == IN_GRID)       ? a.r + base[j] + (long long)n * (lclamp[q] - 1)
                        : (a.in_mode == IN_BOUNDARY) ? a.W + base[j]
                                                     : a.subtab;
    auto load_in = [&](int k, zd (&gv)[RG][RPT]) {
#pragma unroll
        for (int q = 0; q < RG; ++q)
#pragma unroll
            for (int j = 0; j < RPT; ++j) gv[q][j] = inp[q][j][(long long)(k - 1) * ink];
    };

    // unit data enters at i1 = slot + 1 >= ch SRB + 1: the forward results of
    // the blocks before the chunk's first column are zero, so the forward pass
    // starts there and the backward pass reads no results before it
    const int kstart = (a.in_mode == IN_UNIT) ? min(ch * SRB + 1, n) : 1;
    zd gin[RG][RPT];
    load_in(kstart, gin);
    zd shv = a.ax.sh[kstart - 1], isv = a.ax.inv_sh2[kstart - 1];
    fetch(kstart - 1);
    stash(kstart & 1);
    __syncthreads();

    // forward sweep: y_k = S_k^-1 (g_k - E_{k-1} y_{k-1}); block k sits in ring slot k & 1
    cplx<T> yk[RG][RPT];
#pragma unroll
    for (int q = 0; q < RG; ++q)
#pragma unroll
        for (int j = 0; j < RPT; ++j) yk[q][j] = mk<T>(0, 0);
    for (int k = kstart; k <= n; ++k) {
        const int buf = k & 1;
        zd gnx[RG][RPT];
        zd shn = shv, isn = isv;
        if (k < n) {
            load_in(k + 1, gnx);
            shn = a.ax.sh[k];
            isn = a.ax.inv_sh2[k];
            fetch(k);
        }
        const cplx<T> shm = ccast<T>(shv);
        const zd cin = -(coupl * isv);
#pragma unroll
        for (int q = 0; q < RG; ++q) {
            if (!rowv[q]) continue;
            const int i = i0 + q;
            const cplx<T> e = shm * sinv2[q];                       // E_{k-1}, row i
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                cplx<T> g = mk<T>(0, 0);
                if (a.in_mode == IN_GRID)
                    g = in_X[q] ? ccast<T>(gin[q][j]) : mk<T>(0, 0);
                else if (i == grow && a.in_mode == IN_BOUNDARY)
                    g = ccast<T>(gin[q][j] * cin);
                else if (i == grow && slot[j] == k - 1)     // IN_UNIT: unit data at i1 = slot + 1
                    g = ccast<T>(cin);
                if (k > 1) g = g - e * yk[q][j];
                tb[buf][cgi * RPT + j][i] = g;
            }
        }
        __syncthreads();
        product(buf, buf, yk);
#pragma unroll
        for (int q = 0; q < RG; ++q)
#pragma unroll
            for (int j = 0; j < RPT; ++j)
                if (rowv[q]) Y[((long long)(k - 1) * SRB + cgi * RPT + j) * LR + i0 + q] = yk[q][j];
        if (k < n) {
            stash((k + 1) & 1);
#pragma unroll
            for (int q = 0; q < RG; ++q)
#pragma unroll
                for (int j = 0; j < RPT; ++j) gin[q][j] = gnx[q][j];
            shv = shn;
            isv = isn;
        }
    }

    // backward sweep: v_n = y_n, v_k = y_k - S_k^-1 E_k v_{k+1}.  Block n-1 is
    // still in slot (n-1) & 1; block k-1 is loaded during step k.  The y_k and
    // the values the outputs add to are read one step ahead as well.
    const int jout = (d.kind == ASP_SUB_R) ? (d.xe - d.lo) : (d.xs - d.lo);   // OUT_LINE row
    const int omode = (d.kind == ASP_SUB_L) ? a.out_mode_L : a.out_mode;
    zd* const outp = (d.kind == ASP_SUB_L) ? a.out_L : a.out;
    const bool set_u = (omode == OUT_GRID_ADD_U) ||
                       (omode == OUT_GRID_ACC && d.kind == ASP_SUB_L && d.p == 1);
    const bool add_out = !set_u && omode == OUT_GRID_ACC;
    const bool grid_out = omode != OUT_LINE;
    const bool use_add = set_u || add_out;
    const zd* addp[RG][RPT];
#pragma unroll
    for (int q = 0; q < RG; ++q)
#pragma unroll
        for (int j = 0; j < RPT; ++j)
            addp[q][j] = use_add ? (set_u ? a.Ugrid : outp) + (long long)rid[j] * N +
                                       (long long)n * (lclamp[q] - 1)
                                 : a.subtab;
    const int addk = use_add ? 1 : 0;
    auto load_add = [&](int k, zd (&av)[RG][RPT]) {
#pragma unroll
        for (int q = 0; q < RG; ++q)
#pragma unroll
            for (int j = 0; j < RPT; ++j) av[q][j] = addp[q][j][(long long)(k - 1) * addk];
    };
    auto load_y = [&](int k, cplx<T> (&yv)[RG][RPT]) {
        const long long kk = max(k, kstart);     // blocks before kstart: y = 0
#pragma unroll
        for (int q = 0; q < RG; ++q)
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const cplx<T> yv0 = Y[((kk - 1) * SRB + cgi * RPT + j) * LR + i0 + q];
                yv[q][j] = (k >= kstart) ? yv0 : mk<T>(0, 0);
            }
    };
    auto emit = [&](int k, const cplx<T> (&v)[RG][RPT], const zd (&av)[RG][RPT]) {
#pragma unroll
        for (int q = 0; q < RG; ++q) {
            if (!rowv[q]) continue;
            const int i = i0 + q;
            if (!grid_out) {
                if (i != jout) continue;
                cplx<T>* Tp = reinterpret_cast<cplx<T>*>(a.Tout) + d.tr_off;
#pragma unroll
                for (int j = 0; j < RPT; ++j)
                    if (valid[j]) Tp[(long long)slot[j] * n + (k - 1)] = v[q][j];
                continue;
            }
            if (!in_X[q]) continue;
            const long long off = (k - 1) + (long long)n * (line[q] - 1);
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                if (!valid[j]) continue;
                outp[(long long)rid[j] * N + off] =
                    use_add ? ccast<double>(v[q][j]) + av[q][j] : ccast<double>(v[q][j]);
            }
        }
    };
    zd acur[RG][RPT];
    load_add(n, acur);
    emit(n, yk, acur);
    cplx<T> (&vk)[RG][RPT] = yk;
    cplx<T> ycur[RG][RPT];
    if (n >= 2) {
        load_y(n - 1, ycur);
        load_add(n - 1, acur);
    }
    shv = a.ax.sh[n - 1];
    for (int k = n - 1; k >= 1; --k) {
        const int buf = k & 1;
        cplx<T> ynx[RG][RPT];
        zd anx[RG][RPT];
        zd shn = shv;
        if (k > 1) {
            load_y(k - 1, ynx);
            load_add(k - 1, anx);
            shn = a.ax.sh[k - 1];
            fetch(k - 2);
        }
        const cplx<T> shp = ccast<T>(shv);
#pragma unroll
        for (int q = 0; q < RG; ++q) {
            const cplx<T> e = shp * sinv2[q];                       // E_k, row i
#pragma unroll
            for (int j = 0; j < RPT; ++j)
                if (rowv[q]) tb[buf][cgi * RPT + j][i0 + q] = e * vk[q][j];
        }
        __syncthreads();
        cplx<T> acc[RG][RPT];
        product(buf, buf, acc);
#pragma unroll
        for (int q = 0; q < RG; ++q)
#pragma unroll
            for (int j = 0; j < RPT; ++j) vk[q][j] = ycur[q][j] - acc[q][j];
        emit(k, vk, acur);
        if (k > 1) {
            stash((k - 1) & 1);
#pragma unroll
            for (int q = 0; q < RG; ++q)
#pragma unroll
                for (int j = 0; j < RPT; ++j) {
                    ycur[q][j] = ynx[q][j];
                    acur[q][j] = anx[q][j];
                }
            shv = shn;
        }
    }
}

// ----------------------------------------------------------------------------
// one step of the two boundary-value sweeps of Algorithm 2, with the
// boundary-to-boundary maps T (column c holds the outgoing line produced by
// unit data at i1 = c + 1):
//   right-going: W^R_{p+1} = T^R_p W^R_p + u~_{p,p} on the last line of X_p
//   left-going:  W^L_{p-1} = T^L_p W^L_p + u~_{p,p} on the first line of X_p
// ----------------------------------------------------------------------------
struct SweepArgs {
    const void* T;
    long long t_off[2];      // map of the problem stepped from (R, L)
    const void* Wt_in[2];    // W transposed: [i1][slot], row stride ws, type of the maps
    void* Wt_out[2];
    zd* W;                   // W rows [rhs][i1] (complex128) of the problems stepped into
    long long w_out[2];
    int line[2];             // line of u~_{p,p} added (last of X_p / first of X_p)
    const zd* Ugrid;
    const int* act;
    int nact;
    int ws;                  // padded slot count (multiple of SW_RT)
    int n;
    long long N;
};

constexpr int SW_ROWS = 16;    // output rows (i1) per block: one matrix-core tile
constexpr int SW_RT = 32;      // right-hand sides per block: two tiles
constexpr int SW_W = 8;        // wavefronts per block, splitting the columns of T

// W_out = T W_in for 16 outputs i1 and 32 right-hand sides: a complex product
// on the matrix cores.  Each wavefront takes a contiguous eighth of the
// columns of T, four k-steps of operands in flight at a time; the partial
// tiles meet in LDS and are added in wavefront order (fixed, so a result does
// not depend on the other right-hand sides or on scheduling).  The two blocks
// of a row tile are 64 block ids apart and so share an XCD and its L2 copy of T.
template <typename T>
__global__ __launch_bounds__(64 * SW_W) void sweep_step_kernel(SweepArgs a) {
    __shared__ cplx<T> red[SW_W][2][64][4];
    const int side = blockIdx.z;
    const int n = a.n;
    const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = l & 15, lk = l >> 4;
    const int k0 = blockIdx.x * SW_ROWS;
    const int s0 = blockIdx.y * SW_RT;
    if (s0 >= a.nact) return;
    const cplx<T>* __restrict__ Tm = reinterpret_cast<const cplx<T>*>(a.T) + a.t_off[side];
    const cplx<T>* __restrict__ Wi = reinterpret_cast<const cplx<T>*>(a.Wt_in[side]);
    const int ws = a.ws;
    const int kr = min(k0 + li, n - 1);               // rows past n repeat the last (not stored)
    const int per = (n + 16 * SW_W - 1) / (16 * SW_W) * 16;
    const int cb = wv * per;
    CTile<T> acc[2];
    acc[0].zero();
    acc[1].zero();
    // operands of 4 k-steps (16 columns); the next batch is loaded before the
    // current batch's products
    struct Batch {
        cplx<T> av[4], bv[4][2];
    };
    auto load = [&](Batch& B, int c0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + 4 * u + lk;
            const int cc = min(c, n - 1);
            B.av[u] = Tm[(long long)cc * n + kr];
#pragma unroll
            for (int t2 = 0; t2 < 2; ++t2) B.bv[u][t2] = Wi[(long long)cc * ws + s0 + 16 * t2 + li];
            if (c >= n) B.av[u] = mk<T>(T(0), T(0));
        }
    };
    Batch cur, nxt;
    load(cur, cb);
    for (int c0 = cb; c0 < cb + per; c0 += 16) {
        if (c0 + 16 < cb + per) load(nxt, c0 + 16);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t2 = 0; t2 < 2; ++t2) cmac(acc[t2], cur.av[u], cur.bv[u][t2]);
        cur = nxt;
    }
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wv][t2][l][v] = mk<T>(acc[t2].re[v], acc[t2].im[v]);
    __syncthreads();
    // one output per thread: tile t2, lane l2, element v
    const int tid = threadIdx.x;
    const int v = tid & 3, l2 = (tid >> 2) & 63, t2 = tid >> 8;
    const int ko = k0 + Mfma<T>::row(l2, v);
    const int slot = s0 + 16 * t2 + (l2 & 15);
    if (ko >= n || slot >= a.nact) return;
    cplx<T> sum = red[0][t2][l2][v];
#pragma unroll
    for (int q = 1; q < SW_W; ++q) sum = sum + red[q][t2][l2][v];
    const int id = a.act ? a.act[slot] : slot;
    const zd val = ccast<double>(sum) +
                   a.Ugrid[(long long)id * a.N + (long long)n * (a.line[side] - 1) + ko];
    a.W[a.w_out[side] + (long long)id * n + ko] = val;
    reinterpret_cast<cplx<T>*>(a.Wt_out[side])[(long long)ko * ws + slot] = ccast<T>(val);
}

// W rows of the first sweep step: u~_{1,1} on the last line of X_1 (right-going)
// and u~_{m,m} on the first line of X_m (left-going), plus their transposed copies
// (padding slots zero)
template <typename T>
__global__ void sweep_seed_kernel(const zd* __restrict__ Ugrid, zd* __restrict__ W,
                                  long long outR, long long outL, int lineR, int lineL,
                                  cplx<T>* __restrict__ WtR, cplx<T>* __restrict__ WtL,
                                  const int* __restrict__ act, int nact, int ws, int n,
                                  long long N) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int slot = blockIdx.y;
    if (slot >= nact) {
        WtR[(long long)k * ws + slot] = mk<T>(0, 0);
        WtL[(long long)k * ws + slot] = mk<T>(0, 0);
        return;
    }
    const int id = act ? act[slot] : slot;
    const long long u = (long long)id * N + k;
    const zd vR = Ugrid[u + (long long)n * (lineR - 1)];
    const zd vL = Ugrid[u + (long long)n * (lineL - 1)];
    W[outR + (long long)id * n + k] = vR;
    W[outL + (long long)id * n + k] = vL;
    WtR[(long long)k * ws + slot] = ccast<T>(vR);
    WtL[(long long)k * ws + slot] = ccast<T>(vL);
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

template <int LR>
static hipError_t launch_solve_lr(const asp_plan* P, const SolveArgs& a, int blocks, hipStream_t st) {
    if (P->prec == ASP_PREC_FP32)
        hipLaunchKernelGGL((solve2d_kernel<float, LR>), dim3(blocks), dim3(SB), 0, st, a);
    else
        hipLaunchKernelGGL((solve2d_kernel<double, LR>), dim3(blocks), dim3(SB), 0, st, a);
    return hipGetLastError();
}

int solve_rhs_per_block(int LR) { return SB / LR; }

long long solve_scratch_per_block(const asp_plan* P) { return (long long)P->n * SB; }

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
    a.out_mode_L = L.out_L ? L.out_mode_L : L.out_mode;
    a.out_L = L.out_L ? L.out_L : L.out;
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
    a.y_per_wave = solve_scratch_per_block(P);
    a.n = P->n;
    a.N = P->N;
    const int LR = L.rl ? P->LR_RL : P->LR_M;   // every job of one launch shares its row count
    const int srb = solve_rhs_per_block(LR);
    const long long B = (long long)L.njobs * ((L.nact + srb - 1) / srb);
    if (B > P->y_waves) return hipErrorInvalidValue;   // scratch too small
    const int blocks = (int)(((B + 7) / 8) * 8);
    if (LR == 16) return launch_solve_lr<16>(P, a, blocks, st);
    return launch_solve_lr<32>(P, a, blocks, st);
}

static int sweep_slots(int nact) { return (nact + SW_RT - 1) / SW_RT * SW_RT; }

int sweep_wt_len(const asp_plan* P, int nrhs) { return 4 * P->n * sweep_slots(nrhs); }

// transposed sweep buffers: [side][ping-pong][n][ws]
static void* wt_buf(const asp_plan* P, int side, int pp, int ws) {
    const size_t esz = P->prec == ASP_PREC_FP32 ? sizeof(zf) : sizeof(zd);
    return static_cast<char*>(P->d_wt) + ((size_t)(side * 2 + pp) * P->n * ws) * esz;
}

hipError_t launch_sweep_seed(const asp_plan* P, zd* W, long long outR, long long outL,
                             const int* act, int nact, hipStream_t st) {
    if (nact <= 0) return hipSuccess;
    const int lineR = P->X[0][1];
    const int lineL = P->X[P->m - 1][0];
    const int ws = sweep_slots(nact);
    if ((long long)4 * P->n * ws > P->wt_elems) return hipErrorInvalidValue;
    dim3 grid((P->n + 255) / 256, ws);
    if (P->prec == ASP_PREC_FP32)
        hipLaunchKernelGGL(sweep_seed_kernel<float>, grid, dim3(256), 0, st, P->d_U, W, outR, outL,
                           lineR, lineL, (zf*)wt_buf(P, 0, 0, ws), (zf*)wt_buf(P, 1, 0, ws), act,
                           nact, ws, P->n, P->N);
    else
        hipLaunchKernelGGL(sweep_seed_kernel<double>, grid, dim3(256), 0, st, P->d_U, W, outR, outL,
                           lineR, lineL, (zd*)wt_buf(P, 0, 0, ws), (zd*)wt_buf(P, 1, 0, ws), act,
                           nact, ws, P->n, P->N);
    return hipGetLastError();
}

hipError_t launch_sweep_step(const asp_plan* P, int t, zd* W, int w_rhs, const int* act, int nact,
                             hipStream_t st) {
    // step t moves the right-going sweep from layer p = t+1 to p+1 and the
    // left-going sweep from layer p' = m-t to p'-1; the transposed inputs of
    // step t are ping-pong buffer (t-1) & 1
    const int m = P->m;
    const int pR = t + 1, pL = m - t;
    const int ws = sweep_slots(nact);
    if ((long long)4 * P->n * ws > P->wt_elems) return hipErrorInvalidValue;
    SweepArgs a;
    a.T = P->d_T;
    a.t_off[0] = P->subs[P->idx_R(pR)].tr_off;
    a.t_off[1] = P->subs[P->idx_L(pL)].tr_off;
    for (int side = 0; side < 2; ++side) {
        a.Wt_in[side] = wt_buf(P, side, (t - 1) & 1, ws);
        a.Wt_out[side] = wt_buf(P, side, t & 1, ws);
    }
    a.W = W;
    a.w_out[0] = (long long)P->wrow(P->idx_R(pR + 1)) * w_rhs * P->n;
    a.w_out[1] = (long long)P->wrow(P->idx_L(pL - 1)) * w_rhs * P->n;
    a.line[0] = P->X[pR - 1][1];
    a.line[1] = P->X[pL - 1][0];
    a.Ugrid = P->d_U;
    a.act = act;
    a.nact = nact;
    a.ws = ws;
    a.n = P->n;
    a.N = P->N;
    dim3 grid((P->n + SW_ROWS - 1) / SW_ROWS, ws / SW_RT, 2);
    if (P->prec == ASP_PREC_FP32)
        hipLaunchKernelGGL(sweep_step_kernel<float>, grid, dim3(64 * SW_W), 0, st, a);
    else
        hipLaunchKernelGGL(sweep_step_kernel<double>, grid, dim3(64 * SW_W), 0, st, a);
    return hipGetLastError();
}
