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
#include <algorithm>

#include "asp_internal.h"
#include "mfma.h"

namespace {

constexpr int WAVE = 64;
constexpr int MAXL = 64;   // the most sweep lines of a 2D auxiliary problem
static_assert(WAVE * 16 <= SINK_ELEMS, "sixteen discard entries per lane");

// raw buffer stores: dword 3 of the resource (32-bit data format) and an
// offset past any range, whose writes the hardware drops
constexpr int BUF_DW3 = 0x00020000;
constexpr unsigned BUF_OOB = 0x80000000u;
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned off, zd v) {
    u32x4 d;
    __builtin_memcpy(&d, &v, sizeof(d));
    __builtin_amdgcn_raw_buffer_store_b128(d, r, off, 0, 0);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned off, zf v) {
    u32x2 d;
    __builtin_memcpy(&d, &v, sizeof(d));
    __builtin_amdgcn_raw_buffer_store_b64(d, r, off, 0, 0);
}

// ----------------------------------------------------------------------------
// factorization: one 256-thread workgroup per auxiliary problem.  With LR
// columns, thread (j, g) holds rows g RPL .. g RPL + RPL - 1 of column j of the
// current block in registers (LR = 64: 4 row groups of 16; LR = 32: 8 of 4;
// LR = 16: 16 of 1);
// S_k is formed from S_{k-1}^-1 in place and inverted by Gauss-Jordan
// elimination without pivoting (at a few points per wavelength the blocks are
// close to diagonally dominant; a zero or non-finite pivot is reported as a
// breakdown).  The pivot row and column pass through LDS, double-buffered by
// pivot parity: one barrier per pivot.  Arithmetic in double; the stored
// factor is rounded to TS.
// ----------------------------------------------------------------------------
constexpr int FB = 256;   // threads per factor workgroup

template <typename TS, int LR, int ML>
__device__ __forceinline__ void factor2d_body(const SubDesc& d, AxisTables ax,
                                              const zd* __restrict__ subtab,
                                              const double* __restrict__ ksq, int n,
                                              cplx<TS>* __restrict__ fac, int* __restrict__ flag,
                                              zd (&rowbuf)[2][ML + 1], zd (&colbuf)[2][ML],
                                              zd (&srow)[ML]) {
    constexpr int G = FB / LR, RPL = LR / G;
    const int L = d.L;
    const int t = threadIdx.x;
    const int j = t % LR, g = t / LR;
    const bool cj = j < L;
    const zd* tab = subtab + d.tab_off;
    const zd* ssh = tab;                // s at half lines lo-1/2 .. hi+1/2
    const zd* sinv2 = tab + L + 1;      // 1/(s h^2) on lines lo..hi
    const zd* sinv = tab + 2 * L + 1;   // 1/s on lines lo..hi
    const int jc = min(j, L - 1);
    // tables that do not change along axis 1: 1/(s h^2) per row (LDS, zero
    // past L) and, for this thread's column j, the couplings to rows j -+ 1
    if (g == 0) srow[j] = csel(cj, sinv2[jc], mk(0.0, 0.0));
    const zd sj = csel(cj, sinv2[jc], mk(0.0, 0.0));
    const zd c_lo = ssh[jc], c_hi = ssh[jc + 1], sinvj = sinv[jc];
    const double* ksq_j = ksq + (long long)n * (d.lo + jc - 1);
    // S_k^-1 column-major with leading dimension LR through a buffer resource:
    // columns past L give an offset past the range (dropped writes)
    const __amdgpu_buffer_rsrc_t rf =
        __builtin_amdgcn_make_buffer_rsrc(fac + d.fac_off, 0, 0x7fffffff, BUF_DW3);
    const unsigned foff = cj ? (unsigned)((j * LR + g * RPL) * sizeof(cplx<TS>)) : BUF_OOB;
    const unsigned fstep = (unsigned)(L * LR * sizeof(cplx<TS>));
    bool bad = false;
    zd v[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) v[q] = mk(0.0, 0.0);

    // the tables of block k (couplings s1 at k -+ 1/2, 1/(s1 h^2), 1/s1 and
    // omega^2/c^2 on this thread's diagonal point), fetched one block ahead
    struct Step {
        zd sh_m, sh_p, is2, is;
        double kq;
    };
    auto fetch = [&](Step& S, int k) {
        S.sh_m = ax.sh[k - 1];
        S.sh_p = ax.sh[k];
        S.is2 = ax.inv_sh2[k - 1];
        S.is = ax.inv_s[k - 1];
        S.kq = ksq_j[k - 1];
    };
    Step cur, nxt;
    fetch(cur, 1);
    // nothing outstanding on entry: the waits in the loop count its own operations
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    int pc = 0;   // pivots so far: their parity picks the LDS buffer
    for (int k = 1; k <= n; ++k) {
        fetch(nxt, min(k + 1, n));
        // S_k = D_k - E_{k-1} S_{k-1}^-1 E_{k-1} over S_{k-1}^-1; identity padding
        const zd ej = cur.sh_m * sj;
        const zd diag = (cur.kq * cur.is) * sinvj - (cur.sh_p + cur.sh_m) * sj -
                        (c_hi + c_lo) * cur.is2;
        const zd off_lo = c_lo * cur.is2;   // row j - 1
        const zd off_hi = c_hi * cur.is2;   // row j + 1
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int i = g * RPL + q;
            zd val = csel(k > 1, -((cur.sh_m * srow[i]) * v[q] * ej), mk(0.0, 0.0));
            const zd add = csel(i == j, diag,
                                csel(i == j - 1, off_lo, csel(i == j + 1, off_hi, mk(0.0, 0.0))));
            val = val + add;
            const bool inside = i < L && cj;
            v[q] = csel(inside, val, mk(i == j ? 1.0 : 0.0, 0.0));
        }
        // in-place inverse; the pivots run in groups of RPL with the pivot's
        // register index fixed at compile time
        for (int kb = 0; kb < L; kb += RPL) {
            const int gb = kb / RPL;
#pragma unroll
            for (int pq = 0; pq < RPL; ++pq) {
                const int kk = kb + pq;
                if (kk >= L) continue;
                const int b = pc & 1;
                ++pc;
                const bool jp = j == kk, gp = g == gb;
                if (gp) rowbuf[b][j] = v[pq];
                if (jp)
#pragma unroll
                    for (int q = 0; q < RPL; ++q) colbuf[b][g * RPL + q] = v[q];
                // the pivot's owner checks it and publishes 1 / p
                if (jp && gp) {
                    const zd p = v[pq];
                    const double pa = abs2(p);
                    if (!(pa > 1e-300) || !isfinite(pa)) bad = true;
                    rowbuf[b][ML] = cinv(p);
                }
                __syncthreads();
                const zd pinv = rowbuf[b][ML];
                // A[kk][j] / p; the pivot column is scaled by 1 / p instead
                const zd rp = csel(jp, pinv, rowbuf[b][j] * pinv);
                // A[i][j] - A[i][kk] A[kk][j] / p off the pivot row and column,
                // -A[i][kk] / p on the pivot column, A[kk][j] / p on the pivot
                // row and 1 / p at the pivot
#pragma unroll
                for (int q = 0; q < RPL; ++q) {
                    const zd ci = colbuf[b][g * RPL + q];     // A[i][kk]
                    zd x = csel(jp, mk(0.0, 0.0), v[q]) - ci * rp;
                    if (q == pq) x = csel(gp, rp, x);
                    v[q] = x;
                }
            }
        }
        // store S_k^-1 (rows past L zero)
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int i = g * RPL + q;
            buf_store(rf, foff + (unsigned)(k - 1) * fstep + (unsigned)(q * sizeof(cplx<TS>)),
                      ccast<TS>(csel(i < L, v[q], mk(0.0, 0.0))));
        }
        cur = nxt;
    }
    if (bad) *flag = 1;
}

// ML: the largest LR of the launch (32, or 64 when a problem has more than 32
// lines: that body's registers would halve the occupancy of the others)
template <typename TS, int ML>
__global__ __launch_bounds__(FB) void factor2d_kernel(const SubDesc* __restrict__ desc,
                                                     AxisTables ax,
                                                     const zd* __restrict__ subtab,
                                                     const double* __restrict__ ksq, int n,
                                                     cplx<TS>* __restrict__ fac,
                                                     int* __restrict__ flag) {
    static_assert(ML == 32 || ML == MAXL, "row counts");
    __shared__ zd rowbuf[2][ML + 1];   // pivot row; [ML]: the pivot's reciprocal
    __shared__ zd colbuf[2][ML];
    __shared__ zd srow[ML];
    const SubDesc d = desc[blockIdx.x];
    if (d.LR == 16)
        factor2d_body<TS, 16, ML>(d, ax, subtab, ksq, n, fac, flag, rowbuf, colbuf, srow);
    else if (ML == 32 || d.LR == 32)
        factor2d_body<TS, 32, ML>(d, ax, subtab, ksq, n, fac, flag, rowbuf, colbuf, srow);
    else
        factor2d_body<TS, ML, ML>(d, ax, subtab, ksq, n, fac, flag, rowbuf, colbuf, srow);
}

// ----------------------------------------------------------------------------
// The diagonal blocks G_k of H^-1 of a map problem (R_p or L_p, 1 < p < m),
// from the stored S_k^-1: G_n = S_n^-1 and, towards block 1,
//   G_k = S_k^-1 + S_k^-1 E_k G_{k+1} E_k S_k^-1,
// E_k the diagonal coupling of blocks k and k+1 (H, S_k^-1 and G_k are complex
// symmetric).  The boundary maps then start from two columns of every G_k
// (IN_TWIST solves).  One 256-thread workgroup per problem, k from n down to 1;
// thread (j, g) holds rows g RPL .. of column j of G in double, the two
// products of a step go through LDS.  Columns grow and jout of each G_k are
// stored (type TS) at the problem's g_off in the map buffer, [k][2][LR].
// ----------------------------------------------------------------------------
template <typename TS, int LR>
__device__ __forceinline__ void rgf2d_body(const SubDesc& d, AxisTables ax, const zd* __restrict__ subtab,
                                           int n, const cplx<TS>* __restrict__ fac, cplx<TS>* __restrict__ tbuf,
                                           zd (*A)[LR + 1], zd (*Bm)[LR + 1]) {
    constexpr int G = FB / LR, RPL = LR / G;
    const int L = d.L;
    const int t = threadIdx.x, j = t % LR, g = t / LR;
    const zd* sinv2 = subtab + d.tab_off + L + 1;        // 1/(s h^2) on lines lo..hi
    const zd ecol = j < L ? sinv2[min(j, L - 1)] : mk(0.0, 0.0);
    zd erow[RPL];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
        const int r = g * RPL + q;
        erow[q] = r < L ? sinv2[min(r, L - 1)] : mk(0.0, 0.0);
    }
    const int grow = (d.kind == ASP_SUB_R) ? 0 : L - 1;
    const int jout = (d.kind == ASP_SUB_R) ? (d.xe - d.lo) : (d.xs - d.lo);
    const cplx<TS>* F = fac + d.fac_off;
    cplx<TS>* Gout = tbuf + d.g_off;
    zd Gv[RPL], sv[RPL];
    for (int k = n; k >= 1; --k) {
        // S_k^-1 (block k - 1, column-major, rows past L zero): column j
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int r = g * RPL + q;
            sv[q] = (j < L && r < L) ? ccast<double>(F[(long long)(k - 1) * L * LR + (long long)j * LR + r])
                                     : mk(0.0, 0.0);
        }
        if (k == n) {
#pragma unroll
            for (int q = 0; q < RPL; ++q) Gv[q] = sv[q];
        } else {
            const zd sh = ax.sh[k];                            // s at the half line k + 1/2
            // A = G_{k+1} E_k, Bm = S_k^-1
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                const int r = g * RPL + q;
                A[r][j] = Gv[q] * (sh * ecol);
                Bm[r][j] = sv[q];
            }
            __syncthreads();
            // X = E_k (A Bm) = E_k G_{k+1} E_k S_k^-1
            zd xv[RPL];
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                const int r = g * RPL + q;
                zd acc = mk(0.0, 0.0);
                for (int l = 0; l < L; ++l) acc = cfma(A[r][l], Bm[l][j], acc);
                xv[q] = (sh * erow[q]) * acc;
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < RPL; ++q) A[g * RPL + q][j] = xv[q];
            __syncthreads();
            // G_k = S_k^-1 + S_k^-1 X, with (S_k^-1)[r][l] = Bm[l][r] (symmetric)
#pragma unroll
            for (int q = 0; q < RPL; ++q) {
                const int r = g * RPL + q;
                zd acc = mk(0.0, 0.0);
                for (int l = 0; l < L; ++l) acc = cfma(Bm[l][r], A[l][j], acc);
                Gv[q] = sv[q] + acc;
            }
            __syncthreads();   // A and Bm are written again at the next step
        }
#pragma unroll
        for (int q = 0; q < RPL; ++q) {
            const int r = g * RPL + q;
            if (r < L && j == grow) Gout[(long long)(k - 1) * 2 * LR + r] = ccast<TS>(Gv[q]);
            if (r < L && j == jout) Gout[(long long)(k - 1) * 2 * LR + LR + r] = ccast<TS>(Gv[q]);
        }
    }
}

template <typename TS, int LR>
__global__ __launch_bounds__(FB) void rgf2d_kernel(const SubDesc* __restrict__ desc,
                                                  const int* __restrict__ jobs0,
                                                  const int* __restrict__ jobs1, AxisTables ax,
                                                  const zd* __restrict__ subtab, int n,
                                                  const cplx<TS>* __restrict__ fac,
                                                  cplx<TS>* __restrict__ tbuf) {
    __shared__ zd A[LR][LR + 1];
    __shared__ zd Bm[LR][LR + 1];
    // blockIdx.y picks one of two job lists (the map problems of the two sweeps)
    const SubDesc d = desc[(blockIdx.y ? jobs1 : jobs0)[blockIdx.x]];
    rgf2d_body<TS, LR>(d, ax, subtab, n, fac, tbuf, A, Bm);
}

// ----------------------------------------------------------------------------
// batched solves on the matrix cores: one 256-thread workgroup per (auxiliary
// problem, chunk of 1024 / LR right-hand sides).  A block step is the product
// of S_k^-1 (L x L, staged in an LDS ring; the next block's load overlaps the
// step) with the chunk's step vectors (LDS), as four 16 x 16 tiles, one per
// wavefront.  Each lane owns the four (row, rhs) entries of its tile: it forms
// their next step inputs in registers and writes them back to LDS, so a step
// needs one barrier.  Forward results go to scratch for the backward pass.
// ----------------------------------------------------------------------------
// complex 16 x 16 FP32 accumulator of the three-product (Gauss) form:
// p1 = (a_r + a_i) b_r, p2 = a_r (b_i - b_r), p3 = a_i (b_r + b_i);
// re = p1 - p3, im = p1 + p2 (three real products instead of four)
struct KTile3 {
    f32x4 p1, p2, p3;
    __device__ __forceinline__ void zero() {
#pragma unroll
        for (int v = 0; v < 4; ++v) p1[v] = p2[v] = p3[v] = 0.f;
    }
};
__device__ __forceinline__ void kmac3(KTile3& c, zf a, zf b) {
    c.p1 = Mfma<float>::mac(a.x + a.y, b.x, c.p1);
    c.p2 = Mfma<float>::mac(a.x, b.y - b.x, c.p2);
    c.p3 = Mfma<float>::mac(a.y, b.x + b.y, c.p3);
}

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
    zd* out;             // OUT_GRID_STORE: grid vectors
    void* Tout;          // OUT_LINE: boundary-to-boundary maps
    void* y;
    long long y_per_wave;   // scratch entries per workgroup
    zd* sink;               // discard buffer: four entries per thread
    int buf_ok;             // output byte offsets fit the 31-bit buffer range
    int twist_kind;         // IN_TWIST: 0 map columns on and above the diagonal, 1 below
    int n;
    long long N;
};

constexpr int SB = 256;        // threads per solve workgroup: four wavefronts, one tile each

// SPL (ASP_PREC_BF16X3, T = float): every block product as real-split bf16
// products with FP32 accumulation (cmac_split), 16x16x32 steps over the block
template <typename T, int LR, int INM, bool SPL = false>
__global__ __launch_bounds__(SB) void solve2d_kernel(SolveArgs a) {
    static_assert(!SPL || std::is_same<T, float>::value, "the split products take FP32 operands");
    static_assert(INM == IN_GRID || INM == IN_BOUNDARY || INM == IN_TWIST, "input mode");
    constexpr bool NOSTAGE = INM == IN_TWIST;   // map outputs: no staging
    constexpr int SRB = 1024 / LR;          // right-hand sides per workgroup
    constexpr int NCT = SRB / 16;           // right-hand-side tiles
    static_assert((LR / 16) * NCT == 4, "four 16 x 16 tiles, one per wavefront");
    static_assert(SB * 4 <= SINK_ELEMS, "four discard entries per thread");
    constexpr int FMAX = max_lines_2d<T>(LR) * LR;   // largest block
    constexpr int FPT = FMAX / SB;
    constexpr int TBS = SRB + 1;            // padded row stride of the step vectors
    __shared__ cplx<T> Fs[2][FMAX];
    __shared__ cplx<T> tb[2][LR][TBS];      // step vectors [row][rhs]
    // grid outputs of the first SROW lines of X for KO steps, by group parity
    constexpr int KO = sizeof(T) == 4 ? 8 : 2;
    constexpr int SROW = 4;
    __shared__ cplx<T> stg[NOSTAGE ? 1 : 2 * KO * SROW * SRB];

    const int nchunk = (a.nact + SRB - 1) / SRB;
    const int B = a.njobs * nchunk;
    int w, jl, ch;
    if constexpr (INM == IN_TWIST) {
        // chunk ch of a map problem is a chain of min((ch + 1) SRB, n) steps:
        // the longest chains of every problem first, in dispatch order (and so
        // spread over the XCDs), so that no long chain starts near the end
        w = (int)blockIdx.x;
        if (w >= B) return;
        ch = nchunk - 1 - w / a.njobs;
        jl = w % a.njobs;
    } else {
        // XCD-aware order: the chunks of one problem are consecutive work items
        const int per = (B + 7) / 8;
        w = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
        if (w >= B) return;
        jl = w / nchunk;
        ch = w % nchunk;
    }
    const SubDesc d = a.desc[a.jobs[jl]];
    const int L = d.L, n = a.n;
    const long long N = a.N;
    const int tid = threadIdx.x;
    const int l = tid & 63, wv = tid >> 6;
    const int li = l & 15, lk = l >> 4;
    const int rt = wv / NCT, ct = wv % NCT;   // this wavefront's tile
    const int rloc = 16 * ct + li;            // this lane's right-hand side in the chunk
    const cplx<T>* F = reinterpret_cast<const cplx<T>*>(a.fac) + d.fac_off;
    const int FS = L * LR;                  // entries of one block
    const zd* tab = a.subtab + d.tab_off;
    cplx<T>* Y = reinterpret_cast<cplx<T>*>(a.y) + (long long)w * a.y_per_wave;

    const int slot = ch * SRB + rloc;
    const bool valid = slot < a.nact;
    const int rid = valid ? (a.act ? a.act[slot] : slot) : 0;
    const int grow = (d.kind == ASP_SUB_R) ? 0 : L - 1;          // row carrying boundary data
    const zd coupl = (d.kind == ASP_SUB_R) ? tab[0] : tab[L];    // s at lo-1/2 or hi+1/2
    int row[4], lcl[4];
    bool rowv[4], inX[4];
    cplx<T> sinv2[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        row[v] = 16 * rt + Mfma<T>::row(l, v);
        rowv[v] = row[v] < L;
        const int line = d.lo + row[v];
        lcl[v] = min(line, n);
        inX[v] = rowv[v] && line >= d.xs && line <= d.xe;
        sinv2[v] = rowv[v] ? ccast<T>(tab[L + 1 + row[v]]) : mk<T>(0, 0);
    }

    // rows and columns past L stay zero in both rings
    for (int e = tid; e < 2 * LR * TBS; e += SB) (&tb[0][0][0])[e] = mk<T>(0, 0);
    for (int e = tid; e < 2 * FMAX; e += SB) (&Fs[0][0])[e] = mk<T>(0, 0);
    __syncthreads();
    const int LP = (L + 3) & ~3;
    // loads below are unconditional (from clamped, always valid addresses) and
    // their values selected where used: a load under a divergent branch makes
    // the compiler wait for every earlier load at the branch join
    // this wavefront's tile of S^-1 (ring slot fb) times the step vectors tb[buf]
    auto product = [&](int fb, int buf) {
        CTile<T> acc;
        if constexpr (SPL) {
            // lane l takes k = kh + 8 (l / 16) .. + 7 of each 32-wide k range;
            // columns past L are zero in the factor ring, rows past LR of the
            // step vectors are masked
            acc.zero();
            const int lq = l >> 4;
#pragma unroll
            for (int kh = 0; kh < FMAX / LR; kh += 32) {
                float ar[8], ai[8], br[8], bi[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int c = kh + 8 * lq + j;
                    const cplx<T> av = Fs[fb][c * LR + 16 * rt + li];
                    const cplx<T> bv = tb[buf][min(c, LR - 1)][rloc];
                    const bool in = c < LR;
                    ar[j] = av.x;
                    ai[j] = av.y;
                    br[j] = in ? bv.x : 0.f;
                    bi[j] = in ? bv.y : 0.f;
                }
                cmac_split(acc, ar, ai, br, bi);
            }
        } else if constexpr (std::is_same<T, float>::value) {
            KTile3 k3;
            k3.zero();
            for (int c0 = 0; c0 < LP; c0 += 4) {
                const int c = c0 + lk;
                kmac3(k3, Fs[fb][c * LR + 16 * rt + li], tb[buf][c][rloc]);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                acc.re[v] = k3.p1[v] - k3.p3[v];
                acc.im[v] = k3.p1[v] + k3.p2[v];
            }
        } else {
            acc.zero();
            for (int c0 = 0; c0 < LP; c0 += 4) {
                const int c = c0 + lk;
                cmac(acc, Fs[fb][c * LR + 16 * rt + li], tb[buf][c][rloc]);
            }
        }
        return acc;
    };

    // Every memory operation of the step loops is issued by every lane, from a
    // valid address (loads clamp their index; a store a lane does not keep
    // goes to the discard buffer), and the loops have no branch inside: the
    // wait for a load issued two steps ahead then counts exactly the
    // operations issued after it.  (The vector memory counter also counts
    // stores, and a branch makes the compiler assume the shorter path.)
    zd* const sink = a.sink + tid * 4;
    cplx<T>* const sinkT = reinterpret_cast<cplx<T>*>(sink);

    // step data of this lane's rows (complex128): grid data (IN_GRID) or the
    // boundary data of its right-hand side (IN_BOUNDARY)
    // Rows whose data the step ignores read a fixed table entry instead (stride
    // 0), so that they cost no memory traffic.
    const zd* inp[4];
    int ink[4];
    const long long bbase = ((long long)d.wrow * a.w_rhs + rid) * n;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const bool used = (INM == IN_GRID) ? inX[v]
                          : (INM == IN_BOUNDARY) ? (rowv[v] && row[v] == grow)
                                                       : false;
        inp[v] = !used                      ? a.subtab
                 : (INM == IN_GRID) ? a.r + (long long)rid * N + (long long)n * (lcl[v] - 1)
                                          : a.W + bbase;
        ink[v] = used ? 1 : 0;
    }
    auto load_in = [&](int k, zd (&g)[4]) {
#pragma unroll
        for (int v = 0; v < 4; ++v) g[v] = inp[v][(long long)(k - 1) * ink[v]];
    };
    // t_k = g_k - E_{k-1} y_{k-1} for this lane's entries into tb[k & 1]
    // (shm, ism: s at line k - 1/2 and 1 / s^2 at line k - 1 of axis 1).  The
    // data term is g_k (grid rows of X), g_k times the Dirichlet coupling
    // (boundary data on the carrying row), selected per lane; each input mode
    // forms only its own term (a select where the mode needs no product).
    bool carry[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) carry[v] = rowv[v] && row[v] == grow;
    auto put_input = [&](int k, const zd (&g)[4], const cplx<T> (&y)[4], zd shm, zd ism) {
        const cplx<T> shc = ccast<T>(shm);
        zd cin = mk(0.0, 0.0);
        if constexpr (INM != IN_GRID) cin = -(coupl * ism);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            zd dv;
            if constexpr (INM == IN_GRID)
                dv = csel(inX[v], g[v], mk(0.0, 0.0));
            else
                dv = csel(carry[v], g[v] * cin, mk(0.0, 0.0));
            cplx<T> t = ccast<T>(dv);
            t = t - (shc * sinv2[v]) * y[v];              // y = 0 at the first step
            tb[k & 1][row[v]][rloc] = rowv[v] ? t : mk<T>(0, 0);
        }
    };

    // The loads of a step are issued two steps ahead into one of two register
    // slots; the step loops run in pairs so that the slots stay in fixed
    // registers (a register copy would wait for its load).
    auto fetch_to = [&](cplx<T> (&p)[FPT], int blk) {
        const cplx<T>* Fk = F + (long long)blk * FS;
#pragma unroll
        for (int u = 0; u < FPT; ++u) p[u] = Fk[min(tid + u * SB, FS - 1)];
    };
    auto stash_from = [&](const cplx<T> (&p)[FPT], int buf) {
#pragma unroll
        for (int u = 0; u < FPT; ++u) {
            const int e = tid + u * SB;
            Fs[buf][e] = (e < FS) ? p[u] : mk<T>(0, 0);
        }
    };
    cplx<T> yk[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) yk[v] = mk<T>(0, 0);

    // IN_TWIST has no forward sweep: the maps' solutions start from columns of
    // the diagonal blocks of H^-1 and only propagate towards block 1
    if constexpr (INM != IN_TWIST) {
        // forward sweep: y_k = S_k^-1 t_k; block k-1 (S_k^-1) sits in ring slot
        // k & 1.  Slot of step k: the input g_{k+1}, the couplings of lines k, k+1
        // and block k, all used at the end of step k.  The last step stashes block
        // n-2 (already in its ring slot) and forms an input nobody reads: the
        // backward pass finds block n-2 where it expects it and overwrites tb.
        struct FwdSlot {
            cplx<T> pf[FPT];
            zd g[4];
            zd sh, ism;
        };
        auto prefetch_f = [&](FwdSlot& S, int k) {
            load_in(min(k + 1, n), S.g);
            fetch_to(S.pf, k <= n - 1 ? k : max(n - 2, 0));
            const int kc = min(k, n - 1);
            S.sh = a.ax.sh[kc];
            S.ism = a.ax.inv_sh2[kc];
        };
        FwdSlot fsl[2];
        {
            zd g0[4];
            load_in(1, g0);
            fetch_to(fsl[0].pf, 0);
            const zd sh0 = a.ax.sh[0], ism0 = a.ax.inv_sh2[0];
            stash_from(fsl[0].pf, 1);
            put_input(1, g0, yk, sh0, ism0);
        }
        prefetch_f(fsl[0], 1);
        prefetch_f(fsl[1], 2);
        // one full wait before the loop: with nothing outstanding on entry, the
        // waits inside the loop count only the loop's own operations (otherwise the
        // compiler merges in the prologue's shorter history and waits for all)
        __builtin_amdgcn_s_waitcnt(0);
        auto fwd_step = [&](int k, FwdSlot& S, auto pre) {
            const int buf = k & 1;
            __syncthreads();
            const CTile<T> acc = product(buf, buf);
    #pragma unroll
            for (int v = 0; v < 4; ++v) {
                yk[v] = mk<T>(acc.re[v], acc.im[v]);
                Y[((long long)(k - 1) * LR + row[v]) * SRB + rloc] = yk[v];   // rows past L: zero
            }
            stash_from(S.pf, (k + 1) & 1);                               // block k
            put_input(k + 1, S.g, yk, S.sh, S.ism);
            // the slot's next loads after its last use, so that they reuse its registers
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (decltype(pre)::value) prefetch_f(S, k + 2);
        };
        int kf = 1;
        for (; kf + 1 <= n; kf += 2) {
            fwd_step(kf, fsl[0], std::true_type{});
            fwd_step(kf + 1, fsl[1], std::true_type{});
        }
        if (kf <= n) fwd_step(kf, fsl[0], std::false_type{});   // the last step: nothing to fetch
    }

    // backward sweep: v_n = y_n, v_k = y_k - S_k^-1 E_k v_{k+1}; block k-1 in
    // ring slot k & 1.  Slot of step k: y_k, the values its outputs add to and
    // the coupling of lines k-1, k (used in step k), and block k-2 (stashed at
    // the end of step k).  Step 1 stashes and forms data nobody reads.
    const int jout = (d.kind == ASP_SUB_R) ? (d.xe - d.lo) : (d.xs - d.lo);   // OUT_LINE row
    // IN_TWIST: the solutions of this chunk start at blocks slot + 1 <= kmax
    // and are zero above; kind 0 reads its map entries on line jout, kind 1
    // (unit data on line jout) on the data line grow
    const int kmax = (INM == IN_TWIST) ? min((ch + 1) * SRB, n) : n;
    const bool tw1 = INM == IN_TWIST && a.twist_kind == 1;
    const int jrow = tw1 ? grow : jout;
    const int omode = (d.kind == ASP_SUB_L) ? a.out_mode_L : a.out_mode;
    zd* const outp = (d.kind == ASP_SUB_L) ? a.out_L : a.out;
    // map modes write the outgoing line only (known at compile time, so the
    // grid-output state takes no registers); the others store v on X_p
    const bool grid_out = NOSTAGE ? false : omode != OUT_LINE;
    // Grid outputs on the first SROW lines of X are staged in LDS and written
    // KO steps at a time (whole 128-byte lines per right-hand side and line);
    // the other lines of X (the first and last layers are wider) are written
    // at every step.
    const bool bufo = a.buf_ok != 0;
    const bool staging = !NOSTAGE && grid_out && bufo;
    int xr[4];
    bool stgd[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        xr[v] = d.lo + row[v] - d.xs;
        stgd[v] = staging && inX[v] && xr[v] < SROW;
    }
    // IN_TWIST: y_k is the starting vector of the solution that starts at
    // block k (slot = k - 1), zero otherwise: column grow (kind 0, times the
    // unit data's coupling) or jout (kind 1) of G_k, the diagonal block of H^-1
    const cplx<T>* const Gcol = reinterpret_cast<const cplx<T>*>(a.Tout) +
                                (INM == IN_TWIST ? d.g_off : 0) + (tw1 ? LR : 0);
    const cplx<T> cin_s = tw1 ? mk<T>(T(1), T(0))
                              : ccast<T>(-(coupl * a.ax.inv_sh2[min(slot, n - 1)]));
    auto load_y = [&](int k, cplx<T> (&yv)[4]) {
        if constexpr (INM == IN_TWIST) {
            const long long kk = max(k, 1);
            const bool st = valid && slot == k - 1;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const cplx<T> g0 = Gcol[(kk - 1) * 2 * LR + row[v]];
                yv[v] = (st && rowv[v]) ? cin_s * g0 : mk<T>(0, 0);
            }
        } else {
            const long long kk = max(k, 1);     // blocks before the first: y = 0
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const cplx<T> y0 = Y[((kk - 1) * LR + row[v]) * SRB + rloc];
                yv[v] = (k >= 1) ? y0 : mk<T>(0, 0);
            }
        }
    };
    // the one entry of this lane on the OUT_LINE row, if any
    int jsel = -1;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (rowv[e] && row[e] == jrow) jsel = e;
    // boundary maps in row tiles of 16: entry (row r, column c) at (r / 16) n 16 +
    // 16 c + r % 16, so that a sweep workgroup's 16 rows are one contiguous run
    cplx<T>* const Tbase = reinterpret_cast<cplx<T>*>(a.Tout) + d.tr_off;
    const bool tkeep = valid && jsel >= 0;
    auto tidx = [&](int k) { return ((long long)((k - 1) >> 4) * n + slot) * 16 + ((k - 1) & 15); };
    // IN_TWIST kind 1: the entry (row slot, column k - 1)
    auto tidx1 = [&](int k) { return ((long long)(slot >> 4) * n + (k - 1)) * 16 + (slot & 15); };
    bool keep[4];
    zd* gout[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        keep[e] = valid && inX[e];
        gout[e] = outp + (long long)rid * N + (long long)n * (lcl[e] - 1);
    }
    // With a.buf_ok the outputs go through a buffer resource: a lane that keeps
    // nothing gives an offset past the range and the hardware drops the write
    // (no memory traffic, no branch).  Otherwise such writes go to the discard
    // buffer.
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        grid_out ? static_cast<void*>(outp) : static_cast<void*>(Tbase), 0, 0x7fffffff, BUF_DW3);
    unsigned boff[4];   // byte offsets at step 1
#pragma unroll
    for (int e = 0; e < 4; ++e)
        boff[e] = grid_out ? ((keep[e] && !stgd[e])
                                  ? (unsigned)(((long long)rid * N + (long long)n * (lcl[e] - 1)) * 16)
                                  : BUF_OOB)
                           : BUF_OOB;   // OUT_LINE offsets are formed per step
    auto emit = [&](int k, const cplx<T> (&v)[4]) {
        if (!grid_out) {
            cplx<T> x = v[0];
#pragma unroll
            for (int e = 1; e < 4; ++e) x = csel(jsel == e, v[e], x);
            bool kp = tkeep;
            long long ti = tidx(k);
            if constexpr (INM == IN_TWIST) {
                if (tw1) {
                    // entry (slot, k - 1) below the diagonal, with the unit data's
                    // coupling of column k - 1
                    kp = kp && k - 1 < slot;
                    ti = tidx1(k);
                    x = ccast<T>(-(coupl * a.ax.inv_sh2[k - 1])) * x;
                } else {
                    kp = kp && k - 1 <= slot;   // on and above the diagonal
                }
            }
            if (bufo)
                buf_store(rs, kp ? (unsigned)(ti * sizeof(cplx<T>)) : BUF_OOB, x);
            else
                *(kp ? Tbase + ti : sinkT) = x;
            return;
        }
        if constexpr (!NOSTAGE) {
            if (staging) {
                cplx<T>* sg = stg + ((((k - 1) / KO) & 1) * KO + (k - 1) % KO) * SROW * SRB;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (stgd[e]) sg[xr[e] * SRB + rloc] = v[e];
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const zd x = ccast<double>(v[e]);
            if (bufo)
                buf_store(rs, boff[e] + (unsigned)(k - 1) * 16u, x);
            else
                *(keep[e] ? gout[e] + (k - 1) : sink + e) = x;
        }
    };
    // write out the staged steps g KO + 1 .. g KO + KO: thread (line, rhs) of
    // the staged block writes KO consecutive entries; lanes past the block
    // pass offsets past the range
    const int fx = min(tid / SRB, SROW - 1), frl = tid % SRB;
    const int fslot = ch * SRB + frl;
    const int nxs = min(d.xe - d.xs + 1, SROW);
    const bool fvalid = staging && tid < SROW * SRB && tid / SRB < nxs && fslot < a.nact;
    const int frid = fvalid ? (a.act ? a.act[fslot] : fslot) : 0;
    const unsigned fbase =
        fvalid ? (unsigned)(((long long)frid * N + (long long)n * (d.xs + fx - 1)) * 16) : BUF_OOB;
    auto flush = [&](int g) {
        if constexpr (!NOSTAGE) {
            const cplx<T>* sg = stg + (g & 1) * KO * SROW * SRB + fx * SRB + frl;
#pragma unroll
            for (int q = 0; q < KO; ++q) {
                const int st = g * KO + 1 + q;
                const unsigned off = (st <= n) ? fbase + (unsigned)(st - 1) * 16u : BUF_OOB;
                buf_store(rs, off, ccast<double>(sg[q * SROW * SRB]));
            }
        }
    };
    // E_k v_{k+1} for this lane's entries into tb[k & 1] (shk: s at line k + 1/2)
    auto put_coupled = [&](int k, const cplx<T> (&v)[4], zd shk) {
        const cplx<T> shc = ccast<T>(shk);
#pragma unroll
        for (int e = 0; e < 4; ++e) tb[k & 1][row[e]][rloc] = (shc * sinv2[e]) * v[e];
    };
    struct BwdSlot {
        cplx<T> pf[FPT];
        cplx<T> y[4];
        zd sh;
    };
    auto prefetch_b = [&](BwdSlot& S, int k) {
        load_y(k, S.y);
        fetch_to(S.pf, max(k - 2, 0));
        S.sh = a.ax.sh[max(k - 1, 0)];
    };
    BwdSlot bsl[2];
    {
        const zd shn = a.ax.sh[max(kmax - 1, 0)];
        if constexpr (INM == IN_TWIST) {
            // no forward sweep: the starting vectors at the top block, and block
            // kmax - 2 (S_{kmax-1}^-1) into the ring slot the first step reads
            load_y(kmax, yk);
            cplx<T> pf0[FPT];
            fetch_to(pf0, max(kmax - 2, 0));
            stash_from(pf0, (kmax - 1) & 1);
        }
        emit(kmax, yk);
        put_coupled(kmax - 1, yk, shn);    // kmax = 1: data nobody reads
    }
    cplx<T> (&vk)[4] = yk;
    prefetch_b(bsl[0], kmax - 1);
    prefetch_b(bsl[1], kmax - 2);
    __builtin_amdgcn_s_waitcnt(0);
    auto bwd_step = [&](int k, BwdSlot& S, auto pre) {
        const int buf = k & 1;
        __syncthreads();
        if (staging && k % KO == 0) flush(k / KO);   // steps k+1 .. k+KO are staged
        const CTile<T> acc = product(buf, buf);
#pragma unroll
        for (int e = 0; e < 4; ++e) vk[e] = S.y[e] - mk<T>(acc.re[e], acc.im[e]);
        emit(k, vk);
        stash_from(S.pf, (k - 1) & 1);                               // block k-2
        put_coupled(k - 1, vk, S.sh);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (decltype(pre)::value) prefetch_b(S, k - 2);
    };
    int kb = kmax - 1;
    for (; kb - 1 >= 1; kb -= 2) {
        bwd_step(kb, bsl[0], std::true_type{});
        bwd_step(kb - 1, bsl[1], std::true_type{});
    }
    if (kb >= 1) bwd_step(kb, bsl[0], std::false_type{});
    if (staging) {
        __syncthreads();
        flush(0);
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
// columns of T in batches of 16 (four k-steps); two batches sit in two fixed
// register slots, and a slot is refilled right after its products, so one
// batch is in flight while the other is multiplied.  Every load is issued
// (columns past the wavefront's range read its last column again) and the
// columns past the range are zeroed where used: a value selected at the load
// makes the compiler wait for that load at once.  The partial tiles meet in
// LDS and are added in wavefront order (fixed, so a result does not depend on
// the other right-hand sides or on scheduling).  The two blocks of a row tile
// are 64 block ids apart and so share an XCD and its L2 copy of T.
template <typename T, bool SPL = false>
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
    // this block's 16 rows of T: one contiguous run of row-tile blockIdx.x (rows
    // past n are padding, their outputs are not stored)
    const cplx<T>* __restrict__ Tt = Tm + (long long)blockIdx.x * n * 16 + li;
    const int per = (n + 16 * SW_W - 1) / (16 * SW_W) * 16;
    const int cb = wv * per, ce = min(cb + per, n);
    // one output per thread (tile t2o, lane l2, element v_); its u~ value is
    // read now, ahead of the products.  Column li of tile t2 is right-hand side
    // 2 li + t2, so that a lane's two right-hand sides of a column of W are
    // adjacent (one 16-byte load in FP32).
    const int tid = threadIdx.x;
    const int v_ = tid & 3, l2 = (tid >> 2) & 63, t2o = tid >> 8;
    const int ko = k0 + Mfma<T>::row(l2, v_);
    const int slot = s0 + 2 * (l2 & 15) + t2o;
    const bool okout = ko < n && slot < a.nact;
    const int id = okout ? (a.act ? a.act[slot] : slot) : 0;
    const zd uval = a.Ugrid[(long long)id * a.N + (long long)n * (a.line[side] - 1) + (okout ? ko : 0)];
    // FP32: three real products per complex one (p1 = (ar + ai) br,
    // p2 = ar (bi - br), p3 = ai (br + bi); re = p1 - p3, im = p1 + p2), the
    // matrix-core work of the step down by a quarter; FP64: the four products
    KTile3 kacc[2];
    CTile<T> acc[2];
    acc[0].zero();
    acc[1].zero();
    kacc[0].zero();
    kacc[1].zero();
    struct Batch {
        cplx<T> av[4], bv[4][2];
        bool ok[4];
    };
    auto load = [&](Batch& B, int c0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + 4 * u + lk;
            const int cc = min(c, ce - 1);
            B.av[u] = Tt[(long long)cc * 16];
#pragma unroll
            for (int t2 = 0; t2 < 2; ++t2) B.bv[u][t2] = Wi[(long long)cc * ws + s0 + 2 * li + t2];
            B.ok[u] = c < ce;
        }
    };
    auto multiply = [&](const Batch& B) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const cplx<T> av = csel(B.ok[u], B.av[u], mk<T>(T(0), T(0)));
#pragma unroll
            for (int t2 = 0; t2 < 2; ++t2) {
                if constexpr (sizeof(T) == 4)
                    kmac3(kacc[t2], av, B.bv[u][t2]);
                else
                    cmac(acc[t2], av, B.bv[u][t2]);
            }
        }
    };
    // SPL: the two batches (32 columns) as the k range of one split product;
    // slot j < 4 of a lane holds batch 0's column 4 j + lk, slot j >= 4 batch 1's
    auto multiply_split = [&](const Batch& B0, const Batch& B1) {
        if constexpr (SPL) {
#pragma unroll
            for (int t2 = 0; t2 < 2; ++t2) {
                float ar[8], ai[8], br[8], bi[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const Batch& B = j < 4 ? B0 : B1;
                    const int u = j & 3;
                    const cplx<T> av = csel(B.ok[u], B.av[u], mk<T>(T(0), T(0)));
                    ar[j] = av.x;
                    ai[j] = av.y;
                    br[j] = B.bv[u][t2].x;
                    bi[j] = B.bv[u][t2].y;
                }
                cmac_split(acc[t2], ar, ai, br, bi);
            }
        }
    };
    Batch b0, b1;
    load(b0, cb);
    load(b1, cb + 16);
    // nothing outstanding on entry: the waits in the loop count its own loads
    __builtin_amdgcn_s_waitcnt(0);
    for (int c0 = cb; c0 < cb + per; c0 += 32) {
        if constexpr (SPL) {
            multiply_split(b0, b1);
            __builtin_amdgcn_sched_barrier(0);
            load(b0, c0 + 32);
            load(b1, c0 + 48);
            __builtin_amdgcn_sched_barrier(0);
        } else {
            multiply(b0);
            __builtin_amdgcn_sched_barrier(0);
            load(b0, c0 + 32);
            __builtin_amdgcn_sched_barrier(0);
            multiply(b1);
            __builtin_amdgcn_sched_barrier(0);
            load(b1, c0 + 48);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    if constexpr (sizeof(T) == 4 && !SPL) {
#pragma unroll
        for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                acc[t2].re[v] = kacc[t2].p1[v] - kacc[t2].p3[v];
                acc[t2].im[v] = kacc[t2].p1[v] + kacc[t2].p2[v];
            }
    }
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wv][t2][l][v] = mk<T>(acc[t2].re[v], acc[t2].im[v]);
    __syncthreads();
    if (!okout) return;
    cplx<T> sum = red[0][t2o][l2][v_];
#pragma unroll
    for (int q = 1; q < SW_W; ++q) sum = sum + red[q][t2o][l2][v_];
    const zd val = ccast<double>(sum) + uval;
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

// Sequential sweep step: the boundary line R_{t+1} hands to R_{t+2} (its
// output a plus u~ on the last line of its layer) and the one L_{m-t} hands to
// L_{m-t-1} (c plus u~ on the first line of its layer) into their W rows
__global__ void sweep_hand_kernel(const zd* __restrict__ z, const zd* __restrict__ stage,
                                  const zd* __restrict__ Ugrid, zd* __restrict__ W,
                                  long long rowR, int lineR, long long rowL, int lineL,
                                  const int* __restrict__ act, int n, long long N) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int id = act ? act[blockIdx.y] : (int)blockIdx.y;
    const long long u = (long long)id * N + k;
    if (rowR >= 0) {
        const long long g = u + (long long)n * (lineR - 1);
        W[rowR + (long long)id * n + k] = z[g] + Ugrid[g];
    }
    if (rowL >= 0) {
        const long long g = u + (long long)n * (lineL - 1);
        W[rowL + (long long)id * n + k] = stage[g] + Ugrid[g];
    }
}

}  // namespace

hipError_t launch_sweep_hand(const asp_plan* P, const zd* z, const zd* stage, zd* W,
                             long long rowR, int lineR, long long rowL, int lineL, const int* act,
                             int nact, hipStream_t st) {
    if (nact <= 0) return hipSuccess;
    dim3 grid((P->n + 255) / 256, nact);
    hipLaunchKernelGGL(sweep_hand_kernel, grid, dim3(256), 0, st, z, stage, P->d_U, W, rowR, lineR,
                       rowL, lineL, act, P->n, P->N);
    return hipGetLastError();
}

hipError_t launch_factor2d(const asp_plan* P, hipStream_t st) {
    const int nsub = (int)P->subs.size();
    AxisTables ax{P->d_axis, P->d_axis + (P->n + 1), P->d_axis + (2 * P->n + 1)};
    const bool wide = std::max(P->LR_M, P->LR_RL) > 32;
    if (P->prec != ASP_PREC_FP64) {
        auto k = wide ? factor2d_kernel<float, MAXL> : factor2d_kernel<float, 32>;
        hipLaunchKernelGGL(k, dim3(nsub), dim3(FB), 0, st, P->d_desc, ax, P->d_subtab, P->d_ksq,
                           P->n, reinterpret_cast<zf*>(P->d_fac), P->d_flag);
    } else {
        auto k = wide ? factor2d_kernel<double, MAXL> : factor2d_kernel<double, 32>;
        hipLaunchKernelGGL(k, dim3(nsub), dim3(FB), 0, st, P->d_desc, ax, P->d_subtab, P->d_ksq,
                           P->n, reinterpret_cast<zd*>(P->d_fac), P->d_flag);
    }
    return hipGetLastError();
}

template <typename TS>
static hipError_t launch_rgf_t(const asp_plan* P, const int* jobs0, const int* jobs1, int nlists,
                               int njobs, hipStream_t st) {
    AxisTables ax{P->d_axis, P->d_axis + (P->n + 1), P->d_axis + (2 * P->n + 1)};
    const cplx<TS>* fac = reinterpret_cast<const cplx<TS>*>(P->d_fac);
    cplx<TS>* tb = reinterpret_cast<cplx<TS>*>(P->d_T);
    const dim3 grid(njobs, nlists);
    if (P->LR_RL == 16)
        hipLaunchKernelGGL((rgf2d_kernel<TS, 16>), grid, dim3(FB), 0, st, P->d_desc, jobs0, jobs1, ax,
                           P->d_subtab, P->n, fac, tb);
    else if (P->LR_RL == 32)
        hipLaunchKernelGGL((rgf2d_kernel<TS, 32>), grid, dim3(FB), 0, st, P->d_desc, jobs0, jobs1, ax,
                           P->d_subtab, P->n, fac, tb);
    else
        hipLaunchKernelGGL((rgf2d_kernel<TS, 64>), grid, dim3(FB), 0, st, P->d_desc, jobs0, jobs1, ax,
                           P->d_subtab, P->n, fac, tb);
    return hipGetLastError();
}

hipError_t launch_rgf2d(const asp_plan* P, int job0, int job1, int njobs, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    const int* j0 = P->d_jobs + job0;
    const int* j1 = job1 >= 0 ? P->d_jobs + job1 : j0;
    const int nl = job1 >= 0 ? 2 : 1;
    if (P->prec != ASP_PREC_FP64) return launch_rgf_t<float>(P, j0, j1, nl, njobs, st);
    return launch_rgf_t<double>(P, j0, j1, nl, njobs, st);
}

// one kernel per (precision, row count, input mode): the M-solves, the R/L
// solves and the transfer-map solves are separate kernels
template <int LR, int INM>
static hipError_t launch_solve_lr(const asp_plan* P, const SolveArgs& a, int blocks, hipStream_t st) {
    if (P->prec == ASP_PREC_BF16X3)
        hipLaunchKernelGGL((solve2d_kernel<float, LR, INM, true>), dim3(blocks), dim3(SB), 0, st, a);
    else if (P->prec != ASP_PREC_FP64)
        hipLaunchKernelGGL((solve2d_kernel<float, LR, INM>), dim3(blocks), dim3(SB), 0, st, a);
    else
        hipLaunchKernelGGL((solve2d_kernel<double, LR, INM>), dim3(blocks), dim3(SB), 0, st, a);
    return hipGetLastError();
}

template <int LR>
static hipError_t launch_solve_mode(const asp_plan* P, const SolveArgs& a, int blocks,
                                    hipStream_t st) {
    if (a.in_mode == IN_GRID) return launch_solve_lr<LR, IN_GRID>(P, a, blocks, st);
    if (a.in_mode == IN_BOUNDARY) return launch_solve_lr<LR, IN_BOUNDARY>(P, a, blocks, st);
    if (a.in_mode == IN_TWIST) return launch_solve_lr<LR, IN_TWIST>(P, a, blocks, st);
    return hipErrorInvalidValue;
}

int solve_rhs_per_block(int LR) { return 1024 / LR; }

// forward results of one workgroup: n blocks x LR rows x 1024 / LR right-hand sides
long long solve_scratch_per_block(const asp_plan* P) { return (long long)P->n * 1024; }

hipError_t launch_solve2d(const asp_plan* P, const SolveLaunch& L, hipStream_t st) {
    if (L.njobs <= 0 || L.nact <= 0) return hipSuccess;
    // the map solves write the outgoing line, the others store v on X_p
    const bool twist = L.in_mode == IN_TWIST;
    if (twist ? L.out_mode != OUT_LINE
              : (L.out_mode != OUT_GRID_STORE || (L.out_L && L.out_mode_L != OUT_GRID_STORE)))
        return hipErrorInvalidValue;
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
    a.Tout = P->d_T;
    a.y = P->d_y;
    a.y_per_wave = solve_scratch_per_block(P);
    a.sink = P->d_sink;
    {
        const size_t esz = P->prec != ASP_PREC_FP64 ? sizeof(zf) : sizeof(zd);
        const long long lim = 1LL << 31;
        const long long grid_bytes = (long long)std::max(P->ws_rhs, L.nact) * P->N * (long long)sizeof(zd);
        const long long line_bytes = (long long)((P->n + 15) / 16 * 16) * P->n * (long long)esz;
        // map outputs (OUT_LINE) address the map only
        a.buf_ok = ((L.out_mode == OUT_LINE || grid_bytes < lim) && line_bytes < lim) ? 1 : 0;
    }
    a.twist_kind = L.twist_kind;
    a.n = P->n;
    a.N = P->N;
    const int LR = L.rl ? P->LR_RL : P->LR_M;   // every job of one launch shares its row count
    const int srb = solve_rhs_per_block(LR);
    const long long B = (long long)L.njobs * ((L.nact + srb - 1) / srb);
    // IN_TWIST uses no forward-result scratch
    if (!twist && B > P->y_waves) return hipErrorInvalidValue;
    const int blocks = (int)(((B + 7) / 8) * 8);
    if (LR == 16) return launch_solve_mode<16>(P, a, blocks, st);
    if (LR == 32) return launch_solve_mode<32>(P, a, blocks, st);
    return launch_solve_mode<64>(P, a, blocks, st);
}

static int sweep_slots(int nact) { return (nact + SW_RT - 1) / SW_RT * SW_RT; }

int sweep_wt_len(const asp_plan* P, int nrhs) { return 4 * P->n * sweep_slots(nrhs); }

// transposed sweep buffers: [side][ping-pong][n][ws]
static void* wt_buf(const asp_plan* P, int side, int pp, int ws) {
    const size_t esz = P->prec != ASP_PREC_FP64 ? sizeof(zf) : sizeof(zd);
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
    if (P->prec != ASP_PREC_FP64)
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
    if (P->prec == ASP_PREC_BF16X3)
        hipLaunchKernelGGL((sweep_step_kernel<float, true>), grid, dim3(64 * SW_W), 0, st, a);
    else if (P->prec != ASP_PREC_FP64)
        hipLaunchKernelGGL(sweep_step_kernel<float>, grid, dim3(64 * SW_W), 0, st, a);
    else
        hipLaunchKernelGGL(sweep_step_kernel<double>, grid, dim3(64 * SW_W), 0, st, a);
    return hipGetLastError();
}
