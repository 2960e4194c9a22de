// 3D auxiliary problems (Section 4.1, Algorithms 3 and 4).
//
// Reordered with the sweep axis fastest inside x1-blocks, a 3D auxiliary
// problem on sweep lines lo..hi is block tridiagonal in i1 with n dense
// blocks of size n L (the quasi-2D cross-section of one x1 index).  The
// factorization runs the block recurrence
//     S_1 = D_1,   S_k = D_k - E_k S_{k-1}^-1 E_k     (E_k diagonal)
// and stores every S_k^-1; each inverse is an in-place blocked Gauss-Jordan
// elimination whose panel and trailing updates are complex products of 64 x 64
// tiles on the matrix cores.  A solve is the forward pass y_k = S_k^-1 (g_k -
// E_k y_{k-1}) and the backward pass x_k = y_k - S_k^-1 E_{k+1} x_{k+1}, one
// launch per block step, each step a product of S_k^-1 with 16 right-hand sides.
//
// The Gauss-Jordan elimination does not pivot: at a few points per wavelength
// the blocks are close to diagonally dominant (the shift omega^2 h^2 / c^2 is
// small next to the 6 of the diagonal), and a zero or non-finite pivot is
// reported as a breakdown.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "asp_internal.h"
#include "mfma.h"

namespace {

constexpr int TB = 64;        // panel width of the inversion, edge of a tile
constexpr int LDT = TB + 1;   // LDS row stride of a tile (complex entries)
constexpr int NT = 256;       // threads of a factor or solve workgroup (4 waves)
constexpr int RW = 16;        // right-hand sides per solve chunk (one matrix-core tile)

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// ---------------------------------------------------------------------------
// 64 x 64 tiles: LDS copies with row stride LDT, products on the matrix cores
// ---------------------------------------------------------------------------
// S[r][c] = A(r0 + r, c0 + c) of a column-major matrix with leading dimension ld
template <typename T>
__device__ __forceinline__ void load_tile(cplx<T>* S, const cplx<T>* A, long long ld, int r0,
                                          int c0) {
    const int r = threadIdx.x & 63, cg = threadIdx.x >> 6;
#pragma unroll 4
    for (int e = 0; e < 16; ++e) {
        const int c = cg + 4 * e;
        S[r * LDT + c] = A[(long long)(c0 + c) * ld + r0 + r];
    }
}

// half tiles for the trailing update: S[r][k] = A(r0 + r, c0 + k), 64 rows by
// 32 columns with row stride KLD, and S[k][c] = A(r0 + k, c0 + c), 32 rows by
// 64 columns with row stride LDT (column-major sources, leading dimension ld)
constexpr int KLD = TB / 2 + 1;
template <typename T>
__device__ __forceinline__ void load_half_cols(cplx<T>* S, const cplx<T>* A, long long ld, int r0,
                                               int c0) {
    const int r = threadIdx.x & 63, cg = threadIdx.x >> 6;
#pragma unroll 4
    for (int e = 0; e < 8; ++e) {
        const int c = cg + 4 * e;
        S[r * KLD + c] = A[(long long)(c0 + c) * ld + r0 + r];
    }
}
template <typename T>
__device__ __forceinline__ void load_half_rows(cplx<T>* S, const cplx<T>* A, long long ld, int r0,
                                               int c0) {
    const int r = threadIdx.x & 31, cg = threadIdx.x >> 5;
#pragma unroll 4
    for (int e = 0; e < 8; ++e) {
        const int c = cg + 8 * e;
        S[r * LDT + c] = A[(long long)(c0 + c) * ld + r0 + r];
    }
}

// C = P Q for tiles in LDS (P[r][k], Q[k][c]).  Wave w computes rows
// 32 (w / 2) .. + 32 and columns 32 (w % 2) .. + 32 as four transposed 16 x 16
// blocks: acc[a][b], lane l, element v is C(R0 + 16 b + l % 16, C0 + 16 a +
// row(l, v)), so that a column of C leaves the lanes contiguously.
// FP32 uses the three-product (Gauss) form, seeded from the accumulators:
// p1 = 0, p2 = im, p3 = -re, then p1 += (q_r + q_i) p_r, p2 += q_r (p_i - p_r),
// p3 += q_i (p_r + p_i), and re = p1 - p3, im = p1 + p2 (three real products
// per complex one instead of four).
// KL: the k extent (64, or 32 for half tiles); PLD, QLD: the LDS row strides
// of P and Q.
template <typename T, int KL = TB, int PLD = LDT, int QLD = LDT>
__device__ __forceinline__ void tile_product(const cplx<T>* P, const cplx<T>* Q,
                                             CTile<T> acc[2][2]) {
    const int l = lane_id(), w = wave_id();
    const int R0 = 32 * (w >> 1), C0 = 32 * (w & 1);
    const int li = l & 15, lk = l >> 4;
    if constexpr (std::is_same<T, float>::value) {
        f32x4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    p1[a][b][v] = 0.f;
                    p2[a][b][v] = acc[a][b].im[v];
                    p3[a][b][v] = -acc[a][b].re[v];
                }
#pragma unroll 2
        for (int k0 = 0; k0 < KL; k0 += 4) {
            const int kq = k0 + lk;
            zf qa[2], pb[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) qa[a] = Q[kq * QLD + C0 + 16 * a + li];
#pragma unroll
            for (int b = 0; b < 2; ++b) pb[b] = P[(R0 + 16 * b + li) * PLD + kq];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const float qs = qa[a].x + qa[a].y;
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    p1[a][b] = Mfma<float>::mac(qs, pb[b].x, p1[a][b]);
                    p2[a][b] = Mfma<float>::mac(qa[a].x, pb[b].y - pb[b].x, p2[a][b]);
                    p3[a][b] = Mfma<float>::mac(qa[a].y, pb[b].x + pb[b].y, p3[a][b]);
                }
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    acc[a][b].re[v] = p1[a][b][v] - p3[a][b][v];
                    acc[a][b].im[v] = p1[a][b][v] + p2[a][b][v];
                }
    } else {
#pragma unroll 2
        for (int k0 = 0; k0 < KL; k0 += 4) {
            const int kq = k0 + lk;
            cplx<T> qa[2], pb[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) qa[a] = Q[kq * QLD + C0 + 16 * a + li];
#pragma unroll
            for (int b = 0; b < 2; ++b) pb[b] = P[(R0 + 16 * b + li) * PLD + kq];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) cmac(acc[a][b], qa[a], pb[b]);
        }
    }
}

// global tile (column-major, leading dimension ld, origin r0, c0) <-> accumulators
template <typename T>
__device__ __forceinline__ void load_acc(CTile<T> acc[2][2], const cplx<T>* A, long long ld,
                                         int r0, int c0) {
    const int l = lane_id(), w = wave_id();
    const int R0 = 32 * (w >> 1), C0 = 32 * (w & 1);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = R0 + 16 * b + (l & 15), c = C0 + 16 * a + Mfma<T>::row(l, v);
                const cplx<T> x = A[(long long)(c0 + c) * ld + r0 + r];
                acc[a][b].re[v] = x.x;
                acc[a][b].im[v] = x.y;
            }
}

template <typename T>
__device__ __forceinline__ void store_acc(cplx<T>* A, long long ld, int r0, int c0,
                                          const CTile<T> acc[2][2], T sign) {
    const int l = lane_id(), w = wave_id();
    const int R0 = 32 * (w >> 1), C0 = 32 * (w & 1);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = R0 + 16 * b + (l & 15), c = C0 + 16 * a + Mfma<T>::row(l, v);
                A[(long long)(c0 + c) * ld + r0 + r] =
                    mk<T>(sign * acc[a][b].re[v], sign * acc[a][b].im[v]);
            }
}

// ---------------------------------------------------------------------------
// factorization
// ---------------------------------------------------------------------------
struct Form3Args {
    const SubDesc* desc;
    const int* jobs;
    void* fac;
    AxisTables ax;
    const zd* subtab;
    const double* ksq;
    const zd* e3;
    int n, k;
    long long S;
};

// Block k of the symmetric-form operator of the auxiliary problem reordered
// (x1-blocks, sweep axis fastest), minus the Schur term of the previous block.
// Entry (r, c): 7-point couplings inside the cross-section, the diagonal with
// all six half-line terms, identity on the padding.
template <typename T>
__global__ __launch_bounds__(256) void form3d_kernel(Form3Args a) {
    const SubDesc d = a.desc[a.jobs[blockIdx.z]];
    const int Bp = d.B, L = d.L, B = a.n * d.L;
    const int r = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (r >= Bp || c >= Bp) return;
    cplx<T>* A = static_cast<cplx<T>*>(a.fac) + d.fac_off + (long long)a.k * Bp * Bp;
    zd val = mk(0.0, 0.0);
    if (r >= B || c >= B) {
        if (r == c) val = mk(1.0, 0.0);
    } else {
        const int k = a.k;
        const int i3r = r % L, i2r = r / L, i3c = c % L, i2c = c / L;
        const zd* sh3 = a.subtab + d.tab_off;     // s3 at half lines lo - 1/2 ..
        const zd* ish3 = sh3 + L + 1;             // 1 / (s3 h^2)
        const zd* is3 = sh3 + 2 * L + 1;          // 1 / s3
        if (r == c) {
            const zd s23 = a.ax.inv_s[i2r] * ish3[i3r];     // 1 / (s2 s3 h^2)
            const zd s13 = a.ax.inv_s[k] * ish3[i3r];       // 1 / (s1 s3 h^2)
            const zd s12 = a.ax.inv_s[k] * a.ax.inv_sh2[i2r];
            const zd c1 = (a.ax.sh[k + 1] + a.ax.sh[k]) * s23;
            const zd c2 = (a.ax.sh[i2r + 1] + a.ax.sh[i2r]) * s13;
            const zd c3 = (sh3[i3r + 1] + sh3[i3r]) * s12;
            const long long g = (long long)k + (long long)a.n * i2r + a.S * (d.lo - 1 + i3r);
            val = ((a.ksq[g] * a.ax.inv_s[k]) * a.ax.inv_s[i2r]) * is3[i3r] - (c1 + c2 + c3);
        } else if (i2r == i2c && (i3r - i3c == 1 || i3c - i3r == 1)) {
            val = sh3[max(i3r, i3c)] * (a.ax.inv_s[k] * a.ax.inv_sh2[i2r]);
        } else if (i3r == i3c && (i2r - i2c == 1 || i2c - i2r == 1)) {
            val = a.ax.sh[max(i2r, i2c)] * (a.ax.inv_s[k] * ish3[i3r]);
        }
        if (k > 0) {
            const zd* e = a.e3 + d.vec_off;
            const cplx<T>* prev = A - (long long)Bp * Bp;
            const zd sk = a.ax.sh[k];
            const zd er = sk * e[r], ec = sk * e[c];
            const zd pv = ccast<double>(prev[(long long)c * Bp + r]);
            val = val - (er * pv) * ec;
        }
    }
    A[(long long)c * Bp + r] = ccast<T>(val);
}

struct GjArgs {
    const SubDesc* desc;
    const int* jobs;
    const NdFront* fr;   // non-NULL: nested-dissection fronts (only the separator part pivots)
    void* fac;
    void* Rbuf;     // [job][Bmax][64]: the panel rows before the step
    void* Dbuf;     // [job][64][64]: the inverse of the pivot tile
    int* flag;
    long long rstride;
    int k, jp, ntmax;
    // fronts, two panels per pass (look-ahead): the panel rows of panel J1 in
    // R slot 0 and of J2 in slot 1 (rsel), its columns kept in slot 2 (save_c);
    // the update after J1 covers only what panel J2 needs (GJ_NARROW), the one
    // after J2 applies both panels to the rest (GJ_COMBINED)
    int mode, rsel, save_c;
};

enum { GJ_FULL = 0, GJ_NARROW = 1, GJ_COMBINED = 2 };

// the matrix of job js: block k of a problem (all panels pivot), or a front
// whose first ipad / 64 panels pivot
struct GjMat {
    long long off, roff;
    int Bp, npiv;
};

__device__ __forceinline__ GjMat gj_mat(const GjArgs& a, int js) {
    GjMat m;
    if (a.fr) {
        const NdFront& f = a.fr[js];
        m.off = f.foff;
        m.roff = f.roff;
        m.Bp = f.f;
        m.npiv = f.ipad / TB;
    } else {
        const SubDesc& d = a.desc[a.jobs[js]];
        m.Bp = d.B;
        m.off = d.fac_off + (long long)a.k * d.B * d.B;
        m.roff = js * a.rstride;
        m.npiv = d.B / TB;
    }
    return m;
}

// Pivot tile of panel jp: Dbuf = D^-1 for D = A[J,J], one workgroup of PVG
// waves per job.  Gauss-Jordan elimination without pivoting: thread t holds
// row t % 64, columns t / 64 + PVG e (e = 0 .. PVE - 1); the pivot row and
// column pass through LDS, double-buffered (one barrier per pivot).  Sixteen
// waves give the shortest chain of 64 dependent pivots (few jobs per launch);
// four waves do the same work with less per-entry overhead and several
// workgroups per CU (many jobs per launch, the small fronts of nested
// dissection).  A zero or non-finite pivot sets the breakdown flag.
template <typename T, int PVG>
__global__ __launch_bounds__(64 * PVG) void gj_pivot_kernel(GjArgs a) {
    constexpr int PVE = TB / PVG;   // columns per thread
    __shared__ cplx<T> rowbuf[2][TB], colbuf[2][TB];
    __shared__ int bad;
    const int js = blockIdx.x;
    const GjMat gm = gj_mat(a, js);
    const int Bp = gm.Bp;
    if (a.jp >= gm.npiv) return;
    const cplx<T>* A = static_cast<const cplx<T>*>(a.fac) + gm.off;
    const int r = threadIdx.x & 63, cg = threadIdx.x >> 6;     // cg = 0 .. PVG - 1
    const int J0 = a.jp * TB;
    if (threadIdx.x == 0) bad = 0;
    cplx<T> v[PVE];
#pragma unroll
    for (int e = 0; e < PVE; ++e) v[e] = A[(long long)(J0 + cg + PVG * e) * Bp + J0 + r];
    const T tiny = sizeof(T) == 4 ? T(1e-36) : T(1e-300);
    __syncthreads();
    for (int piv = 0; piv < TB; ++piv) {
        cplx<T>* rb = rowbuf[piv & 1];
        cplx<T>* cb = colbuf[piv & 1];
        if (r == piv)
#pragma unroll
            for (int e = 0; e < PVE; ++e) rb[cg + PVG * e] = v[e];
        if (piv % PVG == cg) {
            cplx<T> pc = v[0];
#pragma unroll
            for (int e = 1; e < PVE; ++e) {
                const bool hit = e == piv / PVG;
                pc.x = hit ? v[e].x : pc.x;
                pc.y = hit ? v[e].y : pc.y;
            }
            cb[r] = pc;
        }
        __syncthreads();
        const cplx<T> p = rb[piv];
        const T p2 = abs2(p);
        if (!(p2 > tiny) || !(p2 < T(1) / tiny)) bad = 1;
        const cplx<T> pinv = mk<T>(p.x / p2, -p.y / p2);
        // every entry: v -= (A[r][piv] / p) A[piv][c]; then the pivot row is
        // A[piv][c] / p and the pivot column -A[r][piv] / p (1 / p at the pivot).
        // Both row cases are one multiply-subtract: x = v' - m A[piv][c] with
        // (v', m) = (0, -1 / p) on the pivot row, (v, A[r][piv] / p) elsewhere.
        const bool prow = r == piv;
        const cplx<T> crp = cb[r] * pinv;
        const cplx<T> colv = csel(prow, pinv, -crp);
        const cplx<T> m = csel(prow, -pinv, crp);
#pragma unroll
        for (int e = 0; e < PVE; ++e) {
            const cplx<T> rc = rb[cg + PVG * e];
            cplx<T> x = csel(prow, mk<T>(T(0), T(0)), v[e]) - m * rc;
            const bool pcol = (cg + PVG * e) == piv;
            x.x = pcol ? colv.x : x.x;
            x.y = pcol ? colv.y : x.y;
            v[e] = x;
        }
    }
    cplx<T>* D = static_cast<cplx<T>*>(a.Dbuf) + (long long)js * TB * TB;
#pragma unroll
    for (int e = 0; e < PVE; ++e) D[(cg + PVG * e) * TB + r] = v[e];
    __syncthreads();
    if (threadIdx.x == 0 && bad) *a.flag = 1;
}

// Panel step of panel jp: row-tile workgroups set A[I,J] = -A[I,J] D^-1,
// column-tile workgroups keep A[J,C] in Rbuf and set A[J,C] = D^-1 A[J,C].
template <typename T>
__global__ __launch_bounds__(NT) void gj_panel_kernel(GjArgs a) {
    // the products run over the panel in two halves of 32 through half-size LDS
    // copies (33.5 KB in FP32, 67 KB in FP64 instead of 66.5 and 133)
    __shared__ cplx<T> sP[TB * KLD];
    __shared__ cplx<T> sQ[(TB / 2) * LDT];
    const int js = blockIdx.y;
    const GjMat gm = gj_mat(a, js);
    const int Bp = gm.Bp, nt = Bp / TB;
    if (a.jp >= gm.npiv) return;
    const bool rowt = (int)blockIdx.x < a.ntmax;
    const int t = rowt ? blockIdx.x : blockIdx.x - a.ntmax;
    if (t >= nt || t == a.jp) return;
    cplx<T>* A = static_cast<cplx<T>*>(a.fac) + gm.off;
    const int J0 = a.jp * TB;
    const cplx<T>* D = static_cast<const cplx<T>*>(a.Dbuf) + (long long)js * TB * TB;
    CTile<T> acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j].zero();
    // panel buffers of a front: slots of Bp x 64 entries (rows of J1, rows of
    // J2, columns of J1), column-major with leading dimension 64 / Bp
    const long long slot = (long long)Bp * TB;
    if (rowt) {
        // acc = A[t, J] D
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            __syncthreads();
            load_half_cols(sP, A, Bp, t * TB, J0 + (TB / 2) * h);
            load_half_rows(sQ, D, TB, (TB / 2) * h, 0);
            __syncthreads();
            tile_product<T, TB / 2, KLD, LDT>(sP, sQ, acc);
        }
        store_acc(A, Bp, t * TB, J0, acc, T(-1));
        if (a.save_c)
            store_acc(static_cast<cplx<T>*>(a.Rbuf) + gm.roff + 2 * slot, Bp, t * TB, 0, acc, T(-1));
    } else {
        // acc = D A[J, t]; A[J, t] also goes to the row buffer R
        cplx<T>* R = static_cast<cplx<T>*>(a.Rbuf) + gm.roff + a.rsel * slot;
        const int rl = threadIdx.x & 31, cg = threadIdx.x >> 5;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            __syncthreads();
            load_half_cols(sP, D, TB, 0, (TB / 2) * h);
            load_half_rows(sQ, A, Bp, J0 + (TB / 2) * h, t * TB);
            __syncthreads();
#pragma unroll 4
            for (int e = 0; e < 8; ++e) {
                const int c = cg + 8 * e;
                R[(long long)(t * TB + c) * TB + (TB / 2) * h + rl] = sQ[rl * LDT + c];
            }
            tile_product<T, TB / 2, KLD, LDT>(sP, sQ, acc);
        }
        store_acc(A, Bp, J0, t * TB, acc, T(1));
    }
}

// Trailing update of panel jp: A[I,C] += A[I,J] R[J,C] for I, C outside the
// panel; the pivot tile becomes D^-1.
// acc += P Q for the trailing update, P = Pm(pr0.., pc0..) (64 x 64, leading
// dimension pld) and Q = Qm(0.., qc0..) (leading dimension TB), the k range in
// two halves of 32 through half-size LDS copies
template <typename T>
__device__ __forceinline__ void gj_update_product(cplx<T>* sP, cplx<T>* sQ, const cplx<T>* Pm, long long pld,
                                                  int pr0, int pc0, const cplx<T>* Qm, int qc0,
                                                  CTile<T> (&acc)[2][2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        __syncthreads();   // the previous half's reads are done
        load_half_cols(sP, Pm, pld, pr0, pc0 + (TB / 2) * h);
        load_half_rows(sQ, Qm, TB, (TB / 2) * h, qc0);
        __syncthreads();
        tile_product<T, TB / 2, KLD, LDT>(sP, sQ, acc);
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void gj_update_kernel(GjArgs a) {
    // the products run over the panel in two halves of 32, so that the LDS
    // copies take half a tile each (33.5 KB in FP32, 67 KB in FP64 instead of
    // 66.5 and 133): more workgroups share a CU
    __shared__ cplx<T> sP[TB * KLD];
    __shared__ cplx<T> sQ[(TB / 2) * LDT];
    const int js = blockIdx.y;
    const GjMat gm = gj_mat(a, js);
    const int Bp = gm.Bp, nt = Bp / TB;
    if (a.jp >= gm.npiv) return;
    const int ti = blockIdx.x % a.ntmax, tj = blockIdx.x / a.ntmax;
    if (ti >= nt || tj >= nt) return;
    cplx<T>* A = static_cast<cplx<T>*>(a.fac) + gm.off;
    const int J0 = a.jp * TB;
    if (tj == a.jp) {
        if (ti == a.jp) {
            const cplx<T>* D = static_cast<const cplx<T>*>(a.Dbuf) + (long long)js * TB * TB;
            const int r = threadIdx.x & 63, cg = threadIdx.x >> 6;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int c = cg + 4 * e;
                A[(long long)(J0 + c) * Bp + J0 + r] = D[c * TB + r];
            }
        }
        return;
    }
    if (ti == a.jp) return;
    // GJ_NARROW (a front with a next panel): only the next panel's row and
    // column tiles now, the rest with the next panel's update
    const bool narrow = a.mode == GJ_NARROW && a.jp + 1 < gm.npiv;
    if (narrow && ti != a.jp + 1 && tj != a.jp + 1) return;
    // a front's boundary rows in already eliminated separator columns hold
    // -F_BI F_II^-1, which nothing reads again (the solves use its transpose
    // K^T from the separator rows): not updated
    if (!narrow && a.fr && ti >= gm.npiv && tj < a.jp) return;
    const long long slot = (long long)Bp * TB;
    const cplx<T>* R = static_cast<const cplx<T>*>(a.Rbuf) + gm.roff + a.rsel * slot;
    // the first half's loads are issued before the accumulators', so that its
    // LDS copies wait for them alone
    CTile<T> acc[2][2];
    load_half_cols(sP, A, Bp, ti * TB, J0);
    load_half_rows(sQ, R, TB, 0, tj * TB);
    load_acc(acc, A, Bp, ti * TB, tj * TB);
    __syncthreads();
    tile_product<T, TB / 2, KLD, LDT>(sP, sQ, acc);
    __syncthreads();
    load_half_cols(sP, A, Bp, ti * TB, J0 + TB / 2);
    load_half_rows(sQ, R, TB, TB / 2, tj * TB);
    __syncthreads();
    tile_product<T, TB / 2, KLD, LDT>(sP, sQ, acc);
    if (a.mode == GJ_COMBINED && ti != a.jp - 1 && tj != a.jp - 1) {
        // the deferred update of panel J1 = jp - 1: its columns (slot 2) times
        // its rows (slot 0)
        const cplx<T>* R1 = static_cast<const cplx<T>*>(a.Rbuf) + gm.roff;
        gj_update_product(sP, sQ, R1 + 2 * slot, Bp, ti * TB, 0, R1, tj * TB, acc);
    }
    store_acc(A, Bp, ti * TB, tj * TB, acc, T(1));
}

// Trailing update with real-split bf16 products (ASP_PREC_BF16X3): the same
// tiles as gj_update_kernel<float>; P = A[I,J] and Q = R[J,C] are split into
// bf16 hi/lo planes in LDS (k contiguous), and every real product is
// hi*hi + hi*lo + lo*hi on the 16x16x32 bf16 matrix-core instruction with FP32
// accumulation onto the FP32 tile of A.
constexpr int LDB = TB + 8;   // padded k stride of a bf16 plane

struct SplitPlanes {          // one 64 x 64 complex tile: [row][k] planes
    __bf16 rh[TB * LDB], rl[TB * LDB], ih[TB * LDB], il[TB * LDB];
};

__device__ __forceinline__ void split_store(SplitPlanes& S, int i, int k, zf v) {
    const __bf16 rh = (__bf16)v.x, ih = (__bf16)v.y;
    S.rh[i * LDB + k] = rh;
    S.rl[i * LDB + k] = (__bf16)(v.x - (float)rh);
    S.ih[i * LDB + k] = ih;
    S.il[i * LDB + k] = (__bf16)(v.y - (float)ih);
}

__device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }


__global__ __launch_bounds__(NT) void gj_update_bf16x3_kernel(GjArgs a) {
    __shared__ SplitPlanes sP, sQ;   // P[r][k], Q^T[c][k]
    const int js = blockIdx.y;
    const GjMat gm = gj_mat(a, js);
    const int Bp = gm.Bp, nt = Bp / TB;
    if (a.jp >= gm.npiv) return;
    const int ti = blockIdx.x % a.ntmax, tj = blockIdx.x / a.ntmax;
    if (ti >= nt || tj >= nt) return;
    zf* A = static_cast<zf*>(a.fac) + gm.off;
    const int J0 = a.jp * TB;
    if (tj == a.jp) {
        if (ti == a.jp) {
            const zf* D = static_cast<const zf*>(a.Dbuf) + (long long)js * TB * TB;
            const int r = threadIdx.x & 63, cg = threadIdx.x >> 6;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int c = cg + 4 * e;
                A[(long long)(J0 + c) * Bp + J0 + r] = D[c * TB + r];
            }
        }
        return;
    }
    if (ti == a.jp) return;
    // a front's boundary rows in already eliminated separator columns hold
    // -F_BI F_II^-1, which nothing reads again (the solves use its transpose
    // K^T from the separator rows): not updated
    if (a.fr && ti >= gm.npiv && tj < a.jp) return;
    const zf* R = static_cast<const zf*>(a.Rbuf) + gm.roff;
    {
        // P(r, k) = A(ti*64 + r, J0 + k): reads coalesced over r
        const int r = threadIdx.x & 63, kg = threadIdx.x >> 6;
#pragma unroll 4
        for (int e = 0; e < 16; ++e) {
            const int k = kg + 4 * e;
            split_store(sP, r, k, A[(long long)(J0 + k) * Bp + ti * TB + r]);
        }
        // Q^T(c, k) = R(k, tj*64 + c) at [(tj*64 + c) * 64 + k]: reads coalesced over k
        const int k2 = threadIdx.x & 63, cg = threadIdx.x >> 6;
#pragma unroll 4
        for (int e = 0; e < 16; ++e) {
            const int c = cg + 4 * e;
            split_store(sQ, c, k2, R[(long long)(tj * TB + c) * TB + k2]);
        }
    }
    CTile<float> acc[2][2];
    load_acc(acc, A, Bp, ti * TB, tj * TB);
    __syncthreads();
    // C^T = Q^T P^T: MFMA rows are columns c of C, MFMA columns rows r
    const int l = lane_id(), w = wave_id();
    const int R0 = 32 * (w >> 1), C0 = 32 * (w & 1);
    const int li = l & 15, kq = 8 * (l >> 4);
#pragma unroll
    for (int kc = 0; kc < TB; kc += 32) {
        bf16x8 qrh[2], qrl[2], qih[2], qil[2], prh[2], prl[2], pih[2], pil[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int qo = (C0 + 16 * t + li) * LDB + kc + kq;
            qrh[t] = ld8(sQ.rh + qo);
            qrl[t] = ld8(sQ.rl + qo);
            qih[t] = ld8(sQ.ih + qo);
            qil[t] = ld8(sQ.il + qo);
            const int po = (R0 + 16 * t + li) * LDB + kc + kq;
            prh[t] = ld8(sP.rh + po);
            prl[t] = ld8(sP.rl + po);
            pih[t] = ld8(sP.ih + po);
            pil[t] = ld8(sP.il + po);
        }
#pragma unroll
        for (int ta = 0; ta < 2; ++ta)
#pragma unroll
            for (int tb = 0; tb < 2; ++tb) {
                CTile<float>& c = acc[ta][tb];
                // re += Qr Pr - Qi Pi ; im += Qr Pi + Qi Pr
                c.re = split_mac(qrh[ta], qrl[ta], prh[tb], prl[tb], c.re);
                c.re = split_mac(qih[ta], qil[ta], neg8(pih[tb]), neg8(pil[tb]), c.re);
                c.im = split_mac(qrh[ta], qrl[ta], pih[tb], pil[tb], c.im);
                c.im = split_mac(qih[ta], qil[ta], prh[tb], prl[tb], c.im);
            }
    }
    store_acc(A, Bp, ti * TB, tj * TB, acc, 1.0f);
}

// ---------------------------------------------------------------------------
// solves
// ---------------------------------------------------------------------------
struct Solve3Args {
    const SubDesc* desc;
    const int* jobs;
    int njobs;
    const void* fac;
    void* Y;               // [chunk][job][k][Bmax][RW]
    const void* G;         // gathered M data, same layout
    long long yj;          // entries per (chunk, job)
    int Bmax;
    int k, fwd;
    int n;
    long long N, S;
    AxisTables ax;
    const zd* e3;
    const zd* gv3;
    int in_mode;
    const zd* Win;
    zd* Wout;
    int ws;
    int two_sided;
    int out_mode0, out_mode1;
    zd* out0;
    zd* out1;
    const zd* U;
    const int* act;
    int nact;
};

// Operands of one batch (4 k-steps, 16 columns) of a block step: RT row tiles
// of S_k^-1 and the raw terms of t(c) = g(c) - cf e(c) v(c).
template <typename T, int RT>
struct StepBatch {
    cplx<T> m[RT][4], g[4], v[4];
    zd e[4];
};

template <typename T, int RT, bool with_g>
__device__ __forceinline__ void load_batch(StepBatch<T, RT>& B, const cplx<T>* __restrict__ Mk,
                                           int Bp, int r0, int c0, const cplx<T>* __restrict__ g,
                                           const cplx<T>* __restrict__ v,
                                           const zd* __restrict__ e, bool with_v) {
    const int l = lane_id();
    const int li = l & 15, lk = l >> 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int c = c0 + 4 * u + lk;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) B.m[rt][u] = Mk[(long long)c * Bp + r0 + 16 * rt + li];
        if (with_g) B.g[u] = g[(long long)c * RW + li];
        if (with_v) {
            B.v[u] = v[(long long)c * RW + li];
            B.e[u] = e[c];
        }
    }
}

template <typename T, int RT, bool with_g>
__device__ __forceinline__ void mac_batch(CTile<T> (&acc)[RT], const StepBatch<T, RT>& B, zd cf,
                                          bool with_v) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        cplx<T> t = csel(with_g, B.g[u], mk<T>(T(0), T(0)));
        if (with_v) t = t - ccast<T>(cf * B.e[u]) * B.v[u];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) cmac(acc[rt], B.m[rt][u], t);
    }
}

// acc += S_k^-1 (RT row tiles from r0) t over the batches b = w, w + NW, ...
// of 16 columns, where t(c) = g(c) - cf e(c) v(c) (with_g) or -cf e(c) v(c):
// g the gathered data, v the previous / next block's vector, cf the x1
// coupling without its cross-section factor e.  The next batch's operands are
// loaded before the current batch's products.
template <typename T, int NW, int RT, bool with_g>
__device__ __forceinline__ void step_product(CTile<T> (&acc)[RT], const cplx<T>* __restrict__ Mk,
                                             int Bp, int r0, const cplx<T>* __restrict__ g,
                                             const cplx<T>* __restrict__ v,
                                             const zd* __restrict__ e, zd cf, bool with_v) {
    const int nb = Bp / 16;
    int b = wave_id();
    if (b >= nb) return;
    StepBatch<T, RT> cur, nxt;
    load_batch<T, RT, with_g>(cur, Mk, Bp, r0, 16 * b, g, v, e, with_v);
    for (;;) {
        const int bn = b + NW;
        if (bn < nb) load_batch<T, RT, with_g>(nxt, Mk, Bp, r0, 16 * bn, g, v, e, with_v);
        mac_batch<T, RT, with_g>(acc, cur, cf, with_v);
        if (bn >= nb) break;
        cur = nxt;
        b = bn;
    }
}

// One block step for RT x 16 rows of every job and one chunk of 16
// right-hand sides; NW waves split the inner dimension and reduce through LDS
// in a fixed order.  R/L data (nonzero on one line of the cross-section)
// enters through a separate product over the columns of that line.
template <typename T, int NW, int RT>
__global__ __launch_bounds__(64 * NW) void solve3d_step_kernel(Solve3Args a) {
    __shared__ cplx<T> red[NW][RT][64][4];
    const int js = blockIdx.y, chunk = blockIdx.z;
    const SubDesc d = a.desc[a.jobs[js]];
    const int Bp = d.B, L = d.L;
    const int r0 = blockIdx.x * 16 * RT;
    if (r0 >= Bp) return;
    const int k = a.k;
    const int l = lane_id(), w = wave_id();
    const int li = l & 15, lk = l >> 4;
    const cplx<T>* Mk = static_cast<const cplx<T>*>(a.fac) + d.fac_off + (long long)k * Bp * Bp;
    cplx<T>* Yc = static_cast<cplx<T>*>(a.Y) + ((long long)chunk * a.njobs + js) * a.yj;
    const long long blk = (long long)a.Bmax * RW;
    const zd* e = a.e3 + d.vec_off;
    const int slot_l = chunk * RW + li;       // this lane's right-hand side in the B operand
    const bool live_l = slot_l < a.nact;
    CTile<T> acc[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) acc[rt].zero();
    const bool skip = !a.fwd && k == a.n - 1;   // x_n = y_n
    // rows r0 + 16 RT may pass Bp when Bp is not a multiple of 16 RT: the
    // last row tiles then read (and later drop) the next block's rows
    if (!skip) {
        if (a.fwd) {
            const cplx<T>* yp = Yc + (long long)(k - 1) * blk;
            const zd sk = a.ax.sh[k];                      // coupling of blocks k-1, k
            if (a.in_mode == IN_GRID) {
                const cplx<T>* g = static_cast<const cplx<T>*>(a.G) +
                                   ((long long)chunk * a.njobs + js) * a.yj + (long long)k * blk;
                step_product<T, NW, RT, true>(acc, Mk, Bp, r0, g, yp, e, sk, k > 0);
            } else {
                if (k > 0) step_product<T, NW, RT, false>(acc, Mk, Bp, r0, nullptr, yp, e, sk, true);
                // data on the line next to the Dirichlet data: columns c = L i2 + dl
                const int dl = (d.kind == ASP_SUB_R) ? 0 : L - 1;
                const zd* gv = a.gv3 + d.vec_off;
                const zd* win = a.Win + (long long)js * a.S * a.ws;
                const zd is1 = a.ax.inv_s[k];
                const int nsteps = (a.n + 3) / 4;
                for (int s4 = w; s4 < nsteps; s4 += NW) {
                    const int i2 = 4 * s4 + lk;
                    const int i2c = min(i2, a.n - 1);
                    const int c = L * i2c + dl;
                    const zd wv = win[((long long)k + (long long)a.n * i2c) * a.ws + slot_l];
                    const bool on = i2 < a.n && live_l;
                    const cplx<T> t = csel(on, ccast<T>((is1 * gv[c]) * wv), mk<T>(T(0), T(0)));
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
                        cmac(acc[rt], Mk[(long long)c * Bp + r0 + 16 * rt + li], t);
                }
            }
        } else {
            const cplx<T>* xn = Yc + (long long)(k + 1) * blk;
            const zd sk = a.ax.sh[k + 1];                  // coupling of blocks k, k+1
            step_product<T, NW, RT, false>(acc, Mk, Bp, r0, nullptr, xn, e, -sk, true);
        }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[w][rt][l][v] = mk<T>(acc[rt].re[v], acc[rt].im[v]);
    __syncthreads();
    // one output per thread: row tile rt, lane l2, element v
    const int tid = threadIdx.x;
    if (tid >= RT * 256) return;
    const int v = tid & 3, l2 = (tid >> 2) & 63, rt = tid >> 8;
    cplx<T> s = red[0][rt][l2][v];
#pragma unroll
    for (int q = 1; q < NW; ++q) s = s + red[q][rt][l2][v];
    const int row = r0 + 16 * rt + Mfma<T>::row(l2, v);
    if (row >= Bp) return;
    const int slot = chunk * RW + (l2 & 15);
    cplx<T>* yk = Yc + (long long)k * blk + (long long)row * RW + (l2 & 15);
    if (a.fwd) {
        *yk = s;
        return;
    }
    const cplx<T> x = csel(skip, *yk, *yk - s);
    *yk = x;
    const int B = a.n * L;
    if (row >= B || slot >= a.nact) return;
    const int i3l = row % L, i2 = row / L;
    const int line = d.lo + i3l;
    if (line < d.xs || line > d.xe) return;
    const int rhs = a.act ? a.act[slot] : slot;
    const long long gidx = (long long)rhs * a.N + k + (long long)a.n * i2 + a.S * (line - 1);
    const zd xv = ccast<double>(x);
    const int side = a.two_sided ? js : 0;
    const int mode = side ? a.out_mode1 : a.out_mode0;
    zd* out = side ? a.out1 : a.out0;
    if (mode == OUT_GRID_STORE) out[gidx] = xv;
    else if (mode == OUT_GRID_ADD_U) out[gidx] = a.U[gidx] + xv;
    else out[gidx] = out[gidx] + xv;
    if (a.Wout) {
        // the data entering the next problem of this sweep: R_p hands over its
        // last line, L_p its first line, each with u~_{p,p} added
        const int hand = (d.kind == ASP_SUB_R) ? d.xe : d.xs;
        if (line == hand)
            a.Wout[((long long)js * a.S + k + (long long)a.n * i2) * a.ws + slot] = a.U[gidx] + xv;
    }
}

// G[chunk][job][k][j][16] = r at block k, entry j if its line lies in X_q, else 0
template <typename T>
__global__ __launch_bounds__(256) void gather3d_kernel(const SubDesc* desc, const int* jobs,
                                                       int njobs, const zd* r, const int* act,
                                                       int nact, cplx<T>* G, long long yj,
                                                       int Bmax, int n, long long N, long long S) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    const int c = idx >> 4, li = idx & 15;
    const int k = blockIdx.y;
    const int js = blockIdx.z % njobs, chunk = blockIdx.z / njobs;
    if (c >= Bmax) return;
    const SubDesc d = desc[jobs[js]];
    zd v = mk(0.0, 0.0);
    const int slot = chunk * RW + li;
    if (c < n * d.L && slot < nact) {
        const int line = d.lo + c % d.L;
        if (line >= d.xs && line <= d.xe) {
            const int rhs = act ? act[slot] : slot;
            v = r[(long long)rhs * N + k + (long long)n * (c / d.L) + S * (line - 1)];
        }
    }
    G[((long long)chunk * njobs + js) * yj + ((long long)k * Bmax + c) * RW + li] = ccast<T>(v);
}

// W[job][i1 + n i2][slot] = U(i1, i2, line_job)
__global__ __launch_bounds__(256) void plane3d_kernel(const zd* U, int line0, int line1, zd* W,
                                                      int ws, const int* act, int nact, int n,
                                                      long long N, long long S) {
    const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
    if (p >= S) return;
    const int slot = blockIdx.y, job = blockIdx.z;
    const int rhs = act ? act[slot] : slot;
    const int line = job ? line1 : line0;
    W[((long long)job * S + p) * ws + slot] = U[(long long)rhs * N + S * (line - 1) + p];
}

// z = U + C on lines 1..split, z += C on lines split+1..upto; with all_u
// (z holding the R outputs without U) also z += U on lines split+1..lines
__global__ __launch_bounds__(256) void combine3d_kernel(zd* z, const zd* U, const zd* C, int split,
                                                        int upto, int lines, int all_u,
                                                        const int* act, long long N, long long S) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= S * lines) return;
    const int rhs = act ? act[blockIdx.y] : blockIdx.y;
    const long long g = (long long)rhs * N + i;
    const int line = (int)(i / S) + 1;
    if (line <= split) {
        z[g] = U[g] + C[g];
    } else if (line <= upto) {
        z[g] = all_u ? z[g] + C[g] + U[g] : z[g] + C[g];
    } else {
        z[g] = z[g] + U[g];
    }
}

AxisTables axis_of(const asp_plan* P) {
    AxisTables t;
    t.sh = P->d_axis;
    t.inv_sh2 = P->d_axis + P->n + 1;
    t.inv_s = P->d_axis + 2 * P->n + 1;
    return t;
}

}  // namespace

hipError_t launch_form3d(const asp_plan* P, const int* jobs, int njobs, int k, hipStream_t st) {
    Form3Args a;
    a.desc = P->d_desc;
    a.jobs = jobs;
    a.fac = P->d_fac;
    a.ax = axis_of(P);
    a.subtab = P->d_subtab;
    a.ksq = P->d_ksq;
    a.e3 = P->d_e3;
    a.n = P->n;
    a.k = k;
    a.S = P->S;
    dim3 grid((P->Bmax + 255) / 256, P->Bmax, njobs);
    if (P->prec != ASP_PREC_FP64)
        hipLaunchKernelGGL(form3d_kernel<float>, grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(form3d_kernel<double>, grid, dim3(256), 0, st, a);
    return hipGetLastError();
}

namespace {

// jobs per launch above which the pivot tiles use the four-wave workgroups
// (two sixteen-wave workgroups fit a CU: 512 run at once on 256 CUs)
constexpr int PIVOT_MANY = 512;

void launch_gj(const asp_plan* P, const GjArgs& a, int njobs, hipStream_t st) {
    dim3 g0(njobs), g1(2 * a.ntmax, njobs), g2(a.ntmax * a.ntmax, njobs);
    if (P->prec != ASP_PREC_FP64) {
        if (njobs > PIVOT_MANY)
            hipLaunchKernelGGL((gj_pivot_kernel<float, 4>), g0, dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((gj_pivot_kernel<float, 16>), g0, dim3(1024), 0, st, a);
        hipLaunchKernelGGL(gj_panel_kernel<float>, g1, dim3(NT), 0, st, a);
        if (P->prec == ASP_PREC_BF16X3)
            hipLaunchKernelGGL(gj_update_bf16x3_kernel, g2, dim3(NT), 0, st, a);
        else
            hipLaunchKernelGGL(gj_update_kernel<float>, g2, dim3(NT), 0, st, a);
    } else {
        if (njobs > PIVOT_MANY)
            hipLaunchKernelGGL((gj_pivot_kernel<double, 4>), g0, dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((gj_pivot_kernel<double, 16>), g0, dim3(1024), 0, st, a);
        hipLaunchKernelGGL(gj_panel_kernel<double>, g1, dim3(NT), 0, st, a);
        hipLaunchKernelGGL(gj_update_kernel<double>, g2, dim3(NT), 0, st, a);
    }
}

}  // namespace

hipError_t launch_gj_fronts(const asp_plan* P, const NdFront* fr, int nfr, void* Flevel, int jp,
                            int ntmax, void* Rbuf, void* Dbuf, int mode, hipStream_t st) {
    const size_t esz = P->prec != ASP_PREC_FP64 ? sizeof(zf) : sizeof(zd);
    constexpr int YMAX = 65535;
    for (int y0 = 0; y0 < nfr; y0 += YMAX) {
        GjArgs a{};
        a.fr = fr + y0;
        a.fac = Flevel;
        a.Rbuf = Rbuf;
        a.Dbuf = static_cast<char*>(Dbuf) + (size_t)y0 * TB * TB * esz;
        a.flag = P->d_flag;
        a.jp = jp;
        a.ntmax = ntmax;
        a.mode = mode;
        a.rsel = mode == GJ_COMBINED ? 1 : 0;
        a.save_c = mode == GJ_NARROW ? 1 : 0;
        launch_gj(P, a, std::min(YMAX, nfr - y0), st);
    }
    return hipGetLastError();
}

hipError_t launch_gj3d(const asp_plan* P, const int* jobs, int njobs, int k, int jp, void* Rbuf,
                       void* Dbuf, hipStream_t st) {
    GjArgs a;
    a.desc = P->d_desc;
    a.jobs = jobs;
    a.fr = nullptr;
    a.mode = GJ_FULL;
    a.rsel = 0;
    a.save_c = 0;
    a.fac = P->d_fac;
    a.Rbuf = Rbuf;
    a.Dbuf = Dbuf;
    a.flag = P->d_flag;
    a.rstride = (long long)P->Bmax * TB;
    a.k = k;
    a.jp = jp;
    a.ntmax = P->Bmax / TB;
    launch_gj(P, a, njobs, st);
    return hipGetLastError();
}

hipError_t launch_gj_blocks(const asp_plan* P, const SubDesc* desc, const int* jobs, int njobs,
                            void* fac, int k, int jp, int Bmax, void* Rbuf, void* Dbuf,
                            hipStream_t st) {
    GjArgs a;
    a.desc = desc;
    a.jobs = jobs;
    a.fr = nullptr;
    a.mode = GJ_FULL;
    a.rsel = 0;
    a.save_c = 0;
    a.fac = fac;
    a.Rbuf = Rbuf;
    a.Dbuf = Dbuf;
    a.flag = P->d_flag;
    a.rstride = (long long)Bmax * TB;
    a.k = k;
    a.jp = jp;
    a.ntmax = Bmax / TB;
    launch_gj(P, a, njobs, st);
    return hipGetLastError();
}

hipError_t launch_block_step(const asp_plan* P, const BlockSolve& s, int k, int fwd,
                             hipStream_t st) {
    Solve3Args a{};
    a.desc = s.desc;
    a.jobs = s.jobs;
    a.njobs = s.njobs;
    a.fac = s.fac;
    a.Y = s.Y;
    a.G = s.G;
    a.yj = (long long)P->n * s.Bmax * RW;
    a.Bmax = s.Bmax;
    a.k = k;
    a.fwd = fwd;
    a.n = P->n;
    a.N = P->N;
    a.S = P->S;
    a.ax = axis_of(P);
    a.e3 = s.e;
    a.gv3 = nullptr;
    a.in_mode = IN_GRID;
    a.nact = s.nact;
    const int chunks = (s.nact + RW - 1) / RW;
    if (s.narrow) {
        dim3 grid(s.Bmax / 16, s.njobs, chunks);
        if (P->prec != ASP_PREC_FP64)
            hipLaunchKernelGGL((solve3d_step_kernel<float, 16, 1>), grid, dim3(1024), 0, st, a);
        else
            hipLaunchKernelGGL((solve3d_step_kernel<double, 8, 1>), grid, dim3(512), 0, st, a);
    } else {
        dim3 grid(s.Bmax / 32, s.njobs, chunks);
        if (P->prec != ASP_PREC_FP64)
            hipLaunchKernelGGL((solve3d_step_kernel<float, 8, 2>), grid, dim3(512), 0, st, a);
        else
            hipLaunchKernelGGL((solve3d_step_kernel<double, 8, 2>), grid, dim3(512), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_gather3d(const asp_plan* P, const int* jobs, int njobs, const zd* r,
                           const int* act, int nact, hipStream_t st) {
    const int chunks = (nact + RW - 1) / RW;
    const long long yj = (long long)P->n * P->Bmax * RW;
    dim3 grid((P->Bmax * RW + 255) / 256, P->n, njobs * chunks);
    if (P->prec != ASP_PREC_FP64)
        hipLaunchKernelGGL(gather3d_kernel<float>, grid, dim3(256), 0, st, P->d_desc, jobs, njobs, r,
                           act, nact, static_cast<zf*>(P->d_g3), yj, P->Bmax, P->n, P->N, P->S);
    else
        hipLaunchKernelGGL(gather3d_kernel<double>, grid, dim3(256), 0, st, P->d_desc, jobs, njobs,
                           r, act, nact, static_cast<zd*>(P->d_g3), yj, P->Bmax, P->n, P->N, P->S);
    return hipGetLastError();
}

hipError_t launch_solve3d_step(const asp_plan* P, const Solve3Launch& L, int k, int fwd,
                               hipStream_t st) {
    Solve3Args a;
    a.desc = P->d_desc;
    a.jobs = L.jobs;
    a.njobs = L.njobs;
    a.fac = P->d_fac;
    a.Y = P->d_y3;
    a.G = P->d_g3;
    a.yj = (long long)P->n * P->Bmax * RW;
    a.Bmax = P->Bmax;
    a.k = k;
    a.fwd = fwd;
    a.n = P->n;
    a.N = P->N;
    a.S = P->S;
    a.ax = axis_of(P);
    a.e3 = P->d_e3;
    a.gv3 = P->d_gv3;
    a.in_mode = L.in_mode;
    a.Win = L.Win;
    a.Wout = L.Wout;
    a.ws = P->ws3;
    a.two_sided = L.two_sided ? 1 : 0;
    a.out_mode0 = L.out_mode[0];
    a.out_mode1 = L.out_mode[1];
    a.out0 = L.out[0];
    a.out1 = L.out[1];
    a.U = L.Ugrid;
    a.act = L.act;
    a.nact = L.nact;
    const int chunks = (L.nact + RW - 1) / RW;
    // the sweeps (two problems per step) are latency bound: 16 rows per block and
    // 16 wavefronts over the inner dimension; the M-solves share each loaded
    // vector between two row tiles
    if (L.two_sided) {
        // (FP64 operands take twice the registers: 8 wavefronts, 256 registers each)
        dim3 grid(P->Bmax / 16, L.njobs, chunks);
        if (P->prec != ASP_PREC_FP64)
            hipLaunchKernelGGL((solve3d_step_kernel<float, 16, 1>), grid, dim3(1024), 0, st, a);
        else
            hipLaunchKernelGGL((solve3d_step_kernel<double, 8, 1>), grid, dim3(512), 0, st, a);
    } else {
        dim3 grid(P->Bmax / 32, L.njobs, chunks);
        if (P->prec != ASP_PREC_FP64)
            hipLaunchKernelGGL((solve3d_step_kernel<float, 8, 2>), grid, dim3(512), 0, st, a);
        else
            hipLaunchKernelGGL((solve3d_step_kernel<double, 8, 2>), grid, dim3(512), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_plane3d(const asp_plan* P, const zd* U, int line0, int line1, zd* W,
                          const int* act, int nact, hipStream_t st) {
    dim3 grid((unsigned)((P->S + 255) / 256), nact, 2);
    hipLaunchKernelGGL(plane3d_kernel, grid, dim3(256), 0, st, U, line0, line1, W, P->ws3, act,
                       nact, P->n, P->N, P->S);
    return hipGetLastError();
}

hipError_t launch_combine3d(const asp_plan* P, zd* z, const zd* U, const zd* C, int split,
                            int upto, bool all_u, const int* act, int nact, hipStream_t st) {
    const int lines = all_u ? (int)(P->N / P->S) : upto;
    const long long cnt = P->S * lines;
    dim3 grid((unsigned)((cnt + 255) / 256), nact);
    hipLaunchKernelGGL(combine3d_kernel, grid, dim3(256), 0, st, z, U, C, split, upto, lines,
                       all_u ? 1 : 0, act, P->N, P->S);
    return hipGetLastError();
}
