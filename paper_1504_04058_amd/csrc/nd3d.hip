// Kernels of the nested-dissection path (Section 4.1): front assembly with
// extend-add, the copy of the eliminated fronts into the factor, and the
// forward / backward passes of the multifrontal solve.
//
// Front rows: [0, ipad) the separator part (column c of the node's separator
// list at rows c L .. c L + L - 1, rows from nI L identity padding), [ipad, f)
// the boundary part (boundary column b at rows ipad + b L .., then zero
// padding).  A slab vector holds the n^2 L unknowns of one problem at
// (column i1 + n i2) L + (sweep line - lo), 16 right-hand sides per entry.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "asp_internal.h"
#include "mfma.h"

namespace {

constexpr int RW = 16;       // right-hand sides per chunk
constexpr int NT = 256;      // threads of a workgroup
constexpr int RT = 4;        // 16-row tiles of one product workgroup (64 rows)
constexpr int NW = 4;        // waves splitting the inner dimension of a product
constexpr int YMAX = 65535;  // largest grid y

struct Part {
    int c;      // front column (separator columns first, then boundary columns); -1 padding
    int k;      // sweep line within the column
    int part;   // 0 separator, 1 boundary, 2 separator padding, 3 boundary padding
};

__device__ __forceinline__ Part decode(int r, int ipad, int nI, int nB, int L) {
    Part p;
    if (r < ipad) {
        const int c = r / L;
        const bool in = r < nI * L;
        p.c = in ? c : -1;
        p.k = r - c * L;
        p.part = in ? 0 : 2;
    } else {
        const int q = r - ipad, b = q / L;
        const bool in = q < nB * L;
        p.c = in ? nI + b : -1;
        p.k = q - b * L;
        p.part = in ? 1 : 3;
    }
    return p;
}

__device__ __forceinline__ int front_col(const int* cols, const NdNode& nd, int c) {
    return c < nd.nI ? cols[nd.i_off + c] : cols[nd.b_off + c - nd.nI];
}

struct AsmArgs {
    const NdFront* fr;       // every front
    long long fbase;         // first front of this launch
    long long child0;        // first front of the next level, -1: none
    int nn, nnc;             // nodes of this level / of the next level
    long long front0;        // first front of this level
    const NdNode* nodes;
    const int* cols;
    const int* inv;
    void* F;
    const void* Fc;
    AxisTables ax;
    const zd* subtab;
    const double* ksq;
    const SubDesc* desc;
    int n;
    long long S;
};

constexpr int CPW = 16;      // front columns of one assembly / copy-out workgroup

// F(r, c): the symmetric-form couplings of the 7-point operator between the
// unknowns of rows r and c if one of them is a separator unknown, plus the
// children's Schur complements on the pairs they share; identity / zero on
// the padding.  One workgroup per CPW consecutive front columns: what depends
// on a column (its part and line, grid point, the children's columns) is
// decoded once into LDS, each thread decodes a row once and writes it in all
// CPW columns (one coalesced row segment per wave and column).
template <typename T>
__global__ __launch_bounds__(NT) void nd_assemble_kernel(AsmArgs a) {
    const long long fi = a.fbase + blockIdx.y;
    const NdFront F = a.fr[fi];
    const int c0 = blockIdx.x * CPW;
    if (c0 >= F.f) return;
    const int nc = min(CPW, F.f - c0);
    const NdNode nd = a.nodes[F.node];
    const int L = F.L;
    const SubDesc d = a.desc[F.sub];
    const zd* sh3 = a.subtab + d.tab_off;   // s3 at the half lines lo - 1/2 ..
    const zd* ish3 = sh3 + L + 1;           // 1 / (s3 h^2)
    const zd* is3 = sh3 + 2 * L + 1;        // 1 / s3
    __shared__ int s_pk[CPW];               // part | line << 2
    __shared__ int s_col[CPW];              // grid column, -1 padding
    __shared__ int s_12[CPW];               // i1 | i2 << 16
    __shared__ const cplx<T>* s_u[2][CPW];  // the children's columns from their row ipad, or null
    int io[2] = {-1, -1};
    if (a.child0 >= 0) {
        io[0] = nd.inv_off[0];
        io[1] = nd.inv_off[1];
    }
    if (threadIdx.x < nc) {
        const int c = c0 + threadIdx.x;
        const Part pc = decode(c, F.ipad, nd.nI, nd.nB, L);
        s_pk[threadIdx.x] = pc.part | (pc.k << 2);
        const int colc = pc.part < 2 ? front_col(a.cols, nd, pc.c) : -1;
        s_col[threadIdx.x] = colc;
        s_12[threadIdx.x] = colc < 0 ? 0 : (colc % a.n) | ((colc / a.n) << 16);
        for (int ch = 0; ch < 2; ++ch) {
            const cplx<T>* u = nullptr;
            if (pc.part < 2 && io[ch] >= 0) {
                const int cc = a.inv[io[ch] + pc.c];
                if (cc >= 0) {
                    const NdFront C = a.fr[a.child0 + (long long)F.sub * a.nnc + nd.ch[ch]];
                    u = static_cast<const cplx<T>*>(a.Fc) + C.foff +
                        (long long)(C.ipad + cc * L + pc.k) * C.f + C.ipad;
                }
            }
            s_u[ch][threadIdx.x] = u;
        }
    }
    __syncthreads();
    cplx<T>* out0 = static_cast<cplx<T>*>(a.F) + F.foff + (long long)c0 * F.f;
    for (int r = threadIdx.x; r < F.f; r += NT) {
        const Part pr = decode(r, F.ipad, nd.nI, nd.nB, L);
        const int k = pr.k;
        const bool live = pr.part < 2;
        const bool rsep = pr.part == 0;
        const int colr = live ? front_col(a.cols, nd, pr.c) : -1;
        const int i1r = live ? colr % a.n : 0, i2r = live ? colr / a.n : 0;
        const int cr0 = live && io[0] >= 0 ? a.inv[io[0] + pr.c] : -1;
        const int cr1 = live && io[1] >= 0 ? a.inv[io[1] + pr.c] : -1;
        for (int q = 0; q < nc; ++q) {
            const int c = c0 + q;
            const int cpk = s_pk[q], cpart = cpk & 3, ck = cpk >> 2;
            cplx<T>* out = out0 + (long long)q * F.f;
            if (cpart >= 2 || !live) {
                const bool one = r == c && (cpart == 2 || (cpart < 2 && pr.part == 2));
                out[r] = mk<T>(one ? T(1) : T(0), T(0));
                continue;
            }
            zd val = mk(0.0, 0.0);
            if (cpart == 0 || rsep) {
                const int colc = s_col[q];
                if (colr == colc) {
                    if (k == ck) {
                        const zd s23 = a.ax.inv_s[i2r] * ish3[k];
                        const zd s13 = a.ax.inv_s[i1r] * ish3[k];
                        const zd s12 = a.ax.inv_s[i1r] * a.ax.inv_sh2[i2r];
                        const zd cf1 = (a.ax.sh[i1r + 1] + a.ax.sh[i1r]) * s23;
                        const zd cf2 = (a.ax.sh[i2r + 1] + a.ax.sh[i2r]) * s13;
                        const zd cf3 = (sh3[k + 1] + sh3[k]) * s12;
                        const long long g = (long long)colr + a.S * (d.lo - 1 + k);
                        val = ((a.ksq[g] * a.ax.inv_s[i1r]) * a.ax.inv_s[i2r]) * is3[k] - (cf1 + cf2 + cf3);
                    } else if (k - ck == 1 || ck - k == 1) {
                        val = sh3[max(k, ck)] * (a.ax.inv_s[i1r] * a.ax.inv_sh2[i2r]);
                    }
                } else if (k == ck) {
                    const int i1c = s_12[q] & 0xffff, i2c = s_12[q] >> 16;
                    if (i2r == i2c && (i1r - i1c == 1 || i1c - i1r == 1))
                        val = a.ax.sh[max(i1r, i1c)] * (a.ax.inv_s[i2r] * ish3[k]);
                    else if (i1r == i1c && (i2r - i2c == 1 || i2c - i2r == 1))
                        val = a.ax.sh[max(i2r, i2c)] * (a.ax.inv_s[i1r] * ish3[k]);
                }
            }
            const cplx<T>* u0 = s_u[0][q];
            const cplx<T>* u1 = s_u[1][q];
            if (u0 && cr0 >= 0) val = val + ccast<double>(u0[cr0 * L + k]);
            if (u1 && cr1 >= 0) val = val + ccast<double>(u1[cr1 * L + k]);
            out[r] = ccast<T>(val);
        }
    }
}

// factor block [F_II^-1 | F_II^-1 F_IB] = the first ipad rows of the front;
// one workgroup per CPW consecutive front columns
template <typename T>
__global__ __launch_bounds__(NT) void nd_copyout_kernel(const NdFront* fr, const void* F, void* fac) {
    const NdFront f = fr[blockIdx.y];
    const int c0 = blockIdx.x * CPW;
    const int c1 = min(c0 + CPW, f.f);
    const cplx<T>* src = static_cast<const cplx<T>*>(F) + f.foff;
    cplx<T>* dst = static_cast<cplx<T>*>(fac) + f.moff;
    for (int c = c0; c < c1; ++c)
        for (int r = threadIdx.x; r < f.ipad; r += NT)
            dst[(long long)c * f.ipad + r] = src[(long long)c * f.f + r];
}

struct SolveNdArgs {
    const NdFront* fr;
    const NdNode* nodes;
    const int* cols;
    const int* inv;
    const SubDesc* desc;
    const int* jobs;
    long long front0, child0;
    int nn, nnc;
    int ybase;               // first (job, node) pair of this launch
    const void* fac;
    void* v;                 // front vectors
    void* x;                 // slab vectors
    long long vtot, xtot;    // entries per chunk
};

// front vector = separator data from the slab vector + the children's updates
template <typename T>
__global__ __launch_bounds__(NT) void nd_vec_kernel(SolveNdArgs a) {
    const int y = a.ybase + blockIdx.y;
    const int j = y / a.nn, pos = y - j * a.nn;
    const int sub = a.jobs[j];
    const NdFront F = a.fr[a.front0 + (long long)sub * a.nn + pos];
    const int idx = blockIdx.x * NT + threadIdx.x;
    const int r = idx >> 4, li = idx & 15;
    if (r >= F.f) return;
    const NdNode nd = a.nodes[F.node];
    const Part p = decode(r, F.ipad, nd.nI, nd.nB, F.L);
    cplx<T>* v = static_cast<cplx<T>*>(a.v) + blockIdx.z * a.vtot;
    const cplx<T>* x = static_cast<const cplx<T>*>(a.x) + blockIdx.z * a.xtot + a.desc[sub].xoff;
    cplx<T> val = mk<T>(T(0), T(0));
    if (p.part == 0) val = x[((long long)a.cols[nd.i_off + p.c] * F.L + p.k) * RW + li];
    if (p.part <= 1 && a.child0 >= 0) {
        const long long base = a.child0 + (long long)sub * a.nnc;
        for (int ch = 0; ch < 2; ++ch) {
            const int cs = nd.inv_off[ch] < 0 ? -1 : a.inv[nd.inv_off[ch] + p.c];
            if (cs >= 0) {
                const NdFront C = a.fr[base + nd.ch[ch]];
                val = val + v[C.voff + (long long)(C.ipad + cs * F.L + p.k) * RW + li];
            }
        }
    }
    v[F.voff + (long long)r * RW + li] = val;
}

// Forward (FWD): v_B -= K^T v_I over the boundary rows.  Backward: x_I =
// F_II^-1 v_I - K x_B into the slab vector.  64 output rows x 16 right-hand
// sides per workgroup; four waves split the inner dimension in batches of 16
// (next batch loaded before the current products) and reduce through LDS in a
// fixed order.
template <typename T, bool FWD>
__global__ __launch_bounds__(NT) void nd_prod_kernel(SolveNdArgs a) {
    __shared__ cplx<T> red[NW][RT][64][4];
    const int y = a.ybase + blockIdx.y;
    const int j = y / a.nn, pos = y - j * a.nn;
    const int sub = a.jobs[j];
    const NdFront F = a.fr[a.front0 + (long long)sub * a.nn + pos];
    const int rows = FWD ? F.f - F.ipad : F.ipad;
    const int r0 = blockIdx.x * 64;
    if (r0 >= rows) return;
    const NdNode nd = a.nodes[F.node];
    const int L = F.L;
    const int inner = FWD ? F.ipad : F.f;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int li = l & 15, lk = l >> 4;
    const cplx<T>* M = static_cast<const cplx<T>*>(a.fac) + F.moff;
    cplx<T>* v = static_cast<cplx<T>*>(a.v) + blockIdx.z * a.vtot + F.voff;
    cplx<T>* x = static_cast<cplx<T>*>(a.x) + blockIdx.z * a.xtot + a.desc[sub].xoff;
    const long long ld = F.ipad;
    CTile<T> acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t].zero();
    f32x4 p1[RT], p2[RT], p3[RT];   // FP32: the three products of each row tile
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) p1[t][e] = p2[t][e] = p3[t][e] = 0.f;
    // operands of one batch: A(row, c) for the RT row tiles, the vector at c
    auto load = [&](int c0, cplx<T> (&m)[RT][4], cplx<T> (&t)[4]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + 4 * u + lk;
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const int row = r0 + 16 * rt + li;
                m[rt][u] = FWD ? M[(long long)(F.ipad + row) * ld + c] : M[(long long)c * ld + row];
            }
            if (FWD || c < F.ipad) {
                t[u] = v[(long long)c * RW + li];
            } else {
                const int q = c - F.ipad, b = q / L;
                const bool in = q < nd.nB * L;
                const int col = a.cols[nd.b_off + (in ? b : 0)];
                const cplx<T> xv = x[((long long)col * L + (q - b * L)) * RW + li];
                t[u] = csel(in, mk<T>(-xv.x, -xv.y), mk<T>(T(0), T(0)));
            }
        }
    };
    const int nb = inner / 16;
    int b = w;
    if (b < nb) {
        cplx<T> mc[RT][4], tc[4], mn[RT][4], tn[4];
        load(16 * b, mc, tc);
        for (;;) {
            const int bn = b + NW;
            if (bn < nb) load(16 * bn, mn, tn);
            if constexpr (std::is_same<T, float>::value) {
                // three-product form: p1 += (m_r + m_i) t_r, p2 += m_r (t_i - t_r),
                // p3 += m_i (t_r + t_i); re = p1 - p3, im = p1 + p2
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const float td = tc[u].y - tc[u].x, ts = tc[u].x + tc[u].y;
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt) {
                        p1[rt] = Mfma<float>::mac(mc[rt][u].x + mc[rt][u].y, tc[u].x, p1[rt]);
                        p2[rt] = Mfma<float>::mac(mc[rt][u].x, td, p2[rt]);
                        p3[rt] = Mfma<float>::mac(mc[rt][u].y, ts, p3[rt]);
                    }
                }
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt) cmac(acc[rt], mc[rt][u], tc[u]);
            }
            if (bn >= nb) break;
            // the next batch becomes the current one (register renames)
            for (int u = 0; u < 4; ++u) {
                tc[u] = tn[u];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) mc[rt][u] = mn[rt][u];
            }
            b = bn;
        }
    }
    if constexpr (std::is_same<T, float>::value) {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                acc[rt].re[e] = p1[rt][e] - p3[rt][e];
                acc[rt].im[e] = p1[rt][e] + p2[rt][e];
            }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int e = 0; e < 4; ++e) red[w][rt][l][e] = mk<T>(acc[rt].re[e], acc[rt].im[e]);
    __syncthreads();
#pragma unroll
    for (int o = 0; o < RT; ++o) {
        const int id = threadIdx.x + NT * o;   // (rt, lane, element)
        const int e = id & 3, l2 = (id >> 2) & 63, rt = id >> 8;
        cplx<T> s = red[0][rt][l2][e];
#pragma unroll
        for (int q = 1; q < NW; ++q) s = s + red[q][rt][l2][e];
        const int row = r0 + 16 * rt + Mfma<T>::row(l2, e);
        const int rhs = l2 & 15;
        if (FWD) {
            cplx<T>* dst = v + (long long)(F.ipad + row) * RW + rhs;
            *dst = *dst - s;
        } else if (row < nd.nI * L) {
            const int c = row / L;
            x[((long long)a.cols[nd.i_off + c] * L + (row - c * L)) * RW + rhs] = s;
        }
    }
}

struct IoArgs {
    const SubDesc* desc;
    const int* jobs;
    void* x;
    long long xtot;
    int in_mode;
    const zd* r;
    const zd* Win;
    int ws;
    const int* act;
    int nact;
    AxisTables ax;
    const zd* gv3;
    int n;
    long long N, S;
    // outputs
    int two_sided;
    int mode0, mode1;
    zd* out0;
    zd* out1;
    const zd* U;
    zd* Wout;
};

// slab vector of job blockIdx.y: M data on the lines of X_q, or R/L data
// (the coupling to the Dirichlet data times the boundary plane) on the line
// next to it; zero elsewhere and for unused right-hand-side slots
template <typename T>
__global__ __launch_bounds__(NT) void nd_input_kernel(IoArgs a) {
    const int js = blockIdx.y;
    const SubDesc d = a.desc[a.jobs[js]];
    const long long idx = (long long)blockIdx.x * NT + threadIdx.x;
    const long long e = idx >> 4;
    const int li = (int)(idx & 15);
    if (e >= a.S * d.L) return;
    const long long col = e / d.L;
    const int k = (int)(e - col * d.L);
    const int slot = blockIdx.z * RW + li;
    zd val = mk(0.0, 0.0);
    if (slot < a.nact) {
        if (a.in_mode == IN_GRID) {
            const int line = d.lo + k;
            if (line >= d.xs && line <= d.xe) {
                const int rhs = a.act ? a.act[slot] : slot;
                val = a.r[(long long)rhs * a.N + col + a.S * (line - 1)];
            }
        } else {
            const int dl = (d.kind == ASP_SUB_R) ? 0 : d.L - 1;
            if (k == dl) {
                const int i1 = (int)(col % a.n), i2 = (int)(col / a.n);
                val = (a.ax.inv_s[i1] * a.gv3[d.vec_off + (long long)d.L * i2 + dl]) *
                      a.Win[((long long)js * a.S + col) * a.ws + slot];
            }
        }
    }
    static_cast<cplx<T>*>(a.x)[blockIdx.z * a.xtot + d.xoff + e * RW + li] = ccast<T>(val);
}

// outputs on the lines of X_p: store, or U + solution; the outgoing boundary
// plane (+ U) of a sweep: R_p hands its last line on, L_p its first
template <typename T>
__global__ __launch_bounds__(NT) void nd_output_kernel(IoArgs a) {
    const int js = blockIdx.y;
    const SubDesc d = a.desc[a.jobs[js]];
    const long long idx = (long long)blockIdx.x * NT + threadIdx.x;
    const long long e = idx >> 4;
    const int li = (int)(idx & 15);
    if (e >= a.S * d.L) return;
    const long long col = e / d.L;
    const int k = (int)(e - col * d.L);
    const int line = d.lo + k;
    const int slot = blockIdx.z * RW + li;
    if (line < d.xs || line > d.xe || slot >= a.nact) return;
    const zd xv =
        ccast<double>(static_cast<const cplx<T>*>(a.x)[blockIdx.z * a.xtot + d.xoff + e * RW + li]);
    const int rhs = a.act ? a.act[slot] : slot;
    const long long g = (long long)rhs * a.N + col + a.S * (line - 1);
    const int side = a.two_sided ? js : 0;
    const int mode = side ? a.mode1 : a.mode0;
    zd* out = side ? a.out1 : a.out0;
    if (mode == OUT_GRID_STORE) out[g] = xv;
    else if (mode == OUT_GRID_ADD_U) out[g] = a.U[g] + xv;
    else out[g] = out[g] + xv;
    if (a.Wout) {
        const int hand = (d.kind == ASP_SUB_R) ? d.xe : d.xs;
        if (line == hand) a.Wout[((long long)js * a.S + col) * a.ws + slot] = a.U[g] + xv;
    }
}

AxisTables axes(const asp_plan* P) {
    AxisTables t;
    t.sh = P->d_axis;
    t.inv_sh2 = P->d_axis + P->n + 1;
    t.inv_s = P->d_axis + 2 * P->n + 1;
    return t;
}

int max_L(const asp_plan* P) {
    int L = 0;
    for (const auto& s : P->subs) L = std::max(L, s.L);
    return L;
}

}  // namespace

hipError_t launch_nd_assemble(const asp_plan* P, const NdLevel& lv, int s0, int s1, void* Flevel,
                              const void* Fchild, int fmax, hipStream_t st) {
    AsmArgs a;
    a.fr = lv.fr_all;
    a.child0 = lv.child0;
    a.nn = lv.nn;
    a.nnc = lv.nnc;
    a.front0 = lv.front0;
    a.nodes = P->d_nd_nodes;
    a.cols = P->d_nd_cols;
    a.inv = P->d_nd_inv;
    a.F = Flevel;
    a.Fc = Fchild;
    a.ax = axes(P);
    a.subtab = P->d_subtab;
    a.ksq = P->d_ksq;
    a.desc = P->d_desc;
    a.n = P->n;
    a.S = P->S;
    const long long nfr = (long long)(s1 - s0) * lv.nn;
    const unsigned gx = (unsigned)((fmax + CPW - 1) / CPW);
    for (long long y0 = 0; y0 < nfr; y0 += YMAX) {
        a.fbase = lv.front0 + (long long)s0 * lv.nn + y0;
        dim3 grid(gx, (unsigned)std::min<long long>(YMAX, nfr - y0));
        if (P->prec != ASP_PREC_FP64)
            hipLaunchKernelGGL(nd_assemble_kernel<float>, grid, dim3(NT), 0, st, a);
        else
            hipLaunchKernelGGL(nd_assemble_kernel<double>, grid, dim3(NT), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_nd_copyout(const asp_plan* P, const NdFront* fr, int nfr, const void* Flevel,
                             int fmax, hipStream_t st) {
    const unsigned gx = (unsigned)((fmax + CPW - 1) / CPW);
    for (int y0 = 0; y0 < nfr; y0 += YMAX) {
        dim3 grid(gx, (unsigned)std::min(YMAX, nfr - y0));
        if (P->prec != ASP_PREC_FP64)
            hipLaunchKernelGGL(nd_copyout_kernel<float>, grid, dim3(NT), 0, st, fr + y0, Flevel, P->d_fac);
        else
            hipLaunchKernelGGL(nd_copyout_kernel<double>, grid, dim3(NT), 0, st, fr + y0, Flevel, P->d_fac);
    }
    return hipGetLastError();
}

hipError_t launch_nd_level(const asp_plan* P, const NdLevel& lv, const int* jobs, int njobs,
                           int fwd, int fmax, int nact, hipStream_t st) {
    SolveNdArgs a;
    a.fr = lv.fr_all;
    a.nodes = P->d_nd_nodes;
    a.cols = P->d_nd_cols;
    a.inv = P->d_nd_inv;
    a.desc = P->d_desc;
    a.jobs = jobs;
    a.front0 = lv.front0;
    a.child0 = lv.child0;
    a.nn = lv.nn;
    a.nnc = lv.nnc;
    a.fac = P->d_fac;
    a.v = P->d_nd_v;
    a.x = P->d_nd_x;
    a.vtot = P->nd_vtot;
    a.xtot = P->nd_xtot;
    const int chunks = (nact + RW - 1) / RW;
    const int ny = njobs * lv.nn;
    const bool f32 = P->prec != ASP_PREC_FP64;
    for (int y0 = 0; y0 < ny; y0 += YMAX) {
        a.ybase = y0;
        const unsigned gy = (unsigned)std::min(YMAX, ny - y0);
        if (fwd) {
            dim3 gv((unsigned)(((long long)fmax * RW + NT - 1) / NT), gy, chunks);
            dim3 gp((unsigned)((fmax + 63) / 64), gy, chunks);
            if (f32) {
                hipLaunchKernelGGL(nd_vec_kernel<float>, gv, dim3(NT), 0, st, a);
                hipLaunchKernelGGL((nd_prod_kernel<float, true>), gp, dim3(NT), 0, st, a);
            } else {
                hipLaunchKernelGGL(nd_vec_kernel<double>, gv, dim3(NT), 0, st, a);
                hipLaunchKernelGGL((nd_prod_kernel<double, true>), gp, dim3(NT), 0, st, a);
            }
        } else {
            dim3 gp((unsigned)((fmax + 63) / 64), gy, chunks);
            if (f32)
                hipLaunchKernelGGL((nd_prod_kernel<float, false>), gp, dim3(NT), 0, st, a);
            else
                hipLaunchKernelGGL((nd_prod_kernel<double, false>), gp, dim3(NT), 0, st, a);
        }
    }
    return hipGetLastError();
}

hipError_t launch_nd_input(const asp_plan* P, const int* jobs, int njobs, int in_mode,
                           const zd* r, const zd* Win, const int* act, int nact, hipStream_t st) {
    IoArgs a{};
    a.desc = P->d_desc;
    a.jobs = jobs;
    a.x = P->d_nd_x;
    a.xtot = P->nd_xtot;
    a.in_mode = in_mode;
    a.r = r;
    a.Win = Win;
    a.ws = P->ws3;
    a.act = act;
    a.nact = nact;
    a.ax = axes(P);
    a.gv3 = P->d_gv3;
    a.n = P->n;
    a.N = P->N;
    a.S = P->S;
    const int chunks = (nact + RW - 1) / RW;
    dim3 grid((unsigned)((P->S * max_L(P) * RW + NT - 1) / NT), njobs, chunks);
    if (P->prec != ASP_PREC_FP64)
        hipLaunchKernelGGL(nd_input_kernel<float>, grid, dim3(NT), 0, st, a);
    else
        hipLaunchKernelGGL(nd_input_kernel<double>, grid, dim3(NT), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_nd_output(const asp_plan* P, const int* jobs, int njobs, bool two_sided,
                            const int out_mode[2], zd* const out[2], const zd* U, zd* Wout,
                            const int* act, int nact, hipStream_t st) {
    IoArgs a{};
    a.desc = P->d_desc;
    a.jobs = jobs;
    a.x = P->d_nd_x;
    a.xtot = P->nd_xtot;
    a.ws = P->ws3;
    a.act = act;
    a.nact = nact;
    a.n = P->n;
    a.N = P->N;
    a.S = P->S;
    a.two_sided = two_sided ? 1 : 0;
    a.mode0 = out_mode[0];
    a.mode1 = out_mode[1];
    a.out0 = out[0];
    a.out1 = out[1];
    a.U = U;
    a.Wout = Wout;
    const int chunks = (nact + RW - 1) / RW;
    dim3 grid((unsigned)((P->S * max_L(P) * RW + NT - 1) / NT), njobs, chunks);
    if (P->prec != ASP_PREC_FP64)
        hipLaunchKernelGGL(nd_output_kernel<float>, grid, dim3(NT), 0, st, a);
    else
        hipLaunchKernelGGL(nd_output_kernel<double>, grid, dim3(NT), 0, st, a);
    return hipGetLastError();
}
