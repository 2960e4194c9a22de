// Kernels of the recursive sweep of the 3D auxiliary problems (Section 5):
// the block recurrence of the inner problems along x1 (their blocks formed
// here, inverted by the block Gauss-Jordan kernels), and the data movement of
// the inner sweep along x2 between slab vectors, inner problems and the outer
// grid.  The inner block solves run on the 3D block-step kernel.
//
// Layouts (T = the factor precision; 16 right-hand sides per chunk):
//   slab vectors  SV[b][slot][chunk][k][i2][i3][16], b = 0 input, 1 u~ of the
//                 inner layers, 2 inner R results, 3 inner L results; i2 the
//                 0-based x2 line, i3 the 0-based line of the outer problem
//   inner planes  W2[slot][side][pingpong][chunk][k][i3][16]: the x2 line
//                 entering the next inner R (side 0) or L (side 1) problem
//   block data    G, Y[chunk][job][k][Bmax][16] (the block-step layout)
#include "asp_internal.h"

namespace {

constexpr int RW = 16;

struct RecArgs {
    const RecDesc* rd;
    const SubDesc* desc;
    const zd* subtab;
    AxisTables ax;
    const double* ksq;
    const zd* e;
    void* fac;
    int n;
    long long N, S;
    int Lmax, Bmax, k;
    int nslot, chunks, nact;
    const int* act;
    const int* slot_outer;
    const int* jobs;
    const int* jslot;
    int njobs;
    int mode, pp;
    const zd* rin;
    zd* out0;
    zd* out1;
    const zd* U;
    zd* Wout;
    int ws;
    void* sv;
    long long svlen;
    void* w2;
    void* G;
    void* Y;
    int lineR1, lineLm;   // last x2 line of inner layer 1, first of inner layer m
};

__device__ __forceinline__ long long sv_idx(const RecArgs& a, int slot, int chunk, int k, int i2,
                                            int i3, int r) {
    return (((((long long)slot * a.chunks + chunk) * a.n + k) * a.n + i2) * a.Lmax + i3) * RW + r;
}
__device__ __forceinline__ long long w2_idx(const RecArgs& a, int slot, int side, int pp, int chunk,
                                            int k, int i3, int r) {
    return ((((((long long)slot * 2 + side) * 2 + pp) * a.chunks + chunk) * a.n + k) * a.Lmax + i3) * RW + r;
}
__device__ __forceinline__ long long blk_idx(const RecArgs& a, int chunk, int js, int k, int j, int r) {
    return (((long long)chunk * a.njobs + js) * a.n + k) * a.Bmax * RW + (long long)j * RW + r;
}

// Block k of every inner problem: the symmetric-form operator on the box
// x1 = k, x2 in the inner problem's lines (its x2 profile), x3 in the outer
// problem's lines (its sweep-axis profile), minus the Schur term of block k-1;
// identity on the padding.
template <typename T>
__global__ __launch_bounds__(256) void rec_form_kernel(RecArgs a) {
    const RecDesc rd = a.rd[blockIdx.z];
    const SubDesc so = a.desc[rd.outer], si = a.desc[rd.inner];
    const int Bp = rd.B, L = so.L, L2 = si.L, BB = L * L2;
    const int r = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (r >= Bp || c >= Bp) return;
    const int k = a.k;
    cplx<T>* A = static_cast<cplx<T>*>(a.fac) + rd.fac_off + (long long)k * Bp * Bp;
    zd val = mk(0.0, 0.0);
    if (r >= BB || c >= BB) {
        if (r == c) val = mk(1.0, 0.0);
    } else {
        const int i3r = r % L, i2r = r / L, i3c = c % L, i2c = c / L;
        const zd* sh3 = a.subtab + so.tab_off;   // s3 at half lines lo - 1/2 ..
        const zd* ish3 = sh3 + L + 1;            // 1 / (s3 h^2)
        const zd* is3 = sh3 + 2 * L + 1;         // 1 / s3
        const zd* sh2 = a.subtab + si.tab_off;   // the inner x2 profile, same layout
        const zd* ish2 = sh2 + L2 + 1;
        const zd* is2 = sh2 + 2 * L2 + 1;
        const zd is1 = a.ax.inv_s[k];
        if (r == c) {
            const zd s23 = is2[i2r] * ish3[i3r];   // 1 / (s2 s3 h^2)
            const zd s13 = is1 * ish3[i3r];
            const zd s12 = is1 * ish2[i2r];
            const zd c1 = (a.ax.sh[k + 1] + a.ax.sh[k]) * s23;
            const zd c2 = (sh2[i2r + 1] + sh2[i2r]) * s13;
            const zd c3 = (sh3[i3r + 1] + sh3[i3r]) * s12;
            const long long g = (long long)k + (long long)a.n * (si.lo - 1 + i2r) + a.S * (so.lo - 1 + i3r);
            val = ((a.ksq[g] * is1) * is2[i2r]) * is3[i3r] - (c1 + c2 + c3);
        } else if (i2r == i2c && (i3r - i3c == 1 || i3c - i3r == 1)) {
            val = sh3[max(i3r, i3c)] * (is1 * ish2[i2r]);
        } else if (i3r == i3c && (i2r - i2c == 1 || i2c - i2r == 1)) {
            val = sh2[max(i2r, i2c)] * (is1 * ish3[i3r]);
        }
        if (k > 0) {
            const zd* e = a.e + rd.vec_off;
            const cplx<T>* prev = A - (long long)Bp * Bp;
            const zd sk = a.ax.sh[k];
            const zd er = sk * e[r], ec = sk * e[c];
            const zd pv = ccast<double>(prev[(long long)c * Bp + r]);
            val = val - (er * pv) * ec;
        }
    }
    A[(long long)c * Bp + r] = ccast<T>(val);
}

// Slab input of every slot.  mode IN_GRID: the grid data on the outer
// problem's layer lines (zero on its pads); IN_BOUNDARY: the outer Dirichlet
// data term on its first (R) or last (L) line, -s3(half line) / (s1 s2 h^2)
// times the incoming plane rin[side][i1 + n i2][slot].
template <typename T>
__global__ __launch_bounds__(256) void rec_slab_in_kernel(RecArgs a) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int i3 = t / RW, rl = t % RW;
    if (i3 >= a.Lmax) return;
    const int p = blockIdx.y, k = p % a.n, i2 = p / a.n;
    const int slot = blockIdx.z / a.chunks, chunk = blockIdx.z % a.chunks;
    const SubDesc so = a.desc[a.slot_outer[slot]];
    const int rs = chunk * RW + rl;
    zd v = mk(0.0, 0.0);
    if (i3 < so.L && rs < a.nact) {
        const int rid = a.act ? a.act[rs] : rs;
        if (a.mode == IN_GRID) {
            const int line = so.lo + i3;
            if (line >= so.xs && line <= so.xe) v = a.rin[(long long)rid * a.N + p + a.S * (line - 1)];
        } else {
            const bool right = so.kind == ASP_SUB_R;
            if (i3 == (right ? 0 : so.L - 1)) {
                const zd* sh3 = a.subtab + so.tab_off;
                const zd sdat = right ? sh3[0] : sh3[so.L];
                const zd w = a.rin[((right ? 0 : 1) * a.S + p) * a.ws + rs];
                v = -((sdat * (a.ax.inv_s[k] * a.ax.inv_sh2[i2])) * w);
            }
        }
    }
    static_cast<cplx<T>*>(a.sv)[sv_idx(a, slot, chunk, k, i2, i3, rl)] = ccast<T>(v);
}

// Data of the inner problems of every job into G: an inner M problem takes the
// slab input on its inner layer's x2 lines (zero on its pads); an inner R / L
// problem the x2 Dirichlet data term on its first / last x2 line,
// -s2(half line) / (s1 s3 h^2) times the inner plane.
template <typename T>
__global__ __launch_bounds__(256) void rec_gather_kernel(RecArgs a) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int j = t / RW, rl = t % RW;
    if (j >= a.Bmax) return;
    const int k = blockIdx.y;
    const int js = blockIdx.z % a.njobs, chunk = blockIdx.z / a.njobs;
    const RecDesc rd = a.rd[a.jobs[js]];
    const int slot = a.jslot[js];
    const SubDesc so = a.desc[rd.outer], si = a.desc[rd.inner];
    const int L = so.L, L2 = si.L;
    cplx<T> v = mk<T>(0, 0);
    if (j < L * L2 && chunk * RW + rl < a.nact) {
        const int i3 = j % L, i2l = j / L, i2 = si.lo + i2l;
        const cplx<T>* sv = static_cast<const cplx<T>*>(a.sv);
        if (si.kind == ASP_SUB_M) {
            if (i2 >= si.xs && i2 <= si.xe) v = sv[sv_idx(a, slot, chunk, k, i2 - 1, i3, rl)];
        } else {
            const bool right = si.kind == ASP_SUB_R;
            if (i2l == (right ? 0 : L2 - 1)) {
                const zd* sh2 = a.subtab + si.tab_off;
                const zd s2d = right ? sh2[0] : sh2[L2];
                const zd* ish3 = a.subtab + so.tab_off + L + 1;
                const cplx<T> w = static_cast<const cplx<T>*>(a.w2)[w2_idx(a, slot, right ? 0 : 1, a.pp,
                                                                          chunk, k, i3, rl)];
                v = -(ccast<T>(s2d * (a.ax.inv_s[k] * ish3[i3])) * w);
            }
        }
    }
    static_cast<cplx<T>*>(a.G)[blk_idx(a, chunk, js, k, j, rl)] = v;
}

// Results of the inner problems of every job (Y after the backward pass) on
// their inner layer's x2 lines into the slab vectors (M: u~, R, L), and with
// a.mode != 0 the outgoing x2 line of an inner R (last line of its layer) or
// L problem (first line) plus u~ there into inner plane pingpong a.pp.
template <typename T>
__global__ __launch_bounds__(256) void rec_scatter_kernel(RecArgs a) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int j = t / RW, rl = t % RW;
    if (j >= a.Bmax) return;
    const int k = blockIdx.y;
    const int js = blockIdx.z % a.njobs, chunk = blockIdx.z / a.njobs;
    const RecDesc rd = a.rd[a.jobs[js]];
    const int slot = a.jslot[js];
    const SubDesc so = a.desc[rd.outer], si = a.desc[rd.inner];
    const int L = so.L, L2 = si.L;
    if (j >= L * L2 || chunk * RW + rl >= a.nact) return;
    const int i3 = j % L, i2 = si.lo + j / L;
    if (i2 < si.xs || i2 > si.xe) return;
    const cplx<T> v = static_cast<const cplx<T>*>(a.Y)[blk_idx(a, chunk, js, k, j, rl)];
    cplx<T>* sv = static_cast<cplx<T>*>(a.sv);
    const int buf = si.kind == ASP_SUB_M ? 1 : (si.kind == ASP_SUB_R ? 2 : 3);
    const long long o = sv_idx(a, slot, chunk, k, i2 - 1, i3, rl);
    sv[buf * a.svlen + o] = v;
    if (a.mode && si.kind != ASP_SUB_M) {
        const bool right = si.kind == ASP_SUB_R;
        if (i2 == (right ? si.xe : si.xs))
            static_cast<cplx<T>*>(a.w2)[w2_idx(a, slot, right ? 0 : 1, a.pp, chunk, k, i3, rl)] =
                v + sv[a.svlen + o];
    }
}

// The planes that start the two inner sweeps: u~ on the last x2 line of inner
// layer 1 and on the first x2 line of inner layer m
template <typename T>
__global__ __launch_bounds__(256) void rec_seed_kernel(RecArgs a) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int i3 = t / RW, rl = t % RW;
    if (i3 >= a.Lmax) return;
    const int k = blockIdx.y;
    const int slot = blockIdx.z / a.chunks, chunk = blockIdx.z % a.chunks;
    const cplx<T>* su = static_cast<const cplx<T>*>(a.sv) + a.svlen;
    cplx<T>* w2 = static_cast<cplx<T>*>(a.w2);
    w2[w2_idx(a, slot, 0, 0, chunk, k, i3, rl)] = su[sv_idx(a, slot, chunk, k, a.lineR1 - 1, i3, rl)];
    w2[w2_idx(a, slot, 1, 0, chunk, k, i3, rl)] = su[sv_idx(a, slot, chunk, k, a.lineLm - 1, i3, rl)];
}

// The approximate G~ of every slot, u~ + the inner R results (x2 past inner
// layer 1) + the inner L results (x2 before inner layer m), on the outer
// problem's layer lines.  mode 0: out0 = v;  mode 1 (the outer sweeps): an
// outer R problem writes out0 = U + v and hands U + v on its last line to the
// plane Wout (side 0), an outer L problem writes out1 = v and hands U + v on
// its first line (side 1).
template <typename T>
__global__ __launch_bounds__(256) void rec_slab_out_kernel(RecArgs a) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int i3 = t / RW, rl = t % RW;
    if (i3 >= a.Lmax) return;
    const int p = blockIdx.y, i2 = p / a.n;
    const int slot = blockIdx.z / a.chunks, chunk = blockIdx.z % a.chunks;
    const SubDesc so = a.desc[a.slot_outer[slot]];
    const int rs = chunk * RW + rl;
    if (i3 >= so.L || rs >= a.nact) return;
    const int line = so.lo + i3;
    if (line < so.xs || line > so.xe) return;
    const cplx<T>* sv = static_cast<const cplx<T>*>(a.sv);
    const long long o = sv_idx(a, slot, chunk, p % a.n, i2, i3, rl);
    cplx<T> v = sv[a.svlen + o];
    if (i2 + 1 > a.lineR1) v = v + sv[2 * a.svlen + o];
    if (i2 + 1 < a.lineLm) v = v + sv[3 * a.svlen + o];
    const int rid = a.act ? a.act[rs] : rs;
    const long long g = (long long)rid * a.N + p + a.S * (line - 1);
    const zd vd = ccast<double>(v);
    if (a.mode == 0) {
        a.out0[g] = vd;
    } else if (so.kind == ASP_SUB_R) {
        const zd x = a.U[g] + vd;
        a.out0[g] = x;
        if (a.Wout && line == so.xe) a.Wout[(long long)p * a.ws + rs] = x;
    } else {
        a.out1[g] = vd;
        if (a.Wout && line == so.xs) a.Wout[(a.S + p) * a.ws + rs] = a.U[g] + vd;
    }
}

RecArgs base_args(const asp_plan* P) {
    RecArgs a{};
    a.rd = P->d_rec;
    a.desc = P->d_desc;
    a.subtab = P->d_subtab;
    a.ax = AxisTables{P->d_axis, P->d_axis + (P->n + 1), P->d_axis + (2 * P->n + 1)};
    a.ksq = P->d_ksq;
    a.e = P->d_rec_e;
    a.fac = P->d_fac;
    a.n = P->n;
    a.N = P->N;
    a.S = P->S;
    a.Lmax = P->rec_Lmax;
    a.Bmax = P->rec_Bmax;
    a.ws = P->ws3;
    a.sv = P->d_rec_sv;
    a.svlen = (long long)std::max(P->m, 2) * P->rec_chunks * P->S * P->rec_Lmax * RW;
    a.w2 = P->d_rec_w2;
    a.G = P->d_rec_g;
    a.Y = P->d_rec_y;
    a.lineR1 = P->X[0][1];
    a.lineLm = P->X[P->m - 1][0];
    return a;
}

RecArgs launch_args(const asp_plan* P, const RecLaunch& L) {
    RecArgs a = base_args(P);
    a.nslot = L.nslot;
    a.chunks = L.chunks;
    a.nact = L.nact;
    a.act = L.act;
    a.slot_outer = L.slot_outer;
    a.jobs = L.jobs;
    a.jslot = L.jslot;
    a.njobs = L.njobs;
    a.mode = L.mode;
    a.pp = L.pp;
    a.rin = L.rin;
    a.out0 = L.out0;
    a.out1 = L.out1;
    a.U = L.U;
    a.Wout = L.Wout;
    return a;
}

#define ASP_REC_LAUNCH(kernel, grid, a)                                                  \
    do {                                                                                 \
        if (P->prec != ASP_PREC_FP64)                                                    \
            hipLaunchKernelGGL(kernel<float>, grid, dim3(256), 0, st, a);                \
        else                                                                             \
            hipLaunchKernelGGL(kernel<double>, grid, dim3(256), 0, st, a);               \
    } while (0)

}  // namespace

hipError_t launch_rec_form(const asp_plan* P, int k, hipStream_t st) {
    RecArgs a = base_args(P);
    a.k = k;
    dim3 grid((P->rec_Bmax + 255) / 256, P->rec_Bmax, (unsigned)P->rec_desc.size());
    ASP_REC_LAUNCH(rec_form_kernel, grid, a);
    return hipGetLastError();
}

hipError_t launch_rec_slab_in(const asp_plan* P, const RecLaunch& L, hipStream_t st) {
    RecArgs a = launch_args(P, L);
    dim3 grid((P->rec_Lmax * RW + 255) / 256, (unsigned)P->S, L.nslot * L.chunks);
    ASP_REC_LAUNCH(rec_slab_in_kernel, grid, a);
    return hipGetLastError();
}

hipError_t launch_rec_gather(const asp_plan* P, const RecLaunch& L, hipStream_t st) {
    RecArgs a = launch_args(P, L);
    dim3 grid((P->rec_Bmax * RW + 255) / 256, P->n, L.njobs * L.chunks);
    ASP_REC_LAUNCH(rec_gather_kernel, grid, a);
    return hipGetLastError();
}

hipError_t launch_rec_scatter(const asp_plan* P, const RecLaunch& L, hipStream_t st) {
    RecArgs a = launch_args(P, L);
    dim3 grid((P->rec_Bmax * RW + 255) / 256, P->n, L.njobs * L.chunks);
    ASP_REC_LAUNCH(rec_scatter_kernel, grid, a);
    return hipGetLastError();
}

hipError_t launch_rec_seed(const asp_plan* P, const RecLaunch& L, hipStream_t st) {
    RecArgs a = launch_args(P, L);
    dim3 grid((P->rec_Lmax * RW + 255) / 256, P->n, L.nslot * L.chunks);
    ASP_REC_LAUNCH(rec_seed_kernel, grid, a);
    return hipGetLastError();
}

hipError_t launch_rec_slab_out(const asp_plan* P, const RecLaunch& L, hipStream_t st) {
    RecArgs a = launch_args(P, L);
    dim3 grid((P->rec_Lmax * RW + 255) / 256, (unsigned)P->S, L.nslot * L.chunks);
    ASP_REC_LAUNCH(rec_slab_out_kernel, grid, a);
    return hipGetLastError();
}
