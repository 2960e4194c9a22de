// The recursive sweep of the 3D auxiliary problems (Section 5: the quasi-2D
// problems solved by sweeping along x2 with the same technique).  Each outer
// auxiliary problem's solve H^-1 g is replaced by one application of the
// additive sweeping preconditioner over the slab's x2 lines: inner layers and
// inner M, R and L problems by the rules of Section 2 (with equal layer widths
// the inner partition along x2 is the outer one along x3, so an inner problem
// takes an outer problem's line range and PML profile along x2); the inner
// problems are quasi-1D along x1 and factored by the block recurrence with
// blocks of L_outer x L_inner unknowns (Algorithm 1 one dimension up).
// Setup O(n^3 L^6 m^2 / ...) flops in blocks of (L L2)^3; apply: Algorithm 4
// outside, Algorithm 2 along x2 inside every G~.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <type_traits>

#include "asp_internal.h"

namespace {

constexpr int RW = 16;   // right-hand sides per chunk
constexpr int TB = 64;   // panel width of the block inversions

size_t esz(const asp_plan* P) { return P->prec != ASP_PREC_FP64 ? sizeof(zf) : sizeof(zd); }

template <typename T>
asp_status ralloc(asp_plan* P, T** p, size_t bytes) {
    if (devmem_alloc(reinterpret_cast<void**>(p), bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return plan_fail(P, ASP_ERR_OOM, "device allocation failed");
    }
    return ASP_OK;
}

void rfree(void* p) {
    devmem_free(p);
}

int nsub_of(const asp_plan* P) { return (int)P->subs.size(); }

// job lists (ids into rec_list_off / rec_list_len)
//   0                      every inner problem (the factorization)
//   1                      outer M phase: inner M problems of every outer M problem
//   2 .. m                 outer M phase: inner sweep step t2 = 1..m-1
//   then per outer sweep step t = 1..m-1: its inner M list and m-1 inner sweep lists
//   then per outer problem s: its inner M list and m-1 inner sweep lists (one slot)
int list_M_phase(const asp_plan*) { return 1; }
int list_step(const asp_plan* P, int t) { return 1 + P->m + (t - 1) * P->m; }
int list_single(const asp_plan* P, int s) { return 1 + P->m + (P->m - 1) * P->m + s * P->m; }

size_t sv_len(const asp_plan* P, int chunks) {
    return (size_t)std::max(P->m, 2) * chunks * P->S * P->rec_Lmax * RW;
}
size_t w2_len(const asp_plan* P, int chunks) {
    return (size_t)std::max(P->m, 2) * 4 * chunks * P->n * P->rec_Lmax * RW;
}
long long njobs_max(const asp_plan* P) {
    long long mx = 1;
    for (size_t l = 1; l < P->rec_list_len.size(); ++l) mx = std::max<long long>(mx, P->rec_list_len[l]);
    return mx;
}
size_t blk_len(const asp_plan* P, int chunks) {
    return (size_t)chunks * njobs_max(P) * P->n * P->rec_Bmax * RW;
}

// one application of the inner sweep (Algorithm 2 along x2) to the slab
// inputs of nslot slots, lists [l0, l0 + m): inner M problems, then the m-1
// inner sweep steps; results in the slab vectors (u~, R, L)
asp_status inner_apply(asp_plan* P, int l0, RecLaunch L) {
    hipStream_t st = P->stream;
    const int m = P->m;
    auto solve = [&](int list, int pp, int handoff) -> asp_status {
        L.jobs = P->d_rec_jobs + P->rec_list_off[list];
        L.jslot = P->d_rec_jobs + P->rec_jobs_len + P->rec_list_off[list];
        L.njobs = P->rec_list_len[list];
        L.pp = pp;
        L.mode = 0;
        ASP_HIP(P, launch_rec_gather(P, L, st));
        BlockSolve b;
        b.desc = P->d_rec_sd;
        b.jobs = L.jobs;
        b.njobs = L.njobs;
        b.fac = P->d_fac;
        b.Y = P->d_rec_y;
        b.G = P->d_rec_g;
        b.Bmax = P->rec_Bmax;
        b.e = P->d_rec_e;
        b.nact = L.nact;
        b.narrow = L.njobs <= 8;
        for (int k = 0; k < P->n; ++k) ASP_HIP(P, launch_block_step(P, b, k, 1, st));
        for (int k = P->n - 1; k >= 0; --k) ASP_HIP(P, launch_block_step(P, b, k, 0, st));
        L.pp = handoff >= 0 ? handoff : 0;
        L.mode = handoff >= 0 ? 1 : 0;
        ASP_HIP(P, launch_rec_scatter(P, L, st));
        return ASP_OK;
    };
    asp_status s = solve(l0, 0, -1);
    if (s != ASP_OK || m == 1) return s;
    ASP_HIP(P, launch_rec_seed(P, L, st));
    for (int t2 = 1; t2 <= m - 1; ++t2)
        if ((s = solve(l0 + t2, (t2 - 1) & 1, t2 < m - 1 ? (t2 & 1) : -1)) != ASP_OK) return s;
    return ASP_OK;
}

// kernel launches of one inner_apply
int inner_launches(const asp_plan* P) {
    return P->m * (2 + 2 * P->n) + (P->m > 1 ? 1 : 0);
}

// algorithmic work of the inner block solves of one inner sweep per outer
// problem listed (forward + backward: each factor block read twice)
void inner_cost(const asp_plan* P, const std::vector<int>& outers, int nact, double* bytes,
                double* flops) {
    const int ns = nsub_of(P);
    for (int o : outers)
        for (int i = 0; i < ns; ++i) {
            const double BB = (double)P->subs[o].L * P->subs[i].L;
            *bytes += 2.0 * P->n * BB * BB * esz(P);
            *flops += 2.0 * P->n * BB * BB * 8.0 * nact;
        }
}

}  // namespace

asp_status rec_setup(asp_plan* P) {
    const int ns = nsub_of(P), m = P->m, n = P->n;
    P->rec = true;
    P->rec_desc.clear();
    long long fac = 0, vec = 0;
    P->rec_Bmax = 0;
    P->rec_Lmax = 0;
    for (int o = 0; o < ns; ++o) P->rec_Lmax = std::max(P->rec_Lmax, P->subs[o].L);
    for (int o = 0; o < ns; ++o)
        for (int i = 0; i < ns; ++i) {
            RecDesc d{};
            d.outer = o;
            d.inner = i;
            d.B = (P->subs[o].L * P->subs[i].L + TB - 1) / TB * TB;
            d.fac_off = fac;
            d.vec_off = vec;
            fac += (long long)n * d.B * d.B;
            vec += d.B;
            P->rec_Bmax = std::max(P->rec_Bmax, d.B);
            P->rec_desc.push_back(d);
        }
    P->rec_vec_elems = vec;
    P->fac_elems = fac;
    P->fac_bytes = (size_t)fac * esz(P);
    // job lists (inner problem = outer * ns + inner)
    std::vector<std::vector<std::pair<int, int>>> lists;
    std::vector<std::pair<int, int>> all;
    for (int j = 0; j < ns * ns; ++j) all.push_back({j, 0});
    lists.push_back(all);
    auto inner_lists = [&](const std::vector<int>& outers) {
        std::vector<std::pair<int, int>> lm;
        for (size_t sl = 0; sl < outers.size(); ++sl)
            for (int q = 1; q <= m; ++q) lm.push_back({outers[sl] * ns + P->idx_M(q), (int)sl});
        lists.push_back(lm);
        for (int t2 = 1; t2 <= m - 1; ++t2) {
            std::vector<std::pair<int, int>> ls;
            for (size_t sl = 0; sl < outers.size(); ++sl) {
                ls.push_back({outers[sl] * ns + P->idx_R(t2 + 1), (int)sl});
                ls.push_back({outers[sl] * ns + P->idx_L(m - t2), (int)sl});
            }
            lists.push_back(ls);
        }
    };
    std::vector<int> mo;
    for (int q = 1; q <= m; ++q) mo.push_back(P->idx_M(q));
    inner_lists(mo);
    for (int t = 1; t <= m - 1; ++t) inner_lists({P->idx_R(t + 1), P->idx_L(m - t)});
    for (int s = 0; s < ns; ++s) inner_lists({s});
    P->rec_list_off.clear();
    P->rec_list_len.clear();
    long long off = 0;
    for (auto& l : lists) {
        P->rec_list_off.push_back(off);
        P->rec_list_len.push_back((int)l.size());
        off += (long long)l.size();
    }
    P->rec_jobs_len = off;
    P->rec_jobs_host.assign(2 * (size_t)off, 0);
    for (size_t l = 0; l < lists.size(); ++l)
        for (size_t i = 0; i < lists[l].size(); ++i) {
            P->rec_jobs_host[P->rec_list_off[l] + i] = lists[l][i].first;
            P->rec_jobs_host[off + P->rec_list_off[l] + i] = lists[l][i].second;
        }
    return ASP_OK;
}

asp_status rec_upload(asp_plan* P) {
    const double h2 = P->h * P->h;
    std::vector<SubDesc> sd(P->rec_desc.size());
    std::vector<zd> e((size_t)P->rec_vec_elems, mk(0.0, 0.0));
    for (size_t j = 0; j < P->rec_desc.size(); ++j) {
        const RecDesc& d = P->rec_desc[j];
        SubDesc b{};
        b.kind = ASP_SUB_M;
        b.L = 1;
        b.B = d.B;
        b.xs = 1;      // no grid output from the block-step kernel
        b.xe = 0;
        b.fac_off = d.fac_off;
        b.vec_off = d.vec_off;
        sd[j] = b;
        const int L = P->subs[d.outer].L, L2 = P->subs[d.inner].L;
        for (int r = 0; r < L * L2; ++r) {
            const std::complex<double> s3 = P->sub_int[d.outer][r % L], s2 = P->sub_int[d.inner][r / L];
            const std::complex<double> v = 1.0 / (s2 * s3 * h2);
            e[d.vec_off + r] = mk(v.real(), v.imag());
        }
    }
    auto put = [&](auto** dst, const auto* src, size_t count) -> asp_status {
        using T = std::remove_pointer_t<std::remove_pointer_t<decltype(dst)>>;
        if (ralloc(P, dst, count * sizeof(T)) != ASP_OK) return ASP_ERR_OOM;
        ASP_HIP(P, hipMemcpyAsync(*dst, src, count * sizeof(T), hipMemcpyHostToDevice, P->stream));
        return ASP_OK;
    };
    asp_status s;
    if ((s = put(&P->d_rec, P->rec_desc.data(), P->rec_desc.size())) != ASP_OK) return s;
    if ((s = put(&P->d_rec_sd, sd.data(), sd.size())) != ASP_OK) return s;
    if ((s = put(&P->d_rec_e, e.data(), e.size())) != ASP_OK) return s;
    if ((s = put(&P->d_rec_jobs, P->rec_jobs_host.data(), P->rec_jobs_host.size())) != ASP_OK) return s;
    ASP_HIP(P, hipStreamSynchronize(P->stream));
    return ASP_OK;
}

size_t rec_factor_work_estimate(const asp_plan* P) {
    const size_t nall = P->rec_desc.size();
    return nall * ((size_t)P->rec_Bmax * TB + (size_t)TB * TB) * esz(P);
}

// Algorithm 1 for every inner problem of every outer problem at once: block k
// after block k-1, each block inverted by 64-wide Gauss-Jordan panels
asp_status rec_factor(asp_plan* P) {
    hipStream_t st = P->stream;
    const int nall = (int)P->rec_desc.size();
    char* Rbuf = nullptr;
    char* Dbuf = nullptr;
    if (ralloc(P, &Rbuf, (size_t)nall * P->rec_Bmax * TB * esz(P)) != ASP_OK) return ASP_ERR_OOM;
    if (ralloc(P, &Dbuf, (size_t)nall * TB * TB * esz(P)) != ASP_OK) {
        rfree(Rbuf);
        return ASP_ERR_OOM;
    }
    double fb = 0, fl = 0;
    for (const RecDesc& d : P->rec_desc) {
        const double BB = (double)P->subs[d.outer].L * P->subs[d.inner].L;
        fb += (double)P->n * BB * BB * esz(P);
        fl += (double)P->n * BB * BB * BB * 8.0;   // one inverse per block (the stored factor)
    }
    const int np = P->rec_Bmax / TB;
    asp_status s = ASP_OK;
    {
        KTimer t(P, ASP_K_FACTOR, fb, fl, P->n * (1 + 3 * np));
        const int* all = P->d_rec_jobs + P->rec_list_off[0];
        for (int k = 0; k < P->n && s == ASP_OK; ++k) {
            hipError_t e = launch_rec_form(P, k, st);
            for (int jp = 0; jp < np && e == hipSuccess; ++jp)
                e = launch_gj_blocks(P, P->d_rec_sd, all, nall, P->d_fac, k, jp, P->rec_Bmax, Rbuf, Dbuf, st);
            if (e != hipSuccess)
                s = plan_fail(P, ASP_ERR_DEVICE, std::string("recursive factor launch: ") + hipGetErrorString(e));
        }
        t.end();
    }
    (void)hipStreamSynchronize(st);
    rfree(Rbuf);
    rfree(Dbuf);
    return s;
}

size_t rec_workspace_estimate(const asp_plan* P, int nrhs) {
    const int chunks = (nrhs + RW - 1) / RW;
    const double vec = (double)nrhs * P->N * sizeof(zd);
    const double we = 4.0 * P->S * chunks * RW * sizeof(zd);
    return (size_t)(2.0 * vec + we +
                    (4.0 * sv_len(P, chunks) + w2_len(P, chunks) + 2.0 * blk_len(P, chunks)) * esz(P));
}

void rec_free_ws(asp_plan* P) {
    void* b[] = {P->d_rec_sv, P->d_rec_w2, P->d_rec_g, P->d_rec_y};
    for (void* p : b) rfree(p);
    P->d_rec_sv = P->d_rec_w2 = P->d_rec_g = P->d_rec_y = nullptr;
    P->rec_chunks = 0;
    P->rec_ws_bytes = 0;
}

asp_status rec_ensure_ws(asp_plan* P, int nrhs) {
    if (nrhs <= P->ws_rhs) return ASP_OK;
    ASP_HIP(P, hipStreamSynchronize(P->stream));
    void* old[] = {P->d_U, P->d_stage, P->d_w3};
    for (void* b : old) rfree(b);
    P->d_U = P->d_stage = P->d_w3 = nullptr;
    rec_free_ws(P);
    P->ws_rhs = 0;
    P->ws_bytes = 0;
    const int chunks = (nrhs + RW - 1) / RW;
    const size_t vec = (size_t)nrhs * P->N * sizeof(zd);
    P->ws3 = chunks * RW;
    const long long we = 2LL * 2 * P->S * P->ws3;
    char *sv = nullptr, *w2 = nullptr, *g = nullptr, *y = nullptr;
    if (ralloc(P, &P->d_U, vec) != ASP_OK || ralloc(P, &P->d_stage, vec) != ASP_OK ||
        ralloc(P, &P->d_w3, (size_t)we * sizeof(zd)) != ASP_OK ||
        ralloc(P, &sv, 4 * sv_len(P, chunks) * esz(P)) != ASP_OK ||
        ralloc(P, &w2, w2_len(P, chunks) * esz(P)) != ASP_OK ||
        ralloc(P, &g, blk_len(P, chunks) * esz(P)) != ASP_OK ||
        ralloc(P, &y, blk_len(P, chunks) * esz(P)) != ASP_OK) {
        rfree(sv);
        rfree(w2);
        rfree(g);
        rfree(y);
        return ASP_ERR_OOM;
    }
    P->d_rec_sv = sv;
    P->d_rec_w2 = w2;
    P->d_rec_g = g;
    P->d_rec_y = y;
    P->rec_chunks = chunks;
    P->w3_elems = we;
    P->ws_rhs = nrhs;
    P->ws_bytes = rec_workspace_estimate(P, nrhs);
    return ASP_OK;
}

// Algorithm 4 with every G~ applied by the inner sweep, for the right-hand
// sides act[0..nact) (NULL: 0..nact-1)
asp_status rec_apply(asp_plan* P, const zd* r, zd* z, const int* act, int nact) {
    hipStream_t st = P->stream;
    const int m = P->m, ns = nsub_of(P);
    RecLaunch L;
    L.chunks = (nact + RW - 1) / RW;
    L.nact = nact;
    L.act = act;
    {
        std::vector<int> outers;
        for (int q = 1; q <= m; ++q) outers.push_back(P->idx_M(q));
        double by = 2.0 * nact * (double)P->N * sizeof(zd), fl = 0;
        inner_cost(P, outers, nact, &by, &fl);
        KTimer t(P, ASP_K_SOLVE_M, by, fl, 2 + inner_launches(P));
        L.nslot = m;
        L.slot_outer = P->d_jobs;
        L.mode = IN_GRID;
        L.rin = r;
        ASP_HIP(P, launch_rec_slab_in(P, L, st));
        asp_status s = inner_apply(P, list_M_phase(P), L);
        if (s != ASP_OK) return s;
        L.mode = 0;
        L.out0 = (m == 1) ? z : P->d_U;
        ASP_HIP(P, launch_rec_slab_out(P, L, st));
        t.end();
    }
    if (m == 1) return ASP_OK;
    {
        std::vector<int> outers;
        for (int t1 = 1; t1 <= m - 1; ++t1) {
            outers.push_back(P->idx_R(t1 + 1));
            outers.push_back(P->idx_L(m - t1));
        }
        double by = 2.0 * nact * (double)P->N * sizeof(zd), fl = 0;
        inner_cost(P, outers, nact, &by, &fl);
        KTimer t(P, ASP_K_SOLVE_RL, by, fl, 1 + (m - 1) * (2 + inner_launches(P)));
        const long long plane = 2LL * P->S * P->ws3;
        ASP_HIP(P, launch_plane3d(P, P->d_U, P->X[0][1], P->X[m - 1][0], P->d_w3, act, nact, st));
        for (int t1 = 1; t1 <= m - 1; ++t1) {
            L.nslot = 2;
            L.slot_outer = P->d_jobs + ns + 2 * (t1 - 1);
            L.mode = IN_BOUNDARY;
            L.rin = P->d_w3 + ((t1 - 1) & 1) * plane;
            ASP_HIP(P, launch_rec_slab_in(P, L, st));
            asp_status s = inner_apply(P, list_step(P, t1), L);
            if (s != ASP_OK) return s;
            L.mode = 1;
            L.out0 = z;
            L.out1 = P->d_stage;
            L.U = P->d_U;
            L.Wout = (t1 < m - 1) ? P->d_w3 + (t1 & 1) * plane : nullptr;
            ASP_HIP(P, launch_rec_slab_out(P, L, st));
        }
        t.end();
    }
    {
        KTimer t(P, ASP_K_COMBINE, 4.0 * nact * (double)P->N * sizeof(zd), 0.0);
        ASP_HIP(P, launch_combine3d(P, z, P->d_U, P->d_stage, P->X[0][1], P->X[m - 2][1], false,
                                    act, nact, st));
        t.end();
    }
    return ASP_OK;
}

// One approximate auxiliary Green's operator: M data on X_q, or R/L data on
// the Dirichlet line; the output restricted to X_p.
asp_status rec_subsolve(asp_plan* P, int idx, const void* in, void* out, int nrhs) {
    hipStream_t st = P->stream;
    const SubDesc& d = P->subs[idx];
    const size_t row = sizeof(zd);
    const long long Np = P->S * (d.xe - d.xs + 1);
    RecLaunch L;
    L.chunks = (nrhs + RW - 1) / RW;
    L.nact = nrhs;
    L.nslot = 1;
    L.slot_outer = P->d_jobs + idx;
    if (d.kind == ASP_SUB_M) {
        ASP_HIP(P, hipMemcpy2DAsync(P->d_U + (long long)(d.xs - 1) * P->S, P->N * row, in,
                                    Np * row, Np * row, nrhs, hipMemcpyDeviceToDevice, st));
        L.mode = IN_GRID;
        L.rin = P->d_U;
    } else {
        ASP_HIP(P, hipMemcpy2DAsync(P->d_U, P->N * row, in, P->S * row, P->S * row, nrhs,
                                    hipMemcpyDeviceToDevice, st));
        ASP_HIP(P, launch_plane3d(P, P->d_U, 1, 1, P->d_w3, nullptr, nrhs, st));
        L.mode = IN_BOUNDARY;
        L.rin = P->d_w3;
    }
    ASP_HIP(P, launch_rec_slab_in(P, L, st));
    asp_status s = inner_apply(P, list_single(P, idx), L);
    if (s != ASP_OK) return s;
    L.mode = 0;
    L.out0 = P->d_stage;
    ASP_HIP(P, launch_rec_slab_out(P, L, st));
    ASP_HIP(P, hipMemcpy2DAsync(out, Np * row, P->d_stage + (long long)(d.xs - 1) * P->S,
                                P->N * row, Np * row, nrhs, hipMemcpyDeviceToDevice, st));
    return ASP_OK;
}
