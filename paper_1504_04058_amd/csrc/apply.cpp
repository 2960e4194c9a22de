// Factor (Algorithm 1 and the boundary-to-boundary maps), apply (Algorithm 2),
// the stencil, the single-operator hook and per-kernel timing of the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "asp_internal.h"

namespace {

size_t elem_bytes(const asp_plan* P) { return P->prec != ASP_PREC_FP64 ? sizeof(zf) : sizeof(zd); }

template <typename T>
asp_status dev_alloc(asp_plan* P, T** p, size_t count) {
    if (devmem_alloc(reinterpret_cast<void**>(p), count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return plan_fail(P, ASP_ERR_OOM, "device allocation failed");
    }
    return ASP_OK;
}

void dev_free(void* p) {
    devmem_free(p);
}

// workgroups of a solve launch per problem of LR rows over `nact` right-hand sides
int groups_of(int nact, int LR) {
    const int srb = solve_rhs_per_block(LR);
    return (nact + srb - 1) / srb;
}

// workgroups of the layer solves of one apply over nrhs right-hand sides: the
// M-solves, then the R and L solves in one launch
long long apply_groups(const asp_plan* P, int nrhs) {
    return std::max((long long)P->m * groups_of(nrhs, P->LR_M),
                    (long long)std::max(2 * P->m - 2, 1) * groups_of(nrhs, P->LR_RL));
}

// forward-substitution scratch for at least `waves` workgroups
asp_status ensure_y(asp_plan* P, long long waves) {
    if (waves <= P->y_waves) return ASP_OK;
    ASP_HIP(P, hipStreamSynchronize(P->stream));
    dev_free(P->d_y);
    P->d_y = nullptr;
    P->y_waves = 0;
    char* y = nullptr;
    if (dev_alloc(P, &y, (size_t)waves * solve_scratch_per_block(P) * elem_bytes(P)) != ASP_OK)
        return ASP_ERR_OOM;
    P->d_y = y;
    P->y_waves = waves;
    return ASP_OK;
}

// algorithmic bytes and flops of a batch of layer solves: each factor entry
// read once per launch, each grid value read and written once per right-hand side
void solve_cost(const asp_plan* P, int sub0, int nsub, int nact, double io_vectors, double* bytes,
                double* flops) {
    double fb = 0, fl = 0;
    for (int s = sub0; s < sub0 + nsub; ++s) {
        fb += factor_bytes_of(P, P->subs[s]);
        const double L = P->subs[s].L;
        fl += 2.0 * P->n * L * L * 8.0;   // forward + backward, L^2 complex MACs per block
    }
    *bytes = fb + io_vectors * nact * (double)P->N * sizeof(zd);
    *flops = fl * nact;
}

}  // namespace

long long apply_scratch_groups(const asp_plan* P, int nrhs) { return apply_groups(P, nrhs); }

size_t solve_scratch_bytes(const asp_plan* P) {
    return (size_t)P->y_waves * solve_scratch_per_block(P) * elem_bytes(P);
}

size_t factor_work_estimate(const asp_plan* P) {
    if (P->dim == 3)
        return P->rec ? rec_factor_work_estimate(P)
                      : P->nd ? nd_factor_work_estimate(P) : factor3d_work_estimate(P);
    return 0;   // 2D: the factorization and the boundary maps use no work buffers
}

double factor_bytes_of(const asp_plan* P, const SubDesc& d) {
    const double B = (P->dim == 2) ? d.L : (double)P->n * d.L;
    return (double)P->n * B * B * elem_bytes(P);
}

// ---------------------------------------------------------------------------
// timing
// ---------------------------------------------------------------------------
KTimer::KTimer(asp_plan* p, int c, double bytes, double flops, int launches)
    : P(p), cls(c), on(p->timing) {
    if (!on) return;
    if (P->tpool_used + 2 > P->tpool.size()) {
        for (int k = 0; k < 64; ++k) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) {
                on = false;
                return;
            }
            P->tpool.push_back(e);
        }
    }
    hipEvent_t a = P->tpool[P->tpool_used++], b = P->tpool[P->tpool_used++];
    P->tev[cls].push_back({a, b, launches});
    P->tbytes[cls] += bytes;
    P->tflops[cls] += flops;
    (void)hipEventRecord(a, P->stream);
}

void KTimer::end() {
    if (on) (void)hipEventRecord(P->tev[cls].back().b, P->stream);
    on = false;
}

extern "C" asp_status asp_timing_enable(asp_plan* P, int enable) {
    if (!P) return ASP_ERR_ARG;
    if (enable) {
        ASP_HIP(P, hipStreamSynchronize(P->stream));
        for (int c = 0; c < ASP_K_COUNT; ++c) {
            P->tev[c].clear();
            P->tbytes[c] = P->tflops[c] = 0;
        }
        P->tpool_used = 0;
    }
    P->timing = enable != 0;
    return ASP_OK;
}

extern "C" asp_status asp_timing_read(asp_plan* P, int cls, int* launches, double* ms,
                                      double* bytes, double* flops) {
    if (!P || cls < 0 || cls >= ASP_K_COUNT) return ASP_ERR_ARG;
    ASP_HIP(P, hipStreamSynchronize(P->stream));
    double tot = 0;
    int nl = 0;
    for (auto& sp : P->tev[cls]) {
        float t = 0;
        ASP_HIP(P, hipEventElapsedTime(&t, sp.a, sp.b));
        tot += t;
        nl += sp.launches;
    }
    if (launches) *launches = nl;
    if (ms) *ms = tot;
    if (bytes) *bytes = P->tbytes[cls];
    if (flops) *flops = P->tflops[cls];
    return ASP_OK;
}

// ---------------------------------------------------------------------------
// workspaces
// ---------------------------------------------------------------------------
asp_status ensure_apply_ws(asp_plan* P, int nrhs) {
    if (P->dim == 3)
        return P->rec ? rec_ensure_ws(P, nrhs) : P->nd ? nd_ensure_ws(P, nrhs) : ensure_apply_ws3(P, nrhs);
    if (nrhs <= P->ws_rhs) return ASP_OK;
    ASP_HIP(P, hipStreamSynchronize(P->stream));
    dev_free(P->d_U);
    dev_free(P->d_W);
    dev_free(P->d_stage);
    dev_free(P->d_wt);
    P->d_U = P->d_W = P->d_stage = nullptr;
    P->d_wt = nullptr;
    P->wt_elems = 0;
    P->ws_rhs = 0;
    P->ws_bytes = 0;
    const size_t vec = (size_t)nrhs * P->N;
    const size_t wlen = (size_t)std::max(2 * P->m - 2, 1) * nrhs * P->n;
    if (dev_alloc(P, &P->d_U, vec) != ASP_OK) return ASP_ERR_OOM;
    if (dev_alloc(P, &P->d_W, wlen) != ASP_OK) return ASP_ERR_OOM;
    if (dev_alloc(P, &P->d_stage, vec) != ASP_OK) return ASP_ERR_OOM;
    {
        const long long we = sweep_wt_len(P, nrhs);
        char* wt = nullptr;
        if (dev_alloc(P, &wt, (size_t)we * elem_bytes(P)) != ASP_OK) return ASP_ERR_OOM;
        P->d_wt = wt;
        P->wt_elems = we;
    }
    asp_status s = ensure_y(P, apply_groups(P, nrhs));
    if (s != ASP_OK) return s;
    P->ws_rhs = nrhs;
    P->ws_bytes = (2 * vec + wlen) * sizeof(zd) + (size_t)P->wt_elems * elem_bytes(P);
    return ASP_OK;
}

// ---------------------------------------------------------------------------
// apply (Algorithm 2)
// ---------------------------------------------------------------------------
// z = M^-1 r for the right-hand-side ids act[0..nact) (device list, NULL for
// 0..nact-1) of batches laid out with stride N.
asp_status apply_internal(asp_plan* P, const zd* r, zd* z, const int* act, int nact) {
    if (P->dim == 3)
        return P->rec ? rec_apply(P, r, z, act, nact)
                      : P->nd ? nd_apply(P, r, z, act, nact) : apply3d_internal(P, r, z, act, nact);
    hipStream_t st = P->stream;
    const int m = P->m;
    const int w_rhs = P->ws_rhs;
    double by, fl;
    // u~_{q,q} = G~^M_q f_q for q = 1..m, all at once
    {
        SolveLaunch L;
        L.job0 = 0;
        L.njobs = m;
        L.act = act;
        L.nact = nact;
        L.in_mode = IN_GRID;
        L.out_mode = OUT_GRID_STORE;
        L.r = r;
        L.out = (m == 1) ? z : P->d_U;
        solve_cost(P, 0, m, nact, 2.0, &by, &fl);
        KTimer t(P, ASP_K_SOLVE_M, by, fl);
        ASP_HIP(P, launch_solve2d(P, L, st));
        t.end();
    }
    if (m == 1) return ASP_OK;
    if (P->sweep_seq) {
        // Algorithm 2 as stated: R_{t+1} and L_{m-t} solved in step t (one launch),
        // each handing its outgoing boundary line (plus u~) to the next problem of
        // its sweep; R outputs a_p in z, L outputs c_p in the staging grid
        double sb = 0, sf = 0;
        for (int t = 1; t <= m - 1; ++t) {
            double b1, f1;
            solve_cost(P, P->idx_R(t + 1), 1, nact, 2.0, &b1, &f1);
            sb += b1;
            sf += f1;
            solve_cost(P, P->idx_L(m - t), 1, nact, 2.0, &b1, &f1);
            sb += b1;
            sf += f1;
        }
        KTimer t(P, ASP_K_SWEEP, sb, sf, 1 + (m - 1) + (m - 2));
        const long long rowR = (long long)P->wrow(P->idx_R(2)) * w_rhs * P->n;
        const long long rowL = (long long)P->wrow(P->idx_L(m - 1)) * w_rhs * P->n;
        ASP_HIP(P, launch_sweep_seed(P, P->d_W, rowR, rowL, act, nact, st));
        const int nsub = (int)P->subs.size();
        for (int s = 1; s <= m - 1; ++s) {
            SolveLaunch L;
            L.job0 = nsub + 2 * (s - 1);
            L.njobs = 2;
            L.rl = true;
            L.act = act;
            L.nact = nact;
            L.in_mode = IN_BOUNDARY;
            L.out_mode = OUT_GRID_STORE;
            L.out = z;
            L.out_mode_L = OUT_GRID_STORE;
            L.out_L = P->d_stage;
            L.W = P->d_W;
            L.w_rhs = w_rhs;
            ASP_HIP(P, launch_solve2d(P, L, st));
            if (s < m - 1)
                ASP_HIP(P, launch_sweep_hand(
                               P, z, P->d_stage, P->d_W,
                               (long long)P->wrow(P->idx_R(s + 2)) * w_rhs * P->n, P->X[s][1],
                               (long long)P->wrow(P->idx_L(m - s - 1)) * w_rhs * P->n,
                               P->X[m - s - 1][0], act, nact, st));
        }
        t.end();
        KTimer tc(P, ASP_K_COMBINE, 5.0 * nact * (double)P->N * sizeof(zd), 0.0);
        ASP_HIP(P, launch_combine3d(P, z, P->d_U, P->d_stage, P->X[0][1], P->X[m - 2][1], true,
                                    act, nact, st));
        tc.end();
        return ASP_OK;
    }
    // the two sweeps: the boundary values u~^R_{p,1:p} and u~^L_{p,p:m}
    // accumulated layer by layer (W rows hold the data entering R_p / L_p); the
    // seed and the m-2 steps are timed as one span of m-1 launches
    {
        const double esz = elem_bytes(P);
        const double nn = (double)P->n * P->n;
        const double steps = m - 2;
        KTimer t(P, ASP_K_SWEEP,
                 4.0 * nact * P->n * sizeof(zd) + steps * (2.0 * nn * esz + 6.0 * nact * P->n * sizeof(zd)),
                 steps * 2.0 * nn * nact * 8.0, m - 1);
        const long long rowR = (long long)P->wrow(P->idx_R(2)) * w_rhs * P->n;
        const long long rowL = (long long)P->wrow(P->idx_L(m - 1)) * w_rhs * P->n;
        ASP_HIP(P, launch_sweep_seed(P, P->d_W, rowR, rowL, act, nact, st));
        for (int s = 1; s <= m - 2; ++s) ASP_HIP(P, launch_sweep_step(P, s, P->d_W, w_rhs, act, nact, st));
        t.end();
    }
    // u~_p = u~_{p,1:p-1} + u~_{p,p} + u~_{p,p+1:m}: one launch of every R_p
    // (z = a on X_p, p > 1) and L_p (c into the staging grid), then
    // z = U + c on X_1, z += U + c on X_p (1 < p < m) and z += U on X_m
    {
        SolveLaunch L;
        L.job0 = P->idx_R(2);
        L.njobs = 2 * m - 2;
        L.rl = true;
        L.act = act;
        L.nact = nact;
        L.in_mode = IN_BOUNDARY;
        L.out_mode = OUT_GRID_STORE;
        L.out = z;
        L.out_mode_L = OUT_GRID_STORE;
        L.out_L = P->d_stage;
        L.W = P->d_W;
        L.w_rhs = w_rhs;
        solve_cost(P, L.job0, 2 * m - 2, nact, 2.0, &by, &fl);
        KTimer t(P, ASP_K_SOLVE_RL, by, fl);
        ASP_HIP(P, launch_solve2d(P, L, st));
        t.end();
    }
    {
        KTimer t(P, ASP_K_COMBINE, 5.0 * nact * (double)P->N * sizeof(zd), 0.0);
        ASP_HIP(P, launch_combine3d(P, z, P->d_U, P->d_stage, P->X[0][1], P->X[m - 2][1], true,
                                    act, nact, st));
        t.end();
    }
    return ASP_OK;
}

// boundary-to-boundary maps: T^R_p = (G~^R_p e_c) on the last line of X_p and
// T^L_p = (G~^L_p e_c) on the first line of X_p, c = 1..n, for 1 < p < m
// The boundary maps T^R_p, T^L_p (1 < p < m): column c of a map is the outgoing
// line of G~ applied to unit data at i1 = c + 1.  With the forward factors
// S_k^-1 and the diagonal blocks G_k of H^-1 (launch_rgf2d), the solution for
// unit data at block c + 1 is the coupling times column grow of G_{c+1} there
// and, towards block 1, x_k = -S_k^-1 E_k x_{k+1}: the map entries on and
// above the diagonal (IN_TWIST kind 0).  The entries below it come from the
// solutions for unit data on the outgoing line (column jout of G_{r+1}), read
// on the data line, since H is complex symmetric (kind 1).  No forward sweep
// and no scratch: a chunk of columns is one chain of at most (ch + 1) SRB steps.
static asp_status compute_transfer(asp_plan* P) {
    const int m = P->m;
    if (m < 3) return ASP_OK;
    const double esz = elem_bytes(P);
    const int nj = m - 2;
    // the diagonal blocks of H^-1 of both sweeps' map problems in one launch
    {
        double fb = 0, fl = 0;
        for (int side = 0; side < 2; ++side) {
            const int first = side == 0 ? P->idx_R(2) : P->idx_L(2);
            for (int s = first; s < first + nj; ++s) {
                const SubDesc& d = P->subs[s];
                fb += factor_bytes_of(P, d);
                fl += (double)P->n * 2.0 * d.L * d.L * d.L * 8.0;   // two L^3 complex products per block
            }
        }
        KTimer t(P, ASP_K_TRANSFER, fb + 2.0 * nj * P->n * 2 * P->LR_RL * esz, fl);
        ASP_HIP(P, launch_rgf2d(P, P->idx_R(2), P->idx_L(2), nj, P->stream));
        t.end();
    }
    for (int side = 0; side < 2; ++side) {
        const int first = side == 0 ? P->idx_R(2) : P->idx_L(2);
        double fb = 0, L2 = 0;
        for (int s = first; s < first + nj; ++s) {
            const SubDesc& d = P->subs[s];
            fb += factor_bytes_of(P, d);
            L2 += (double)d.L * d.L;
        }
        for (int kind = 0; kind < 2; ++kind) {
            SolveLaunch L;
            L.job0 = first;
            L.njobs = nj;
            L.rl = true;
            L.nact = P->n;
            L.in_mode = IN_TWIST;
            L.out_mode = OUT_LINE;
            L.twist_kind = kind;
            // about n^2 / 2 block steps of L^2 complex MACs per problem and kind;
            // the factor read once per chunk over half the blocks on average
            const double chunks = (P->n + solve_rhs_per_block(P->LR_RL) - 1) / solve_rhs_per_block(P->LR_RL);
            const double by = 0.5 * chunks * fb + 0.5 * (double)nj * P->n * P->n * esz;
            const double flk = 0.5 * (double)P->n * P->n * L2 * 8.0;
            KTimer t(P, ASP_K_TRANSFER, by, flk);
            ASP_HIP(P, launch_solve2d(P, L, P->stream));
            t.end();
        }
    }
    return ASP_OK;
}

extern "C" asp_status asp_factor(asp_plan* P) {
    if (!P) return ASP_ERR_ARG;
    if (P->host_only) return plan_fail(P, ASP_ERR_STATE, "host-only plan");
    P->factored = false;
    if (!P->d_fac) {
        char* f = nullptr;
        if (dev_alloc(P, &f, P->fac_bytes) != ASP_OK) return ASP_ERR_OOM;
        P->d_fac = f;
    }
    if (P->dim == 3) {
        ASP_HIP(P, hipMemsetAsync(P->d_flag, 0, sizeof(int), P->stream));
        asp_status s3 = P->rec ? rec_factor(P) : P->nd ? nd_factor(P) : factor3d(P);
        if (s3 != ASP_OK) return s3;
        int flag3 = 0;
        ASP_HIP(P, hipMemcpyAsync(&flag3, P->d_flag, sizeof(int), hipMemcpyDeviceToHost, P->stream));
        ASP_HIP(P, hipStreamSynchronize(P->stream));
        if (flag3)
            return plan_fail(P, ASP_ERR_BREAKDOWN, "zero or non-finite pivot in a layer factorization");
        P->factored = true;
        return ASP_OK;
    }
    if (!P->d_T && P->t_bytes > 0) {
        char* t = nullptr;
        if (dev_alloc(P, &t, P->t_bytes) != ASP_OK) return ASP_ERR_OOM;
        P->d_T = t;
    }
    asp_status s = ASP_OK;
    ASP_HIP(P, hipMemsetAsync(P->d_flag, 0, sizeof(int), P->stream));
    {
        double fb = 0, fl = 0;
        for (const auto& d : P->subs) {
            fb += factor_bytes_of(P, d);
            fl += (double)P->n * ((double)d.L * d.L * d.L + 2.0 * d.L * d.L) * 8.0;
        }
        KTimer t(P, ASP_K_FACTOR, fb + P->N * sizeof(double), fl);
        ASP_HIP(P, launch_factor2d(P, P->stream));
        t.end();
    }
    int flag = 0;
    ASP_HIP(P, hipMemcpyAsync(&flag, P->d_flag, sizeof(int), hipMemcpyDeviceToHost, P->stream));
    ASP_HIP(P, hipStreamSynchronize(P->stream));
    if (flag) return plan_fail(P, ASP_ERR_BREAKDOWN, "zero or non-finite pivot in a layer factorization");
    if (!P->sweep_seq && (s = compute_transfer(P)) != ASP_OK) return s;
    ASP_HIP(P, hipStreamSynchronize(P->stream));
    P->factored = true;
    return ASP_OK;
}

extern "C" asp_status asp_apply(asp_plan* P, const void* r, void* z, int nrhs) {
    if (!P) return ASP_ERR_ARG;
    if (!r || !z || nrhs < 1) return plan_fail(P, ASP_ERR_ARG, "asp_apply: bad arguments");
    if (r == z) return plan_fail(P, ASP_ERR_ARG, "asp_apply: r and z must not alias");
    if (!P->factored) return plan_fail(P, ASP_ERR_STATE, "asp_apply before asp_factor");
    asp_status s = ensure_apply_ws(P, nrhs);
    if (s != ASP_OK) return s;
    return apply_internal(P, static_cast<const zd*>(r), static_cast<zd*>(z), nullptr, nrhs);
}

extern "C" asp_status asp_matvec(asp_plan* P, const void* x, void* y, int nrhs) {
    if (!P) return ASP_ERR_ARG;
    if (!x || !y || nrhs < 1 || x == y) return plan_fail(P, ASP_ERR_ARG, "asp_matvec: bad arguments");
    if (P->host_only) return plan_fail(P, ASP_ERR_STATE, "host-only plan");
    KTimer t(P, ASP_K_STENCIL, (double)nrhs * P->N * 32.0 + P->N * 8.0, 40.0 * nrhs * P->N);
    ASP_HIP(P, launch_stencil(P, static_cast<const zd*>(x), static_cast<zd*>(y), nullptr, nrhs,
                              P->stream));
    t.end();
    return ASP_OK;
}

extern "C" asp_status asp_subsolve(asp_plan* P, int kind, int p, const void* in, void* out,
                                   int nrhs) {
    if (!P) return ASP_ERR_ARG;
    if (!in || !out || nrhs < 1) return plan_fail(P, ASP_ERR_ARG, "asp_subsolve: bad arguments");
    const int m = P->m;
    int idx;
    if (kind == ASP_SUB_M && p >= 1 && p <= m) idx = P->idx_M(p);
    else if (kind == ASP_SUB_R && p >= 2 && p <= m) idx = P->idx_R(p);
    else if (kind == ASP_SUB_L && p >= 1 && p <= m - 1) idx = P->idx_L(p);
    else return plan_fail(P, ASP_ERR_ARG, "asp_subsolve: no such auxiliary problem");
    if (!P->factored) return plan_fail(P, ASP_ERR_STATE, "asp_subsolve before asp_factor");
    asp_status s = ensure_apply_ws(P, nrhs);
    if (s != ASP_OK) return s;
    if (P->dim == 3)
        return P->rec ? rec_subsolve(P, idx, in, out, nrhs)
                      : P->nd ? nd_subsolve(P, idx, in, out, nrhs) : subsolve3d(P, idx, in, out, nrhs);
    const SubDesc& d = P->subs[idx];
    hipStream_t st = P->stream;
    const size_t row = sizeof(zd);
    const long long Np = P->S * (d.xe - d.xs + 1);
    SolveLaunch L;
    L.job0 = idx;
    L.njobs = 1;
    L.rl = kind != ASP_SUB_M;
    L.nact = nrhs;
    L.out_mode = OUT_GRID_STORE;
    L.out = P->d_stage;
    if (kind == ASP_SUB_M) {
        // y on X_p into a grid-shaped copy of the input
        ASP_HIP(P, hipMemcpy2DAsync(P->d_U + (long long)(d.xs - 1) * P->S, P->N * row, in,
                                    Np * row, Np * row, nrhs, hipMemcpyDeviceToDevice, st));
        L.in_mode = IN_GRID;
        L.r = P->d_U;
    } else {
        // w into this problem's boundary-data rows
        ASP_HIP(P, hipMemcpyAsync(P->d_W + (long long)d.wrow * P->ws_rhs * P->n, in,
                                  (size_t)nrhs * P->n * row, hipMemcpyDeviceToDevice, st));
        L.in_mode = IN_BOUNDARY;
        L.W = P->d_W;
        L.w_rhs = P->ws_rhs;
    }
    ASP_HIP(P, launch_solve2d(P, L, st));
    ASP_HIP(P, hipMemcpy2DAsync(out, Np * row, P->d_stage + (long long)(d.xs - 1) * P->S,
                                P->N * row, Np * row, nrhs, hipMemcpyDeviceToDevice, st));
    return ASP_OK;
}

// ---------------------------------------------------------------------------
// workspace accounting
// ---------------------------------------------------------------------------
extern "C" asp_status asp_workspace_estimate(const asp_plan* P, int nrhs, int restart,
                                             size_t* bytes) {
    if (!P || !bytes || nrhs < 1 || restart < 1) return ASP_ERR_ARG;
    const double esz = elem_bytes(P);
    if (P->dim == 3) {
        const double vec3 = (double)nrhs * P->N * sizeof(zd);
        const double kr3 = vec3 * (2.0 * restart + 2.0) + krylov_small_bytes(P->N, nrhs);
        *bytes = (P->rec ? rec_workspace_estimate(P, nrhs)
                  : P->nd ? nd_workspace_estimate(P, nrhs) : workspace_estimate3(P, nrhs)) + (size_t)kr3;
        return ASP_OK;
    }
    const double vec = (double)nrhs * P->N * sizeof(zd);
    const double wrows = (double)std::max(2 * P->m - 2, 1) * nrhs * P->n * sizeof(zd);
    const double wt = (double)sweep_wt_len(P, nrhs) * esz;
    const double y = (double)apply_groups(P, nrhs) * solve_scratch_per_block(P) * esz;
    const double krylov = vec * (2.0 * restart + 2.0) + krylov_small_bytes(P->N, nrhs);
    *bytes = (size_t)(2.0 * vec + wrows + wt + y + krylov);
    return ASP_OK;
}

extern "C" asp_status asp_release_workspace(asp_plan* P) {
    if (!P) return ASP_ERR_ARG;
    if (P->host_only) return ASP_OK;
    ASP_HIP(P, hipStreamSynchronize(P->stream));
    void* bufs[] = {P->d_U, P->d_W, P->d_stage, P->d_wt, P->d_V, P->d_Z, P->d_b, P->d_red,
                    P->d_small, P->d_act, P->d_y3, P->d_g3, P->d_w3, P->d_nd_v, P->d_nd_x,
                    P->d_nd_lb[0], P->d_nd_lb[1], P->d_nd_rb, P->d_nd_db};
    for (void* b : bufs) dev_free(b);
    P->d_nd_v = P->d_nd_x = nullptr;
    rec_free_ws(P);
    P->d_nd_lb[0] = P->d_nd_lb[1] = nullptr;
    P->d_nd_rb = P->d_nd_db = nullptr;
    P->nd_work_bytes = 0;
    P->d_y3 = P->d_g3 = nullptr;
    P->d_w3 = nullptr;
    P->y3_elems = P->w3_elems = 0;
    P->d_U = P->d_W = P->d_stage = nullptr;
    P->d_wt = nullptr;
    P->d_V = P->d_Z = P->d_b = P->d_red = P->d_small = nullptr;
    P->d_act = nullptr;
    P->ws_rhs = 0;
    P->ws_bytes = 0;
    P->wt_elems = 0;
    P->kr_rhs = P->kr_restart = 0;
    P->kr_bytes = 0;
    // the layer solves' scratch (shared by asp_factor and the applies)
    dev_free(P->d_y);
    P->d_y = nullptr;
    P->y_waves = 0;
    return ASP_OK;
}
