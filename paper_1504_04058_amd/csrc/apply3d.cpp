// 3D factor and apply (Algorithms 3 and 4): the block recurrence of every
// auxiliary problem, the M-solves, the two sweeps of R/L solves handing a
// boundary plane from layer to layer, and the accumulation of the layer sums.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "asp_internal.h"

namespace {

constexpr int RW3 = 16;   // right-hand sides per solve chunk
constexpr int TB3 = 64;   // panel width of the block inversion

size_t esz(const asp_plan* P) { return P->prec != ASP_PREC_FP64 ? sizeof(zf) : sizeof(zd); }

template <typename T>
asp_status alloc3(asp_plan* P, T** p, size_t bytes) {
    if (devmem_alloc(reinterpret_cast<void**>(p), bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return plan_fail(P, ASP_ERR_OOM, "device allocation failed");
    }
    return ASP_OK;
}

void free3(void* p) {
    devmem_free(p);
}

int chunks_of(int nrhs) { return (nrhs + RW3 - 1) / RW3; }

// forward / backward results of one launch set: chunks x jobs x n x Bmax x 16
long long y3_len(const asp_plan* P, int nrhs) {
    return (long long)chunks_of(nrhs) * std::max(P->m, 2) * P->n * P->Bmax * RW3;
}

// work of one solve (forward + backward) of the given jobs over nact right-hand sides
void solve3_cost(const asp_plan* P, const int* host_jobs, int njobs, int nact, double* bytes,
                 double* flops) {
    double fb = 0, fl = 0;
    for (int j = 0; j < njobs; ++j) {
        const SubDesc& d = P->subs[host_jobs[j]];
        const double B = (double)P->n * d.L;
        fb += 2.0 * factor_bytes_of(P, d);
        fl += 2.0 * P->n * B * B * 8.0;
    }
    *bytes = fb + 2.0 * nact * (double)P->N * sizeof(zd);
    *flops = fl * nact;
}

// forward pass k = 1..n, then backward pass k = n..1
asp_status run_solve3(asp_plan* P, const Solve3Launch& L) {
    for (int k = 0; k < P->n; ++k) ASP_HIP(P, launch_solve3d_step(P, L, k, 1, P->stream));
    for (int k = P->n - 1; k >= 0; --k) ASP_HIP(P, launch_solve3d_step(P, L, k, 0, P->stream));
    return ASP_OK;
}

}  // namespace

asp_status ensure_apply_ws3(asp_plan* P, int nrhs) {
    if (nrhs <= P->ws_rhs) return ASP_OK;
    ASP_HIP(P, hipStreamSynchronize(P->stream));
    void* old[] = {P->d_U, P->d_stage, P->d_y3, P->d_g3, P->d_w3};
    for (void* b : old) free3(b);
    P->d_U = P->d_stage = nullptr;
    P->d_y3 = P->d_g3 = nullptr;
    P->d_w3 = nullptr;
    P->ws_rhs = 0;
    P->ws_bytes = 0;
    const size_t vec = (size_t)nrhs * P->N * sizeof(zd);
    const long long ye = y3_len(P, nrhs);
    P->ws3 = chunks_of(nrhs) * RW3;
    const long long we = 2LL * 2 * P->S * P->ws3;
    if (alloc3(P, &P->d_U, vec) != ASP_OK) return ASP_ERR_OOM;
    if (alloc3(P, &P->d_stage, vec) != ASP_OK) return ASP_ERR_OOM;
    char* y = nullptr;
    char* g = nullptr;
    if (alloc3(P, &y, (size_t)ye * esz(P)) != ASP_OK) return ASP_ERR_OOM;
    P->d_y3 = y;
    if (alloc3(P, &g, (size_t)ye * esz(P)) != ASP_OK) return ASP_ERR_OOM;
    P->d_g3 = g;
    if (alloc3(P, &P->d_w3, (size_t)we * sizeof(zd)) != ASP_OK) return ASP_ERR_OOM;
    P->y3_elems = ye;
    P->w3_elems = we;
    P->ws_rhs = nrhs;
    P->ws_bytes = 2 * vec + 2 * (size_t)ye * esz(P) + (size_t)we * sizeof(zd);
    return ASP_OK;
}

size_t workspace_estimate3(const asp_plan* P, int nrhs) {
    const double vec = (double)nrhs * P->N * sizeof(zd);
    const double ye = (double)y3_len(P, nrhs) * esz(P);
    const double we = 4.0 * P->S * chunks_of(nrhs) * RW3 * sizeof(zd);
    return (size_t)(2.0 * vec + 2.0 * ye + we);
}

size_t factor3d_work_estimate(const asp_plan* P) {
    const size_t nsub = P->subs.size();
    return nsub * ((size_t)P->Bmax * TB3 + (size_t)TB3 * TB3) * esz(P);
}

// Algorithm 3: every auxiliary problem at once, block k after block k-1; each
// block inverse is a sequence of 64-wide Gauss-Jordan panels.
asp_status factor3d(asp_plan* P) {
    hipStream_t st = P->stream;
    const int nsub = (int)P->subs.size();
    char* Rbuf = nullptr;
    char* Dbuf = nullptr;
    if (alloc3(P, &Rbuf, (size_t)nsub * P->Bmax * TB3 * esz(P)) != ASP_OK) return ASP_ERR_OOM;
    if (alloc3(P, &Dbuf, (size_t)nsub * TB3 * TB3 * esz(P)) != ASP_OK) {
        free3(Rbuf);
        return ASP_ERR_OOM;
    }
    asp_status s = ASP_OK;
    double fb = 0, fl = 0;
    for (const auto& d : P->subs) {
        const double B = (double)P->n * d.L;
        fb += factor_bytes_of(P, d);
        fl += (double)P->n * B * B * B * 8.0;
    }
    {
        KTimer t(P, ASP_K_FACTOR, fb, fl);
        const int ntmax = P->Bmax / TB3;
        for (int k = 0; k < P->n && s == ASP_OK; ++k) {
            hipError_t e = launch_form3d(P, P->d_jobs, nsub, k, st);
            for (int jp = 0; jp < ntmax && e == hipSuccess; ++jp)
                e = launch_gj3d(P, P->d_jobs, nsub, k, jp, Rbuf, Dbuf, st);
            if (e != hipSuccess)
                s = plan_fail(P, ASP_ERR_DEVICE, std::string("3D factor launch: ") + hipGetErrorString(e));
        }
        t.end();
    }
    (void)hipStreamSynchronize(st);
    free3(Rbuf);
    free3(Dbuf);
    return s;
}

// Algorithm 4 for the right-hand sides act[0..nact) (NULL: 0..nact-1)
asp_status apply3d_internal(asp_plan* P, const zd* r, zd* z, const int* act, int nact) {
    hipStream_t st = P->stream;
    const int m = P->m;
    const int nsub = (int)P->subs.size();
    double by, fl;
    // u~_{q,q} = G~^M_q f_q, q = 1..m
    {
        std::vector<int> hj(m);
        for (int q = 0; q < m; ++q) hj[q] = q;
        solve3_cost(P, hj.data(), m, nact, &by, &fl);
        KTimer t(P, ASP_K_SOLVE_M, by, fl);
        ASP_HIP(P, launch_gather3d(P, P->d_jobs, m, r, act, nact, st));
        Solve3Launch L;
        L.jobs = P->d_jobs;
        L.njobs = m;
        L.act = act;
        L.nact = nact;
        L.in_mode = IN_GRID;
        L.out_mode[0] = OUT_GRID_STORE;
        L.out[0] = (m == 1) ? z : P->d_U;
        asp_status s = run_solve3(P, L);
        t.end();
        if (s != ASP_OK) return s;
    }
    if (m == 1) return ASP_OK;
    // the two sweeps, side by side: step t solves R_{t+1} (data: u~ + a on the
    // last line of X_t) and L_{m-t} (data: u~ + c on the first line of X_{m-t+1});
    // R_p writes z = u~_{p,p} + a_p on X_p, L_p writes c_p into the staging grid
    {
        by = fl = 0;
        for (int t1 = 1; t1 <= m - 1; ++t1) {
            const int hj[2] = {P->idx_R(t1 + 1), P->idx_L(m - t1)};
            double b1, f1;
            solve3_cost(P, hj, 2, nact, &b1, &f1);
            by += b1;
            fl += f1;
        }
        KTimer t(P, ASP_K_SOLVE_RL, by, fl);
        const long long plane = 2LL * P->S * P->ws3;   // both sides of one ping-pong half
        ASP_HIP(P, launch_plane3d(P, P->d_U, P->X[0][1], P->X[m - 1][0], P->d_w3, act, nact, st));
        for (int t1 = 1; t1 <= m - 1; ++t1) {
            Solve3Launch L;
            L.jobs = P->d_jobs + nsub + 2 * (t1 - 1);
            L.njobs = 2;
            L.two_sided = true;
            L.act = act;
            L.nact = nact;
            L.in_mode = IN_BOUNDARY;
            L.Win = P->d_w3 + ((t1 - 1) & 1) * plane;
            L.Wout = (t1 < m - 1) ? P->d_w3 + (t1 & 1) * plane : nullptr;
            L.out_mode[0] = OUT_GRID_ADD_U;
            L.out[0] = z;
            L.out_mode[1] = OUT_GRID_STORE;
            L.out[1] = P->d_stage;
            L.Ugrid = P->d_U;
            asp_status s = run_solve3(P, L);
            if (s != ASP_OK) return s;
        }
        t.end();
    }
    // u~_1 = u~_{1,1} + c_1;  u~_p += c_p for 1 < p < m
    {
        KTimer t(P, ASP_K_COMBINE, 4.0 * nact * (double)P->N * sizeof(zd), 0.0);
        ASP_HIP(P, launch_combine3d(P, z, P->d_U, P->d_stage, P->X[0][1], P->X[m - 2][1], false,
                                    act, nact, st));
        t.end();
    }
    return ASP_OK;
}

// One auxiliary Green's operator (test hook): M data on X_q, or R/L data on
// the Dirichlet line; the output restricted to X_p.
asp_status subsolve3d(asp_plan* P, int idx, const void* in, void* out, int nrhs) {
    hipStream_t st = P->stream;
    const SubDesc& d = P->subs[idx];
    const size_t row = sizeof(zd);
    const long long Np = P->S * (d.xe - d.xs + 1);
    Solve3Launch L;
    L.jobs = P->d_jobs + idx;
    L.njobs = 1;
    L.nact = nrhs;
    L.out_mode[0] = OUT_GRID_STORE;
    L.out[0] = P->d_stage;
    if (d.kind == ASP_SUB_M) {
        ASP_HIP(P, hipMemcpy2DAsync(P->d_U + (long long)(d.xs - 1) * P->S, P->N * row, in,
                                    Np * row, Np * row, nrhs, hipMemcpyDeviceToDevice, st));
        ASP_HIP(P, launch_gather3d(P, L.jobs, 1, P->d_U, nullptr, nrhs, st));
        L.in_mode = IN_GRID;
    } else {
        // the plane data into line 1 of a grid-shaped buffer, then into the plane layout
        ASP_HIP(P, hipMemcpy2DAsync(P->d_U, P->N * row, in, P->S * row, P->S * row, nrhs,
                                    hipMemcpyDeviceToDevice, st));
        ASP_HIP(P, launch_plane3d(P, P->d_U, 1, 1, P->d_w3, nullptr, nrhs, st));
        L.in_mode = IN_BOUNDARY;
        L.Win = P->d_w3;
    }
    asp_status s = run_solve3(P, L);
    if (s != ASP_OK) return s;
    ASP_HIP(P, hipMemcpy2DAsync(out, Np * row, P->d_stage + (long long)(d.xs - 1) * P->S,
                                P->N * row, Np * row, nrhs, hipMemcpyDeviceToDevice, st));
    return ASP_OK;
}
