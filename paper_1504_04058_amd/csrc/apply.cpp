// Factor (Algorithm 1), apply (Algorithm 2), the stencil and the single
// auxiliary-operator hook of the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "asp_internal.h"

namespace {

size_t elem_bytes(const asp_plan* P) { return P->prec == ASP_PREC_FP32 ? sizeof(zf) : sizeof(zd); }

template <typename T>
asp_status dev_alloc(asp_plan* P, T** p, size_t count) {
    if (hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return plan_fail(P, ASP_ERR_OOM, "device allocation failed");
    }
    return ASP_OK;
}

}  // namespace

// apply workspaces for right-hand-side ids 0..nrhs-1
asp_status ensure_apply_ws(asp_plan* P, int nrhs) {
    if (nrhs <= P->ws_rhs) return ASP_OK;
    ASP_HIP(P, hipStreamSynchronize(P->stream));
    zd** vecs[] = {&P->d_U, &P->d_AR, &P->d_CL};
    for (zd** v : vecs)
        if (*v) {
            (void)hipFree(*v);
            *v = nullptr;
        }
    if (P->d_y) (void)hipFree(P->d_y);
    if (P->d_rhs_id) (void)hipFree(P->d_rhs_id);
    P->d_y = nullptr;
    P->d_rhs_id = nullptr;
    P->ws_rhs = 0;
    P->ws_bytes = 0;
    const size_t vec = (size_t)nrhs * P->N;
    for (zd** v : vecs)
        if (dev_alloc(P, v, vec) != ASP_OK) return ASP_ERR_OOM;
    // forward-substitution scratch: one n x L block column per (problem, rhs) wave
    P->y_per_wave = (long long)P->n * P->max_L;
    const long long waves = (long long)std::max(P->m, 2) * nrhs;
    char* y = nullptr;
    if (dev_alloc(P, &y, (size_t)waves * P->y_per_wave * elem_bytes(P)) != ASP_OK) return ASP_ERR_OOM;
    P->d_y = y;
    std::vector<int> ids(nrhs);
    for (int i = 0; i < nrhs; ++i) ids[i] = i;
    if (dev_alloc(P, &P->d_rhs_id, ids.size()) != ASP_OK) return ASP_ERR_OOM;
    ASP_HIP(P, hipMemcpyAsync(P->d_rhs_id, ids.data(), ids.size() * sizeof(int),
                              hipMemcpyHostToDevice, P->stream));
    ASP_HIP(P, hipStreamSynchronize(P->stream));
    P->ws_rhs = nrhs;
    P->ws_bytes = 3 * vec * sizeof(zd) + (size_t)waves * P->y_per_wave * elem_bytes(P);
    return ASP_OK;
}

// z = M^-1 r for the right-hand-side ids act[0..nact) (device list) of batches
// laid out with stride N; Algorithm 2.
asp_status apply_internal(asp_plan* P, const zd* r, zd* z, const int* act, int nact) {
    hipStream_t st = P->stream;
    const int m = P->m;
    // u~_{q,q} = G~^M_q f_q, q = 1..m, all at once
    SolveIO io{r, nullptr, nullptr, nullptr, P->d_U, P->d_AR, P->d_CL};
    ASP_HIP(P, launch_solve2d(P, 0, m, false, act, nact, io, st));
    // step t: u~_{t+1,1:t} = G~^R_{t+1}(...) and u~_{m-t,m-t+1:m} = G~^L_{m-t}(...),
    // their boundary data being the accumulated value on the adjacent line
    // (u~_{p,p} plus the wave accumulated so far).
    for (int t = 1; t < m; ++t) {
        SolveIO s{nullptr, P->d_U, t > 1 ? P->d_AR : nullptr, t > 1 ? P->d_CL : nullptr,
                  P->d_U, P->d_AR, P->d_CL};
        ASP_HIP(P, launch_solve2d(P, m + 2 * (t - 1), 2, true, act, nact, s, st));
    }
    ASP_HIP(P, launch_combine(P, P->d_U, P->d_AR, P->d_CL, z, act, nact, st));
    return ASP_OK;
}

extern "C" asp_status asp_factor(asp_plan* P) {
    if (!P) return ASP_ERR_ARG;
    if (P->factored) return ASP_OK;
    if (P->host_only) return plan_fail(P, ASP_ERR_STATE, "host-only plan");
    if (P->dim != 2) return plan_fail(P, ASP_ERR_ARG, "3D factorization is not available in this build");
    if (!P->d_fac) {
        char* f = nullptr;
        if (dev_alloc(P, &f, P->fac_bytes) != ASP_OK) return ASP_ERR_OOM;
        P->d_fac = f;
    }
    ASP_HIP(P, hipMemsetAsync(P->d_flag, 0, sizeof(int), P->stream));
    ASP_HIP(P, launch_factor2d(P, P->stream));
    int flag = 0;
    ASP_HIP(P, hipMemcpyAsync(&flag, P->d_flag, sizeof(int), hipMemcpyDeviceToHost, P->stream));
    ASP_HIP(P, hipStreamSynchronize(P->stream));
    if (flag) return plan_fail(P, ASP_ERR_BREAKDOWN, "zero or non-finite pivot in a layer factorization");
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
    ASP_HIP(P, launch_stencil(P, static_cast<const zd*>(x), static_cast<zd*>(y), nullptr, nrhs,
                              P->stream));
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
    const SubDesc& d = P->subs[idx];
    hipStream_t st = P->stream;
    const size_t row = sizeof(zd);
    const long long Np = P->S * (d.xe - d.xs + 1);
    zd* tin = P->d_AR;    // grid-shaped staging of the input
    zd* tout = P->d_CL;   // grid-shaped output
    if (kind == ASP_SUB_M) {
        ASP_HIP(P, hipMemcpy2DAsync(tin + (long long)(d.xs - 1) * P->S, P->N * row, in, Np * row,
                                    Np * row, nrhs, hipMemcpyDeviceToDevice, st));
    } else {
        ASP_HIP(P, hipMemcpy2DAsync(tin + (long long)(d.src_line - 1) * P->S, P->N * row, in,
                                    P->S * row, P->S * row, nrhs, hipMemcpyDeviceToDevice, st));
    }
    const int job0 = m + 2 * (m - 1) + idx;   // the "every problem once" job list
    SolveIO io{tin, tin, nullptr, nullptr, tout, tout, tout};
    ASP_HIP(P, launch_solve2d(P, job0, 1, kind != ASP_SUB_M, nullptr, nrhs, io, st));
    ASP_HIP(P, hipMemcpy2DAsync(out, Np * row, tout + (long long)(d.xs - 1) * P->S, P->N * row,
                                Np * row, nrhs, hipMemcpyDeviceToDevice, st));
    return ASP_OK;
}
