// Restarted GMRES with right preconditioning by the additive sweeping
// preconditioner (the outer solver of Sections 3.2 and 4.2), in its flexible
// form: the preconditioned vectors z_j = M^-1 v_j are kept and x = x0 + Z y, so
// the Arnoldi relation A Z_j = V_{j+1} Hbar_j holds whatever precision M^-1
// runs in.  Arnoldi uses classical Gram-Schmidt applied twice, in complex
// double, on the device (the second pass's coefficients from the Gram matrix
// of the basis, so the basis is read twice per step); the Hessenberg least-squares problem (Givens
// rotations) runs on the host in double.  Each right-hand side has its own
// Krylov space; right-hand sides that stop are dropped from every later launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "asp_internal.h"

namespace {

using cd = std::complex<double>;
constexpr int CH = 8;          // vectors per multi-dot / multi-axpy launch
constexpr int SMALL = 256;     // per-RHS slots of the small device array
// layout of the small array per RHS: [0,64) first Gram-Schmidt pass,
// [64,128) second pass, [128] |w|^2, [129,129+CGS_SLOTS) the dots and |w|^2
// after the fused second pass, [192,256) update coefficients
constexpr int OFF_H1 = 0, OFF_H2 = 64, OFF_NRM = 128, OFF_D = 129, OFF_COEF = 192;
static_assert(OFF_D + CGS_SLOTS <= OFF_COEF, "small-array layout");
constexpr int MAX_RESTART = 64;

// elements of the partial-sum buffer per right-hand side
size_t krylov_red_elems(long long N) {
    return std::max((size_t)krylov_blocks(N) * CH, (size_t)cgs_blocks(N) * CGS_SLOTS);
}

template <typename T>
asp_status dev_alloc(asp_plan* P, T** p, size_t count) {
    if (devmem_alloc(reinterpret_cast<void**>(p), count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return plan_fail(P, ASP_ERR_OOM, "device allocation of GMRES workspace failed");
    }
    return ASP_OK;
}

asp_status ensure_krylov_ws(asp_plan* P, int nrhs, int restart) {
    if (nrhs <= P->kr_rhs && restart <= P->kr_restart) return ASP_OK;
    ASP_HIP(P, hipStreamSynchronize(P->stream));
    void* old[] = {P->d_V, P->d_Z, P->d_b, P->d_red, P->d_small, P->d_act};
    for (void* b : old)
        devmem_free(b);
    P->d_V = P->d_Z = P->d_b = P->d_red = P->d_small = nullptr;
    P->d_act = nullptr;
    P->kr_rhs = P->kr_restart = 0;
    P->kr_bytes = 0;
    const size_t vec = (size_t)nrhs * P->N;
    if (dev_alloc(P, &P->d_V, vec * (restart + 1)) != ASP_OK) return ASP_ERR_OOM;
    if (dev_alloc(P, &P->d_Z, vec * restart) != ASP_OK) return ASP_ERR_OOM;
    if (dev_alloc(P, &P->d_b, vec) != ASP_OK) return ASP_ERR_OOM;
    const size_t red = krylov_red_elems(P->N);
    if (dev_alloc(P, &P->d_red, (size_t)nrhs * red) != ASP_OK) return ASP_ERR_OOM;
    // small array, the scales 1/beta, the Gram-matrix columns of each basis
    if (dev_alloc(P, &P->d_small, (size_t)nrhs * (SMALL + 1 + CGS_MAXV * CGS_MAXV)) != ASP_OK)
        return ASP_ERR_OOM;
    if (dev_alloc(P, &P->d_act, (size_t)nrhs) != ASP_OK) return ASP_ERR_OOM;
    P->kr_rhs = nrhs;
    P->kr_restart = restart;
    P->kr_bytes = vec * (2 * restart + 2) * sizeof(zd) + (size_t)nrhs * red * sizeof(zd) +
                  (size_t)nrhs * (SMALL + 1 + CGS_MAXV * CGS_MAXV) * sizeof(zd);
    return ASP_OK;
}

struct RhsState {
    double bnorm = 0, relres = 1;
    int iters = 0;
    bool done = false;
    int steps = 0;                      // Arnoldi steps in the current cycle
    bool inner = false;                 // still iterating in the current cycle
    std::vector<cd> H;                  // (restart+1) x restart, column-major
    std::vector<cd> cs, sn, g;
};

}  // namespace

extern "C" asp_status asp_gmres(asp_plan* P, const void* f_, void* u_, int nrhs, double tol,
                                int restart, int maxit, int* iters, double* relres) {
    if (!P) return ASP_ERR_ARG;
    if (!f_ || !u_ || !iters || !relres || nrhs < 1 || f_ == u_)
        return plan_fail(P, ASP_ERR_ARG, "asp_gmres: bad arguments");
    if (!(tol > 0.0) || restart < 1 || maxit < 1)
        return plan_fail(P, ASP_ERR_ARG, "asp_gmres: need tol > 0, restart >= 1, maxit >= 1");
    if (restart > MAX_RESTART) return plan_fail(P, ASP_ERR_ARG, "asp_gmres: restart > 64");
    asp_status s;
    if (!P->factored && (s = asp_factor(P)) != ASP_OK) return s;
    if ((s = ensure_apply_ws(P, nrhs)) != ASP_OK) return s;
    if ((s = ensure_krylov_ws(P, nrhs, restart)) != ASP_OK) return s;

    hipStream_t st = P->stream;
    const zd* f = static_cast<const zd*>(f_);
    zd* x = static_cast<zd*>(u_);
    const long long N = P->N;
    const long long vs = (long long)nrhs * N;   // stride between Krylov vectors
    zd* V = P->d_V;
    zd* Z = P->d_Z;
    zd* b = P->d_b;
    zd* small = P->d_small;
    zd* scal = P->d_small + (size_t)nrhs * SMALL;
    zd* gram = scal + nrhs;   // [rhs][CGS_MAXV][CGS_MAXV]
    const int nblk = krylov_blocks(N);
    std::vector<zd> hsmall((size_t)nrhs * SMALL + nrhs);
    std::vector<int> act;

    auto upload_act = [&](const std::vector<int>& a) -> asp_status {
        ASP_HIP(P, hipMemcpyAsync(P->d_act, a.data(), a.size() * sizeof(int), hipMemcpyHostToDevice, st));
        return ASP_OK;
    };
    auto download_small = [&]() -> asp_status {
        ASP_HIP(P, hipMemcpyAsync(hsmall.data(), small, hsmall.size() * sizeof(zd),
                                  hipMemcpyDeviceToHost, st));
        ASP_HIP(P, hipStreamSynchronize(st));
        return ASP_OK;
    };
    // |v[r]|^2 for the active list into small[r][OFF_NRM]
    auto norms = [&](const zd* v, int nact) -> asp_status {
        ASP_TIMED(P, ASP_K_KRYLOV, 16.0 * nact * N, 4.0 * nact * N,
                  launch_norms(v, N, P->d_act, nact, P->d_red, st));
        ASP_HIP(P, launch_reduce(P->d_red, nblk, 1, P->d_act, nact, small + OFF_NRM, SMALL, st));
        return ASP_OK;
    };

    // b = f / prod s (symmetric form), x0 = 0
    ASP_TIMED(P, ASP_K_KRYLOV, 32.0 * nrhs * N, 6.0 * nrhs * N, launch_scale_by_s(P, f, b, nrhs, st));
    ASP_HIP(P, hipMemsetAsync(x, 0, (size_t)nrhs * N * sizeof(zd), st));
    std::vector<RhsState> R(nrhs);
    act.resize(nrhs);
    for (int r = 0; r < nrhs; ++r) act[r] = r;
    if ((s = upload_act(act)) != ASP_OK) return s;
    if ((s = norms(b, nrhs)) != ASP_OK) return s;
    if ((s = download_small()) != ASP_OK) return s;
    for (int r = 0; r < nrhs; ++r) {
        R[r].bnorm = std::sqrt(hsmall[(size_t)r * SMALL + OFF_NRM].x);
        R[r].H.assign((size_t)(restart + 1) * restart, 0.0);
        R[r].cs.assign(restart, 0.0);
        R[r].sn.assign(restart, 0.0);
        R[r].g.assign(restart + 1, 0.0);
        if (!(R[r].bnorm > 0.0)) {
            R[r].done = true;   // f = 0: u = 0 exactly
            R[r].relres = 0.0;
            if (!std::isfinite(R[r].bnorm)) return plan_fail(P, ASP_ERR_ARG, "asp_gmres: non-finite f");
        }
    }

    bool first = true;
    while (true) {
        // true residual r0 = b - A x into V_0 for the right-hand sides still running
        act.clear();
        for (int r = 0; r < nrhs; ++r)
            if (!R[r].done) act.push_back(r);
        if (act.empty()) break;
        if ((s = upload_act(act)) != ASP_OK) return s;
        const int na = (int)act.size();
        // the first cycle's residual is b itself (x0 = 0): its norm is |b|,
        // already known, and v_0 = b / |b| is formed straight from b below
        const bool from_b = first;
        if (!from_b) {
            int nb = 0;
            ASP_TIMED(P, ASP_K_STENCIL, 64.0 * na * N + 8.0 * N, 48.0 * na * N,
                      launch_residual(P, b, x, V, P->d_act, na, P->d_red, &nb, st));
            ASP_HIP(P, launch_reduce(P->d_red, nb, 1, P->d_act, na, small + OFF_NRM, SMALL, st));
            if ((s = download_small()) != ASP_OK) return s;
        }
        first = false;
        std::vector<int> cyc;
        for (int r : act) {
            const double beta = from_b ? R[r].bnorm : std::sqrt(hsmall[(size_t)r * SMALL + OFF_NRM].x);
            R[r].relres = beta / R[r].bnorm;
            if (!std::isfinite(beta)) return plan_fail(P, ASP_ERR_BREAKDOWN, "asp_gmres: non-finite residual");
            if (R[r].relres <= tol || R[r].iters >= maxit) {
                R[r].done = true;
                continue;
            }
            std::fill(R[r].H.begin(), R[r].H.end(), cd(0.0));
            std::fill(R[r].g.begin(), R[r].g.end(), cd(0.0));
            R[r].g[0] = beta;
            R[r].steps = 0;
            R[r].inner = true;
            hsmall[(size_t)nrhs * SMALL + r] = mk(1.0 / beta, 0.0);
            cyc.push_back(r);
        }
        if (cyc.empty()) break;
        // v_0 = r0 / beta
        if ((s = upload_act(cyc)) != ASP_OK) return s;
        ASP_HIP(P, hipMemcpyAsync(scal, hsmall.data() + (size_t)nrhs * SMALL, nrhs * sizeof(zd),
                                  hipMemcpyHostToDevice, st));
        ASP_TIMED(P, ASP_K_KRYLOV, 32.0 * cyc.size() * N, 6.0 * cyc.size() * N,
                  launch_scale_vec(from_b ? b : V, V, scal, N, P->d_act, (int)cyc.size(), st));

        std::vector<int> inner = cyc;
        for (int j = 0; j < restart && !inner.empty(); ++j) {
            const int ni = (int)inner.size();
            if ((s = upload_act(inner)) != ASP_OK) return s;
            zd* vj = V + (long long)j * vs;
            zd* zj = Z + (long long)j * vs;
            zd* w = V + (long long)(j + 1) * vs;
            // z_j = M^-1 v_j ; w = A z_j
            if ((s = apply_internal(P, vj, zj, P->d_act, ni)) != ASP_OK) return s;
            ASP_TIMED(P, ASP_K_STENCIL, 32.0 * ni * N + 8.0 * N, 40.0 * ni * N,
                      launch_stencil(P, zj, w, P->d_act, ni, st));
            // classical Gram-Schmidt applied twice against v_0..v_j
            const bool fused = j + 1 <= CGS_MAXV;
            if (fused) {
                // two reads of the basis: h1 = V^H w; the second pass's
                // coefficients h2 = -E h1 from the Gram matrix of the basis
                // (launch_gram); w -= V (h1 + h2) with V^H w (the Gram column of
                // the next basis vector) and |w|^2
                const int nv = j + 1, cb = cgs_blocks(N);
                const double vb = 16.0 * ni * N;
                ASP_TIMED(P, ASP_K_KRYLOV, vb * (nv + 1), 8.0 * nv * ni * N,
                          launch_cgs(0, nv, V, vs, nullptr, 0, w, N, P->d_act, ni, P->d_red, st));
                ASP_HIP(P, launch_cgs_reduce(P->d_red, cb, nv, P->d_act, ni, small + OFF_H1, SMALL, st));
                ASP_HIP(P, launch_gram(small, SMALL, OFF_H1, OFF_H2, OFF_COEF, OFF_D, scal, gram, j,
                                       P->d_act, ni, st));
                ASP_TIMED(P, ASP_K_KRYLOV, vb * (nv + 2), 16.0 * nv * ni * N + 4.0 * ni * N,
                          launch_cgs(1, nv, V, vs, small + OFF_COEF, SMALL, w, N, P->d_act, ni,
                                     P->d_red, st));
                ASP_HIP(P, launch_cgs_reduce(P->d_red, cb, nv + 1, P->d_act, ni, small + OFF_D, SMALL, st));
            } else {
                for (int pass = 0; pass < 2; ++pass) {
                    const int off = pass == 0 ? OFF_H1 : OFF_H2;
                    for (int c0 = 0; c0 <= j; c0 += CH) {
                        const int c1 = std::min(j + 1, c0 + CH);
                        ASP_TIMED(P, ASP_K_KRYLOV, 16.0 * (c1 - c0 + 1) * ni * N, 8.0 * (c1 - c0) * ni * N,
                                  launch_multidot(V, vs, c0, c1, w, N, P->d_act, ni, P->d_red, st));
                        ASP_HIP(P, launch_reduce(P->d_red, nblk, c1 - c0, P->d_act, ni, small + off + c0,
                                                 SMALL, st));
                    }
                    for (int c0 = 0; c0 <= j; c0 += CH) {
                        const int c1 = std::min(j + 1, c0 + CH);
                        const bool last = (pass == 1) && (c1 == j + 1);
                        ASP_TIMED(P, ASP_K_KRYLOV, 16.0 * (c1 - c0 + 2) * ni * N, 8.0 * (c1 - c0) * ni * N,
                                  launch_axpy_multi(V, vs, c0, c1, small + off, SMALL, w, N, P->d_act,
                                                    ni, last ? P->d_red : nullptr, st));
                    }
                }
                ASP_HIP(P, launch_reduce(P->d_red, nblk, 1, P->d_act, ni, small + OFF_NRM, SMALL, st));
            }
            if ((s = download_small()) != ASP_OK) return s;
            std::vector<int> next;
            for (int r : inner) {
                RhsState& q = R[r];
                const zd* hs = hsmall.data() + (size_t)r * SMALL;
                cd* Hc = q.H.data() + (size_t)j * (restart + 1);   // column j
                for (int i = 0; i <= j; ++i)
                    Hc[i] = cd(hs[OFF_H1 + i].x, hs[OFF_H1 + i].y) + cd(hs[OFF_H2 + i].x, hs[OFF_H2 + i].y);
                const double hnext = std::sqrt(fused ? hs[OFF_D + j + 1].x : hs[OFF_NRM].x);
                Hc[j + 1] = hnext;
                if (!std::isfinite(hnext)) return plan_fail(P, ASP_ERR_BREAKDOWN, "asp_gmres: non-finite Arnoldi vector");
                // apply the previous rotations, then a new one that zeroes H(j+1, j)
                for (int i = 0; i < j; ++i) {
                    const cd t = q.cs[i] * Hc[i] + q.sn[i] * Hc[i + 1];
                    Hc[i + 1] = -std::conj(q.sn[i]) * Hc[i] + q.cs[i] * Hc[i + 1];
                    Hc[i] = t;
                }
                const cd a = Hc[j];
                const double bb = std::abs(Hc[j + 1]);
                const double rr = std::hypot(std::abs(a), bb);
                cd c, sv;
                if (std::abs(a) == 0.0) {
                    c = 0.0;
                    sv = 1.0;
                } else {
                    c = std::abs(a) / rr;
                    sv = (a / std::abs(a)) * std::conj(Hc[j + 1]) / rr;
                }
                q.cs[j] = c;
                q.sn[j] = sv;
                Hc[j] = c * a + sv * Hc[j + 1];
                Hc[j + 1] = 0.0;
                q.g[j + 1] = -std::conj(sv) * q.g[j];
                q.g[j] = c * q.g[j];
                q.iters += 1;
                q.steps = j + 1;
                const double est = std::abs(q.g[j + 1]) / q.bnorm;
                if (est <= tol || q.iters >= maxit || hnext == 0.0) {
                    q.inner = false;
                } else {
                    next.push_back(r);
                    hsmall[(size_t)nrhs * SMALL + r] = mk(1.0 / hnext, 0.0);
                }
            }
            inner = next;
            if (!inner.empty() && j + 1 < restart) {
                if ((s = upload_act(inner)) != ASP_OK) return s;
                ASP_HIP(P, hipMemcpyAsync(scal, hsmall.data() + (size_t)nrhs * SMALL, nrhs * sizeof(zd),
                                          hipMemcpyHostToDevice, st));
                ASP_TIMED(P, ASP_K_KRYLOV, 32.0 * inner.size() * N, 6.0 * inner.size() * N,
                          launch_scale_vec(w, w, scal, N, P->d_act, (int)inner.size(), st));
            }
        }
        // x += Z y with R y = g (upper triangular), per right-hand side
        int kmax = 0;
        for (int r : cyc) {
            RhsState& q = R[r];
            const int k = q.steps;
            kmax = std::max(kmax, k);
            std::vector<cd> y(k);
            for (int i = k - 1; i >= 0; --i) {
                cd acc = q.g[i];
                for (int l = i + 1; l < k; ++l) acc -= q.H[(size_t)l * (restart + 1) + i] * y[l];
                y[i] = acc / q.H[(size_t)i * (restart + 1) + i];
            }
            zd* co = hsmall.data() + (size_t)r * SMALL + OFF_COEF;
            for (int i = 0; i < 64; ++i) co[i] = mk(0.0, 0.0);
            for (int i = 0; i < k; ++i) co[i] = mk(-y[i].real(), -y[i].imag());   // x -= (-y) Z
        }
        ASP_HIP(P, hipMemcpyAsync(small, hsmall.data(), (size_t)nrhs * SMALL * sizeof(zd),
                                  hipMemcpyHostToDevice, st));
        if ((s = upload_act(cyc)) != ASP_OK) return s;
        for (int c0 = 0; c0 < kmax; c0 += CH) {
            const int c1 = std::min(kmax, c0 + CH);
            ASP_TIMED(P, ASP_K_KRYLOV, 16.0 * (c1 - c0 + 2) * cyc.size() * N,
                      8.0 * (c1 - c0) * cyc.size() * N,
                      launch_axpy_multi(Z, vs, c0, c1, small + OFF_COEF, SMALL, x, N, P->d_act,
                                        (int)cyc.size(), nullptr, st));
        }
    }
    ASP_HIP(P, hipStreamSynchronize(st));
    bool all = true;
    for (int r = 0; r < nrhs; ++r) {
        iters[r] = R[r].iters;
        relres[r] = R[r].relres;
        if (R[r].relres > tol) all = false;
    }
    if (!all) return plan_fail(P, ASP_ERR_NOCONV, "asp_gmres: maxit reached before tol");
    return ASP_OK;
}

double krylov_small_bytes(long long N, int nrhs) {
    return (double)nrhs * (double)(krylov_red_elems(N) + SMALL + 1 + CGS_MAXV * CGS_MAXV) * sizeof(zd);
}
