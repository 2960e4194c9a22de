// Plan construction: argument checks, the layer partition and auxiliary grids
// (Section 2; Section 3.1 / 4.1 "Auxiliary domains"), the PML tables
// (Section 2 PML profile, evaluated at integer and half-integer lines as in
// eq. (1D)), the descriptors of the 3m-2 auxiliary problems and their upload.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "asp_internal.h"

asp_status plan_fail(asp_plan* p, asp_status s, const std::string& msg) {
    if (p) p->err = msg;
    return s;
}

namespace {

using cd = std::complex<double>;

// sigma at grid coordinate t for a profile vanishing on [phi, psi] (line units):
// (C/eta) (dist/eta)^2 with dist the distance to [phi, psi] and eta = gamma h,
// gamma = g_lo below phi and g_hi above psi (a thinner auxiliary pad on a side
// facing another layer, Section 3.1 remarks).
double sigma_at(double t, double phi, double psi, double C, int g_lo, int g_hi, double h) {
    double dist = 0.0;
    int gamma = g_lo;
    if (t < phi) dist = phi - t;
    if (t > psi) {
        dist = t - psi;
        gamma = g_hi;
    }
    const double eta = gamma * h;
    const double r = dist * h / eta;
    return (C / eta) * r * r;
}

cd s_at(double t, double phi, double psi, double C, int g_lo, int g_hi, double h, double omega) {
    return 1.0 / cd(1.0, sigma_at(t, phi, psi, C, g_lo, g_hi, h) / omega);
}

void fill_tables(int lo, int hi, double phi, double psi, int g_lo, int g_hi, const asp_plan* P,
                 std::vector<cd>& s_int, std::vector<cd>& s_half) {
    s_int.resize(hi - lo + 1);
    s_half.resize(hi - lo + 2);
    for (int t = lo; t <= hi; ++t)
        s_int[t - lo] = s_at(t, phi, psi, P->C, g_lo, g_hi, P->h, P->omega);
    for (int k = 0; k <= hi - lo + 1; ++k)
        s_half[k] = s_at(lo - 0.5 + k, phi, psi, P->C, g_lo, g_hi, P->h, P->omega);
}

template <typename T>
asp_status upload(asp_plan* P, T** dst, const T* src, size_t count) {
    if (devmem_alloc(reinterpret_cast<void**>(dst), count * sizeof(T)) != hipSuccess)
        return plan_fail(P, ASP_ERR_OOM, "hipMalloc of a plan table failed");
    ASP_HIP(P, hipMemcpyAsync(*dst, src, count * sizeof(T), hipMemcpyHostToDevice, P->stream));
    return ASP_OK;
}

zd to_zd(cd v) { return mk(v.real(), v.imag()); }

}  // namespace

// Partition along the sweep axis (1-based lines).  g = gamma - 1 lines carry
// sigma > 0 in each boundary PML; the n_phys = n - 2g physical lines are cut
// into m layers of w_1..w_m lines (uniform: m = ceil(n_phys / b) layers of b,
// the last one holding the remainder; or the caller's widths, Section 3.1
// remarks).  With t_p = gamma + w_1 + ... + w_{p-1}: X_1 = [1, t_2 - 1],
// X_p = [t_p, t_{p+1} - 1], X_m = [t_m, n].
static void build_partition(asp_plan* P, const std::vector<int>& w) {
    const int n = P->n, m = (int)w.size();
    P->X.clear();
    int t = P->gamma;
    for (int p = 0; p < m; ++p) {
        P->X.push_back({p == 0 ? 1 : t, p == m - 1 ? n : t + w[p] - 1});
        t += w[p];
    }
    P->m = m;
}

// Auxiliary problems: M_q on [phi_q - g, psi_q + g] with the sweep-axis PML
// vanishing on X_q's physical part [phi_q, psi_q]; R_p on [s_p, psi_p + g]
// vanishing on [s_p - 1, psi_p] (from the Dirichlet line of D^R_p); L_p on
// [phi_p - g, e_p] vanishing on [phi_p, e_p + 1] (up to the Dirichlet line of D^L_p).
// A pad facing a neighbouring layer has gamma_aux - 1 lines and width gamma_aux
// (the thinner auxiliary PML of the Section 3.1 remarks); a pad at the domain
// boundary is the boundary PML (g lines, width gamma).
static void build_subproblems(asp_plan* P) {
    const int n = P->n, gamma = P->gamma, g = P->g, m = P->m;
    const int ga = P->gamma_aux;
    auto pad_lo = [&](int p) { return p == 1 ? g : ga - 1; };
    auto pad_hi = [&](int p) { return p == m ? g : ga - 1; };
    auto wid_lo = [&](int p) { return p == 1 ? gamma : ga; };
    auto wid_hi = [&](int p) { return p == m ? gamma : ga; };
    P->subs.clear();
    auto phys = [&](int p, int& phi, int& psi) {
        phi = std::max(P->X[p - 1][0], gamma);
        psi = std::min(P->X[p - 1][1], n + 1 - gamma);
    };
    for (int q = 1; q <= m; ++q) {
        SubDesc d{};
        int phi, psi;
        phys(q, phi, psi);
        d.kind = ASP_SUB_M; d.p = q; d.lo = phi - pad_lo(q); d.hi = psi + pad_hi(q);
        d.phi = phi; d.psi = psi;
        d.gam_lo = wid_lo(q); d.gam_hi = wid_hi(q);
        d.src_line = 0;
        P->subs.push_back(d);
    }
    for (int p = 2; p <= m; ++p) {
        SubDesc d{};
        int phi, psi;
        phys(p, phi, psi);
        d.kind = ASP_SUB_R; d.p = p; d.lo = P->X[p - 1][0]; d.hi = psi + pad_hi(p);
        d.phi = P->X[p - 1][0] - 1; d.psi = psi;
        d.gam_lo = d.gam_hi = wid_hi(p);
        d.src_line = P->X[p - 2][1];
        P->subs.push_back(d);
    }
    for (int p = 1; p < m; ++p) {
        SubDesc d{};
        int phi, psi;
        phys(p, phi, psi);
        d.kind = ASP_SUB_L; d.p = p; d.lo = phi - pad_lo(p); d.hi = P->X[p - 1][1];
        d.phi = phi; d.psi = P->X[p - 1][1] + 1;
        d.gam_lo = d.gam_hi = wid_lo(p);
        d.src_line = P->X[p][0];
        P->subs.push_back(d);
    }
    for (auto& d : P->subs) {
        d.L = d.hi - d.lo + 1;
        d.xs = P->X[d.p - 1][0];
        d.xe = P->X[d.p - 1][1];
    }
}

static int rows_per_wave(int L) { return L <= 16 ? 16 : L <= 32 ? 32 : 64; }

extern "C" void asp_default_opts(asp_opts* o) {
    if (!o) return;
    o->C = 25.0;
    o->prec = ASP_PREC_FP64;
    o->stream = nullptr;
    o->host_only = 0;
    o->pml_aux = 0;
    o->n_layers = 0;
    o->layer_widths = nullptr;
    o->fact3d = ASP_FACT3D_ND;
    o->sweep2d = ASP_SWEEP2D_MAPS;
}

extern "C" asp_status asp_setup(asp_plan** out, int dim, const double* c, double omega, int n,
                                int layer_b, int pml_eta, const asp_opts* opts) {
    if (!out) return ASP_ERR_ARG;
    *out = nullptr;
    asp_plan* P = new (std::nothrow) asp_plan();
    if (!P) return ASP_ERR_OOM;
    asp_opts o;
    asp_default_opts(&o);
    if (opts) o = *opts;
    auto fail = [&](asp_status s, const char* msg) {
        // a plan is returned even on failure so that asp_last_error can explain it
        P->err = msg;
        *out = P;
        return s;
    };
    if (dim != 2 && dim != 3) return fail(ASP_ERR_ARG, "dim must be 2 or 3");
    if (!c) return fail(ASP_ERR_ARG, "c is NULL");
    if (!(omega > 0.0) || !std::isfinite(omega)) return fail(ASP_ERR_ARG, "omega must be finite and > 0");
    if (pml_eta < 2) return fail(ASP_ERR_ARG, "pml_eta must be >= 2");
    if (n < 1 || n - 2 * (pml_eta - 1) < 1) return fail(ASP_ERR_ARG, "n too small for the PML");
    std::vector<int> widths;
    const int n_phys = n - 2 * (pml_eta - 1);
    if (o.n_layers < 0) return fail(ASP_ERR_ARG, "n_layers must be >= 0");
    if (o.n_layers > 0) {
        if (!o.layer_widths) return fail(ASP_ERR_ARG, "layer_widths is NULL with n_layers > 0");
        long long sum = 0;
        for (int p = 0; p < o.n_layers; ++p) {
            if (o.layer_widths[p] < 1) return fail(ASP_ERR_ARG, "layer_widths must be >= 1");
            sum += o.layer_widths[p];
        }
        if (sum != n_phys)
            return fail(ASP_ERR_ARG, "layer_widths must sum to n - 2(pml_eta - 1)");
        widths.assign(o.layer_widths, o.layer_widths + o.n_layers);
    } else {
        if (layer_b < 1) return fail(ASP_ERR_ARG, "layer_b must be >= 1");
        const int m = (n_phys + layer_b - 1) / layer_b;
        widths.assign(m, layer_b);
        widths.back() = n_phys - (m - 1) * layer_b;
    }
    if (o.pml_aux != 0 && (o.pml_aux < 2 || o.pml_aux > pml_eta))
        return fail(ASP_ERR_ARG, "pml_aux must be 0 or in [2, pml_eta]");
    if (!(o.C >= 0.0) || !std::isfinite(o.C)) return fail(ASP_ERR_ARG, "C must be finite and >= 0");
    if (o.prec != ASP_PREC_FP64 && o.prec != ASP_PREC_FP32 && o.prec != ASP_PREC_BF16X3)
        return fail(ASP_ERR_ARG, "unknown precision");
    if (dim == 3 && (long long)n * n * n > (1LL << 31)) return fail(ASP_ERR_ARG, "grid too large");
    if (o.fact3d != ASP_FACT3D_ND && o.fact3d != ASP_FACT3D_BLOCKS && o.fact3d != ASP_FACT3D_RECURSIVE)
        return fail(ASP_ERR_ARG, "unknown fact3d");
    if (o.sweep2d != ASP_SWEEP2D_MAPS && o.sweep2d != ASP_SWEEP2D_SEQUENTIAL)
        return fail(ASP_ERR_ARG, "unknown sweep2d");
    if (dim == 3 && o.fact3d == ASP_FACT3D_RECURSIVE && o.n_layers > 0)
        return fail(ASP_ERR_ARG, "the recursive sweep takes equal layer widths (n_layers = 0)");

    P->dim = dim;
    P->n = n;
    P->b = *std::max_element(widths.begin(), widths.end());
    P->gamma = pml_eta;
    P->g = pml_eta - 1;
    P->gamma_aux = o.pml_aux ? o.pml_aux : pml_eta;
    P->omega = omega;
    P->h = 1.0 / (n + 1);
    P->C = o.C;
    P->prec = o.prec;
    P->sweep_seq = dim == 2 && o.sweep2d == ASP_SWEEP2D_SEQUENTIAL;
    P->stream = reinterpret_cast<hipStream_t>(o.stream);
    P->S = (dim == 2) ? n : (long long)n * n;
    P->N = P->S * n;
    try {
        P->c.assign(c, c + P->N);
    } catch (...) {
        return fail(ASP_ERR_OOM, "host allocation of c failed");
    }
    for (long long i = 0; i < P->N; ++i)
        if (!(P->c[i] > 0.0) || !std::isfinite(P->c[i])) return fail(ASP_ERR_ARG, "c must be finite and > 0");

    build_partition(P, widths);
    build_subproblems(P);

    // PML tables: the boundary profile of one axis, and the sweep-axis profile
    // of every auxiliary problem
    fill_tables(1, n, P->gamma, n + 1 - P->gamma, P->gamma, P->gamma, P, P->ax_int, P->ax_half);
    P->sub_int.resize(P->subs.size());
    P->sub_half.resize(P->subs.size());
    int maxL_M = 0, maxL_RL = 0;
    for (size_t s = 0; s < P->subs.size(); ++s) {
        const SubDesc& d = P->subs[s];
        fill_tables(d.lo, d.hi, d.phi, d.psi, d.gam_lo, d.gam_hi, P, P->sub_int[s], P->sub_half[s]);
        if (d.kind == ASP_SUB_M) maxL_M = std::max(maxL_M, d.L);
        else maxL_RL = std::max(maxL_RL, d.L);
    }
    P->max_L = std::max(maxL_M, maxL_RL);
    if (dim == 2 && P->prec == ASP_PREC_FP64 && P->max_L > max_lines_2d<double>(64))
        return fail(ASP_ERR_ARG, "2D auxiliary problems are limited to 48 sweep lines in FP64 "
                                 "(widest layer + 2(pml_eta-1) <= 48)");
    if (dim == 2 && P->max_L > max_lines_2d<float>(64))
        return fail(ASP_ERR_ARG, "2D auxiliary problems are limited to 64 sweep lines "
                                 "(widest layer + 2(pml_eta-1) <= 64)");
    P->LR_M = rows_per_wave(maxL_M);
    P->LR_RL = rows_per_wave(maxL_RL > 0 ? maxL_RL : 1);
    long long fac_off = 0, tab_off = 0, tr_off = 0, vec_off = 0;
    P->Bmax = 0;
    for (size_t s = 0; s < P->subs.size(); ++s) {
        SubDesc& d = P->subs[s];
        d.fac_off = fac_off;
        d.tab_off = tab_off;
        tab_off += sub_table_len(d.L);
        d.wrow = (d.kind == ASP_SUB_M) ? -1 : (int)s - P->m;
        d.tr_off = -1;
        d.g_off = -1;
        d.vec_off = -1;
        if (dim == 2) {
            d.LR = (d.kind == ASP_SUB_M) ? P->LR_M : P->LR_RL;
            d.B = 0;
            fac_off += (long long)n * d.L * d.LR;
            // the sweeps step through R_p and L_p for 1 < p < m with their dense
            // maps, stored in row tiles of 16 (rows padded to a multiple of 16)
            if (!P->sweep_seq && d.kind != ASP_SUB_M && d.p > 1 && d.p < P->m) {
                d.tr_off = tr_off;
                tr_off += (long long)((n + 15) / 16 * 16) * n;
            }
        } else {
            // dense x1-blocks of n L unknowns, padded to a multiple of 64
            d.LR = 0;
            d.B = (n * d.L + 63) / 64 * 64;
            d.vec_off = vec_off;
            vec_off += d.B;
            fac_off += (long long)n * d.B * d.B;
            P->Bmax = std::max(P->Bmax, d.B);
        }
    }
    P->vec_elems = vec_off;
    const size_t esz = (P->prec != ASP_PREC_FP64 ? sizeof(zf) : sizeof(zd));
    P->fac_elems = fac_off;
    P->fac_bytes = (size_t)fac_off * esz;
    if (dim == 3 && o.fact3d == ASP_FACT3D_ND) {
        // nested dissection: the tree, the fronts and the factor size
        P->nd = true;
        asp_status s_nd = nd_setup(P);
        if (s_nd != ASP_OK) return fail(s_nd, P->err.c_str());
    }
    if (dim == 3 && o.fact3d == ASP_FACT3D_RECURSIVE) {
        // the recursive sweep: inner problems along x2 of every slab and their factor size
        asp_status s_rec = rec_setup(P);
        if (s_rec != ASP_OK) return fail(s_rec, P->err.c_str());
    }
    // after the maps: per map problem, columns grow and jout of the diagonal
    // blocks of H^-1 (the boundary maps are built from them)
    for (SubDesc& d : P->subs)
        if (dim == 2 && d.tr_off >= 0) {
            d.g_off = tr_off;
            tr_off += (long long)n * 2 * d.LR;
        }
    P->t_elems = tr_off;
    P->t_bytes = (size_t)tr_off * esz;

    // device tables
    const double h2 = P->h * P->h;
    std::vector<zd> axis(3 * (size_t)n + 1);
    for (int k = 0; k <= n; ++k) axis[k] = to_zd(P->ax_half[k]);
    for (int i = 0; i < n; ++i) axis[n + 1 + i] = to_zd(1.0 / (P->ax_int[i] * h2));
    for (int i = 0; i < n; ++i) axis[2 * n + 1 + i] = to_zd(1.0 / P->ax_int[i]);
    std::vector<zd> subtab((size_t)tab_off);
    for (size_t s = 0; s < P->subs.size(); ++s) {
        const SubDesc& d = P->subs[s];
        zd* t = subtab.data() + d.tab_off;
        for (int k = 0; k <= d.L; ++k) t[k] = to_zd(P->sub_half[s][k]);
        for (int j = 0; j < d.L; ++j) t[d.L + 1 + j] = to_zd(1.0 / (P->sub_int[s][j] * h2));
        for (int j = 0; j < d.L; ++j) t[2 * d.L + 1 + j] = to_zd(1.0 / P->sub_int[s][j]);
    }
    std::vector<double> ksq((size_t)P->N);
    for (long long i = 0; i < P->N; ++i) ksq[i] = (omega * omega) / (P->c[i] * P->c[i]);
    // 3D per-entry vectors: the x1 coupling without its s1 factor, and the
    // Dirichlet data weights of R/L problems (on their first / last line)
    std::vector<zd> e3((size_t)vec_off), gv3((size_t)vec_off);
    if (dim == 3) {
        for (size_t s = 0; s < P->subs.size(); ++s) {
            const SubDesc& d = P->subs[s];
            const int data_line = d.kind == ASP_SUB_R ? 0 : (d.kind == ASP_SUB_L ? d.L - 1 : -1);
            const cd s_data = d.kind == ASP_SUB_R ? P->sub_half[s][0] : P->sub_half[s][d.L];
            for (int j = 0; j < d.B; ++j) {
                zd ev = mk(0.0, 0.0), gv = mk(0.0, 0.0);
                if (j < n * d.L) {
                    const int i3 = j % d.L, i2 = j / d.L;
                    const cd s2 = P->ax_int[i2], s3 = P->sub_int[s][i3];
                    ev = to_zd(1.0 / (s2 * s3 * h2));
                    if (i3 == data_line) gv = to_zd(-s_data / (s2 * h2));
                }
                e3[d.vec_off + j] = ev;
                gv3[d.vec_off + j] = gv;
            }
        }
    }
    P->host_only = (o.host_only != 0);
    if (P->host_only) {
        *out = P;
        return ASP_OK;
    }
    // job list: every auxiliary problem once (M_1..M_m, R_2..R_m, L_1..L_{m-1});
    // a launch takes a contiguous range of it
    std::vector<int> jobs(P->subs.size());
    for (size_t s = 0; s < P->subs.size(); ++s) jobs[s] = (int)s;
    // sweep step t = 1..m-1 runs R_{t+1} and L_{m-t} together (two entries each)
    for (int t = 1; t <= P->m - 1; ++t) {
        jobs.push_back(P->idx_R(t + 1));
        jobs.push_back(P->idx_L(P->m - t));
    }

    asp_status st;
    if ((st = upload(P, &P->d_axis, axis.data(), axis.size())) != ASP_OK) return fail(st, P->err.c_str());
    if ((st = upload(P, &P->d_subtab, subtab.data(), subtab.size())) != ASP_OK) return fail(st, P->err.c_str());
    if ((st = upload(P, &P->d_ksq, ksq.data(), ksq.size())) != ASP_OK) return fail(st, P->err.c_str());
    if ((st = upload(P, &P->d_desc, P->subs.data(), P->subs.size())) != ASP_OK) return fail(st, P->err.c_str());
    if ((st = upload(P, &P->d_jobs, jobs.data(), jobs.size())) != ASP_OK) return fail(st, P->err.c_str());
    if (dim == 3) {
        if ((st = upload(P, &P->d_e3, e3.data(), e3.size())) != ASP_OK) return fail(st, P->err.c_str());
        if ((st = upload(P, &P->d_gv3, gv3.data(), gv3.size())) != ASP_OK) return fail(st, P->err.c_str());
    }
    if (P->nd && (st = nd_upload(P)) != ASP_OK) return fail(st, P->err.c_str());
    if (P->rec && (st = rec_upload(P)) != ASP_OK) return fail(st, P->err.c_str());
    if (devmem_alloc(reinterpret_cast<void**>(&P->d_flag), sizeof(int)) != hipSuccess)
        return fail(ASP_ERR_OOM, "hipMalloc failed");
    if (devmem_alloc(reinterpret_cast<void**>(&P->d_sink), SINK_ELEMS * sizeof(zd)) != hipSuccess)
        return fail(ASP_ERR_OOM, "hipMalloc failed");
    // the host vectors above are released on return: finish the copies first
    if (hipStreamSynchronize(P->stream) != hipSuccess) return fail(ASP_ERR_DEVICE, "upload failed");
    *out = P;
    return ASP_OK;
}

extern "C" void asp_destroy(asp_plan* P) {
    if (!P) return;
    if (P->host_only) {
        delete P;
        return;
    }
    void* bufs[] = {P->d_ksq, P->d_axis, P->d_subtab, P->d_desc, P->d_jobs, P->d_fac, P->d_flag, P->d_sink,
                    P->d_T, P->d_U, P->d_W, P->d_stage, P->d_wt, P->d_y, P->d_V, P->d_Z, P->d_b,
                    P->d_red, P->d_small, P->d_act, P->d_e3, P->d_gv3, P->d_y3,
                    P->d_g3, P->d_w3, P->d_nd_nodes, P->d_nd_cols, P->d_nd_inv, P->d_nd_fronts,
                    P->d_nd_v, P->d_nd_x, P->d_nd_lb[0], P->d_nd_lb[1], P->d_nd_rb, P->d_nd_db,
                    P->d_rec, P->d_rec_sd, P->d_rec_e, P->d_rec_jobs, P->d_rec_sv, P->d_rec_w2,
                    P->d_rec_g, P->d_rec_y};
    (void)hipStreamSynchronize(P->stream);
    for (void* b : bufs)
        devmem_free(b);
    for (hipEvent_t e : P->tpool) (void)hipEventDestroy(e);
    delete P;
}

extern "C" const char* asp_last_error(const asp_plan* P) {
    if (!P) return "no plan";
    return P->err.c_str();
}

extern "C" asp_status asp_set_stream(asp_plan* P, void* stream) {
    if (!P) return ASP_ERR_ARG;
    P->stream = reinterpret_cast<hipStream_t>(stream);
    return ASP_OK;
}

extern "C" asp_status asp_info(const asp_plan* P, asp_plan_info* info) {
    if (!P || !info) return ASP_ERR_ARG;
    info->dim = P->dim;
    info->n = P->n;
    info->m = P->m;
    info->n_sub = (int)P->subs.size();
    info->max_lines = P->max_L;
    info->factor_bytes = P->fac_bytes + P->t_bytes;
    info->workspace_bytes = P->ws_bytes + P->kr_bytes + P->nd_work_bytes + solve_scratch_bytes(P);
    info->factored = P->factored ? 1 : 0;
    info->factor_work_bytes = factor_work_estimate(P);
    return ASP_OK;
}

extern "C" asp_status asp_layers(const asp_plan* P, int* m, int* layers, int* subs) {
    if (!P || !m) return ASP_ERR_ARG;
    *m = P->m;
    if (layers)
        for (int p = 0; p < P->m; ++p) {
            layers[2 * p] = P->X[p][0];
            layers[2 * p + 1] = P->X[p][1];
        }
    if (subs)
        for (size_t s = 0; s < P->subs.size(); ++s) {
            const SubDesc& d = P->subs[s];
            int* o = subs + 6 * s;
            o[0] = d.kind; o[1] = d.p; o[2] = d.lo; o[3] = d.hi; o[4] = d.phi; o[5] = d.psi;
        }
    return ASP_OK;
}

extern "C" asp_status asp_tables(const asp_plan* P, int sub, double* s_int, double* s_half) {
    if (!P || !s_int || !s_half) return ASP_ERR_ARG;
    const std::vector<cd>* a;
    const std::vector<cd>* b;
    if (sub < 0) {
        a = &P->ax_int;
        b = &P->ax_half;
    } else {
        if (sub >= (int)P->subs.size()) return ASP_ERR_ARG;
        a = &P->sub_int[sub];
        b = &P->sub_half[sub];
    }
    for (size_t k = 0; k < a->size(); ++k) {
        s_int[2 * k] = (*a)[k].real();
        s_int[2 * k + 1] = (*a)[k].imag();
    }
    for (size_t k = 0; k < b->size(); ++k) {
        s_half[2 * k] = (*b)[k].real();
        s_half[2 * k + 1] = (*b)[k].imag();
    }
    return ASP_OK;
}
