// Host-side check of the nested-dissection structures of a plan (Section 4.1):
// builds a host-only 3D plan, then factors and solves every auxiliary problem
// on the CPU in complex double exactly as the device path is organised -- the
// plan's elimination tree, front column lists, child maps, front padding,
// separator elimination by Gauss-Jordan without pivoting, forward and backward
// passes using K = F_II^-1 F_IB and its transpose -- and checks the residual of
// each solution against the slab operator's 7-point couplings, written out
// independently of the fronts.  Arguments: n b gamma gamma_aux; exit status 0
// when every relative residual is below 1e-10.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <map>
#include "asp_internal.h"

typedef std::complex<double> C;

int main(int argc, char** argv) {
    int n = argc > 1 ? atoi(argv[1]) : 11;
    int b = argc > 2 ? atoi(argv[2]) : 3;
    int gamma = argc > 3 ? atoi(argv[3]) : 3;
    int aux = argc > 4 ? atoi(argv[4]) : 0;
    std::mt19937 rng(7);
    std::uniform_real_distribution<double> U(0.8, 1.2), Nn(-1, 1);
    std::vector<double> c((size_t)n * n * n);
    for (auto& v : c) v = U(rng);
    asp_opts o;
    asp_default_opts(&o);
    o.host_only = 1;
    o.fact3d = ASP_FACT3D_ND;
    o.pml_aux = aux;
    asp_plan* P = nullptr;
    double omega = 2 * M_PI * (n + 1) / 8.0;
    int st = asp_setup(&P, 3, c.data(), omega, n, b, gamma, &o);
    if (st) { printf("setup failed %d %s\n", st, asp_last_error(P)); return 1; }
    const double h = P->h, h2 = h * h;
    printf("n=%d levels=%d nodes=%zu fronts=%zu groups=%zu fac=%.3f MB\n", n, P->nd_levels, P->nd_nodes.size(),
           P->nd_fronts.size(), P->nd_groups.size(), P->fac_bytes / 1e6);
    for (int d = 0; d < P->nd_levels; ++d) printf("  level %d nodes %d fmax %d\n", d, P->nd_lvl_nodes[d], P->nd_lvl_fmax[d]);
    const long long S = (long long)n * n;
    auto sh = [&](int k) { return P->ax_half.at(k); };
    auto inv_s = [&](int i) { return 1.0 / P->ax_int.at(i); };
    auto inv_sh2 = [&](int i) { return 1.0 / (P->ax_int.at(i) * h2); };
    double worst = 0;
    for (size_t s = 0; s < P->subs.size(); ++s) {
        const SubDesc& d = P->subs[s];
        const int L = d.L;
        auto sh3 = [&](int k) { return P->sub_half[s].at(k); };
        auto ish3 = [&](int j) { return 1.0 / (P->sub_int[s].at(j) * h2); };
        auto is3 = [&](int j) { return 1.0 / P->sub_int[s].at(j); };
        // dense operator entry between (col, k) and (col2, k2)
        auto A = [&](int colr, int kr, int colc, int kc) -> C {
            int i1r = colr % n, i2r = colr / n, i1c = colc % n, i2c = colc / n;
            if (colr == colc) {
                if (kr == kc) {
                    C s23 = inv_s(i2r) * ish3(kr), s13 = inv_s(i1r) * ish3(kr), s12 = inv_s(i1r) * inv_sh2(i2r);
                    C c1 = (sh(i1r + 1) + sh(i1r)) * s23, c2 = (sh(i2r + 1) + sh(i2r)) * s13, c3 = (sh3(kr + 1) + sh3(kr)) * s12;
                    long long g = colr + S * (d.lo - 1 + kr);
                    double ksq = omega * omega / (c[g] * c[g]);
                    return ksq * inv_s(i1r) * inv_s(i2r) * is3(kr) - (c1 + c2 + c3);
                }
                if (std::abs(kr - kc) == 1) return sh3(std::max(kr, kc)) * (inv_s(i1r) * inv_sh2(i2r));
                return 0;
            }
            if (kr != kc) return 0;
            if (i2r == i2c && std::abs(i1r - i1c) == 1) return sh(std::max(i1r, i1c)) * (inv_s(i2r) * ish3(kr));
            if (i1r == i1c && std::abs(i2r - i2c) == 1) return sh(std::max(i2r, i2c)) * (inv_s(i1r) * ish3(kr));
            return 0;
        };
        // multifrontal factorization, emulated
        std::map<long long, std::vector<C>> Fs;   // front index -> dense front (kept for the parent)
        std::map<long long, std::vector<C>> Ms;   // factor blocks
        for (int dl = P->nd_levels - 1; dl >= 0; --dl) {
            int nn = P->nd_lvl_nodes[dl];
            for (int pos = 0; pos < nn; ++pos) {
                long long fi = P->nd_lvl_front0[dl] + (long long)s * nn + pos;
                const NdFront& F = P->nd_fronts.at(fi);
                const NdNode& nd = P->nd_nodes.at(F.node);
                if (F.L != L || F.sub != (int)s) { printf("front mismatch\n"); return 1; }
                int f = F.f, ipad = F.ipad;
                std::vector<C> M((size_t)f * f, 0.0);
                auto decode = [&](int r, int& cc, int& k, int& part) {
                    if (r < ipad) { cc = r / L; k = r % L; part = r < nd.nI * L ? 0 : 2; if (part == 2) cc = -1; }
                    else { int q = r - ipad; cc = nd.nI + q / L; k = q % L; part = q < nd.nB * L ? 1 : 3; if (part == 3) cc = -1; }
                };
                auto fcol = [&](int cc) { return cc < nd.nI ? P->nd_cols.at(nd.i_off + cc) : P->nd_cols.at(nd.b_off + cc - nd.nI); };
                for (int cI = 0; cI < f; ++cI)
                    for (int r = 0; r < f; ++r) {
                        int cr, kr, pr, ccn, kc, pc;
                        decode(r, cr, kr, pr);
                        decode(cI, ccn, kc, pc);
                        C val = 0;
                        if (pr >= 2 || pc >= 2) { val = (r == cI && pr == 2) ? 1.0 : 0.0; }
                        else {
                            if (cr < nd.nI || ccn < nd.nI) val = A(fcol(cr), kr, fcol(ccn), kc);
                            if (dl + 1 < P->nd_levels)
                                for (int ch = 0; ch < 2; ++ch) {
                                    if (nd.inv_off[ch] < 0) continue;
                                    int a1 = P->nd_inv.at(nd.inv_off[ch] + cr), a2 = P->nd_inv.at(nd.inv_off[ch] + ccn);
                                    if (a1 < 0 || a2 < 0) continue;
                                    long long cfi = P->nd_lvl_front0[dl + 1] + (long long)s * P->nd_lvl_nodes[dl + 1] + nd.ch[ch];
                                    const NdFront& Cf = P->nd_fronts.at(cfi);
                                    const std::vector<C>& Uc = Fs.at(cfi);
                                    val += Uc.at((size_t)(Cf.ipad + a2 * L + kc) * Cf.f + Cf.ipad + a1 * L + kr);
                                }
                        }
                        M[(size_t)cI * f + r] = val;
                    }
                // partial Gauss-Jordan over pivots 0..ipad-1 (scalar pivots, no pivoting)
                for (int p = 0; p < ipad; ++p) {
                    C piv = M[(size_t)p * f + p];
                    if (std::abs(piv) < 1e-300) { printf("zero pivot\n"); return 1; }
                    C pinv = 1.0 / piv;
                    std::vector<C> rowp(f), colp(f);
                    for (int j = 0; j < f; ++j) rowp[j] = M[(size_t)j * f + p];
                    for (int i = 0; i < f; ++i) colp[i] = M[(size_t)p * f + i];
                    for (int j = 0; j < f; ++j)
                        for (int i = 0; i < f; ++i) {
                            if (i == p && j == p) M[(size_t)j * f + i] = pinv;
                            else if (i == p) M[(size_t)j * f + i] = rowp[j] * pinv;
                            else if (j == p) M[(size_t)j * f + i] = -colp[i] * pinv;
                            else M[(size_t)j * f + i] -= colp[i] * pinv * rowp[j];
                        }
                }
                std::vector<C> Mk((size_t)ipad * f);
                for (int j = 0; j < f; ++j)
                    for (int i = 0; i < ipad; ++i) Mk[(size_t)j * ipad + i] = M[(size_t)j * f + i];
                Ms[fi] = Mk;
                Fs[fi] = M;
            }
        }
        // solve with a random right-hand side
        const long long Ns = S * L;
        std::vector<C> rhs(Ns), x(Ns);
        for (auto& v : rhs) v = C(Nn(rng), Nn(rng));
        x = rhs;
        std::map<long long, std::vector<C>> V;
        for (int dl = P->nd_levels - 1; dl >= 0; --dl) {
            int nn = P->nd_lvl_nodes[dl];
            for (int pos = 0; pos < nn; ++pos) {
                long long fi = P->nd_lvl_front0[dl] + (long long)s * nn + pos;
                const NdFront& F = P->nd_fronts.at(fi);
                const NdNode& nd = P->nd_nodes.at(F.node);
                int f = F.f, ipad = F.ipad;
                std::vector<C> v(f, 0.0);
                for (int r = 0; r < f; ++r) {
                    int cc = -1, k = 0, part;
                    if (r < ipad) { cc = r / L; k = r % L; part = r < nd.nI * L ? 0 : 2; }
                    else { int q = r - ipad; cc = nd.nI + q / L; k = q % L; part = q < nd.nB * L ? 1 : 3; }
                    if (part == 0) v[r] = x.at((long long)P->nd_cols.at(nd.i_off + cc) * L + k);
                    if (part <= 1 && dl + 1 < P->nd_levels)
                        for (int ch = 0; ch < 2; ++ch) {
                            if (nd.inv_off[ch] < 0) continue;
                            int cs = P->nd_inv.at(nd.inv_off[ch] + cc);
                            if (cs < 0) continue;
                            long long cfi = P->nd_lvl_front0[dl + 1] + (long long)s * P->nd_lvl_nodes[dl + 1] + nd.ch[ch];
                            const NdFront& Cf = P->nd_fronts.at(cfi);
                            v[r] += V.at(cfi).at(Cf.ipad + cs * L + k);
                        }
                }
                const std::vector<C>& Mk = Ms.at(fi);
                for (int j = 0; j < f - ipad; ++j) {
                    C acc = 0;
                    for (int r = 0; r < ipad; ++r) acc += Mk.at((size_t)(ipad + j) * ipad + r) * v[r];
                    v[ipad + j] -= acc;
                }
                V[fi] = v;
            }
        }
        for (int dl = 0; dl < P->nd_levels; ++dl) {
            int nn = P->nd_lvl_nodes[dl];
            for (int pos = 0; pos < nn; ++pos) {
                long long fi = P->nd_lvl_front0[dl] + (long long)s * nn + pos;
                const NdFront& F = P->nd_fronts.at(fi);
                const NdNode& nd = P->nd_nodes.at(F.node);
                int f = F.f, ipad = F.ipad;
                const std::vector<C>& v = V.at(fi);
                const std::vector<C>& Mk = Ms.at(fi);
                std::vector<C> z(f, 0.0);
                for (int cI = 0; cI < f; ++cI) {
                    if (cI < ipad) z[cI] = v[cI];
                    else {
                        int q = cI - ipad;
                        if (q < nd.nB * L) z[cI] = -x.at((long long)P->nd_cols.at(nd.b_off + q / L) * L + q % L);
                    }
                }
                for (int r = 0; r < nd.nI * L; ++r) {
                    C acc = 0;
                    for (int cI = 0; cI < f; ++cI) acc += Mk.at((size_t)cI * ipad + r) * z[cI];
                    x.at((long long)P->nd_cols.at(nd.i_off + r / L) * L + r % L) = acc;
                }
            }
        }
        // residual with the dense operator
        double rn = 0, bn = 0;
        for (long long u = 0; u < Ns; ++u) {
            int col = (int)(u / L), k = (int)(u % L);
            C acc = 0;
            int i1 = col % n, i2 = col / n;
            int nb[7][2] = {{col, k}, {col, k - 1}, {col, k + 1}, {col - 1, k}, {col + 1, k}, {col - n, k}, {col + n, k}};
            bool ok[7] = {true, k > 0, k < L - 1, i1 > 0, i1 < n - 1, i2 > 0, i2 < n - 1};
            for (int t = 0; t < 7; ++t)
                if (ok[t]) acc += A(col, k, nb[t][0], nb[t][1]) * x[(long long)nb[t][0] * L + nb[t][1]];
            rn += std::norm(acc - rhs[u]);
            bn += std::norm(rhs[u]);
        }
        double rel = std::sqrt(rn / bn);
        worst = std::max(worst, rel);
        if (s < 3 || rel > 1e-10) printf("sub %zu kind %d L %d rel residual %.3e\n", s, d.kind, L, rel);
    }
    printf("worst %.3e\n", worst);
    asp_destroy(P);
    return worst < 1e-10 ? 0 : 1;
}
