// Host-side exercise of the plan builder for the sanitizer build: host-only
// plans of 2D and 3D problems with equal and unequal layer widths, thin
// auxiliary PML and both 3D factorizations, every query a host-only plan
// answers (sizes, partition, auxiliary grids, PML tables, workspace
// estimates), and the argument checks of asp_setup.  Exit status 0 when every
// call returns what it should.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "asp.h"

static int failures = 0;

#define EXPECT(cond)                                                          \
    do {                                                                      \
        if (!(cond)) {                                                        \
            std::printf("FAIL line %d: %s\n", __LINE__, #cond);               \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

struct Case {
    int dim, n, b, gamma, aux, fact3d;
    std::vector<int> widths;
};

static void exercise(const Case& k) {
    std::vector<double> c((size_t)std::pow(k.n, k.dim), 1.0);
    for (size_t i = 0; i < c.size(); ++i) c[i] = 0.8 + 0.4 * ((i * 7919) % 101) / 100.0;
    asp_opts o;
    asp_default_opts(&o);
    o.host_only = 1;
    o.pml_aux = k.aux;
    o.fact3d = k.fact3d;
    if (!k.widths.empty()) {
        o.n_layers = (int)k.widths.size();
        o.layer_widths = k.widths.data();
    }
    asp_plan* P = nullptr;
    const int st = asp_setup(&P, k.dim, c.data(), 2 * M_PI * (k.n + 1) / 8.0, k.n, k.b, k.gamma, &o);
    EXPECT(st == ASP_OK);
    if (st != ASP_OK) {
        std::printf("  setup: %s\n", asp_last_error(P));
        asp_destroy(P);
        return;
    }
    asp_plan_info info;
    EXPECT(asp_info(P, &info) == ASP_OK);
    EXPECT(info.dim == k.dim && info.n == k.n && info.n_sub == 3 * info.m - 2);
    EXPECT(info.factor_bytes > 0 && info.factored == 0);
    int m = 0;
    EXPECT(asp_layers(P, &m, nullptr, nullptr) == ASP_OK && m == info.m);
    std::vector<int> layers(2 * m), subs(6 * (3 * m - 2));
    EXPECT(asp_layers(P, &m, layers.data(), subs.data()) == ASP_OK);
    // the layers tile 1..n
    EXPECT(layers[0] == 1 && layers[2 * m - 1] == k.n);
    for (int p = 1; p < m; ++p) EXPECT(layers[2 * p] == layers[2 * p - 1] + 1);
    // PML tables: the boundary profile and every auxiliary problem's
    std::vector<double> si(2 * (size_t)k.n), sh(2 * (size_t)(k.n + 1));
    EXPECT(asp_tables(P, -1, si.data(), sh.data()) == ASP_OK);
    for (int s = 0; s < 3 * m - 2; ++s) {
        const int L = subs[6 * s + 3] - subs[6 * s + 2] + 1;
        std::vector<double> ti(2 * (size_t)L), th(2 * (size_t)(L + 1));
        EXPECT(L >= 1 && L <= info.max_lines);
        EXPECT(asp_tables(P, s, ti.data(), th.data()) == ASP_OK);
        for (double v : ti) EXPECT(std::isfinite(v));
    }
    EXPECT(asp_tables(P, 3 * m - 2, si.data(), sh.data()) == ASP_ERR_ARG);
    size_t prev = 0;
    for (int nrhs : {1, 7, 16, 17, 64}) {
        size_t bytes = 0;
        EXPECT(asp_workspace_estimate(P, nrhs, 20, &bytes) == ASP_OK);
        EXPECT(bytes >= prev);
        prev = bytes;
    }
    size_t bytes = 0;
    EXPECT(asp_workspace_estimate(P, 0, 20, &bytes) == ASP_ERR_ARG);
    // calls that need the device are refused by a host-only plan
    EXPECT(asp_factor(P) == ASP_ERR_STATE);
    EXPECT(std::strlen(asp_last_error(P)) > 0);
    asp_destroy(P);
}

static void refused(int dim, int n, int b, int gamma, double omega, double cval, int aux,
                    const std::vector<int>& widths, int fact3d) {
    std::vector<double> c((size_t)std::pow(n > 0 ? n : 1, dim > 0 && dim < 4 ? dim : 2), cval);
    asp_opts o;
    asp_default_opts(&o);
    o.host_only = 1;
    o.pml_aux = aux;
    o.fact3d = fact3d;
    if (!widths.empty()) {
        o.n_layers = (int)widths.size();
        o.layer_widths = widths.data();
    }
    asp_plan* P = nullptr;
    EXPECT(asp_setup(&P, dim, c.data(), omega, n, b, gamma, &o) == ASP_ERR_ARG);
    EXPECT(std::strlen(asp_last_error(P)) > 0);
    asp_destroy(P);
}

int main() {
    const std::vector<Case> cases = {
        {2, 63, 4, 12, 0, 0, {}},          {2, 100, 4, 12, 0, 0, {}},
        {2, 127, 8, 9, 0, 0, {}},          {2, 48, 3, 5, 0, 0, {}},
        {2, 16, 8, 5, 0, 0, {}},           {2, 17, 8, 5, 0, 0, {}},
        {2, 127, 8, 9, 5, 0, {}},          {2, 47, 0, 9, 0, 0, {1, 4, 16, 10}},
        {3, 19, 4, 4, 0, ASP_FACT3D_ND, {}}, {3, 23, 4, 8, 0, ASP_FACT3D_BLOCKS, {}},
        {3, 31, 4, 9, 5, ASP_FACT3D_ND, {}}, {3, 26, 3, 5, 0, ASP_FACT3D_ND, {}},
        {3, 21, 0, 4, 3, ASP_FACT3D_ND, {2, 5, 1, 3, 4}},
    };
    for (const Case& k : cases) exercise(k);
    const std::vector<int> none;
    refused(4, 15, 4, 4, 1.0, 1.0, 0, none, 0);               // dimension
    refused(2, 5, 4, 4, 1.0, 1.0, 0, none, 0);                // no physical line
    refused(2, 31, 0, 4, 1.0, 1.0, 0, none, 0);               // b < 1
    refused(2, 31, 4, 1, 1.0, 1.0, 0, none, 0);               // gamma < 2
    refused(2, 31, 4, 4, 0.0, 1.0, 0, none, 0);               // omega <= 0
    refused(2, 31, 4, 4, 1.0, -1.0, 0, none, 0);              // c <= 0
    refused(2, 31, 4, 4, 1.0, NAN, 0, none, 0);               // c not finite
    refused(2, 31, 4, 4, 1.0, 1.0, 5, none, 0);               // pml_aux > pml_eta
    refused(2, 31, 4, 4, 1.0, 1.0, 1, none, 0);               // pml_aux < 2
    refused(2, 31, 0, 4, 1.0, 1.0, 0, {4, 4, 4}, 0);          // widths do not sum to n - 2g
    refused(2, 31, 0, 4, 1.0, 1.0, 0, {25, 0}, 0);            // a layer of no line
    refused(3, 15, 4, 4, 1.0, 1.0, 0, none, 7);               // unknown 3D factorization
    asp_destroy(nullptr);
    std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
    return failures ? 1 : 0;
}
