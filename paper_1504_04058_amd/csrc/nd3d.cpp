// 3D auxiliary problems by nested dissection (Section 4.1: the unknowns of a
// quasi-2D slab are grouped along the sweep axis into columns, and the
// columns are ordered by nested dissection; Algorithms 3 and 4 otherwise
// unchanged).
//
// The tree is built once over the n x n columns (i1, i2) and shared by every
// auxiliary problem: a region wider than 4 columns in either direction is cut
// by a line of columns across its longer side (the separator, eliminated at
// the node), the two halves become its children; smaller regions are leaves
// and eliminate all their columns.  The factorization is multifrontal, level
// by level from the leaves: a node's dense front holds the original couplings
// of its separator and the Schur complements of its children (extend-add),
// and a Gauss-Jordan elimination of the separator part leaves
//     [ F_II^-1          F_II^-1 F_IB                ]
//     [ -F_BI F_II^-1    F_BB - F_BI F_II^-1 F_IB    ]
// of which the top rows are kept as the factor and the bottom right block is
// passed to the parent.  The operator is complex symmetric (symmetric form),
// so F_BI F_II^-1 = (F_II^-1 F_IB)^T and one block serves both passes:
//     forward (leaves to root):  w = data on I + children's updates,
//                                update to the parent = (B part) - K^T w_I
//     backward (root to leaves): x_I = F_II^-1 w_I - K x_B,   K = F_II^-1 F_IB.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <unordered_map>

#include "asp_internal.h"

namespace {

constexpr int NDT = 64;                 // padding of a front part: the Gauss-Jordan panel width
constexpr int ND_LEAF = 4;              // regions of at most 4 x 4 columns are leaves
constexpr double ND_TRANSIENT = 24e9;   // level-buffer bytes of one factorization group
constexpr int RW = ND_CHUNK;            // right-hand sides per chunk

long long pad64(long long x) { return (x + NDT - 1) / NDT * NDT; }

size_t esz(const asp_plan* P) { return P->prec != ASP_PREC_FP64 ? sizeof(zf) : sizeof(zd); }

// separator panels eliminated two at a time (one pass of the trailing update
// over the front per pair); the bf16-split updates keep one pass per panel
bool look_ahead(const asp_plan* P) { return P->prec != ASP_PREC_BF16X3; }

struct TNode {
    int depth = 0;
    int ch[2] = {-1, -1};
    std::vector<int> I, B;
};

// region [x0, x1] x [y0, y1] of columns (0-based i1, i2); returns the node index
int build_tree(std::vector<TNode>& T, int n, int x0, int x1, int y0, int y1, int depth) {
    const int id = (int)T.size();
    T.emplace_back();
    T[id].depth = depth;
    const int w = x1 - x0 + 1, h = y1 - y0 + 1;
    auto col = [n](int x, int y) { return x + n * y; };
    std::vector<int> I, B;
    int c0 = -1, c1 = -1;
    if (w <= ND_LEAF && h <= ND_LEAF) {
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x) I.push_back(col(x, y));
    } else if (w >= h) {
        const int mid = x0 + (w - 1) / 2;
        for (int y = y0; y <= y1; ++y) I.push_back(col(mid, y));
        if (mid > x0) c0 = build_tree(T, n, x0, mid - 1, y0, y1, depth + 1);
        if (mid < x1) c1 = build_tree(T, n, mid + 1, x1, y0, y1, depth + 1);
    } else {
        const int mid = y0 + (h - 1) / 2;
        for (int x = x0; x <= x1; ++x) I.push_back(col(x, mid));
        if (mid > y0) c0 = build_tree(T, n, x0, x1, y0, mid - 1, depth + 1);
        if (mid < y1) c1 = build_tree(T, n, x0, x1, mid + 1, y1, depth + 1);
    }
    if (x0 > 0)
        for (int y = y0; y <= y1; ++y) B.push_back(col(x0 - 1, y));
    if (x1 < n - 1)
        for (int y = y0; y <= y1; ++y) B.push_back(col(x1 + 1, y));
    if (y0 > 0)
        for (int x = x0; x <= x1; ++x) B.push_back(col(x, y0 - 1));
    if (y1 < n - 1)
        for (int x = x0; x <= x1; ++x) B.push_back(col(x, y1 + 1));
    std::sort(B.begin(), B.end());
    T[id].I = std::move(I);
    T[id].B = std::move(B);
    T[id].ch[0] = c0;
    T[id].ch[1] = c1;
    return id;
}

template <typename T>
asp_status nd_alloc(asp_plan* P, T** p, size_t bytes) {
    if (devmem_alloc(reinterpret_cast<void**>(p), std::max<size_t>(bytes, 16)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return plan_fail(P, ASP_ERR_OOM, "device allocation failed");
    }
    return ASP_OK;
}

template <typename T>
asp_status nd_put(asp_plan* P, T** d, const std::vector<T>& h) {
    asp_status s = nd_alloc(P, d, h.size() * sizeof(T));
    if (s != ASP_OK) return s;
    if (!h.empty())
        ASP_HIP(P, hipMemcpyAsync(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, P->stream));
    return ASP_OK;
}

NdLevel level_of(const asp_plan* P, int d) {
    NdLevel lv;
    lv.fr_all = P->d_nd_fronts;
    lv.front0 = P->nd_lvl_front0[d];
    lv.nn = P->nd_lvl_nodes[d];
    const bool last = d + 1 >= P->nd_levels;
    lv.child0 = last ? -1 : P->nd_lvl_front0[d + 1];
    lv.nnc = last ? 0 : P->nd_lvl_nodes[d + 1];
    return lv;
}

// largest front of level d over problems [s0, s1)
int level_fmax(const asp_plan* P, int d, int s0, int s1) {
    int fm = 0;
    const int nn = P->nd_lvl_nodes[d];
    for (long long i = P->nd_lvl_front0[d] + (long long)s0 * nn;
         i < P->nd_lvl_front0[d] + (long long)s1 * nn; ++i)
        fm = std::max(fm, P->nd_fronts[i].f);
    return fm;
}

// bytes and flops of one solve of problem `sub` (forward reads K, backward [F_II^-1 K])
void solve_cost_nd(const asp_plan* P, int sub, int nact, double* bytes, double* flops) {
    double e = 0, fl = 0;
    for (int d = 0; d < P->nd_levels; ++d) {
        const int nn = P->nd_lvl_nodes[d];
        for (int p = 0; p < nn; ++p) {
            const NdFront& F = P->nd_fronts[P->nd_lvl_front0[d] + (long long)sub * nn + p];
            const NdNode& nd = P->nd_nodes[F.node];
            const double sI = (double)nd.nI * F.L, tB = (double)nd.nB * F.L;   // unpadded
            const double kb = sI * tB, all = sI * (sI + tB);
            e += kb + all;
            fl += 8.0 * (kb + all);
        }
    }
    const SubDesc& s = P->subs[sub];
    *bytes += e * esz(P) + 2.0 * nact * (double)P->S * s.L * sizeof(zd);
    *flops += fl * nact;
}

// forward levels (leaves to root), then backward levels (root to leaves)
asp_status nd_solve(asp_plan* P, const int* jobs, int njobs, int nact) {
    for (int d = P->nd_levels - 1; d >= 0; --d)
        ASP_HIP(P, launch_nd_level(P, level_of(P, d), jobs, njobs, 1, P->nd_lvl_fmax[d], nact, P->stream));
    for (int d = 0; d < P->nd_levels; ++d)
        ASP_HIP(P, launch_nd_level(P, level_of(P, d), jobs, njobs, 0, P->nd_lvl_fmax[d], nact, P->stream));
    return ASP_OK;
}

int nd_solve_launches(const asp_plan* P) { return 3 * P->nd_levels + 2; }

}  // namespace

// The tree, the fronts and their offsets; factor size into P->fac_elems.
asp_status nd_setup(asp_plan* P) {
    const int n = P->n;
    std::vector<TNode> T;
    T.reserve(4 * (size_t)n * n / (ND_LEAF * ND_LEAF) + 8);
    build_tree(T, n, 0, n - 1, 0, n - 1, 0);
    int D = 0;
    for (const auto& t : T) D = std::max(D, t.depth + 1);
    // level-major order; position within the level
    std::vector<std::vector<int>> lv(D);
    for (int i = 0; i < (int)T.size(); ++i) lv[T[i].depth].push_back(i);
    std::vector<int> pos(T.size()), gid(T.size());
    P->nd_levels = D;
    P->nd_lvl_nodes.assign(D, 0);
    P->nd_node0.assign(D, 0);
    int g = 0;
    for (int d = 0; d < D; ++d) {
        P->nd_node0[d] = g;
        P->nd_lvl_nodes[d] = (int)lv[d].size();
        for (int q = 0; q < (int)lv[d].size(); ++q) {
            pos[lv[d][q]] = q;
            gid[lv[d][q]] = g++;
        }
    }
    P->nd_nodes.assign(T.size(), NdNode{});
    P->nd_cols.clear();
    P->nd_inv.clear();
    for (int d = 0; d < D; ++d)
        for (int t : lv[d]) {
            NdNode& nd = P->nd_nodes[gid[t]];
            nd.i_off = (int)P->nd_cols.size();
            nd.nI = (int)T[t].I.size();
            P->nd_cols.insert(P->nd_cols.end(), T[t].I.begin(), T[t].I.end());
            nd.b_off = (int)P->nd_cols.size();
            nd.nB = (int)T[t].B.size();
            P->nd_cols.insert(P->nd_cols.end(), T[t].B.begin(), T[t].B.end());
            for (int c = 0; c < 2; ++c) {
                nd.ch[c] = -1;
                nd.inv_off[c] = -1;
                const int ct = T[t].ch[c];
                if (ct < 0) continue;
                if (T[ct].depth != d + 1) return plan_fail(P, ASP_ERR_ARG, "nested dissection: bad tree");
                nd.ch[c] = pos[ct];
                std::unordered_map<int, int> where;
                for (int j = 0; j < (int)T[ct].B.size(); ++j) where[T[ct].B[j]] = j;
                nd.inv_off[c] = (int)P->nd_inv.size();
                int found = 0;
                auto look = [&](int colid) {
                    auto it = where.find(colid);
                    if (it == where.end()) return -1;
                    ++found;
                    return it->second;
                };
                for (int x : T[t].I) P->nd_inv.push_back(look(x));
                for (int x : T[t].B) P->nd_inv.push_back(look(x));
                // every boundary column of the child is a column of this front
                if (found != (int)T[ct].B.size())
                    return plan_fail(P, ASP_ERR_ARG, "nested dissection: child boundary outside its parent's front");
            }
        }
    // fronts [level][problem][node]; factor, vector and slab offsets
    const int ns = (int)P->subs.size();
    P->nd_fronts.clear();
    P->nd_lvl_front0.assign(D, 0);
    long long moff = 0, voff = 0, xoff = 0;
    for (int s = 0; s < ns; ++s) {
        P->subs[s].xoff = xoff;
        xoff += P->S * P->subs[s].L * RW;
    }
    for (int d = 0; d < D; ++d) {
        P->nd_lvl_front0[d] = (long long)P->nd_fronts.size();
        for (int s = 0; s < ns; ++s) {
            const int L = P->subs[s].L;
            for (int q = 0; q < (int)lv[d].size(); ++q) {
                const NdNode& nd = P->nd_nodes[P->nd_node0[d] + q];
                NdFront F{};
                F.ipad = (int)pad64((long long)nd.nI * L);
                F.f = F.ipad + (int)pad64((long long)nd.nB * L);
                F.L = L;
                F.sub = s;
                F.node = P->nd_node0[d] + q;
                F.moff = moff;
                moff += (long long)F.ipad * F.f;
                F.voff = voff;
                voff += (long long)F.f * RW;
                P->nd_fronts.push_back(F);
            }
        }
    }
    P->fac_elems = moff;
    P->fac_bytes = (size_t)moff * esz(P);
    P->nd_lvl_fmax.assign(D, 0);
    for (int d = 0; d < D; ++d) P->nd_lvl_fmax[d] = level_fmax(P, d, 0, ns);
    P->nd_vtot = voff;
    P->nd_xtot = xoff;
    // factorization groups: problems whose level buffers (two adjacent levels
    // alive at a time) fit the transient budget
    std::vector<std::vector<long long>> lvl_sz(ns, std::vector<long long>(D, 0));
    for (int d = 0; d < D; ++d)
        for (int s = 0; s < ns; ++s)
            for (int q = 0; q < P->nd_lvl_nodes[d]; ++q) {
                const NdFront& F = P->nd_fronts[P->nd_lvl_front0[d] + (long long)s * P->nd_lvl_nodes[d] + q];
                lvl_sz[s][d] += (long long)F.f * F.f;
            }
    P->nd_groups.clear();
    std::vector<long long> acc(D, 0);
    int s0 = 0;
    auto need = [&](const std::vector<long long>& a) {
        long long m = 0;
        for (int d = 0; d < D; ++d) m = std::max(m, a[d] + (d + 1 < D ? a[d + 1] : 0));
        return m;
    };
    for (int s = 0; s < ns; ++s) {
        std::vector<long long> tryv = acc;
        for (int d = 0; d < D; ++d) tryv[d] += lvl_sz[s][d];
        if (s > s0 && (double)need(tryv) * esz(P) > ND_TRANSIENT) {
            P->nd_groups.push_back({s0, s});
            s0 = s;
            std::fill(acc.begin(), acc.end(), 0);
            for (int d = 0; d < D; ++d) acc[d] = lvl_sz[s][d];
        } else {
            acc = tryv;
        }
    }
    P->nd_groups.push_back({s0, ns});
    // level-buffer, panel-buffer and pivot-tile offsets inside each (group, level)
    P->nd_lvlbuf = P->nd_rbuf = 0;
    P->nd_dbuf = 0;
    for (const auto& gr : P->nd_groups)
        for (int d = 0; d < D; ++d) {
            const int nn = P->nd_lvl_nodes[d];
            long long fo = 0, ro = 0;
            for (long long i = P->nd_lvl_front0[d] + (long long)gr[0] * nn;
                 i < P->nd_lvl_front0[d] + (long long)gr[1] * nn; ++i) {
                NdFront& F = P->nd_fronts[i];
                F.foff = fo;
                F.roff = ro;
                fo += (long long)F.f * F.f;
                ro += (long long)F.f * NDT * (look_ahead(P) ? 3 : 1);
            }
            P->nd_lvlbuf = std::max(P->nd_lvlbuf, fo);
            P->nd_rbuf = std::max(P->nd_rbuf, ro);
            P->nd_dbuf = std::max(P->nd_dbuf, (gr[1] - gr[0]) * nn);
        }
    return ASP_OK;
}

asp_status nd_upload(asp_plan* P) {
    asp_status s;
    if ((s = nd_put(P, &P->d_nd_nodes, P->nd_nodes)) != ASP_OK) return s;
    if ((s = nd_put(P, &P->d_nd_cols, P->nd_cols)) != ASP_OK) return s;
    if ((s = nd_put(P, &P->d_nd_inv, P->nd_inv)) != ASP_OK) return s;
    if ((s = nd_put(P, &P->d_nd_fronts, P->nd_fronts)) != ASP_OK) return s;
    return ASP_OK;
}

// Algorithm 3 by nested dissection: every problem of a group, level by level.
asp_status nd_factor(asp_plan* P) {
    hipStream_t st = P->stream;
    const size_t e = esz(P);
    asp_status s = ASP_OK;
    if (!P->d_nd_lb[0]) {
        char* lb0 = nullptr;
        char* lb1 = nullptr;
        char* rb0 = nullptr;
        char* db0 = nullptr;
        if ((s = nd_alloc(P, &lb0, (size_t)P->nd_lvlbuf * e)) != ASP_OK ||
            (s = nd_alloc(P, &lb1, (size_t)P->nd_lvlbuf * e)) != ASP_OK ||
            (s = nd_alloc(P, &rb0, (size_t)P->nd_rbuf * e)) != ASP_OK ||
            (s = nd_alloc(P, &db0, (size_t)P->nd_dbuf * NDT * NDT * e)) != ASP_OK) {
            for (void* b : {(void*)lb0, (void*)lb1, (void*)rb0})
                devmem_free(b);
            return s;
        }
        P->d_nd_lb[0] = lb0;
        P->d_nd_lb[1] = lb1;
        P->d_nd_rb = rb0;
        P->d_nd_db = db0;
        P->nd_work_bytes = nd_factor_work_estimate(P);
    }
    char* lb[2] = {static_cast<char*>(P->d_nd_lb[0]), static_cast<char*>(P->d_nd_lb[1])};
    char* rb = static_cast<char*>(P->d_nd_rb);
    char* db = static_cast<char*>(P->d_nd_db);
    double fb = 0, fl = 0;
    int launches = 0;
    // the method's work, from the unpadded separator (s) and boundary (t)
    // unknowns of each front: LU elimination of the separator, 8 (s^3/3 +
    // s^2 t + s t^2) real flops, and [F_II^-1 | F_II^-1 F_IB] written once.
    // The Gauss-Jordan kernels execute more (the whole padded front, the
    // explicit inverse), which counts as overhead, not as work.
    for (const auto& F : P->nd_fronts) {
        const NdNode& nd = P->nd_nodes[F.node];
        const double sI = (double)nd.nI * F.L, tB = (double)nd.nB * F.L;
        fb += sI * (sI + tB) * e;
        fl += 8.0 * (sI * sI * sI / 3.0 + sI * sI * tB + sI * tB * tB);
    }
    for (const auto& gr : P->nd_groups)
        for (int d = 0; d < P->nd_levels; ++d) {
            int np = 0;
            for (long long i = P->nd_lvl_front0[d] + (long long)gr[0] * P->nd_lvl_nodes[d];
                 i < P->nd_lvl_front0[d] + (long long)gr[1] * P->nd_lvl_nodes[d]; ++i)
                np = std::max(np, P->nd_fronts[i].ipad / NDT);
            launches += 2 + 3 * np;
        }
    {
        KTimer t(P, ASP_K_FACTOR, fb, fl, launches);
        for (const auto& gr : P->nd_groups) {
            for (int d = P->nd_levels - 1; d >= 0 && s == ASP_OK; --d) {
                const NdLevel lv = level_of(P, d);
                const int fmax = level_fmax(P, d, gr[0], gr[1]);
                const int nfr = (gr[1] - gr[0]) * lv.nn;
                const NdFront* fr = P->d_nd_fronts + lv.front0 + (long long)gr[0] * lv.nn;
                int np = 0;
                for (long long i = lv.front0 + (long long)gr[0] * lv.nn; i < lv.front0 + (long long)gr[1] * lv.nn; ++i)
                    np = std::max(np, P->nd_fronts[i].ipad / NDT);
                hipError_t err = launch_nd_assemble(P, lv, gr[0], gr[1], lb[d & 1], lb[(d + 1) & 1], fmax, st);
                if (look_ahead(P)) {
                    for (int jp = 0; jp < np && err == hipSuccess; jp += 2) {
                        err = launch_gj_fronts(P, fr, nfr, lb[d & 1], jp, fmax / NDT, rb, db, 1, st);
                        if (err == hipSuccess && jp + 1 < np)
                            err = launch_gj_fronts(P, fr, nfr, lb[d & 1], jp + 1, fmax / NDT, rb, db, 2, st);
                    }
                } else {
                    for (int jp = 0; jp < np && err == hipSuccess; ++jp)
                        err = launch_gj_fronts(P, fr, nfr, lb[d & 1], jp, fmax / NDT, rb, db, 0, st);
                }
                if (err == hipSuccess) err = launch_nd_copyout(P, fr, nfr, lb[d & 1], fmax, st);
                if (err != hipSuccess)
                    s = plan_fail(P, ASP_ERR_DEVICE, std::string("nested dissection factor launch: ") +
                                                         hipGetErrorString(err));
            }
        }
        t.end();
    }
    return s;
}

size_t nd_factor_work_estimate(const asp_plan* P) {
    return (2 * (size_t)P->nd_lvlbuf + (size_t)P->nd_rbuf + (size_t)P->nd_dbuf * NDT * NDT) * esz(P);
}

size_t nd_workspace_estimate(const asp_plan* P, int nrhs) {
    const double ch = (nrhs + RW - 1) / RW;
    const double vec = (double)nrhs * P->N * sizeof(zd);
    const double we = 4.0 * P->S * ch * RW * sizeof(zd);
    return (size_t)(2.0 * vec + we + ch * (double)(P->nd_vtot + P->nd_xtot) * esz(P));
}

asp_status nd_ensure_ws(asp_plan* P, int nrhs) {
    if (nrhs <= P->ws_rhs) return ASP_OK;
    ASP_HIP(P, hipStreamSynchronize(P->stream));
    void* old[] = {P->d_U, P->d_stage, P->d_w3, P->d_nd_v, P->d_nd_x};
    for (void* b : old)
        devmem_free(b);
    P->d_U = P->d_stage = P->d_w3 = nullptr;
    P->d_nd_v = P->d_nd_x = nullptr;
    P->ws_rhs = 0;
    P->ws_bytes = 0;
    const int chunks = (nrhs + RW - 1) / RW;
    const size_t vec = (size_t)nrhs * P->N * sizeof(zd);
    P->ws3 = chunks * RW;
    const long long we = 2LL * 2 * P->S * P->ws3;
    char* v = nullptr;
    char* x = nullptr;
    if (nd_alloc(P, &P->d_U, vec) != ASP_OK || nd_alloc(P, &P->d_stage, vec) != ASP_OK ||
        nd_alloc(P, &P->d_w3, (size_t)we * sizeof(zd)) != ASP_OK ||
        nd_alloc(P, &v, (size_t)chunks * P->nd_vtot * esz(P)) != ASP_OK ||
        nd_alloc(P, &x, (size_t)chunks * P->nd_xtot * esz(P)) != ASP_OK)
        return ASP_ERR_OOM;
    P->d_nd_v = v;
    P->d_nd_x = x;
    P->w3_elems = we;
    P->ws_rhs = nrhs;
    P->ws_bytes = nd_workspace_estimate(P, nrhs);
    return ASP_OK;
}

// Algorithm 4 with nested-dissection solves, for the right-hand sides act[0..nact)
asp_status nd_apply(asp_plan* P, const zd* r, zd* z, const int* act, int nact) {
    hipStream_t st = P->stream;
    const int m = P->m;
    const int nsub = (int)P->subs.size();
    const int L1 = nd_solve_launches(P);
    {
        double by = 0, fl = 0;
        for (int q = 0; q < m; ++q) solve_cost_nd(P, q, nact, &by, &fl);
        KTimer t(P, ASP_K_SOLVE_M, by, fl, L1);
        ASP_HIP(P, launch_nd_input(P, P->d_jobs, m, IN_GRID, r, nullptr, act, nact, st));
        asp_status s = nd_solve(P, P->d_jobs, m, nact);
        if (s != ASP_OK) return s;
        const int modes[2] = {OUT_GRID_STORE, OUT_GRID_STORE};
        zd* const outs[2] = {(m == 1) ? z : P->d_U, nullptr};
        ASP_HIP(P, launch_nd_output(P, P->d_jobs, m, false, modes, outs, nullptr, nullptr, act, nact, st));
        t.end();
    }
    if (m == 1) return ASP_OK;
    // the two sweeps side by side (as in the block-recurrence path): step t
    // solves R_{t+1} and L_{m-t}; R_p writes z = u~_{p,p} + a_p on X_p, L_p
    // writes c_p into the staging grid, both hand their boundary plane on
    {
        double by = 0, fl = 0;
        for (int t1 = 1; t1 <= m - 1; ++t1) {
            solve_cost_nd(P, P->idx_R(t1 + 1), nact, &by, &fl);
            solve_cost_nd(P, P->idx_L(m - t1), nact, &by, &fl);
        }
        KTimer t(P, ASP_K_SOLVE_RL, by, fl, 1 + (m - 1) * L1);
        const long long plane = 2LL * P->S * P->ws3;
        ASP_HIP(P, launch_plane3d(P, P->d_U, P->X[0][1], P->X[m - 1][0], P->d_w3, act, nact, st));
        for (int t1 = 1; t1 <= m - 1; ++t1) {
            const int* jobs = P->d_jobs + nsub + 2 * (t1 - 1);
            const zd* Win = P->d_w3 + ((t1 - 1) & 1) * plane;
            zd* Wout = (t1 < m - 1) ? P->d_w3 + (t1 & 1) * plane : nullptr;
            ASP_HIP(P, launch_nd_input(P, jobs, 2, IN_BOUNDARY, nullptr, Win, act, nact, st));
            asp_status s = nd_solve(P, jobs, 2, nact);
            if (s != ASP_OK) return s;
            const int modes[2] = {OUT_GRID_ADD_U, OUT_GRID_STORE};
            zd* const outs[2] = {z, P->d_stage};
            ASP_HIP(P, launch_nd_output(P, jobs, 2, true, modes, outs, P->d_U, Wout, act, nact, st));
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

// One auxiliary Green's operator: M data on X_q, or R/L data on the Dirichlet
// line; the output restricted to X_p.
asp_status nd_subsolve(asp_plan* P, int idx, const void* in, void* out, int nrhs) {
    hipStream_t st = P->stream;
    const SubDesc& d = P->subs[idx];
    const size_t row = sizeof(zd);
    const long long Np = P->S * (d.xe - d.xs + 1);
    const int* jobs = P->d_jobs + idx;
    if (d.kind == ASP_SUB_M) {
        ASP_HIP(P, hipMemcpy2DAsync(P->d_U + (long long)(d.xs - 1) * P->S, P->N * row, in,
                                    Np * row, Np * row, nrhs, hipMemcpyDeviceToDevice, st));
        ASP_HIP(P, launch_nd_input(P, jobs, 1, IN_GRID, P->d_U, nullptr, nullptr, nrhs, st));
    } else {
        ASP_HIP(P, hipMemcpy2DAsync(P->d_U, P->N * row, in, P->S * row, P->S * row, nrhs,
                                    hipMemcpyDeviceToDevice, st));
        ASP_HIP(P, launch_plane3d(P, P->d_U, 1, 1, P->d_w3, nullptr, nrhs, st));
        ASP_HIP(P, launch_nd_input(P, jobs, 1, IN_BOUNDARY, nullptr, P->d_w3, nullptr, nrhs, st));
    }
    asp_status s = nd_solve(P, jobs, 1, nrhs);
    if (s != ASP_OK) return s;
    const int modes[2] = {OUT_GRID_STORE, OUT_GRID_STORE};
    zd* const outs[2] = {P->d_stage, nullptr};
    ASP_HIP(P, launch_nd_output(P, jobs, 1, false, modes, outs, nullptr, nullptr, nullptr, nrhs, st));
    ASP_HIP(P, hipMemcpy2DAsync(out, Np * row, P->d_stage + (long long)(d.xs - 1) * P->S,
                                P->N * row, Np * row, nrhs, hipMemcpyDeviceToDevice, st));
    return ASP_OK;
}
