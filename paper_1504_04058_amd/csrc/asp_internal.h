// Internal declarations of the asp library: plan layout, descriptors of the
// auxiliary problems, complex arithmetic helpers and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/asp.h"

// ---------------------------------------------------------------------------
// complex arithmetic (interleaved re/im, the layout of complex128 / complex64)
// ---------------------------------------------------------------------------
template <typename T>
struct __attribute__((aligned(2 * sizeof(T)))) cplx {
    T x, y;
};
using zd = cplx<double>;
using zf = cplx<float>;

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T a, T b) { return cplx<T>{a, b}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a) { return {-a.x, -a.y}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) { return {s * a.x, s * a.y}; }
// acc + a*b
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cfma(cplx<T> a, cplx<T> b, cplx<T> acc) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
// acc + conj(a)*b
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cfma_conj(cplx<T> a, cplx<T> b, cplx<T> acc) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
    return acc;
}
template <typename T>
__host__ __device__ __forceinline__ T abs2(cplx<T> a) { return a.x * a.x + a.y * a.y; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cinv(cplx<T> a) {
    const T r = T(1) / (a.x * a.x + a.y * a.y);
    return {a.x * r, -a.y * r};
}
// c ? a : b per component (a select of whole structs can become a select of
// their addresses, which puts them in scratch memory)
template <typename T>
__host__ __device__ __forceinline__ cplx<T> csel(bool c, cplx<T> a, cplx<T> b) {
    return {c ? a.x : b.x, c ? a.y : b.y};
}
template <typename To, typename Ti>
__host__ __device__ __forceinline__ cplx<To> ccast(cplx<Ti> a) { return {(To)a.x, (To)a.y}; }

// ---------------------------------------------------------------------------
// auxiliary problems
// ---------------------------------------------------------------------------
// Block-tridiagonal layout of a 2D auxiliary problem on sweep lines lo..hi
// (L lines): block k (k = i1 = 1..n) holds the L unknowns (i1 = k, lo..hi).
// The factor stores, for every k, S_k^-1 (S_k the Schur complement of the
// block recurrence) column-major with leading dimension LR >= L (rows past L
// zero): entry (i, j) of block k at [(k-1) L LR + j LR + i], so that the LR
// lanes holding the rows of one solve load each column coalesced.
//
// 3D: block k (k = i1 = 1..n) holds the n L unknowns (i1 = k, i2, i3 = lo..hi)
// at in-block index j = (i3 - lo) + L (i2 - 1); blocks are padded to B (a
// multiple of 64) with identity rows.  The factor stores S_k^-1 for every k as
// a dense B x B column-major matrix at fac_off + (k-1) B^2.
struct SubDesc {
    int kind;            // ASP_SUB_M / R / L
    int p;               // layer index (1-based)
    int lo, hi, L;       // sweep lines of the extended grid
    int LR;              // 2D: rows per solve wavefront (16 or 32, >= L)
    int B;               // 3D: padded block size (multiple of 64); 2D: 0
    int xs, xe;          // lines of X_p (output lines)
    int src_line;        // R: last line of X_{p-1};  L: first line of X_{p+1};  M: 0
    int phi, psi;        // zero region of the sweep-axis PML profile
    int gam_lo, gam_hi;  // its PML width (grid units) below phi / above psi
    long long fac_off;   // offset of block k = 1 in the factor buffer (complex entries)
    long long tab_off;   // offset of this problem's tables in the table buffer
    long long tr_off;    // offset of its boundary-to-boundary map (R_p, L_p with 1 < p < m), else -1
    long long g_off;     // map problems: offset (in the map buffer) of the columns of the
                         // diagonal blocks of H^-1 the maps start from, [k][2][LR]; else -1
    int wrow;            // R/L problems: row of its boundary data in the sweep buffer, else -1
    long long vec_off;   // 3D: offset of this problem's per-entry vectors (B entries each)
    long long xoff;      // 3D nested dissection: this problem's slab vector (n^2 L x 16 per chunk)
};

// 3D nested dissection (Section 4.1).  The elimination tree is built over the
// n x n columns (i1, i2) of a slab, each column holding the L unknowns of its
// sweep lines; every auxiliary problem shares the tree (only L differs).  A
// node eliminates its separator columns (all columns at a leaf); its boundary
// is the set of columns outside its region next to it, which belong to the
// separators of its ancestors.  Its dense front has the rows and columns
// [I (padded to ipad, a multiple of 64) | B (padded to a multiple of 64)],
// column c of the front column list holding rows c L .. c L + L - 1 of its part.
struct NdNode {
    int i_off, nI;       // separator columns: nd_cols[i_off .. i_off + nI)
    int b_off, nB;       // boundary columns: nd_cols[b_off .. b_off + nB)
    int inv_off[2];      // per child: front column (I then B) -> the child's boundary
                         // column holding it, or -1 (nd_inv[inv_off + c]); -1: no child
    int ch[2];           // children: positions in the next level, or -1
};
// one front: (auxiliary problem, tree node); fronts are ordered [level][problem][node]
struct NdFront {
    long long moff;      // [F_II^-1 | F_II^-1 F_IB] in the factor buffer: ipad x f, column-major
    long long foff;      // the dense front in its level buffer while factoring (f x f)
    long long roff;      // panel rows of the Gauss-Jordan steps (f x 64) while factoring
    long long voff;      // front vector in the solve buffer (f x 16 per chunk)
    int f, ipad, L, sub, node;
};

// 3D recursive sweep (Section 5): inner problem (outer, inner) is the
// auxiliary problem `inner`'s geometry taken along x2 (with equal layer widths
// the inner partition of a slab along x2 is the outer partition along x3) on
// the slab of the auxiliary problem `outer` (its x3 lines and profile).  Block
// k (i1 = k) holds the L_outer x L_inner unknowns (i3, i2) at j = (i3 - lo) +
// L_outer (i2 - lo2), padded to B with identity rows; the factor stores S_k^-1
// for every k (n B x B blocks at fac_off).
struct RecDesc {
    int outer, inner;    // indices into the auxiliary problems
    int B;               // padded block size (multiple of 64) >= L_outer L_inner
    long long fac_off;   // block k = 0 in the factor buffer
    long long vec_off;   // x1 coupling vector e(j) = 1 / (s2 s3 h^2), B entries
};

// solve launch modes
enum { IN_GRID = 0, IN_BOUNDARY = 1, IN_TWIST = 2 };
enum { OUT_GRID_STORE = 0, OUT_GRID_ADD_U = 1, OUT_GRID_ACC = 2, OUT_LINE = 3 };

// Per-problem sweep-axis tables, complex double, at tab_off:
//   [0 .. L]        s at the half lines lo-1/2 .. hi+1/2
//   [L+1 .. 2L]     1 / (s h^2) at the lines lo .. hi
//   [2L+1 .. 3L]    1 / s at the lines lo .. hi
inline long long sub_table_len(int L) { return 3LL * L + 1; }

// Global axis tables (the boundary PML, the same on every axis), complex double:
//   sh[k]      s at t = k + 1/2, k = 0..n
//   inv_sh2[i] 1 / (s(i+1) h^2), i = 0..n-1
//   inv_s[i]   1 / s(i+1)
struct AxisTables {
    const zd* sh;
    const zd* inv_sh2;
    const zd* inv_s;
};

// ---------------------------------------------------------------------------
// the plan
// ---------------------------------------------------------------------------
constexpr int SINK_ELEMS = 1024;   // complex128 entries of the discard buffer

struct asp_plan {
    // problem
    int dim = 0, n = 0, b = 0, gamma = 0, g = 0, m = 0;
    int gamma_aux = 0;                // PML width of the pads facing another layer
    double omega = 0, h = 0, C = 25.0;
    int prec = ASP_PREC_FP64;
    bool sweep_seq = false;           // 2D: the sweeps as sequential R/L solves (no maps)
    hipStream_t stream = nullptr;
    bool host_only = false;  // partition and tables only, no device state
    long long N = 0, S = 0;  // unknowns, unknowns per line
    std::vector<double> c;   // host copy of the velocity

    // partition (1-based lines)
    std::vector<std::array<int, 2>> X;
    std::vector<SubDesc> subs;   // M_1..M_m, R_2..R_m, L_1..L_{m-1}
    int idx_M(int q) const { return q - 1; }
    int idx_R(int p) const { return m + (p - 2); }
    int idx_L(int p) const { return m + (m - 1) + (p - 1); }
    int max_L = 0, LR_M = 0, LR_RL = 0;
    int wrow(int sub) const { return subs[sub].wrow; }

    // host tables
    std::vector<std::complex<double>> ax_int, ax_half;                   // s on lines, half lines
    std::vector<std::vector<std::complex<double>>> sub_int, sub_half;    // per problem

    // device data
    double* d_ksq = nullptr;          // omega^2 / c^2, N
    zd* d_axis = nullptr;             // sh | inv_sh2 | inv_s  (n+1 + n + n)
    zd* d_subtab = nullptr;           // per-problem tables
    SubDesc* d_desc = nullptr;
    int* d_jobs = nullptr;            // [0..m): M jobs; then 2 per sweep step
    void* d_fac = nullptr;
    size_t fac_bytes = 0;
    long long fac_elems = 0;
    int* d_flag = nullptr;            // breakdown flag of the factorization
    zd* d_sink = nullptr;             // SINK_ELEMS entries: target of stores a lane discards
    bool factored = false;

    // boundary-to-boundary maps T^R_p, T^L_p (1 < p < m), n x n each, column-major
    void* d_T = nullptr;
    size_t t_bytes = 0;
    long long t_elems = 0;

    // apply workspaces (grown on demand)
    int ws_rhs = 0;
    zd* d_U = nullptr;      // u~_{p,p} on every layer
    zd* d_W = nullptr;      // sweep boundary data: (2m-2) rows x ws_rhs x n
    zd* d_stage = nullptr;  // grid-shaped staging for asp_subsolve
    void* d_wt = nullptr;   // sweep data, transposed, in the factor precision
    long long wt_elems = 0;
    void* d_y = nullptr;    // forward-substitution scratch, y_waves workgroups
    long long y_waves = 0;
    size_t ws_bytes = 0;

    // per-kernel-class timing (asp_timing_enable / asp_timing_read)
    bool timing = false;
    struct TimedSpan {
        hipEvent_t a, b;
        int launches;        // kernel launches between the two events
    };
    std::vector<TimedSpan> tev[ASP_K_COUNT];
    std::vector<hipEvent_t> tpool;
    size_t tpool_used = 0;
    double tbytes[ASP_K_COUNT] = {0};
    double tflops[ASP_K_COUNT] = {0};

    // 3D: per-entry vectors of every auxiliary problem (B entries at vec_off):
    //   e3[j]  = 1 / (s2(i2) s3(i3) h^2), the coupling between blocks k and k+1
    //            divided by s1 at the half line between them
    //   gv3[j] = R/L problems, on the line next to the Dirichlet data:
    //            -s3(half line to the data) / (s2(i2) h^2); else 0
    int Bmax = 0;                 // largest padded block size
    long long vec_elems = 0;
    zd* d_e3 = nullptr;
    zd* d_gv3 = nullptr;
    // 3D solve workspaces
    void* d_y3 = nullptr;         // forward results / solution blocks [chunk][job][k][B][16]
    void* d_g3 = nullptr;         // gathered M data, same layout
    long long y3_elems = 0;
    zd* d_w3 = nullptr;           // sweep planes [pingpong][side][n^2][ws]
    long long w3_elems = 0;
    int ws3 = 0;                  // right-hand-side stride of the planes (multiple of 16)
    // 3D nested dissection (opts.nd3d): tree and fronts (host and device copies)
    bool nd = false;
    int nd_levels = 0;
    std::vector<int> nd_lvl_nodes;            // nodes per level (root: level 0)
    std::vector<long long> nd_lvl_front0;     // first front of each level
    std::vector<int> nd_lvl_fmax;             // largest front of each level
    std::vector<NdNode> nd_nodes;             // level by level
    std::vector<int> nd_node0;                // first node of each level
    std::vector<int> nd_cols, nd_inv;
    std::vector<NdFront> nd_fronts;
    std::vector<std::array<int, 2>> nd_groups;   // problems factored together [s0, s1)
    long long nd_lvlbuf = 0, nd_rbuf = 0;     // level / panel buffer entries of the factorization
    int nd_dbuf = 0;                          // fronts of the largest (group, level)
    long long nd_vtot = 0, nd_xtot = 0;       // solve vector entries per chunk of 16
    NdNode* d_nd_nodes = nullptr;
    int* d_nd_cols = nullptr;
    int* d_nd_inv = nullptr;
    NdFront* d_nd_fronts = nullptr;
    void* d_nd_v = nullptr;                   // front vectors [chunk][vtot]
    void* d_nd_x = nullptr;                   // slab vectors [chunk][xtot]
    // the factorization's level, panel and pivot-tile buffers, kept between
    // factorizations until asp_release_workspace
    void* d_nd_lb[2] = {nullptr, nullptr};
    void* d_nd_rb = nullptr;
    void* d_nd_db = nullptr;
    size_t nd_work_bytes = 0;

    // 3D recursive sweep (fact3d == ASP_FACT3D_RECURSIVE)
    bool rec = false;
    std::vector<RecDesc> rec_desc;            // (3m-2)^2 inner problems, outer-major
    int rec_Bmax = 0;
    long long rec_vec_elems = 0;
    RecDesc* d_rec = nullptr;
    SubDesc* d_rec_sd = nullptr;              // the same problems as block descriptors (B, fac_off, vec_off)
    zd* d_rec_e = nullptr;
    int* d_rec_jobs = nullptr;                // job lists: inner problem indices, then their slots
    long long rec_jobs_len = 0;               // entries of each of the two halves
    std::vector<int> rec_jobs_host;           // the same on the host
    std::vector<long long> rec_list_off;      // start of every job list
    std::vector<int> rec_list_len;
    int rec_Lmax = 0;
    // recursive solve workspaces (chunks of 16 right-hand sides)
    int rec_chunks = 0;
    void* d_rec_sv = nullptr;                 // slab vectors: in, U, R, L [slot][chunk][k][i2][i3][16]
    void* d_rec_w2 = nullptr;                 // inner sweep planes [slot][side][pingpong][chunk][k][i3][16]
    void* d_rec_g = nullptr;                  // block-solve data and results [chunk][job][k][Bmax][16]
    void* d_rec_y = nullptr;
    size_t rec_ws_bytes = 0;

    // GMRES workspaces
    int kr_rhs = 0, kr_restart = 0;
    zd* d_V = nullptr;      // (restart+1) * nrhs * N
    zd* d_Z = nullptr;      // restart * nrhs * N
    zd* d_b = nullptr;      // nrhs * N
    zd* d_red = nullptr;    // reduction partials
    zd* d_small = nullptr;  // small per-RHS arrays (h, norms, coefficients)
    int* d_act = nullptr;   // active RHS list
    size_t kr_bytes = 0;

    std::string err;
};

// status helpers
asp_status plan_fail(asp_plan* p, asp_status s, const std::string& msg);
#define ASP_HIP(plan, call)                                                              \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return plan_fail((plan), ASP_ERR_DEVICE,                                     \
                             std::string(#call) + ": " + hipGetErrorString(e_));         \
    } while (0)

// ---------------------------------------------------------------------------
// launchers (stream-ordered; return hipSuccess or the launch error)
// ---------------------------------------------------------------------------
// y = A x (symmetric form), rhs indices act[0..nact) of the batch (nullptr: 0..nact-1)
hipError_t launch_stencil(const asp_plan* P, const zd* x, zd* y, const int* act, int nact,
                          hipStream_t st);
// out = b - A x and per-RHS partial sums of |out|^2 into red (nblk per RHS)
hipError_t launch_residual(const asp_plan* P, const zd* b, const zd* x, zd* out,
                           const int* act, int nact, zd* red, int* nblk_out, hipStream_t st);

// factorization of every auxiliary problem (2D)
hipError_t launch_factor2d(const asp_plan* P, hipStream_t st);

// batched layer solves for the jobs d_jobs[job0 .. job0+njobs) (all M, or all
// R/L: rl) and the right-hand sides act[0..nact) (NULL: 0..nact-1).
//   in_mode   IN_GRID: data = r on X_p;  IN_BOUNDARY: boundary data from the
//             W rows of the problems;  IN_TWIST: the boundary-map solutions
//             (nact = n virtual right-hand sides, act ignored)
//   out_mode  OUT_GRID_STORE: out = v on X_p (IN_GRID, IN_BOUNDARY);
//             OUT_LINE: the outgoing boundary line into the problem's
//             boundary map (IN_TWIST); other modes are refused
struct SolveLaunch {
    int job0 = 0, njobs = 0;
    bool rl = false;
    const int* act = nullptr;
    int nact = 0;
    int in_mode = IN_GRID, out_mode = OUT_GRID_STORE;
    const zd* r = nullptr;
    const zd* W = nullptr;
    int w_rhs = 0;
    zd* out = nullptr;
    // a launch over R and L problems: the L problems write here instead (NULL: out)
    int out_mode_L = OUT_GRID_STORE;
    zd* out_L = nullptr;
    // IN_TWIST: 0 = solutions for unit data at column slot (map columns on and
    // above the diagonal), 1 = for unit data on the map's output line at row
    // slot (the entries below the diagonal, by the symmetry of H)
    int twist_kind = 0;
};
hipError_t launch_solve2d(const asp_plan* P, const SolveLaunch& L, hipStream_t st);
// columns grow and jout of the diagonal blocks of H^-1 of the map problems
// jobs[job0 .. job0 + njobs) and, if job1 >= 0, jobs[job1 .. job1 + njobs)
// in the same launch (R_p or L_p with 1 < p < m, after asp_factor)
hipError_t launch_rgf2d(const asp_plan* P, int job0, int job1, int njobs, hipStream_t st);
// device memory of the library (devmem.cpp): blocks may be cached and handed
// to another plan, so a block is freed only once no work is pending on it
// (after a synchronization of the owning plan's stream)
hipError_t devmem_alloc(void** p, size_t bytes);
void devmem_free(void* p);

// right-hand sides handled by one solve workgroup for problems of LR rows, and
// the scratch entries of one workgroup (the same for every LR)
int solve_rhs_per_block(int LR);
// the most sweep lines a 2D auxiliary problem may have with blocks of LR rows
// (LR = 16, 32, 64) in element type T: the solve kernels keep two blocks in
// LDS, which at LR = 64 holds 64 lines of FP32 and 48 of FP64
template <typename T>
constexpr int max_lines_2d(int LR) { return LR <= 32 ? 32 : (sizeof(T) == 4 ? 64 : 48); }
long long solve_scratch_per_block(const asp_plan* P);
// the W rows that start the two sweeps (from u~_{1,1} and u~_{m,m} in U)
hipError_t launch_sweep_seed(const asp_plan* P, zd* W, long long outR, long long outL,
                             const int* act, int nact, hipStream_t st);
// the boundary lines the R_{t+1} / L_{m-t} solves of a sequential sweep step hand
// on: W rows rowR / rowL (R outputs in z, L outputs in stage, both without U)
// get the output plus U on line lineR / lineL
hipError_t launch_sweep_hand(const asp_plan* P, const zd* z, const zd* stage, zd* W,
                             long long rowR, int lineR, long long rowL, int lineL, const int* act,
                             int nact, hipStream_t st);
// sweep step t = 1..m-2 (both directions); workspace sizes for nrhs right-hand sides
int sweep_wt_len(const asp_plan* P, int nrhs);
hipError_t launch_sweep_step(const asp_plan* P, int t, zd* W, int w_rhs, const int* act, int nact,
                             hipStream_t st);

// ---------------------------------------------------------------------------
// 3D auxiliary problems
// ---------------------------------------------------------------------------
// S_k = D_k - diag(E_k) S_{k-1}^-1 diag(E_k) into block k (0-based) of every job
hipError_t launch_form3d(const asp_plan* P, const int* jobs, int njobs, int k, hipStream_t st);
// one panel jp of the in-place block Gauss-Jordan inversion of block k
// (panel step, then trailing update); Rbuf: njobs x 64 x Bmax, Dbuf: njobs x 64 x 64
hipError_t launch_gj3d(const asp_plan* P, const int* jobs, int njobs, int k, int jp, void* Rbuf,
                       void* Dbuf, hipStream_t st);
// M data on X_q gathered into the block layout of the forward pass
hipError_t launch_gather3d(const asp_plan* P, const int* jobs, int njobs, const zd* r,
                           const int* act, int nact, hipStream_t st);
// one block step of the forward (fwd = 1) or backward pass over jobs
struct Solve3Launch {
    const int* jobs = nullptr;   // device job list
    int njobs = 0;
    bool two_sided = false;      // job 0 is an R problem, job 1 an L problem
    const int* act = nullptr;
    int nact = 0;
    int in_mode = IN_GRID;       // IN_GRID: gathered data; IN_BOUNDARY: planes in Win
    const zd* Win = nullptr;     // [job][n^2][ws3]
    zd* Wout = nullptr;          // outgoing boundary plane (+ U) of every job, or NULL
    int out_mode[2] = {OUT_GRID_STORE, OUT_GRID_STORE};
    zd* out[2] = {nullptr, nullptr};
    const zd* Ugrid = nullptr;
};
hipError_t launch_solve3d_step(const asp_plan* P, const Solve3Launch& L, int k, int fwd,
                               hipStream_t st);
// the block-recurrence kernels on other descriptors (only B, fac_off and
// vec_off are read; a descriptor with xs > xe writes no grid output):
// Gauss-Jordan panel jp of block k of desc[jobs[0..njobs)], and one block step
// of their solves with data gathered into G and results kept in Y
// ([chunk][job][k][Bmax][16] each, e the x1 coupling vectors at vec_off)
hipError_t launch_gj_blocks(const asp_plan* P, const SubDesc* desc, const int* jobs, int njobs,
                            void* fac, int k, int jp, int Bmax, void* Rbuf, void* Dbuf,
                            hipStream_t st);
struct BlockSolve {
    const SubDesc* desc = nullptr;
    const int* jobs = nullptr;
    int njobs = 0;
    const void* fac = nullptr;
    void* Y = nullptr;
    const void* G = nullptr;
    int Bmax = 0;
    const zd* e = nullptr;
    int nact = 0;
    bool narrow = false;   // 16 rows per workgroup, 16 wavefronts (few problems)
};
hipError_t launch_block_step(const asp_plan* P, const BlockSolve& s, int k, int fwd, hipStream_t st);
// W[job][i1 + n i2][slot] = U on sweep line `line0` (job 0) and `line1` (job 1)
hipError_t launch_plane3d(const asp_plan* P, const zd* U, int line0, int line1, zd* W,
                          const int* act, int nact, hipStream_t st);
// z = U + C on lines 1..split, z += C on lines split+1..upto
hipError_t launch_combine3d(const asp_plan* P, zd* z, const zd* U, const zd* C, int split,
                            int upto, bool all_u, const int* act, int nact, hipStream_t st);

// timing of one launch: constructed before the launch, end() after it
struct KTimer {
    asp_plan* P;
    int cls;
    bool on;
    // one event pair around `launches` launches of class c (a chain of
    // dependent launches is timed as one span: an event per launch would add
    // its own gap to every step of the chain)
    KTimer(asp_plan* p, int c, double bytes, double flops, int launches = 1);
    void end();
};

// Krylov kernels (complex double)
hipError_t launch_scale_by_s(const asp_plan* P, const zd* f, zd* b, int nrhs, hipStream_t st);
// partial[r][blk][i] = sum conj(V_i[r]) w[r] for i in [i0, i1)
int krylov_blocks(long long N);
// fused Gram-Schmidt passes (modes: 0 dots, 1 update then dots and norm) over
// nv <= CGS_MAXV basis vectors; partial sums [rhs][block][CGS_SLOTS]
constexpr int CGS_MAXV = 24;
constexpr int CGS_SLOTS = CGS_MAXV + 1;
// the second Gram-Schmidt pass from the Gram matrix of the basis (E: per
// right-hand side CGS_MAXV x CGS_MAXV, column j written at step j)
hipError_t launch_gram(zd* small, int small_stride, int off_h1, int off_h2, int off_coef, int off_d,
                       const zd* scal, zd* E, int j, const int* act, int nact, hipStream_t st);
// device bytes of the GMRES partial sums, small arrays and Gram columns
double krylov_small_bytes(long long N, int nrhs);
// partial sums of |v|^2 per right-hand side, reduced by launch_reduce (one value)
hipError_t launch_norms(const zd* v, long long N, const int* act, int nact, zd* partial,
                        hipStream_t st);
int cgs_blocks(long long N);
hipError_t launch_cgs(int mode, int nv, const zd* V, long long vstride, const zd* coef,
                      int coef_stride, zd* w, long long N, const int* act, int nact, zd* partial,
                      hipStream_t st);
hipError_t launch_cgs_reduce(const zd* partial, int nblk, int nv, const int* act, int nact,
                             zd* out, int out_stride, hipStream_t st);
hipError_t launch_multidot(const zd* V, long long vstride, int i0, int i1, const zd* w,
                           long long N, const int* act, int nact, zd* partial, hipStream_t st);
// out[r][i] = sum_blk partial[r][blk][i], i < ni, fixed order
hipError_t launch_reduce(const zd* partial, int nblk, int ni, const int* act, int nact,
                         zd* out, int out_stride, hipStream_t st);
// w[r] -= sum_i coef[r][i] V_i[r], i in [i0,i1); partial |w|^2 if norm_partial
hipError_t launch_axpy_multi(const zd* V, long long vstride, int i0, int i1, const zd* coef,
                             int coef_stride, zd* w, long long N, const int* act, int nact,
                             zd* norm_partial, hipStream_t st);
// v[r] = w[r] * scal[r]  (scal complex, per rhs slot)
hipError_t launch_scale_vec(const zd* w, zd* v, const zd* scal, long long N, const int* act,
                            int nact, hipStream_t st);

// host-side pieces shared by the entry points
asp_status ensure_apply_ws(asp_plan* P, int nrhs);
asp_status apply_internal(asp_plan* P, const zd* r, zd* z, const int* act, int nact);
// workgroups (each with solve_scratch_per_block entries of scratch) of the
// 2D layer solves of one apply over nrhs right-hand sides
long long apply_scratch_groups(const asp_plan* P, int nrhs);
// right-hand sides per chunk of the 3D nested-dissection solves
constexpr int ND_CHUNK = 16;
// device bytes of the 2D layer solves' forward-substitution scratch now allocated
size_t solve_scratch_bytes(const asp_plan* P);
// device bytes of the work buffers asp_factor allocates besides the factors
size_t factor_work_estimate(const asp_plan* P);
size_t nd_factor_work_estimate(const asp_plan* P);
size_t factor3d_work_estimate(const asp_plan* P);
// algorithmic bytes of one auxiliary problem's factor (n dense L x L blocks in
// 2D, n dense nL x nL blocks in 3D)
double factor_bytes_of(const asp_plan* P, const SubDesc& d);
// 3D counterparts (apply3d.cpp)
asp_status ensure_apply_ws3(asp_plan* P, int nrhs);
size_t workspace_estimate3(const asp_plan* P, int nrhs);
asp_status factor3d(asp_plan* P);
asp_status apply3d_internal(asp_plan* P, const zd* r, zd* z, const int* act, int nact);
asp_status subsolve3d(asp_plan* P, int idx, const void* in, void* out, int nrhs);
// nested dissection (nd3d.cpp): tree and fronts at setup (sizes only for a
// host-only plan), factorization, apply, one auxiliary solve
asp_status nd_setup(asp_plan* P);
asp_status nd_upload(asp_plan* P);
asp_status nd_factor(asp_plan* P);
asp_status nd_apply(asp_plan* P, const zd* r, zd* z, const int* act, int nact);
asp_status nd_subsolve(asp_plan* P, int idx, const void* in, void* out, int nrhs);
asp_status nd_ensure_ws(asp_plan* P, int nrhs);
size_t nd_workspace_estimate(const asp_plan* P, int nrhs);

// recursive sweep (rec3d.cpp): inner problems and job lists at setup, factor,
// apply, one auxiliary solve, workspaces
asp_status rec_setup(asp_plan* P);
asp_status rec_upload(asp_plan* P);
asp_status rec_factor(asp_plan* P);
asp_status rec_apply(asp_plan* P, const zd* r, zd* z, const int* act, int nact);
asp_status rec_subsolve(asp_plan* P, int idx, const void* in, void* out, int nrhs);
asp_status rec_ensure_ws(asp_plan* P, int nrhs);
size_t rec_workspace_estimate(const asp_plan* P, int nrhs);
size_t rec_factor_work_estimate(const asp_plan* P);
void rec_free_ws(asp_plan* P);

// recursive-sweep kernels (rec3d.hip).  A launch covers nslot slabs (outer
// problems slot_outer[0..nslot)) and nchunk chunks of 16 right-hand sides.
struct RecLaunch {
    int nslot = 0, chunks = 0, nact = 0;
    const int* act = nullptr;
    const int* slot_outer = nullptr;   // device: outer problem of each slot
    const int* jobs = nullptr;         // device: inner problem of each job
    const int* jslot = nullptr;        // device: slot of each job
    int njobs = 0;
    int mode = 0;                      // launch-specific (see rec3d.hip)
    int pp = 0;                        // ping-pong plane of the inner sweeps
    const zd* rin = nullptr;           // grid data (M) or outer planes (R/L)
    zd* out0 = nullptr;                // outputs (see launch_rec_slab_out)
    zd* out1 = nullptr;
    const zd* U = nullptr;
    zd* Wout = nullptr;
};
hipError_t launch_rec_form(const asp_plan* P, int k, hipStream_t st);
hipError_t launch_rec_slab_in(const asp_plan* P, const RecLaunch& L, hipStream_t st);
hipError_t launch_rec_gather(const asp_plan* P, const RecLaunch& L, hipStream_t st);
hipError_t launch_rec_scatter(const asp_plan* P, const RecLaunch& L, hipStream_t st);
hipError_t launch_rec_seed(const asp_plan* P, const RecLaunch& L, hipStream_t st);
hipError_t launch_rec_slab_out(const asp_plan* P, const RecLaunch& L, hipStream_t st);

// nested-dissection kernels (nd3d.hip); fronts fr[0..nfr) of one level
struct NdLevel {
    const NdFront* fr_all;   // every front
    long long front0;        // first front of the level
    int nn;                  // nodes in the level
    long long child0;        // first front of the next level (children), -1: none
    int nnc;                 // nodes in the next level
};
// dense fronts of problems [s0, s1) at one level: original entries + the
// children's Schur complements (from Fchild); F in Flevel
hipError_t launch_nd_assemble(const asp_plan* P, const NdLevel& lv, int s0, int s1, void* Flevel,
                              const void* Fchild, int fmax, hipStream_t st);
// Gauss-Jordan panel jp of the separator part of nfr fronts.  mode 0: the
// whole trailing update; panels in pairs (look-ahead), Rbuf holding three
// slots of f x 64 per front: mode 1 for the first of a pair (its rows and
// columns kept, only the second panel's tiles updated; the whole update for a
// front without a second panel), mode 2 for the second (both panels' updates
// applied to the rest in one pass)
hipError_t launch_gj_fronts(const asp_plan* P, const NdFront* fr, int nfr, void* Flevel, int jp,
                            int ntmax, void* Rbuf, void* Dbuf, int mode, hipStream_t st);
// [F_II^-1 | F_II^-1 F_IB] of each front into the factor buffer
hipError_t launch_nd_copyout(const asp_plan* P, const NdFront* fr, int nfr, const void* Flevel,
                             int fmax, hipStream_t st);
// solve inputs into the slab vectors: M data on X_q (grid r), or R/L data from planes
hipError_t launch_nd_input(const asp_plan* P, const int* jobs, int njobs, int in_mode,
                           const zd* r, const zd* Win, const int* act, int nact, hipStream_t st);
// forward (fwd = 1) or backward step over one level for the jobs
hipError_t launch_nd_level(const asp_plan* P, const NdLevel& lv, const int* jobs, int njobs,
                           int fwd, int fmax, int nact, hipStream_t st);
// outputs of the solved slabs on X_p, as launch modes of the block solves
hipError_t launch_nd_output(const asp_plan* P, const int* jobs, int njobs, bool two_sided,
                            const int out_mode[2], zd* const out[2], const zd* U, zd* Wout,
                            const int* act, int nact, hipStream_t st);

// a launch bracketed by a KTimer of class cls
#define ASP_TIMED(plan, cls, bytes, flops, call)        \
    do {                                                \
        KTimer t_((plan), (cls), (bytes), (flops));     \
        ASP_HIP((plan), call);                          \
        t_.end();                                       \
    } while (0)
