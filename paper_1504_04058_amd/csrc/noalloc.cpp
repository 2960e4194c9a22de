// asp_apply_noalloc: the preconditioner apply (Algorithm 2 / 4) for callers
// that cannot allocate device memory.  Its work buffers (the u~ grid, the
// sweep boundary data, the staging grid, the layer solves' forward-substitution
// scratch; in 3D the nested-dissection front and slab vectors) are carved out
// of one fixed device array instead of the plan's grown workspaces, and the
// kernels are those of asp_apply.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "asp_internal.h"

namespace {

// The array every call on a device shares (each device holds its own copy).
// In host code `scratch` only names the symbol; its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
static __device__ __align__(256) unsigned char scratch[ASP_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
unsigned char* g_scratch[MAX_DEVICES] = {};

// the device address of this device's `scratch` (set up on the first call)
hipError_t scratch_ptr(unsigned char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

size_t esz(const asp_plan* P) { return P->prec != ASP_PREC_FP64 ? sizeof(zf) : sizeof(zd); }

// consecutive 256-byte aligned pieces of the scratch array
struct Carve {
    unsigned char* base;
    size_t used = 0;
    template <typename T>
    T* take(size_t bytes) {
        T* p = reinterpret_cast<T*>(base ? base + used : nullptr);
        used += (bytes + 255) / 256 * 256;
        return p;
    }
};

// the plan's workspace fields an apply reads, swapped for the call's duration
struct WsFields {
    zd *U, *W, *stage, *w3;
    void *wt, *y, *nd_v, *nd_x;
    long long wt_elems, y_waves, w3_elems;
    int ws_rhs, ws3;
    bool timing;
    void save(const asp_plan* P) {
        U = P->d_U; W = P->d_W; stage = P->d_stage; w3 = P->d_w3;
        wt = P->d_wt; y = P->d_y; nd_v = P->d_nd_v; nd_x = P->d_nd_x;
        wt_elems = P->wt_elems; y_waves = P->y_waves; w3_elems = P->w3_elems;
        ws_rhs = P->ws_rhs; ws3 = P->ws3; timing = P->timing;
    }
    void restore(asp_plan* P) const {
        P->d_U = U; P->d_W = W; P->d_stage = stage; P->d_w3 = w3;
        P->d_wt = wt; P->d_y = y; P->d_nd_v = nd_v; P->d_nd_x = nd_x;
        P->wt_elems = wt_elems; P->y_waves = y_waves; P->w3_elems = w3_elems;
        P->ws_rhs = ws_rhs; P->ws3 = ws3; P->timing = timing;
    }
};

// lay the apply's buffers for nrhs right-hand sides out from `base` (NULL:
// sizes only) into the plan's fields; returns the bytes used
size_t lay_out(asp_plan* P, int nrhs, unsigned char* base) {
    Carve c{base};
    const size_t vec = (size_t)nrhs * P->N * sizeof(zd);
    P->d_U = c.take<zd>(vec);
    P->d_stage = c.take<zd>(vec);
    P->ws_rhs = nrhs;
    if (P->dim == 2) {
        P->d_W = c.take<zd>((size_t)std::max(2 * P->m - 2, 1) * nrhs * P->n * sizeof(zd));
        P->wt_elems = sweep_wt_len(P, nrhs);
        P->d_wt = c.take<void>((size_t)P->wt_elems * esz(P));
        P->y_waves = apply_scratch_groups(P, nrhs);
        P->d_y = c.take<void>((size_t)P->y_waves * solve_scratch_per_block(P) * esz(P));
    } else {
        const int chunks = (nrhs + ND_CHUNK - 1) / ND_CHUNK;
        P->ws3 = chunks * ND_CHUNK;
        P->w3_elems = 2LL * 2 * P->S * P->ws3;
        P->d_w3 = c.take<zd>((size_t)P->w3_elems * sizeof(zd));
        P->d_nd_v = c.take<void>((size_t)chunks * P->nd_vtot * esz(P));
        P->d_nd_x = c.take<void>((size_t)chunks * P->nd_xtot * esz(P));
    }
    return c.used;
}

}  // namespace

extern "C" asp_status asp_apply_noalloc(asp_plan* P, const void* r, void* z, int nrhs) {
    if (!P) return ASP_ERR_ARG;
    if (!r || !z || nrhs < 1) return plan_fail(P, ASP_ERR_ARG, "asp_apply_noalloc: bad arguments");
    if (r == z) return plan_fail(P, ASP_ERR_ARG, "asp_apply_noalloc: r and z must not alias");
    if (P->host_only || !P->factored)
        return plan_fail(P, ASP_ERR_STATE, "asp_apply_noalloc before asp_factor");
    if (P->dim == 3 && !P->nd)
        return plan_fail(P, ASP_ERR_ARG,
                         "asp_apply_noalloc: 3D plans factored by the block recurrence or the recursive "
                         "sweep are not supported");
    WsFields keep;
    keep.save(P);
    const size_t need = lay_out(P, nrhs, nullptr);
    keep.restore(P);
    if (need > ASP_NOALLOC_SCRATCH_BYTES)
        return plan_fail(P, ASP_ERR_ARG,
                         "asp_apply_noalloc: " + std::to_string(need) + " bytes of work buffers for " +
                             std::to_string(nrhs) + " right-hand sides exceed the fixed " +
                             std::to_string((size_t)ASP_NOALLOC_SCRATCH_BYTES) + "-byte scratch");
    unsigned char* base = nullptr;
    ASP_HIP(P, scratch_ptr(&base));
    lay_out(P, nrhs, base);
    P->timing = false;   // no event objects are created on this path
    const asp_status s = apply_internal(P, static_cast<const zd*>(r), static_cast<zd*>(z), nullptr, nrhs);
    keep.restore(P);
    return s;
}
