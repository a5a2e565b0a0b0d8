// Internal declarations shared by the hsla HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <type_traits>

#include "hsla.h"

namespace hsla {

constexpr int kBlock = 256;             // threads per block for every kernel
constexpr int kWave = 64;               // CDNA wavefront width
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kTileRows = 64;           // rows per SpMV tile: one lane per row
constexpr int kTileCap = 512;           // max stored entries staged per tile (LDS, per wave)
constexpr int kXcds = 8;                // MI355X: 8 XCDs, blocks dispatched round-robin
constexpr int kMaxOffsets = 16;         // distinct column offsets of a stencil pattern
// allocation-free solves: size of the per-device static scratch array, and
// the most systems one such call takes (host state mirror sized at creation)
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kNoAllocMaxSystems = 1024;

// Offset-mask form of a CSR pattern whose entries all lie on a few fixed
// diagonals (structured-grid stencils): column = row + ofs[s] for every set
// bit s of mask[row], bits in ascending order = entries in CSR order.  It
// replaces the 4-byte column index of every entry by 2 bytes per row; the
// values keep their CSR layout.  mask == nullptr: not a stencil pattern.
struct Stencil {
    const uint16_t *mask = nullptr;
    int32_t nofs = 0;
    int32_t ofs[kMaxOffsets] = {};
    int32_t diag_slot = -1;  // s with ofs[s] == 0, -1 if none
    int32_t pencil = 1;      // planes per pencil of the half form's SpMV (set per launch)
};

// Per-system solver state (device memory, one record per system).
struct alignas(128) SysState {
    double rho;      // CG: r.z ; BiCGStab: rho = r_hat.r of the previous step
    double rho_new;  // BiCGStab: r_hat.r of the current step
    double alpha, beta, omega;
    double rnorm2;   // last ||r||^2
    double bnorm;    // ||b||
    double tol;      // max(rtol ||b||, atol)
    double snorm2;
    int64_t iters;
    int64_t max_iter;
    int32_t status;  // hsla_status of the system
    int32_t done;    // 1 once the system stopped (converged, failed, exhausted)
    int32_t restarts;
    int32_t s_exit;  // BiCGStab: ||s|| <= tol, finish with x += alpha p_hat
    int32_t restart_pending;
    int32_t bad_diag;  // set when Jacobi finds a missing or zero diagonal
    int32_t xpend;     // CG: the stopping iteration's x += alpha p is still to be applied
    int32_t stall;     // stall window (iterations; 0 = off)
    double win_rr;     // ||r||^2 at the start of the current stall window
    int64_t win_it;    // iteration at the start of the current stall window
    int32_t sr_swept;  // single-reduction CG: a vector sweep has run since the start
};

// Stall test after an iteration with ||r||^2 = rr: once st.stall iterations
// have passed since the window began, the window either shows a 10x fall of
// ||r|| (100x of rr) and a new window begins, or the system has stagnated.
__device__ __forceinline__ bool stall_step(SysState &st, double rr) {
    if (st.stall <= 0 || st.iters - st.win_it < st.stall) return false;
    if (rr <= 0.01 * st.win_rr) {
        st.win_rr = rr;
        st.win_it = st.iters;
        return false;
    }
    return true;
}

// Scalar steps of the CG recurrence (Alg. 1), run by thread 0 of a
// finalize block once the system's sums are complete; shared by the batched
// solver and the segmented ragged solver.
// Start: ||b||, tol = max(rtol ||b||, atol), stop test on r0, rho = r.z.
__device__ __forceinline__ void cg_step_init(SysState &st, double bb, double rr, double rz, double rtol,
                                             double atol) {
    const double bn = sqrt(bb);
    double tol = rtol * bn;
    if (atol > tol) tol = atol;
    st.bnorm = bn;
    st.tol = tol;
    st.rnorm2 = rr;
    st.iters = 0;
    st.win_rr = rr;
    st.win_it = 0;
    const double rn = sqrt(rr);
    if (st.bad_diag) {
        st.status = HSLA_ERR_ZERO_DIAGONAL;
        st.done = 1;
    } else if (!isfinite(rn) || !isfinite(bn)) {
        st.status = HSLA_ERR_NONFINITE;
        st.done = 1;
    } else if (rn <= tol) {
        st.status = HSLA_OK;
        st.done = 1;
    } else if (st.max_iter <= 0) {
        st.status = HSLA_NOT_CONVERGED;
        st.done = 1;
    } else {
        st.rho = rz;
        st.beta = 0.0;
    }
}

// alpha = rho / sigma with sigma = p.Ap, or breakdown when sigma <= 0.
__device__ __forceinline__ void cg_step_alpha(SysState &st, double sigma) {
    if (!isfinite(sigma)) {
        st.status = HSLA_ERR_NONFINITE;
        st.done = 1;
    } else if (!(sigma > 0.0)) {
        st.status = HSLA_BREAKDOWN;
        st.done = 1;
    } else {
        st.alpha = st.rho / sigma;
    }
}

// After r -= alpha q: stop test on ||r|| (a system stopping here still has
// this iteration's x += alpha p to apply: xpend), else, when rz is the new
// r.z (with_rho), beta = rz / rho and rho = rz.
__device__ __forceinline__ void cg_step_beta(SysState &st, double rr, double rz, bool with_rho) {
    st.iters += 1;
    st.rnorm2 = rr;
    const double rn = sqrt(rr);
    if (!isfinite(rn)) {
        st.status = HSLA_ERR_NONFINITE;
        st.done = 1;
        st.xpend = 1;
    } else if (rn <= st.tol) {
        st.status = HSLA_OK;
        st.done = 1;
        st.xpend = 1;
    } else if (st.iters >= st.max_iter) {
        st.status = HSLA_NOT_CONVERGED;
        st.done = 1;
        st.xpend = 1;
    } else if (stall_step(st, rr)) {
        st.status = HSLA_STAGNATED;
        st.done = 1;
        st.xpend = 1;
    } else if (with_rho) {
        st.beta = rz / st.rho;
        st.rho = rz;
    }
}

struct DevInfo {
    int num_cu = 256;
    int wall_khz = 100000;  // device wall clock (wall_clock64) rate
};

}  // namespace hsla

struct hsla_pattern {
    int device = 0;
    int32_t format = HSLA_FORMAT_AUTO;  // requested SpMV format
    int32_t max_row = 0;                // most entries in one row
    // autotuned SpMV configuration of the solvers (hsla_autotune); defaults
    // until tuned: diagonal-major form where available (its symmetric half
    // form for symmetric values), 16 / 8 / 8 blocks per CU
    int32_t tune_dia = 1, tune_tile_cu = 16, tune_dia_cu = 8, tune_sym = 1, tune_sym_cu = 8, tuned = 0;
    uint64_t signature = 0;  // hash of (n, nnz, row_ptr, col): key of stored tunings
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t *row_ptr = nullptr;  // [n+1]
    int32_t *col = nullptr;      // [nnz]
    int32_t *diag = nullptr;     // [n] position of the diagonal entry, -1 if absent
    int2 *meta = nullptr;         // [ntiles+1] (first row, first entry) of each SpMV tile
    int32_t ntiles = 0;
    int32_t *rpT = nullptr, *colT = nullptr, *srcT = nullptr;  // transpose
    int2 *metaT = nullptr;
    int32_t ntilesT = 0;
    int32_t *diagT = nullptr;
    int32_t pattern_symmetric = 0;
    int64_t nnz_lower = 0;
    // lower triangle (incl. diagonal) for factorized approximate inverses
    int32_t *rpL = nullptr, *colL = nullptr, *posL = nullptr;   // posL: position in A
    int2 *metaL = nullptr;
    int32_t ntilesL = 0;
    int32_t *rpU = nullptr, *colU = nullptr, *srcU = nullptr;   // L^T (upper) + perm into L order
    int2 *metaU = nullptr;
    int32_t ntilesU = 0;
    int32_t *rowL = nullptr;     // row of each lower entry
    uint8_t *isdiagL = nullptr;  // lower entry on the diagonal
    // offset-mask forms of A, A^T, L, U (mask == nullptr where not a stencil)
    hsla::Stencil stA, stT, stL, stU;
    // the form the kernels use: the stencil form unless the CSR form was requested
    const hsla::Stencil &use(const hsla::Stencil &s) const {
        static const hsla::Stencil none{};
        return format == HSLA_FORMAT_CSR ? none : s;
    }
};

struct hsla_handle {
    int device = 0;
    hsla::DevInfo dev;
    std::string last_error;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    // set while a call runs on the device-resident scratch array instead of
    // the handle's workspace: ensure_workspace and ensure_host_state then
    // allocate nothing and reject sizes beyond what is there
    bool ws_fixed = false;
    hsla::SysState *h_state = nullptr;  // pinned host mirror
    size_t h_state_cap = 0;
    // cached HIP graphs of iteration chunks (small LRU by launch arguments)
    static constexpr int kGraphCache = 4;
    hipGraphExec_t graph_exec[kGraphCache] = {};
    uint64_t graph_key[kGraphCache] = {};
    uint64_t graph_use[kGraphCache] = {};
    uint64_t graph_clock = 0;
    // private stream (default priority) ordered after the caller's stream
    hipStream_t stream = nullptr;
    hipEvent_t entry_event = nullptr;
    int32_t *d_flags = nullptr;  // small device scratch for yes/no flags
    // profile mode: event pairs around the timed kernel
    hipEvent_t *prof_ev = nullptr;
    int prof_cap = 0;
    // preconditioner network: activations of the last kept forward, probe buffers
    void *mp_ws = nullptr;
    size_t mp_ws_bytes = 0;
    int mp_keep_B = 0;
    const hsla_pattern *mp_keep_pattern = nullptr;
    void *pr_ws = nullptr;
    size_t pr_ws_bytes = 0;
    // workspace allocator (hsla_set_allocator); hipMalloc/hipFree when unset
    hsla_alloc_fn alloc_fn = nullptr;
    hsla_free_fn free_fn = nullptr;
    void *alloc_ctx = nullptr;
};

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
namespace hsla {

hsla_status set_error(hsla_handle *h, hsla_status st, const char *fmt, ...);

#define HSLA_HIP(h, expr)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::hsla::set_error((h), HSLA_ERR_HIP, "%s failed: %s (%s:%d)", #expr,         \
                                     hipGetErrorString(e_), __FILE__, __LINE__);               \
    } while (0)

// Sets the device, and orders the handle's stream after the caller's.
hsla_status enter(hsla_handle *h, hipStream_t user);

// Grows the handle's workspace to at least `bytes` (contents not preserved).
hsla_status ensure_workspace(hsla_handle *h, size_t bytes);
// Workspace memory through the handle's allocator (hipMalloc when unset).
hipError_t dev_alloc(hsla_handle *h, void **p, size_t bytes);
void dev_free(hsla_handle *h, void *p);
hsla_status ensure_host_state(hsla_handle *h, size_t nsys);

// Shared-pattern solve of B systems (hsla_solve / hsla_solve_batched).
hsla_status solve_entry(hsla_handle *h, const hsla_pattern *p, int B, const double *values, const double *b,
                        double *x, const hsla_opts *opts, hsla_info *infos, hipStream_t user);
// Looks up this device's copy of the library's static scratch array (once per
// device; the device must be current).  Called by hsla_create.
hsla_status scratch_init(hsla_handle *h);

// Blocks per system for grid-stride kernels: enough for `units` work items
// at `per_block` each, at most `per_cu` blocks per CU, a multiple of kXcds.
inline int grid_blocks(const hsla_handle *h, int64_t per_block, int64_t units, int nsys, int per_cu = 8) {
    int64_t want = (units + per_block - 1) / per_block;
    int64_t cap = (int64_t)h->dev.num_cu * per_cu / (nsys > 0 ? nsys : 1);
    if (cap < kXcds) cap = kXcds;
    if (want > cap) want = cap;
    if (want < 1) want = 1;
    want = (want + kXcds - 1) / kXcds * kXcds;
    return (int)want;
}

// Shared-pattern CG batches of small systems (or of mid-size systems when
// the batch fills the chip) run as one persistent launch (ragged.hip): no
// per-iteration launches, every system iterating independently.
constexpr int64_t kPersistentMaxNnz = 131072;
bool persistent_eligible(const hsla_handle *h, const hsla_pattern *p, int B, int method, const hsla_opts &o);
// single_reduction: the Chronopoulos-Gear recurrence in the small-system
// kernel (HSLA_METHOD_CG_SR); other persistent solves run Algorithm 1.
hsla_status persistent_solve(hsla_handle *h, const hsla_pattern *p, int B, const double *values, const double *b,
                             double *x, const hsla_opts &o, hsla_info *infos, hipStream_t s,
                             bool single_reduction = false);

// Kernel launch helpers implemented in the .hip files.
hsla_status launch_spmv(hsla_handle *h, const hsla_pattern *p, int B, const double *values,
                        const double *x, double *y, hipStream_t s);

}  // namespace hsla

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
namespace hsla {

// Butterfly sum over the 64 lanes; every lane ends with the same value and
// the association order is fixed, so the result is deterministic.
// A DPP lane move of a double (both 32-bit halves with the same control);
// rows left out by ROW_MASK keep `old`.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_f64(double old, double v) {
    const uint64_t o = (uint64_t)__double_as_longlong(old), x = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)x, CTRL, ROW_MASK,
                                                              0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(x >> 32),
                                                              CTRL, ROW_MASK, 0xf, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum over the 64 lanes of a wavefront (all lanes active), in every lane.
// A fixed tree of data-parallel-primitive moves (no LDS round trips): pairs,
// quads, half rows and rows of 16 lanes (each lane ends with its row's sum),
// then rows 0+1 and 2+3 (row broadcast 15), then all four (row broadcast
// 31, into lane 63), which is read back into every lane.  The order is the
// same on every call, so results are run-to-run deterministic.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0xB1>(0.0, v);        // quad_perm [1, 0, 3, 2]
    v += dpp_f64<0x4E>(0.0, v);        // quad_perm [2, 3, 0, 1]
    v += dpp_f64<0x141>(0.0, v);       // row_half_mirror
    v += dpp_f64<0x140>(0.0, v);       // row_mirror
    v += dpp_f64<0x142, 0xa>(0.0, v);  // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xc>(0.0, v);  // row_bcast:31 into rows 2 and 3
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum over the block of NV values; the result is valid in thread 0.
// `sh` must hold NV * kWavesPerBlock doubles.  Ends with a barrier, so `sh`
// may be reused right after.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *sh) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) sh[j * kWavesPerBlock + w] = v[j];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double s = 0.0;
            for (int q = 0; q < kWavesPerBlock; ++q) s += sh[j * kWavesPerBlock + q];
            v[j] = s;
        }
    }
    __syncthreads();
}

// Block partial of NV values: the block sums of every reducing kernel go to
// part[j * G + block] with plain stores (G = gridDim.x).  A separate
// one-block finalize kernel per system (reduce_partials) adds the G partials
// in a fixed order once the producing kernel has completed, so the result
// does not depend on block scheduling, and no atomics or cross-XCD fences
// sit on the hot path (contended ticket atomics from thousands of blocks
// serialize at the memory side).
template <int NV>
__device__ __forceinline__ void block_partial(double (&v)[NV], double *part) {
    __shared__ double sh[NV * kWavesPerBlock];
    block_sum<NV>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) part[(size_t)j * gridDim.x + blockIdx.x] = v[j];
    }
}

// Sum of the G partials of each of NV values (fixed order); valid in
// thread 0.  Called by all threads of a finalize block.
template <int NV>
__device__ __forceinline__ void reduce_partials(const double *part, int G, double (&tot)[NV]) {
    __shared__ double sh[NV * kWavesPerBlock];
#pragma unroll
    for (int j = 0; j < NV; ++j) tot[j] = 0.0;
    for (int i = threadIdx.x; i < G; i += blockDim.x) {
#pragma unroll
        for (int j = 0; j < NV; ++j) tot[j] += part[(size_t)j * G + i];
    }
    block_sum<NV>(tot, sh);
}

// XCD-aware tile walk.  Blocks are dispatched round-robin over the 8 XCDs,
// so block b runs on XCD b % 8.  Each XCD gets a contiguous range of tiles,
// and the waves of that XCD sweep it together, keeping the x-gather window
// in that XCD's L2.  Returns the number of rounds; tile(round) gives the
// tile of this wave in that round or -1.
struct TileWalk {
    int32_t lo, hi, first, stride;
    __device__ __forceinline__ TileWalk(int32_t ntiles) {
        const int G = gridDim.x;
        const int wave = threadIdx.x / kWave;
        if (G % kXcds == 0) {
            const int xcd = blockIdx.x % kXcds;
            const int per = G / kXcds;
            lo = (int32_t)((int64_t)ntiles * xcd / kXcds);
            hi = (int32_t)((int64_t)ntiles * (xcd + 1) / kXcds);
            first = lo + (blockIdx.x / kXcds) * kWavesPerBlock + wave;
            stride = per * kWavesPerBlock;
        } else {
            lo = 0;
            hi = ntiles;
            first = blockIdx.x * kWavesPerBlock + wave;
            stride = G * kWavesPerBlock;
        }
    }
    __device__ __forceinline__ int rounds() const {
        // identical for all waves of a block (same XCD range)
        const int32_t base = first - (threadIdx.x / kWave);
        const int32_t span = hi - base;
        return span <= 0 ? 0 : (span + stride - 1) / stride;
    }
    __device__ __forceinline__ int32_t tile(int r) const {
        const int32_t t = first + r * stride;
        return t < hi ? t : -1;
    }
};

// Tiled CSR SpMV over the rows of a pattern: y_row = sum_k val[k] x[col[k]].
//
// A tile is a run of consecutive rows, at most kTileRows rows and kTileCap
// stored entries (one lane per row); a row longer than kTileCap is a tile by
// itself and is summed in kTileCap-entry pieces, still in ascending k.  meta[t] = (first row, first entry) of tile t, meta[T] = (n, nnz).
// Per tile, every lane loads kTileCap/64 values and column indices (clamped
// inside the tile, nontemporal: the matrix stream is read once per sweep),
// gathers x, and stages the products in LDS; each row then adds its own
// products in ascending k, which associates exactly like the sequential
// definition.  The walk is software-pipelined: the next tile's value and
// column loads are in flight while the current tile gathers and sums.
// epi(row, y) is called on the lane owning each row.
template <typename VT, class Epi>
__device__ __forceinline__ void spmv_tiles_csr(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                               const VT *__restrict__ val, const double *__restrict__ x,
                                               const int2 *__restrict__ meta, int32_t ntiles, double *lds,
                                               Epi &&epi) {
    constexpr int U = kTileCap / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const TileWalk tw(ntiles);
    const int R = tw.rounds();
    int32_t t = tw.tile(0);
    if (R == 0 || t < 0) return;
    int2 m0 = meta[t], m1 = meta[t + 1];
    VT v[U];
    int32_t c[U];
    int32_t ra = 0, rb = 0;
    auto issue = [&](int2 a, int2 b, VT *vv, int32_t *cc, int32_t &qa, int32_t &qb) {
        const int32_t k0 = a.y, cnt = b.y - a.y;
        const int32_t row = a.x + lane;
        const int32_t rr = row < b.x ? row : a.x;
        qa = rp[rr] - k0;
        qb = rp[rr + 1] - k0;
        if (cnt > 0 && cnt <= kTileCap) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t e = u * kWave + lane;
                const int32_t k = k0 + (e < cnt ? e : cnt - 1);
                vv[u] = __builtin_nontemporal_load(&val[k]);
                cc[u] = __builtin_nontemporal_load(&col[k]);
            }
        }
    };
    issue(m0, m1, v, c, ra, rb);
    for (int r = 0; r < R; ++r) {
        const int32_t tn = tw.tile(r + 1);
        int2 n0 = m1, n1 = m1;
        if (tn >= 0) {
            n0 = meta[tn];
            n1 = meta[tn + 1];
        }
        const int32_t cnt = m1.y - m0.y;
        if (cnt > kTileCap) {
            // one long row, summed like every other row in ascending k: the
            // wave stages kTileCap rounded products at a time in LDS and
            // lane 0 adds them in order (the store rounds each product, so
            // no product is fused into the running sum)
            double s = 0.0;
            for (int32_t e0 = 0; e0 < cnt; e0 += kTileCap) {
                const int32_t m = cnt - e0 < kTileCap ? cnt - e0 : kTileCap;
                for (int32_t e = lane; e < m; e += kWave) {
                    const int32_t k = m0.y + e0 + e;
                    lds[e] = (double)val[k] * x[col[k]];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (lane == 0)
                    for (int32_t e = 0; e < m; ++e) s += lds[e];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
            if (lane == 0) epi(m0.x, s);
        } else {
            double xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) xv[u] = cnt > 0 ? x[c[u]] : 0.0;
            VT vn[U];
            int32_t cn[U];
            int32_t ran = 0, rbn = 0;
            if (tn >= 0) issue(n0, n1, vn, cn, ran, rbn);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t e = u * kWave + lane;
                if (e < cnt) lds[e] = (double)v[u] * xv[u];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int32_t row = m0.x + lane;
            const bool own = row < m1.x;
            double s = 0.0;
            if (own)
                for (int32_t k = ra; k < rb; ++k) s += lds[k];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (own) epi(row, s);
            if (tn >= 0) {
                ra = ran;
                rb = rbn;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    v[u] = vn[u];
                    c[u] = cn[u];
                }
            }
        }
        if (tn < 0) break;
        if (m1.y - m0.y > kTileCap || n1.y - n0.y > kTileCap) {
            // a long row breaks the pipeline: (re)issue the next tile now
            issue(n0, n1, v, c, ra, rb);
        }
        m0 = n0;
        m1 = n1;
    }
}

// The same tiled SpMV on the offset-mask form.  Tiles, value layout, LDS
// staging and the per-row ascending summation are those of the CSR walk, so
// the result is bitwise identical; only the column of each staged entry is
// derived from the row masks: each lane turns its row's mask into column
// offsets (relative to the tile's first row) written at its row's slot in
// LDS (slots = exclusive prefix sum of the rows' entry counts), and every
// lane then reads the column of the entries it loads.  The LDS words that
// held the offsets are overwritten by the products afterwards.
template <typename VT, class Epi>
__device__ __forceinline__ void spmv_tiles_stencil(const Stencil &sn, const VT *__restrict__ val,
                                                   const double *__restrict__ x, const int2 *__restrict__ meta,
                                                   int32_t ntiles, double *lds, Epi &&epi) {
    constexpr int U = kTileCap / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    int32_t *ldc = reinterpret_cast<int32_t *>(lds);
    const uint16_t *__restrict__ mask = sn.mask;
    const TileWalk tw(ntiles);
    const int R = tw.rounds();
    int32_t t = tw.tile(0);
    if (R == 0 || t < 0) return;
    int2 m0 = meta[t], m1 = meta[t + 1];
    VT v[U];
    uint32_t mk = 0;
    auto issue = [&](int2 a, int2 b, VT *vv, uint32_t &mm) {
        const int32_t k0 = a.y, cnt = b.y - a.y;
        const int32_t row = a.x + lane;
        mm = row < b.x ? (uint32_t)__builtin_nontemporal_load(&mask[row]) : 0u;
        if (cnt > 0) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t e = u * kWave + lane;
                vv[u] = __builtin_nontemporal_load(&val[k0 + (e < cnt ? e : cnt - 1)]);
            }
        }
    };
    issue(m0, m1, v, mk);
    for (int r = 0; r < R; ++r) {
        const int32_t tn = tw.tile(r + 1);
        int2 n0 = m1, n1 = m1;
        if (tn >= 0) {
            n0 = meta[tn];
            n1 = meta[tn + 1];
        }
        const int32_t cnt = m1.y - m0.y;
        // this row's entries occupy slots [ra, rb) of the tile
        const int32_t own_cnt = __popc(mk);
        int32_t incl = own_cnt;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int32_t y = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += y;
        }
        const int32_t ra = incl - own_cnt, rb = incl;
        {
            int32_t k = ra;
#pragma unroll
            for (int s = 0; s < kMaxOffsets; ++s)
                if ((mk >> s) & 1u) ldc[k++] = lane + sn.ofs[s];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        int32_t c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t e = u * kWave + lane;
            c[u] = m0.x + (e < cnt ? ldc[e] : 0);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = cnt > 0 ? x[c[u]] : 0.0;
        VT vn[U];
        uint32_t mkn = 0;
        if (tn >= 0) issue(n0, n1, vn, mkn);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t e = u * kWave + lane;
            if (e < cnt) lds[e] = (double)v[u] * xv[u];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int32_t row = m0.x + lane;
        const bool own = row < m1.x;
        double s = 0.0;
        if (own)
            for (int32_t k = ra; k < rb; ++k) s += lds[k];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (own) epi(row, s);
        if (tn < 0) break;
        mk = mkn;
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = vn[u];
        m0 = n0;
        m1 = n1;
    }
}

// Tiled SpMV on whichever form the pattern carries (uniform branch).
template <typename VT, class Epi>
__device__ __forceinline__ void spmv_tiles(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                           const Stencil &sn, const VT *__restrict__ val,
                                           const double *__restrict__ x, const int2 *__restrict__ meta,
                                           int32_t ntiles, double *lds, Epi &&epi) {
    if (sn.mask)
        spmv_tiles_stencil(sn, val, x, meta, ntiles, lds, epi);
    else
        spmv_tiles_csr(rp, col, val, x, meta, ntiles, lds, epi);
}

// Diagonal-major values of an offset-mask pattern are stored in chunks of
// kDiaChunk rows: the entries of chunk c on diagonal s are contiguous at
// [(c * nofs + s) * kDiaChunk, + kDiaChunk), so one chunk's values for all
// diagonals form a single contiguous run (zeros where a row has no entry
// and past the last row).
constexpr int kDiaChunk = 2 * kBlock;

__host__ __device__ inline int64_t dia_chunks(int64_t n) { return (n + kDiaChunk - 1) / kDiaChunk; }
__host__ __device__ inline int64_t dia_index(int64_t i, int s, int nofs) {
    return ((i / kDiaChunk) * nofs + s) * kDiaChunk + (i % kDiaChunk);
}

// XCD-aware walk over row chunks: XCD k (blocks b with b % 8 == k) owns
// chunks [C k / 8, C (k+1) / 8) and its blocks sweep that range, so the
// rows being processed on one XCD at a time stay within a window whose
// stencil neighbours are in that XCD's L2.
struct ChunkWalk {
    int64_t first, stride, hi;
    __device__ __forceinline__ explicit ChunkWalk(int64_t nchunks) {
        const int G = gridDim.x;
        if (G % kXcds == 0) {
            const int xcd = blockIdx.x % kXcds;
            const int per = G / kXcds;
            first = nchunks * xcd / kXcds + blockIdx.x / kXcds;
            hi = nchunks * (xcd + 1) / kXcds;
            stride = per;
        } else {
            first = blockIdx.x;
            hi = nchunks;
            stride = G;
        }
    }
};

// Slot count of the diagonal-major SpMV for a pattern with nofs diagonals:
// the common stencil widths 5, 7 and 9 get exact instantiations (every
// diagonal's loads issued together), others round up to a multiple of 4.
__host__ __device__ inline int dia_slots_for(int nofs) {
    return (nofs == 5 || nofs == 7 || nofs == 9) ? nofs : (nofs + 3) / 4 * 4;
}

// Symmetric half form.  When the offsets come in pairs +-o around the main
// diagonal, the pattern is symmetric and the values are symmetric bit for
// bit, only the main and the upper diagonals are stored (stored slot
// s - nofs/2 for diagonal s >= nofs/2, same chunked layout with nofs/2 + 1
// slots): the entry (i, i - o) of a lower diagonal is the stored entry
// (i - o, i).  When the largest offset o_max is a multiple of kDiaChunk the
// SpMV walks pencils: a block takes one chunk position inside an o_max-row
// plane for kPencil consecutive planes, so the +o_max diagonal loaded for one
// plane is, unchanged, the -o_max diagonal of the next plane's rows; the
// other lower diagonals are re-read from entries that the block or its XCD
// neighbours loaded moments before.  Slot counts above kSymNS select this
// form for NS - kSymNS diagonals.
constexpr int kSymNS = 100;
// Slot counts above kUnitNS select the half form of an operator whose
// diagonal is 1 by construction (Jacobi CG's S A S): the main diagonal is not
// stored either, and its product is p_i itself.
constexpr int kUnitNS = 200;
// Slot counts above kUnitFullNS select the full copy of an operator whose
// diagonal is 1 by construction (right-Jacobi BiCGStab's A D^{-1}): every
// diagonal but the main one is stored.
constexpr int kUnitFullNS = 300;
constexpr int kPencil = 16;  // longest pencil

// Stored diagonals per system of a diagonal-major copy for slot count ns.
__host__ __device__ inline int dia_stored(int ns, int nofs) {
    return ns > kUnitFullNS ? nofs - 1 : ns > kUnitNS ? nofs / 2 : ns > kSymNS ? nofs / 2 + 1 : nofs;
}

inline bool stencil_half_ok(const Stencil &sn) {
    if (!sn.mask || (sn.nofs != 5 && sn.nofs != 7 && sn.nofs != 9)) return false;
    const int ds = sn.nofs / 2;
    if (sn.diag_slot != ds) return false;
    for (int u = 1; u <= ds; ++u)
        if (sn.ofs[ds - u] != -sn.ofs[ds + u]) return false;
    return sn.ofs[sn.nofs - 1] > 0;
}

// The half form walks pencils when the largest offset is a whole number of
// chunks, else chunks.
inline bool half_pencil(const Stencil &sn) { return sn.ofs[sn.nofs - 1] % kDiaChunk == 0; }

// Pencil length for a launch over B systems of n rows: the longest (up to
// kPencil planes) that still gives the grid about 8 pencils per CU.
inline int pencil_len(const Stencil &sn, int64_t n, int B, int num_cu) {
    if (!half_pencil(sn)) return 1;
    const int64_t cols = sn.ofs[sn.nofs - 1] / kDiaChunk;
    const int64_t planes = (dia_chunks(n) + cols - 1) / cols;
    int P = kPencil;
    while (P > 1 && cols * ((planes + P - 1) / P) * (int64_t)B < 8 * (int64_t)num_cu) P /= 2;
    return P;
}

// Pencil items: column col (chunk position inside a plane of cols chunks)
// and segment seg (planes [seg * P, + P), P = sn.pencil).  With a grid that is
// a multiple of kXcds, XCD k owns columns [cols k / 8, cols (k+1) / 8), so
// the neighbouring columns whose entries and x a row gathers are processed
// on the same XCD at the same time.
struct PencilWalk {
    int64_t cols, nch, c0, ncx, items, first, stride;
    __device__ __forceinline__ PencilWalk(int64_t n, int64_t omax, int P) {
        nch = dia_chunks(n);
        cols = omax / kDiaChunk;
        const int64_t planes = (nch + cols - 1) / cols;
        const int64_t segs = (planes + P - 1) / P;
        const int G = gridDim.x;
        if (G % kXcds == 0 && cols >= kXcds) {
            const int xcd = blockIdx.x % kXcds;
            c0 = cols * xcd / kXcds;
            ncx = cols * (xcd + 1) / kXcds - c0;
            first = blockIdx.x / kXcds;
            stride = G / kXcds;
        } else {
            c0 = 0;
            ncx = cols;
            first = blockIdx.x;
            stride = G;
        }
        items = ncx * segs;
    }
};

// SpMV on the chunked diagonal-major copy of the values (see kDiaChunk).
// A block takes one chunk of 512 rows per step, each thread two rows 256
// apart; each row adds its present products in ascending diagonal order,
// which is ascending column order, with products rounded before the add (no
// contraction), so the result equals the CSR and tile forms bit for bit.
// NS is the slot count: exactly nofs for 5, 7 and 9 diagonals, otherwise a
// multiple of 4 >= nofs whose slots past nofs reload the last diagonal and
// are masked out.  epi(row, y) per row, or epi(row, y, x_row) when the
// epilogue takes x of its own row too (it is the diagonal slot's gathered
// value: absent entries gather the row's own x).
template <int NS, bool UNIT, typename VT, class Epi>
__device__ __forceinline__ void spmv_dia_sym(const Stencil &sn, const VT *__restrict__ dv, int64_t n,
                                             const double *__restrict__ x, Epi &&epi);

template <int NS, bool UF, typename VT, class Epi>
__device__ __forceinline__ void spmv_dia_full(const Stencil &sn, const VT *__restrict__ dv, int64_t n,
                                              const double *__restrict__ x, Epi &&epi);

template <int NS, typename VT, class Epi>
__device__ __forceinline__ void spmv_dia(const Stencil &sn, const VT *__restrict__ dv, int64_t n,
                                         const double *__restrict__ x, Epi &&epi) {
    if constexpr (NS > kUnitFullNS)
        spmv_dia_full<NS - kUnitFullNS, true>(sn, dv, n, x, epi);
    else if constexpr (NS > kUnitNS)
        spmv_dia_sym<NS - kUnitNS, true>(sn, dv, n, x, epi);
    else if constexpr (NS > kSymNS)
        spmv_dia_sym<NS - kSymNS, false>(sn, dv, n, x, epi);
    else
        spmv_dia_full<NS, false>(sn, dv, n, x, epi);
}

typedef double dpair __attribute__((ext_vector_type(2)));

// An epilogue that derives from OwnRowsEpi reads per-row data of its own:
// load_one(row) is issued when a step starts, together with the product's
// loads, so that no second memory round trip follows the sum, and
// one(row, y, loaded) finishes the row.  (Strided chunk layout of the full
// copy; the tile walk calls it as epi(row, y).)
struct OwnRowsEpi {};
template <class Epi>
constexpr bool own_rows_epi = std::is_base_of_v<OwnRowsEpi, std::remove_reference_t<Epi>>;

__device__ __forceinline__ int64_t clamp_row(int64_t r, int64_t n) { return r < 0 ? 0 : r < n ? r : n - 1; }

// Whether the paired row layout applies (see full_pair and sym_pair): 5, 7
// or 9 diagonals with the main one in the middle and -1 and +1 beside it,
// every other offset even, n even and x 16-byte aligned.  The host makes the
// same test to report the layout a solve ran.
__host__ __device__ inline bool pairable_stencil(const Stencil &sn, int64_t n) {
    const int ns = sn.nofs, ds = ns / 2;
    if ((ns != 5 && ns != 7 && ns != 9) || (n & 1) != 0 || sn.diag_slot != ds) return false;
    if (sn.ofs[ds - 1] != -1 || sn.ofs[ds + 1] != 1) return false;
    for (int s = 0; s < ns; ++s)
        if (s != ds - 1 && s != ds + 1 && (sn.ofs[s] & 1) != 0) return false;
    return true;
}

template <int NS>
__device__ __forceinline__ bool pairable(const Stencil &sn, int64_t n, const double *x) {
    return sn.nofs == NS && ((uintptr_t)x & 15u) == 0 && pairable_stencil(sn, n);
}

// One chunk of the full copy in the paired layout: rows r0 = 2t and r1 =
// 2t + 1 of the chunk, one 16-byte load per stored diagonal and per x gather
// at an even offset for both rows, the pair's own x as each other's -1 and
// +1 neighbour, and x of rows r0 - 1 and r0 + 2 from the neighbouring lanes
// (DPP).  Same products in the same order as spmv_dia_full, without
// the row masks: an absent entry is stored as 0 and every gather row is
// clamped into [0, n), so its product is 0 * (a finite x) and the add leaves
// the sum as it was (up to the sign of a zero sum).
template <int NS, bool UF, class Epi>
__device__ __forceinline__ void full_pair(const Stencil &sn, const double *__restrict__ dv, int64_t n,
                                          const double *__restrict__ x, int64_t c, Epi &&epi) {
#pragma clang fp contract(off)
    constexpr int DS = NS / 2, NST = UF ? NS - 1 : NS;
    const int64_t r0 = c * kDiaChunk + 2 * (int64_t)threadIdx.x;
    const bool one = r0 < n;  // n is even: r0 and r0 + 1 exist together
    const double *__restrict__ base = dv + c * NST * kDiaChunk + 2 * (int64_t)threadIdx.x;
    double v0[NS], v1[NS], x0[NS], x1[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        if (UF && s == DS) {
            v0[s] = 1.0;
            v1[s] = 1.0;
        } else {
            const dpair t = __builtin_nontemporal_load((const dpair *)(base + (UF && s > DS ? s - 1 : s) * kDiaChunk));
            v0[s] = t.x;
            v1[s] = t.y;
        }
        if (s == DS - 1 || s == DS + 1) {  // the neighbouring lanes' rows, after the loop
            x0[s] = x1[s] = 0.0;
        } else {
            const int64_t a = r0 + sn.ofs[s], pa = a < 0 ? 0 : a > n - 2 ? n - 2 : a;
            const dpair t = *(const dpair *)(x + pa);
            x0[s] = t.x;
            x1[s] = t.y;
        }
    }
    // x of rows r0 - 1 and r0 + 2 from the lanes below and above by DPP wave
    // shifts (the wavefront's first and last lane read theirs)
    {
        const int lane = threadIdx.x & (kWave - 1);
        double xe = 0.0;
        if (lane == 0)
            xe = x[clamp_row(r0 - 1, n)];
        else if (lane == kWave - 1)
            xe = x[clamp_row(r0 + 2, n)];
        x0[DS - 1] = dpp_f64<0x138>(xe, x1[DS]);  // wave_shr:1, lane l <- l - 1
        x1[DS + 1] = dpp_f64<0x130>(xe, x0[DS]);  // wave_shl:1, lane l <- l + 1
    }
    x1[DS - 1] = x0[DS];
    x0[DS + 1] = x1[DS];
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const double p0 = v0[s] * x0[s];
        const double p1 = v1[s] * x1[s];
        a0 = a0 + p0;
        a1 = a1 + p1;
    }
    if (one) {
        if constexpr (std::is_invocable_v<Epi, int64_t, double, double>) {
            epi(r0, a0, x0[DS]);
            epi(r0 + 1, a1, x1[DS]);
        } else {
            epi(r0, a0);
            epi(r0 + 1, a1);
        }
    }
}

// The full copy; UF: the main diagonal is 1 and not stored (slots past it
// move down by one).
template <int NS, bool UF, typename VT, class Epi>
__device__ __forceinline__ void spmv_dia_full(const Stencil &sn, const VT *__restrict__ dv, int64_t n,
                                              const double *__restrict__ x, Epi &&epi) {
#pragma clang fp contract(off)
    constexpr bool kExact = NS == 5 || NS == 7 || NS == 9;
    static_assert(!UF || kExact, "the unit-diagonal copy has 5, 7 or 9 diagonals");
    constexpr int kGroup = kExact ? NS : 4;
    const ChunkWalk cw(dia_chunks(n));
    if constexpr (kExact && std::is_same_v<VT, double> && !own_rows_epi<Epi>) {
        if (pairable<NS>(sn, n, x)) {
            for (int64_t c = cw.first; c < cw.hi; c += cw.stride) full_pair<NS, UF>(sn, dv, n, x, c, epi);
            return;
        }
    }
    const uint16_t *__restrict__ mask = sn.mask;
    const int nofs = kExact ? NS : sn.nofs;
    const int nst = UF ? nofs - 1 : nofs;  // stored diagonals
    for (int64_t c = cw.first; c < cw.hi; c += cw.stride) {
        const int64_t i = c * kDiaChunk + threadIdx.x;
        const int64_t i2 = i + kBlock;
        const bool one = i < n, two = i2 < n;
        const int64_t j1 = one ? i : 0, j2 = two ? i2 : 0;
        [[maybe_unused]] auto own1 = [&] {
            if constexpr (own_rows_epi<Epi>) return epi.load_one(j1);
            else return 0;
        }();
        [[maybe_unused]] auto own2 = [&] {
            if constexpr (own_rows_epi<Epi>) return epi.load_one(j2);
            else return 0;
        }();
        const uint32_t m1 = one ? (uint32_t)mask[i] : 0u;
        const uint32_t m2 = two ? (uint32_t)mask[i2] : 0u;
        const VT *__restrict__ base = dv + c * nst * kDiaChunk + threadIdx.x;
        double a1 = 0.0, a2 = 0.0;
        double c1 = 0.0, c2 = 0.0;  // x of the rows themselves
        const int ds = sn.diag_slot;
#pragma unroll
        for (int g = 0; g < NS; g += kGroup) {
            if (kExact || g < nofs) {
                VT v1[kGroup], v2[kGroup];
                double x1[kGroup], x2[kGroup];
#pragma unroll
                for (int u = 0; u < kGroup; ++u) {
                    const int s = kExact ? g + u : (g + u < nofs ? g + u : nofs - 1);
                    const int64_t d = sn.ofs[s];
                    const bool o1 = (m1 >> (g + u)) & 1u, o2 = (m2 >> (g + u)) & 1u;
                    if (UF && s == sn.diag_slot) {
                        v1[u] = VT(1);
                        v2[u] = VT(1);
                    } else {
                        const int si = UF && s > sn.diag_slot ? s - 1 : s;
                        v1[u] = __builtin_nontemporal_load(&base[si * kDiaChunk]);
                        v2[u] = __builtin_nontemporal_load(&base[si * kDiaChunk + kBlock]);
                    }
                    // rows i and i2 are kBlock apart: at +kBlock row i's
                    // neighbour is row i2, at -kBlock row i2's is row i
                    // (their own x, taken below)
                    const bool up = kExact && ds >= 0 && d == kBlock, dn = kExact && ds >= 0 && d == -kBlock;
                    x1[u] = up ? 0.0 : x[o1 ? i + d : j1];
                    x2[u] = dn ? 0.0 : x[o2 ? i2 + d : j2];
                }
                if constexpr (kExact) {
                    if (ds >= 0) {
                        double own1 = 0.0, own2 = 0.0;
#pragma unroll
                        for (int u = 0; u < kGroup; ++u)
                            if (u == ds) {
                                own1 = x1[u];
                                own2 = x2[u];
                            }
#pragma unroll
                        for (int u = 0; u < kGroup; ++u) {
                            if (sn.ofs[u] == kBlock) x1[u] = own2;
                            if (sn.ofs[u] == -kBlock) x2[u] = own1;
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < kGroup; ++u) {
                    const double p1 = (double)v1[u] * x1[u];
                    const double p2 = (double)v2[u] * x2[u];
                    if ((m1 >> (g + u)) & 1u) a1 = a1 + p1;
                    if ((m2 >> (g + u)) & 1u) a2 = a2 + p2;
                    if (g + u == ds) {
                        c1 = x1[u];
                        c2 = x2[u];
                    }
                }
            }
        }
        if constexpr (own_rows_epi<Epi>) {
            if (one) epi.one(i, a1, own1);
            if (two) epi.one(i2, a2, own2);
        } else if constexpr (std::is_invocable_v<Epi, int64_t, double, double>) {
            if (ds < 0) {
                c1 = x[j1];
                c2 = x[j2];
            }
            if (one) epi(i, a1, c1);
            if (two) epi(i2, a2, c2);
        } else {
            if (one) epi(i, a1);
            if (two) epi(i2, a2);
        }
    }
}

// The half form's SpMV (see kSymNS): the same products as spmv_dia, added
// in the same ascending diagonal order, so the result is bitwise that of the
// full copy, the tiles and CSR.  The upper and main diagonals stream
// (nontemporal loads: each entry is read once per sweep); the lower ones are
// re-reads of the mirrored upper entries.  Along a pencil the
// previous plane's +o_max values are, in registers, this plane's -o_max
// values, and x moves the same way: the previous plane's own x is this
// plane's x at -o_max, and its x at +o_max is this plane's own x.  When o_max
// is not a multiple of kDiaChunk (small planes) the chunks are walked as in
// spmv_dia and every lower value is a re-read.
//
// Two row layouts.  Paired (sym_pair): each thread takes two adjacent rows
// r0 = 2t, r1 = 2t + 1 of the chunk, so that every stream and every gather
// at an even offset is one 16-byte load for both rows, and the pair's own
// entries and x are each other's -1 and +1 neighbours; x of rows r0 - 1 and
// r0 + 2 and row r0 - 1's +1 entry are the neighbouring lanes' own values,
// moved by DPP (measured at 256^3: 134 -> 121 us per SpMV).  It needs the offsets
// -1 and +1 beside the main diagonal, every other offset even, n even and x
// 16-byte aligned: then a pair start clamped into [0, n - 2] reads exactly
// the x of every row that has the entry.  It reads no row masks: an absent
// entry is stored as 0 (a mirror row above the first row is taken as 0), so
// its product adds 0 to the sum.  Otherwise (sym_chunk) each thread takes
// rows t and t + 256, one 8-byte load per row, and the masks gate the adds.
template <typename VT>
struct SymCarry {
    VT v0 = VT(0), v1 = VT(0);
    double xlo0 = 0.0, xlo1 = 0.0, xown0 = 0.0, xown1 = 0.0;
};

template <int NS, bool CONT, bool UNIT, typename VT, class Epi>
__device__ __forceinline__ void sym_chunk(const Stencil &sn, const VT *__restrict__ dv, int64_t n,
                                          const double *__restrict__ x, int64_t c, SymCarry<VT> &cy, Epi &&epi) {
#pragma clang fp contract(off)
    constexpr int DS = NS / 2, NH = UNIT ? DS : DS + 1, U0 = UNIT ? DS + 1 : DS;
    const int64_t i = c * kDiaChunk + threadIdx.x;
    const int64_t i2 = i + kBlock;
    const bool one = i < n, two = i2 < n;
    const int64_t j1 = one ? i : 0, j2 = two ? i2 : 0;
    const uint32_t m1 = one ? (uint32_t)sn.mask[i] : 0u;
    const uint32_t m2 = two ? (uint32_t)sn.mask[i2] : 0u;
    const VT *__restrict__ base = dv + c * NH * kDiaChunk + threadIdx.x;
    VT v1[NS], v2[NS];
    double x1[NS], x2[NS];
    // The thread's two rows are kBlock apart: at offset +kBlock row i's
    // neighbour is row i2, at -kBlock row i2's is row i (x and the mirrored
    // entry), so those come from the thread's own registers after the loop.
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int64_t d = sn.ofs[s];
        const bool up = d == kBlock, dn = d == -kBlock && !(CONT && s == 0);
        // gather rows clamped into [0, n) rather than chosen by the mask, so
        // that no address waits for the mask load; the mask gates the adds
        const int64_t r1 = clamp_row(j1 + d, n);
        const int64_t r2 = clamp_row(j2 + d, n);
        if (UNIT && s == DS) {
            v1[s] = VT(1);
            v2[s] = VT(1);
        } else if (s >= DS) {
            v1[s] = __builtin_nontemporal_load(&base[(s - U0) * kDiaChunk]);
            v2[s] = __builtin_nontemporal_load(&base[(s - U0) * kDiaChunk + kBlock]);
        } else if (CONT && s == 0) {
            v1[s] = cy.v0;
            v2[s] = cy.v1;
        } else {
            v1[s] = dv[dia_index(r1, NS - 1 - s - U0, NH)];
            v2[s] = dn ? VT(0) : dv[dia_index(r2, NS - 1 - s - U0, NH)];
        }
        if (CONT && s == 0) {
            x1[s] = cy.xlo0;
            x2[s] = cy.xlo1;
        } else if (CONT && s == DS) {
            x1[s] = cy.xown0;
            x2[s] = cy.xown1;
        } else {
            x1[s] = up ? 0.0 : x[r1];
            x2[s] = dn ? 0.0 : x[r2];
        }
    }
    {
        VT vup = VT(0);  // row i's +kBlock entry: the mirror of row i2's -kBlock entry
#pragma unroll
        for (int s = DS; s < NS; ++s)
            if (sn.ofs[s] == kBlock) vup = v1[s];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (sn.ofs[s] == kBlock) x1[s] = x2[DS];
            if (sn.ofs[s] == -kBlock && !(CONT && s == 0)) {
                x2[s] = x1[DS];
                v2[s] = vup;
            }
        }
    }
    double a1 = 0.0, a2 = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const double p1 = (double)v1[s] * x1[s];
        const double p2 = (double)v2[s] * x2[s];
        if ((m1 >> s) & 1u) a1 = a1 + p1;
        if ((m2 >> s) & 1u) a2 = a2 + p2;
    }
    cy.v0 = v1[NS - 1];
    cy.v1 = v2[NS - 1];
    cy.xlo0 = x1[DS];
    cy.xlo1 = x2[DS];
    cy.xown0 = x1[NS - 1];
    cy.xown1 = x2[NS - 1];
    if constexpr (std::is_invocable_v<Epi, int64_t, double, double>) {
        if (one) epi(i, a1, x1[DS]);
        if (two) epi(i2, a2, x2[DS]);
    } else {
        if (one) epi(i, a1);
        if (two) epi(i2, a2);
    }
}

template <int NS, bool CONT, bool UNIT, typename VT, class Epi>
__device__ __forceinline__ void sym_pair(const Stencil &sn, const VT *__restrict__ dv, int64_t n,
                                         const double *__restrict__ x, int64_t c, SymCarry<VT> &cy, Epi &&epi) {
#pragma clang fp contract(off)
    static_assert(std::is_same_v<VT, double>, "the paired layout reads FP64 pairs");
    constexpr int DS = NS / 2, NH = UNIT ? DS : DS + 1, U0 = UNIT ? DS + 1 : DS;
    const int64_t r0 = c * kDiaChunk + 2 * (int64_t)threadIdx.x;
    const int64_t npad = dia_chunks(n) * kDiaChunk;  // rows of the padded diagonal-major copy
    const bool one = r0 < n;                         // n is even: r0 and r0 + 1 exist together
    const VT *__restrict__ base = dv + c * NH * kDiaChunk + 2 * (int64_t)threadIdx.x;
    VT v0[NS], v1[NS];
    double x0[NS], x1[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int64_t d = sn.ofs[s];
        const int ms = NS - 1 - s - U0;  // stored slot of the mirrored upper entry
        if (UNIT && s == DS) {
            v0[s] = VT(1);
            v1[s] = VT(1);
        } else if (s >= DS) {
            const dpair t = __builtin_nontemporal_load((const dpair *)(base + (s - U0) * kDiaChunk));
            v0[s] = t.x;
            v1[s] = t.y;
        } else if (CONT && s == 0) {
            v0[s] = cy.v0;
            v1[s] = cy.v1;
        } else if (s == DS - 1) {  // d = -1: taken from the lane below after the loop
            v0[s] = VT(0);
        } else {  // a mirror row above the first row holds no entry: 0
            const int64_t a = r0 + d, pa = a < 0 ? 0 : a > npad - 2 ? npad - 2 : a;
            const dpair t = *(const dpair *)(dv + dia_index(pa, ms, NH));
            v0[s] = a >= 0 ? t.x : VT(0);
            v1[s] = a >= 0 ? t.y : VT(0);
        }
        if (CONT && s == 0) {
            x0[s] = cy.xlo0;
            x1[s] = cy.xlo1;
        } else if (CONT && s == DS) {
            x0[s] = cy.xown0;
            x1[s] = cy.xown1;
        } else if (s == DS - 1 || s == DS + 1) {  // the neighbouring lanes' rows, after the loop
            x0[s] = x1[s] = 0.0;
        } else {
            const int64_t a = r0 + d, pa = a < 0 ? 0 : a > n - 2 ? n - 2 : a;
            const dpair t = *(const dpair *)(x + pa);
            x0[s] = t.x;
            x1[s] = t.y;
        }
    }
    // Rows r0 - 1 and r0 + 2 belong to the lanes below and above: their x
    // and row r0 - 1's +1 entry (the mirror of row r0's -1 entry) move by
    // DPP wave shifts; the wavefront's first and last lane read theirs.
    {
        const int lane = threadIdx.x & (kWave - 1);
        double xe = 0.0;
        VT ve = VT(0);
        if (lane == 0) {
            xe = x[clamp_row(r0 - 1, n)];
            ve = r0 >= 1 ? dv[dia_index(r0 - 1, NS - 1 - (DS - 1) - U0, NH)] : VT(0);
        } else if (lane == kWave - 1) {
            xe = x[clamp_row(r0 + 2, n)];
        }
        x0[DS - 1] = dpp_f64<0x138>(xe, x1[DS]);       // wave_shr:1, lane l <- l - 1
        x1[DS + 1] = dpp_f64<0x130>(xe, x0[DS]);       // wave_shl:1, lane l <- l + 1
        v0[DS - 1] = dpp_f64<0x138>(ve, v1[DS + 1]);
    }
    v1[DS - 1] = v0[DS + 1];
    x1[DS - 1] = x0[DS];
    x0[DS + 1] = x1[DS];
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const double p0 = (double)v0[s] * x0[s];
        const double p1 = (double)v1[s] * x1[s];
        a0 = a0 + p0;
        a1 = a1 + p1;
    }
    cy.v0 = v0[NS - 1];
    cy.v1 = v1[NS - 1];
    cy.xlo0 = x0[DS];
    cy.xlo1 = x1[DS];
    cy.xown0 = x0[NS - 1];
    cy.xown1 = x1[NS - 1];
    if (one) {
        if constexpr (std::is_invocable_v<Epi, int64_t, double, double>) {
            epi(r0, a0, x0[DS]);
            epi(r0 + 1, a1, x1[DS]);
        } else {
            epi(r0, a0);
            epi(r0 + 1, a1);
        }
    }
}

template <int NS, bool UNIT, bool PAIR, typename VT, class Epi>
__device__ __forceinline__ void sym_walk(const Stencil &sn, const VT *__restrict__ dv, int64_t n,
                                         const double *__restrict__ x, Epi &&epi) {
    const int64_t omax = sn.ofs[NS - 1];
    SymCarry<VT> cy;
    auto step = [&](int64_t c, auto cont) {
        if constexpr (PAIR)
            sym_pair<NS, decltype(cont)::value, UNIT>(sn, dv, n, x, c, cy, epi);
        else
            sym_chunk<NS, decltype(cont)::value, UNIT>(sn, dv, n, x, c, cy, epi);
    };
    if (omax % kDiaChunk != 0) {
        const ChunkWalk cw(dia_chunks(n));
        for (int64_t c = cw.first; c < cw.hi; c += cw.stride) step(c, std::false_type{});
        return;
    }
    const int P = sn.pencil;
    const PencilWalk pw(n, omax, P);
    for (int64_t it = pw.first; it < pw.items; it += pw.stride) {
        const int64_t col = pw.c0 + it % pw.ncx, seg = it / pw.ncx;
        int64_t c = seg * P * pw.cols + col;
        if (c >= pw.nch) continue;
        step(c, std::false_type{});
        for (int t = 1; t < P; ++t) {
            c += pw.cols;
            if (c >= pw.nch) break;
            step(c, std::true_type{});
        }
    }
}

template <int NS, bool UNIT, typename VT, class Epi>
__device__ __forceinline__ void spmv_dia_sym(const Stencil &sn, const VT *__restrict__ dv, int64_t n,
                                             const double *__restrict__ x, Epi &&epi) {
    static_assert(NS == 5 || NS == 7 || NS == 9, "half form for 5, 7 or 9 diagonals");
    if (pairable<NS>(sn, n, x))
        sym_walk<NS, UNIT, true>(sn, dv, n, x, epi);
    else
        sym_walk<NS, UNIT, false>(sn, dv, n, x, epi);
}

}  // namespace hsla
