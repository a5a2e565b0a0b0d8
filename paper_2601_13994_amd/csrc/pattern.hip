// Handle, workspace and sparsity-pattern ingest: canonical-CSR validation,
// diagonal positions, the transpose permutation, lower/upper triangles and
// the SpMV tile schedule.  Pattern work is integer-only and deterministic.
#include <climits>
#include <cstdarg>
#include <cstring>
#include <algorithm>
#include <vector>

#include "common.h"

namespace hsla {

hsla_status set_error(hsla_handle *h, hsla_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->last_error = buf;
    return st;
}

hipError_t dev_alloc(hsla_handle *h, void **p, size_t bytes) {
    if (h->alloc_fn) {
        *p = h->alloc_fn(bytes, h->alloc_ctx);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

void dev_free(hsla_handle *h, void *p) {
    if (!p) return;
    if (h->free_fn)
        h->free_fn(p, h->alloc_ctx);
    else
        (void)hipFree(p);
}

hsla_status ensure_workspace(hsla_handle *h, size_t bytes) {
    if (bytes <= h->ws_bytes) return HSLA_OK;
    if (h->ws_fixed)
        return set_error(h, HSLA_ERR_INVALID_ARG,
                         "this call needs %zu bytes of scratch; the allocation-free entry point has %zu", bytes,
                         h->ws_bytes);
    if (h->ws) {
        HSLA_HIP(h, hipDeviceSynchronize());
        dev_free(h, h->ws);
        h->ws = nullptr;
        h->ws_bytes = 0;
        for (int i = 0; i < hsla_handle::kGraphCache; ++i) {
            if (h->graph_exec[i]) (void)hipGraphExecDestroy(h->graph_exec[i]);
            h->graph_exec[i] = nullptr;
            h->graph_key[i] = 0;
        }
    }
    size_t want = bytes + bytes / 8 + 4096;
    hipError_t e = dev_alloc(h, &h->ws, want);
    if (e != hipSuccess) {
        h->ws = nullptr;
        return set_error(h, HSLA_ERR_NO_MEMORY, "workspace of %zu bytes: %s", want, hipGetErrorString(e));
    }
    h->ws_bytes = want;
    // Zero-fill on the handle's own stream and wait for it: that stream does
    // not wait on the legacy null stream, so a plain hipMemset could land in
    // the middle of the solve that follows.
    HSLA_HIP(h, hipMemsetAsync(h->ws, 0, want, h->stream));
    HSLA_HIP(h, hipStreamSynchronize(h->stream));
    return HSLA_OK;
}

hsla_status enter(hsla_handle *h, hipStream_t user) {
    HSLA_HIP(h, hipSetDevice(h->device));
    HSLA_HIP(h, hipEventRecord(h->entry_event, user));
    HSLA_HIP(h, hipStreamWaitEvent(h->stream, h->entry_event, 0));
    return HSLA_OK;
}

hsla_status ensure_host_state(hsla_handle *h, size_t nsys) {
    if (nsys <= h->h_state_cap) return HSLA_OK;
    if (h->ws_fixed)
        return set_error(h, HSLA_ERR_INVALID_ARG, "%zu systems exceed the %zu the allocation-free entry point takes",
                         nsys, h->h_state_cap);
    if (h->h_state) HSLA_HIP(h, hipHostFree(h->h_state));
    h->h_state = nullptr;
    HSLA_HIP(h, hipHostMalloc((void **)&h->h_state, nsys * sizeof(SysState), hipHostMallocDefault));
    h->h_state_cap = nsys;
    return HSLA_OK;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Canonical-CSR check of row i: its entry range [rp[i], rp[i+1]) lies in
// [0, nnz] (checked before any entry is read) and its columns are in
// [0, n) and strictly increasing.  *d receives the position of (i, i) (-1
// if absent) and *lower is advanced by the row's entries with col <= i.
// Shared by the device validation and hsla_csr_check.
__host__ __device__ inline bool csr_row_ok(int32_t i, int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col,
                                           int32_t *d, int64_t *lower) {
    const int32_t lo = rp[i], hi = rp[i + 1];
    *d = -1;
    if (!(lo >= 0 && lo <= hi && (int64_t)hi <= nnz)) return false;
    int32_t prev = -1;
    for (int32_t k = lo; k < hi; ++k) {
        const int32_t c = col[k];
        if (c < 0 || c >= n || c <= prev) return false;
        if (c == i) *d = k;
        if (c <= i) ++*lower;
        prev = c;
    }
    return true;
}

// Per-row canonical-CSR checks.  The first offending row wins via an
// integer atomic minimum (order-independent).  diag[i] = position of (i, i).
__global__ __launch_bounds__(kBlock) void k_validate(int32_t n, int64_t nnz, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col, int32_t *__restrict__ diag,
                                                     int32_t *__restrict__ bad_row, int64_t *__restrict__ nnz_lower) {
    int64_t lower = 0;
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        int32_t d = -1;
        const bool ok = csr_row_ok(i, n, nnz, rp, col, &d, &lower);
        diag[i] = d;
        if (!ok) atomicMin(bad_row, i);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lower += __shfl_xor(lower, o, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0 && lower) atomicAdd((unsigned long long *)nnz_lower, (unsigned long long)lower);
}

__global__ __launch_bounds__(kBlock) void k_find_diag(int32_t n, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ col, int32_t *__restrict__ diag) {
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        int32_t d = -1;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
            if (col[k] == i) d = k;
        diag[i] = d;
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = v;
}

// counts[c + 1] += 1 for every stored entry in column c (integer atomics:
// the totals do not depend on order).
__global__ __launch_bounds__(kBlock) void k_count_cols(int64_t nnz, const int32_t *__restrict__ col,
                                                       int32_t *__restrict__ counts1) {
    for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * kBlock)
        atomicAdd(&counts1[col[k] + 1], 1);
}

// Inclusive scan, phase 1: each block scans kScanItems consecutive values in
// place and records its total.
constexpr int kScanPer = 8;
constexpr int kScanItems = kBlock * kScanPer;

__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t *sh, int32_t *total) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int32_t inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int32_t t = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += t;
    }
    if (lane == kWave - 1) sh[w] = inc;
    __syncthreads();
    int32_t base = 0, tot = 0;
    for (int q = 0; q < kWavesPerBlock; ++q) {
        if (q < w) base += sh[q];
        tot += sh[q];
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_blocks(int32_t *__restrict__ a, int64_t m, int32_t *__restrict__ tot) {
    __shared__ int32_t sh[kWavesPerBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanItems + (int64_t)threadIdx.x * kScanPer;
    int32_t v[kScanPer];
    int32_t s = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        v[j] = base + j < m ? a[base + j] : 0;
        s += v[j];
        v[j] = s;
    }
    int32_t total;
    const int32_t off = block_excl_scan(s, sh, &total);
#pragma unroll
    for (int j = 0; j < kScanPer; ++j)
        if (base + j < m) a[base + j] = v[j] + off;
    if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

// Phase 2: exclusive scan of the block totals by one block.
__global__ __launch_bounds__(kBlock) void k_scan_totals(int32_t *__restrict__ tot, int32_t nb) {
    __shared__ int32_t sh[kWavesPerBlock];
    int32_t carry = 0;
    for (int32_t base = 0; base < nb; base += kBlock) {
        const int32_t i = base + threadIdx.x;
        const int32_t v = i < nb ? tot[i] : 0;
        int32_t total;
        const int32_t ex = block_excl_scan(v, sh, &total);
        if (i < nb) tot[i] = carry + ex;
        carry += total;
    }
}

// Phase 3: add each block's offset.
__global__ __launch_bounds__(kBlock) void k_scan_add(int32_t *__restrict__ a, int64_t m, const int32_t *__restrict__ tot) {
    const int32_t off = tot[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kScanItems;
    for (int j = threadIdx.x; j < kScanItems; j += kBlock)
        if (base + j < m) a[base + j] += off;
}

// Scatter of A's entries into A^T's rows.  Slots inside a row of A^T are
// taken with an atomic cursor (arbitrary order); k_sort_segments restores
// ascending column order, which makes the result unique.
__global__ __launch_bounds__(kBlock) void k_scatter_T(int32_t n, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ col, int32_t *__restrict__ cursor,
                                                      int32_t *__restrict__ colT, int32_t *__restrict__ srcT) {
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int32_t slot = atomicAdd(&cursor[col[k]], 1);
            colT[slot] = i;
            srcT[slot] = k;
        }
}

__global__ __launch_bounds__(kBlock) void k_sort_segments(int32_t n, const int32_t *__restrict__ rpT,
                                                          int32_t *__restrict__ colT, int32_t *__restrict__ srcT) {
    for (int32_t j = blockIdx.x * kBlock + threadIdx.x; j < n; j += gridDim.x * kBlock) {
        const int32_t lo = rpT[j], hi = rpT[j + 1];
        for (int32_t a = lo + 1; a < hi; ++a) {
            const int32_t c = colT[a], s = srcT[a];
            int32_t b = a - 1;
            while (b >= lo && colT[b] > c) {
                colT[b + 1] = colT[b];
                srcT[b + 1] = srcT[b];
                --b;
            }
            colT[b + 1] = c;
            srcT[b + 1] = s;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_compare_i32(const int32_t *__restrict__ a, const int32_t *__restrict__ b,
                                                        int64_t m, int32_t *__restrict__ differ) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock)
        if (a[i] != b[i]) *differ = 1;
}

// Pattern signature: sum over elements of splitmix64(salt ^ (i << 32 | a[i]))
// (position-bound, so any change of an index or its place changes it with
// overwhelming probability); one 64-bit atomic add per block.
__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(kBlock) void k_hash_i32(const int32_t *__restrict__ a, int64_t m, uint64_t salt,
                                                     unsigned long long *acc) {
    __shared__ uint64_t sh[kBlock];
    uint64_t s = 0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock)
        s += mix64(salt ^ (((uint64_t)i << 32) | (uint32_t)a[i]));
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(acc, (unsigned long long)sh[0]);
}

// Lower triangle (col <= row) of a canonical CSR: a prefix of every row.
__global__ __launch_bounds__(kBlock) void k_count_lower(int32_t n, const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col, int32_t *__restrict__ cnt1) {
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        int32_t c = 0;
        for (int32_t k = rp[i]; k < rp[i + 1] && col[k] <= i; ++k) ++c;
        cnt1[i + 1] = c;
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_lower(int32_t n, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col, const int32_t *__restrict__ rpL,
                                                       int32_t *__restrict__ colL, int32_t *__restrict__ posL) {
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const int32_t lo = rpL[i], cnt = rpL[i + 1] - lo;
        for (int32_t j = 0; j < cnt; ++j) {
            colL[lo + j] = col[rp[i] + j];
            posL[lo + j] = rp[i] + j;
        }
    }
}

// Row index and diagonal flag of every entry of a CSR pattern.
__global__ __launch_bounds__(kBlock) void k_row_flags(int32_t n, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ col, int32_t *__restrict__ row,
                                                      uint8_t *__restrict__ isdiag) {
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            row[k] = i;
            isdiag[k] = col[k] == i;
        }
}

// ---------------------------------------------------------------------------
// Host-side helpers
// ---------------------------------------------------------------------------

static int blocks_for(int64_t m) {
    int64_t b = (m + kBlock - 1) / kBlock;
    if (b > 65536) b = 65536;
    return b < 1 ? 1 : (int)b;
}

// Inclusive in-place scan of a[0..m) (int32; totals < 2^31).
static hsla_status scan_inclusive(hsla_handle *h, int32_t *a, int64_t m, hipStream_t s) {
    if (m <= 0) return HSLA_OK;
    const int64_t nb = (m + kScanItems - 1) / kScanItems;
    if (nb > INT_MAX) return set_error(h, HSLA_ERR_INVALID_ARG, "scan too long");
    int32_t *tot = nullptr;
    HSLA_HIP(h, hipMalloc((void **)&tot, sizeof(int32_t) * nb));
    k_scan_blocks<<<(unsigned)nb, kBlock, 0, s>>>(a, m, tot);
    k_scan_totals<<<1, kBlock, 0, s>>>(tot, (int32_t)nb);
    k_scan_add<<<(unsigned)nb, kBlock, 0, s>>>(a, m, tot);
    HSLA_HIP(h, hipGetLastError());
    HSLA_HIP(h, hipStreamSynchronize(s));
    HSLA_HIP(h, hipFree(tot));
    return HSLA_OK;
}

// CSR transpose on the device (deterministic, canonical result).
static hsla_status device_transpose(hsla_handle *h, int32_t n, int64_t nnz, const int32_t *rp, const int32_t *col,
                                    int32_t *rpT, int32_t *colT, int32_t *srcT, hipStream_t s) {
    HSLA_HIP(h, hipMemsetAsync(rpT, 0, sizeof(int32_t) * (n + 1), s));
    if (nnz > 0) k_count_cols<<<blocks_for(nnz), kBlock, 0, s>>>(nnz, col, rpT);
    hsla_status st = scan_inclusive(h, rpT + 1, n, s);
    if (st != HSLA_OK) return st;
    if (nnz > 0) {
        int32_t *cursor = nullptr;
        HSLA_HIP(h, hipMalloc((void **)&cursor, sizeof(int32_t) * (n > 0 ? n : 1)));
        HSLA_HIP(h, hipMemcpyAsync(cursor, rpT, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
        k_scatter_T<<<blocks_for(n), kBlock, 0, s>>>(n, rp, col, cursor, colT, srcT);
        k_sort_segments<<<blocks_for(n), kBlock, 0, s>>>(n, rpT, colT, srcT);
        HSLA_HIP(h, hipGetLastError());
        HSLA_HIP(h, hipStreamSynchronize(s));
        HSLA_HIP(h, hipFree(cursor));
    }
    return HSLA_OK;
}

// Tile schedule: consecutive rows packed while a tile holds at most
// kTileRows rows and kTileCap entries; a row longer than kTileCap forms a
// tile by itself.  Built on the host from a copy of row_ptr; meta[t] =
// (first row, first entry) of tile t and meta[T] = (n, nnz).
static hsla_status build_tiles(hsla_handle *h, int32_t n, const int32_t *d_rp, hipStream_t s, int2 **d_meta,
                               int32_t *ntiles, std::vector<int32_t> &rp) {
    rp.assign((size_t)n + 1, 0);
    HSLA_HIP(h, hipMemcpyAsync(rp.data(), d_rp, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s));
    HSLA_HIP(h, hipStreamSynchronize(s));
    std::vector<int2> t;
    t.reserve(n / kTileRows + 2);
    t.push_back(make_int2(0, rp[0]));
    int32_t r = 0;
    while (r < n) {
        const int32_t len = rp[r + 1] - rp[r];
        if (len > kTileCap) {
            ++r;
        } else {
            int32_t e = r, acc = 0;
            while (e < n && e - r < kTileRows) {
                const int32_t l = rp[e + 1] - rp[e];
                if (l > kTileCap || acc + l > kTileCap) break;
                acc += l;
                ++e;
            }
            r = e;
        }
        t.push_back(make_int2(r, rp[r]));
    }
    *ntiles = (int32_t)t.size() - 1;
    HSLA_HIP(h, hipMalloc((void **)d_meta, sizeof(int2) * t.size()));
    HSLA_HIP(h, hipMemcpyAsync(*d_meta, t.data(), sizeof(int2) * t.size(), hipMemcpyHostToDevice, s));
    HSLA_HIP(h, hipStreamSynchronize(s));
    return HSLA_OK;
}

// Row masks of the offset-mask form: bit s of mask[i] <=> row i stores
// column i + ofs[s].  `bad` is set if an entry lies on no listed diagonal.
// Columns increase within a row and ofs increases, so bit order is entry
// order.
__global__ __launch_bounds__(kBlock) void k_build_mask(int32_t n, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col, Stencil sn,
                                                       uint16_t *__restrict__ mask, int32_t *bad) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        uint32_t m = 0;
        bool ok = true;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int32_t d = col[k] - (int32_t)i;
            int s = -1;
#pragma unroll
            for (int j = 0; j < kMaxOffsets; ++j)
                if (j < sn.nofs && sn.ofs[j] == d) s = j;
            if (s < 0)
                ok = false;
            else
                m |= 1u << s;
        }
        mask[i] = (uint16_t)m;
        if (!ok) *bad = 1;
    }
}

// Offset-mask form of a CSR structure, if it has one.  Candidate diagonals
// come from sampled rows (the first, middle and last rows and 16 spread
// blocks); the device then builds every row's mask and checks that no entry
// lies off the candidates.  Leaves *out empty when the structure has more
// than kMaxOffsets diagonals or the check fails.
static hsla_status build_stencil(hsla_handle *h, int32_t n, int64_t nnz, const std::vector<int32_t> &rp,
                                 const int32_t *d_rp, const int32_t *d_col, hipStream_t s, Stencil *out) {
    *out = Stencil{};
    if (n <= 0 || nnz <= 0) return HSLA_OK;
    std::vector<int64_t> ofs;
    bool too_many = false;
    std::vector<int32_t> c;
    auto sample = [&](int64_t r0, int64_t r1) -> hipError_t {
        r0 = r0 < 0 ? 0 : r0;
        r1 = r1 > n ? n : r1;
        if (too_many || r0 >= r1 || rp[r1] == rp[r0]) return hipSuccess;
        const int32_t k0 = rp[r0], k1 = rp[r1];
        c.resize((size_t)(k1 - k0));
        hipError_t e = hipMemcpyAsync(c.data(), d_col + k0, sizeof(int32_t) * (k1 - k0), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        for (int64_t r = r0; r < r1 && !too_many; ++r)
            for (int32_t k = rp[r]; k < rp[r + 1]; ++k) {
                const int64_t d = (int64_t)c[k - k0] - r;
                bool seen = false;
                for (int64_t o : ofs) seen |= (o == d);
                if (!seen) {
                    if ((int)ofs.size() == kMaxOffsets) {
                        too_many = true;
                        break;
                    }
                    ofs.push_back(d);
                }
            }
        return hipSuccess;
    };
    HSLA_HIP(h, sample(0, 2048));
    HSLA_HIP(h, sample((int64_t)n / 2 - 1024, (int64_t)n / 2 + 1024));
    HSLA_HIP(h, sample((int64_t)n - 2048, n));
    for (int j = 1; j <= 16; ++j) HSLA_HIP(h, sample((int64_t)n * j / 17, (int64_t)n * j / 17 + 128));
    if (too_many || ofs.empty()) return HSLA_OK;
    std::sort(ofs.begin(), ofs.end());
    Stencil st{};
    st.nofs = (int32_t)ofs.size();
    for (int j = 0; j < st.nofs; ++j) {
        st.ofs[j] = (int32_t)ofs[j];
        if (ofs[j] == 0) st.diag_slot = j;
    }
    uint16_t *mask = nullptr;
    int32_t *bad = nullptr;
    int32_t hbad = 0;
    HSLA_HIP(h, hipMalloc((void **)&mask, sizeof(uint16_t) * (size_t)n));
    hipError_t e = hipMalloc((void **)&bad, sizeof(int32_t));
    if (e == hipSuccess) e = hipMemsetAsync(bad, 0, sizeof(int32_t), s);
    if (e == hipSuccess) {
        k_build_mask<<<blocks_for(n), kBlock, 0, s>>>(n, d_rp, d_col, st, mask, bad);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (bad) (void)hipFree(bad);
    if (e != hipSuccess || hbad) {
        (void)hipFree(mask);
        if (e != hipSuccess) return set_error(h, HSLA_ERR_HIP, "stencil form: %s", hipGetErrorString(e));
        return HSLA_OK;
    }
    st.mask = mask;
    *out = st;
    return HSLA_OK;
}

static void free_pattern(hsla_pattern *p) {
    if (!p) return;
    for (const Stencil *st : {&p->stA, &p->stT, &p->stL, &p->stU})
        if (st->mask) (void)hipFree(const_cast<uint16_t *>(st->mask));
    void *bufs[] = {p->row_ptr, p->col, p->diag, p->meta, p->rpT, p->colT, p->srcT, p->metaT, p->diagT,
                    p->rpL, p->colL, p->posL, p->metaL, p->rpU, p->colU, p->srcU, p->metaU, p->rowL, p->isdiagL};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    delete p;
}

hsla_status make_pattern(hsla_handle *h, int32_t n, int64_t nnz, const int32_t *d_row_ptr, const int32_t *d_col,
                         uint32_t flags, hipStream_t s, hsla_pattern **out) {
    if (!h || !out) return set_error(h, HSLA_ERR_INVALID_ARG, "null handle or output");
    *out = nullptr;
    if (flags & ~(uint32_t)HSLA_PATTERN_CSR) return set_error(h, HSLA_ERR_INVALID_ARG, "unknown flags 0x%x", flags);
    const bool stencils = !(flags & HSLA_PATTERN_CSR);
    if (n < 0 || nnz < 0 || nnz >= INT32_MAX)
        return set_error(h, HSLA_ERR_INVALID_ARG, "n=%d nnz=%lld out of range", n, (long long)nnz);
    if (!d_row_ptr || (nnz > 0 && !d_col)) return set_error(h, HSLA_ERR_INVALID_ARG, "null pattern pointer");
    HSLA_HIP(h, hipSetDevice(h->device));
    hsla_pattern *p = new hsla_pattern();
    p->device = h->device;
    p->n = n;
    p->nnz = nnz;
    if (!stencils) p->format = HSLA_FORMAT_CSR;
    auto fail = [&](hsla_status st) {
        free_pattern(p);
        return st;
    };
#define PCHK(expr)                                                                                   \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return fail(set_error(h, HSLA_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)));         \
    } while (0)
    const size_t nn = (size_t)n;
    PCHK(hipMalloc((void **)&p->row_ptr, sizeof(int32_t) * (nn + 1)));
    PCHK(hipMalloc((void **)&p->col, sizeof(int32_t) * (nnz > 0 ? nnz : 1)));
    PCHK(hipMalloc((void **)&p->diag, sizeof(int32_t) * (nn > 0 ? nn : 1)));
    PCHK(hipMemcpyAsync(p->row_ptr, d_row_ptr, sizeof(int32_t) * (nn + 1), hipMemcpyDeviceToDevice, s));
    if (nnz > 0) PCHK(hipMemcpyAsync(p->col, d_col, sizeof(int32_t) * nnz, hipMemcpyDeviceToDevice, s));
    int32_t ends[2];
    PCHK(hipMemcpyAsync(&ends[0], p->row_ptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PCHK(hipMemcpyAsync(&ends[1], p->row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PCHK(hipStreamSynchronize(s));
    if (ends[0] != 0 || ends[1] != nnz)
        return fail(set_error(h, HSLA_ERR_INVALID_CSR, "row_ptr[0]=%d row_ptr[n]=%d, expected 0 and %lld", ends[0],
                              ends[1], (long long)nnz));
    struct Flags {
        int32_t bad_row;
        int32_t differ;
        int64_t nnz_lower;
        unsigned long long hash_rp, hash_col;
    } hf{INT32_MAX, 0, 0, 0, 0}, *df = nullptr;
    PCHK(hipMalloc((void **)&df, sizeof(Flags)));
    PCHK(hipMemcpyAsync(df, &hf, sizeof(Flags), hipMemcpyHostToDevice, s));
    if (n > 0) k_validate<<<blocks_for(n), kBlock, 0, s>>>(n, nnz, p->row_ptr, p->col, p->diag, &df->bad_row, &df->nnz_lower);
    k_hash_i32<<<blocks_for(n + 1), kBlock, 0, s>>>(p->row_ptr, (int64_t)n + 1, 0x5241u, &df->hash_rp);
    if (nnz > 0) k_hash_i32<<<blocks_for(nnz), kBlock, 0, s>>>(p->col, nnz, 0x434Fu, &df->hash_col);
    PCHK(hipGetLastError());
    PCHK(hipMemcpyAsync(&hf, df, sizeof(Flags), hipMemcpyDeviceToHost, s));
    PCHK(hipStreamSynchronize(s));
    if (hf.bad_row != INT32_MAX) {
        (void)hipFree(df);
        return fail(set_error(h, HSLA_ERR_INVALID_CSR, "row %d is not canonical CSR (bounds, column range or order)",
                              hf.bad_row));
    }
    p->nnz_lower = hf.nnz_lower;
    p->signature = mix64(mix64((uint64_t)n) ^ (uint64_t)nnz) + 3ull * hf.hash_rp + hf.hash_col;

    std::vector<int32_t> hrp;
    hsla_status st = build_tiles(h, n, p->row_ptr, s, &p->meta, &p->ntiles, hrp);
    for (int32_t i = 0; st == HSLA_OK && i < n; ++i) p->max_row = std::max(p->max_row, hrp[i + 1] - hrp[i]);
    if (st == HSLA_OK && stencils) st = build_stencil(h, n, nnz, hrp, p->row_ptr, p->col, s, &p->stA);
    if (st != HSLA_OK) { (void)hipFree(df); return fail(st); }

    // transpose and pattern symmetry
    PCHK(hipMalloc((void **)&p->rpT, sizeof(int32_t) * (nn + 1)));
    PCHK(hipMalloc((void **)&p->colT, sizeof(int32_t) * (nnz > 0 ? nnz : 1)));
    PCHK(hipMalloc((void **)&p->srcT, sizeof(int32_t) * (nnz > 0 ? nnz : 1)));
    st = device_transpose(h, n, nnz, p->row_ptr, p->col, p->rpT, p->colT, p->srcT, s);
    if (st != HSLA_OK) { (void)hipFree(df); return fail(st); }
    k_compare_i32<<<blocks_for(n + 1), kBlock, 0, s>>>(p->row_ptr, p->rpT, n + 1, &df->differ);
    if (nnz > 0) k_compare_i32<<<blocks_for(nnz), kBlock, 0, s>>>(p->col, p->colT, nnz, &df->differ);
    PCHK(hipGetLastError());
    PCHK(hipMemcpyAsync(&hf, df, sizeof(Flags), hipMemcpyDeviceToHost, s));
    PCHK(hipStreamSynchronize(s));
    p->pattern_symmetric = hf.differ ? 0 : 1;
    (void)hipFree(df);
    st = build_tiles(h, n, p->rpT, s, &p->metaT, &p->ntilesT, hrp);
    if (st == HSLA_OK && stencils) st = build_stencil(h, n, nnz, hrp, p->rpT, p->colT, s, &p->stT);
    if (st != HSLA_OK) return fail(st);
    PCHK(hipMalloc((void **)&p->diagT, sizeof(int32_t) * (nn > 0 ? nn : 1)));
    if (n > 0) k_find_diag<<<blocks_for(n), kBlock, 0, s>>>(n, p->rpT, p->colT, p->diagT);
    PCHK(hipGetLastError());

    // lower triangle incl. diagonal, and its transpose (the upper triangle)
    PCHK(hipMalloc((void **)&p->rpL, sizeof(int32_t) * (nn + 1)));
    PCHK(hipMemsetAsync(p->rpL, 0, sizeof(int32_t), s));
    const int64_t nL = p->nnz_lower;
    PCHK(hipMalloc((void **)&p->colL, sizeof(int32_t) * (nL > 0 ? nL : 1)));
    PCHK(hipMalloc((void **)&p->posL, sizeof(int32_t) * (nL > 0 ? nL : 1)));
    if (n > 0) {
        k_count_lower<<<blocks_for(n), kBlock, 0, s>>>(n, p->row_ptr, p->col, p->rpL);
        st = scan_inclusive(h, p->rpL + 1, n, s);
        if (st != HSLA_OK) return fail(st);
        k_fill_lower<<<blocks_for(n), kBlock, 0, s>>>(n, p->row_ptr, p->col, p->rpL, p->colL, p->posL);
        PCHK(hipGetLastError());
    }
    st = build_tiles(h, n, p->rpL, s, &p->metaL, &p->ntilesL, hrp);
    if (st == HSLA_OK && stencils) st = build_stencil(h, n, nL, hrp, p->rpL, p->colL, s, &p->stL);
    if (st != HSLA_OK) return fail(st);
    PCHK(hipMalloc((void **)&p->rpU, sizeof(int32_t) * (nn + 1)));
    PCHK(hipMalloc((void **)&p->colU, sizeof(int32_t) * (nL > 0 ? nL : 1)));
    PCHK(hipMalloc((void **)&p->srcU, sizeof(int32_t) * (nL > 0 ? nL : 1)));
    st = device_transpose(h, n, nL, p->rpL, p->colL, p->rpU, p->colU, p->srcU, s);
    if (st != HSLA_OK) return fail(st);
    st = build_tiles(h, n, p->rpU, s, &p->metaU, &p->ntilesU, hrp);
    if (st == HSLA_OK && stencils) st = build_stencil(h, n, nL, hrp, p->rpU, p->colU, s, &p->stU);
    if (st != HSLA_OK) return fail(st);
    PCHK(hipMalloc((void **)&p->rowL, sizeof(int32_t) * (nL > 0 ? nL : 1)));
    PCHK(hipMalloc((void **)&p->isdiagL, (nL > 0 ? nL : 1)));
    if (n > 0) k_row_flags<<<blocks_for(n), kBlock, 0, s>>>(n, p->rpL, p->colL, p->rowL, p->isdiagL);
    PCHK(hipGetLastError());
    PCHK(hipStreamSynchronize(s));
#undef PCHK
    *out = p;
    return HSLA_OK;
}

}  // namespace hsla

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void hsla_opts_default(hsla_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->method = HSLA_METHOD_AUTO;
    o->precond = HSLA_PRECOND_JACOBI;
    o->rtol = 1e-8;
    o->atol = 0.0;
    o->max_iter = 0;
    o->check_every = 0;
    o->use_x0 = 0;
    o->use_graph = 1;
    o->persistent = 1;
    o->stall_window = 0;
    o->s_step = 4;
}

const char *hsla_status_string(int st) {
    switch (st) {
        case HSLA_OK: return "ok";
        case HSLA_NOT_CONVERGED: return "not converged";
        case HSLA_BREAKDOWN: return "breakdown";
        case HSLA_FELL_BACK: return "fell back to Jacobi";
        case HSLA_STAGNATED: return "stagnated";
        case HSLA_ERR_INVALID_ARG: return "invalid argument";
        case HSLA_ERR_INVALID_CSR: return "invalid CSR pattern";
        case HSLA_ERR_NONFINITE: return "non-finite value";
        case HSLA_ERR_HIP: return "HIP runtime error";
        case HSLA_ERR_NO_MEMORY: return "out of device memory";
        case HSLA_ERR_ZERO_DIAGONAL: return "missing or zero diagonal";
        case HSLA_ERR_INTERNAL: return "internal error";
        default: return "unknown status";
    }
}

hsla_status hsla_create(hsla_handle **out, int device) {
    if (!out) return HSLA_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return HSLA_ERR_INVALID_ARG;
    hsla_handle *h = new hsla_handle();
    h->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete h;
        return HSLA_ERR_HIP;
    }
    int cu = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cu > 0)
        h->dev.num_cu = cu;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
        h->dev.wall_khz = khz;
    if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&h->entry_event, hipEventDisableTiming) != hipSuccess ||
        hipMalloc((void **)&h->d_flags, 256) != hipSuccess) {
        hsla_destroy(h);
        return HSLA_ERR_HIP;
    }
    // a host mirror of the per-system state large enough for the
    // allocation-free entry point's batches, and that entry point's scratch
    // array on this device (a failed lookup is retried, and reported, by
    // that entry point's first call)
    if (hsla::ensure_host_state(h, hsla::kNoAllocMaxSystems) != HSLA_OK) {
        hsla_destroy(h);
        return HSLA_ERR_HIP;
    }
    (void)hsla::scratch_init(h);
    *out = h;
    return HSLA_OK;
}

void hsla_destroy(hsla_handle *h) {
    if (!h) return;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    for (int i = 0; i < hsla_handle::kGraphCache; ++i)
        if (h->graph_exec[i]) (void)hipGraphExecDestroy(h->graph_exec[i]);
    hsla::dev_free(h, h->ws);
    if (h->h_state) (void)hipHostFree(h->h_state);
    if (h->d_flags) (void)hipFree(h->d_flags);
    hsla::dev_free(h, h->mp_ws);
    hsla::dev_free(h, h->pr_ws);
    for (int i = 0; i < h->prof_cap; ++i) (void)hipEventDestroy(h->prof_ev[i]);
    delete[] h->prof_ev;
    if (h->entry_event) (void)hipEventDestroy(h->entry_event);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

const char *hsla_last_error(const hsla_handle *h) { return h ? h->last_error.c_str() : "null handle"; }

hsla_status hsla_set_allocator(hsla_handle *h, hsla_alloc_fn alloc, hsla_free_fn free_fn, void *ctx) {
    if (!h) return HSLA_ERR_INVALID_ARG;
    if ((alloc == nullptr) != (free_fn == nullptr))
        return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "alloc and free must both be set or both be NULL");
    HSLA_HIP(h, hipSetDevice(h->device));
    HSLA_HIP(h, hipDeviceSynchronize());
    for (int i = 0; i < hsla_handle::kGraphCache; ++i) {
        if (h->graph_exec[i]) (void)hipGraphExecDestroy(h->graph_exec[i]);
        h->graph_exec[i] = nullptr;
        h->graph_key[i] = 0;
    }
    hsla::dev_free(h, h->ws);
    hsla::dev_free(h, h->mp_ws);
    hsla::dev_free(h, h->pr_ws);
    h->ws = h->mp_ws = h->pr_ws = nullptr;
    h->ws_bytes = h->mp_ws_bytes = h->pr_ws_bytes = 0;
    h->mp_keep_B = 0;
    h->mp_keep_pattern = nullptr;
    h->alloc_fn = alloc;
    h->free_fn = free_fn;
    h->alloc_ctx = ctx;
    return HSLA_OK;
}

hsla_status hsla_reserve(hsla_handle *h, size_t bytes) {
    if (!h) return HSLA_ERR_INVALID_ARG;
    HSLA_HIP(h, hipSetDevice(h->device));
    return hsla::ensure_workspace(h, bytes);
}

hsla_status hsla_csr_check(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col, int32_t *bad_row) {
    if (bad_row) *bad_row = INT32_MAX;
    if (n < 0 || nnz < 0 || nnz >= INT32_MAX || !row_ptr || (nnz > 0 && !col)) return HSLA_ERR_INVALID_ARG;
    if (row_ptr[0] != 0 || (int64_t)row_ptr[n] != nnz) {
        if (bad_row) *bad_row = -1;
        return HSLA_ERR_INVALID_CSR;
    }
    int64_t lower = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t d = -1;
        if (!hsla::csr_row_ok(i, n, nnz, row_ptr, col, &d, &lower)) {
            if (bad_row) *bad_row = i;
            return HSLA_ERR_INVALID_CSR;
        }
    }
    return HSLA_OK;
}

hsla_status hsla_pattern_create(hsla_handle *h, int32_t n, int64_t nnz, const int32_t *d_row_ptr,
                                const int32_t *d_col, uint32_t flags, void *stream, hsla_pattern **out) {
    if (!h) return HSLA_ERR_INVALID_ARG;
    hsla_status st = hsla::enter(h, (hipStream_t)stream);
    if (st != HSLA_OK) return st;
    return hsla::make_pattern(h, n, nnz, d_row_ptr, d_col, flags, h->stream, out);
}

void hsla_pattern_destroy(hsla_pattern *p) {
    if (p) (void)hipSetDevice(p->device);
    hsla::free_pattern(p);
}

hsla_status hsla_pattern_info(const hsla_pattern *p, int32_t *n, int64_t *nnz, int64_t *nnz_lower,
                              int32_t *pattern_symmetric) {
    if (!p) return HSLA_ERR_INVALID_ARG;
    if (n) *n = p->n;
    if (nnz) *nnz = p->nnz;
    if (nnz_lower) *nnz_lower = p->nnz_lower;
    if (pattern_symmetric) *pattern_symmetric = p->pattern_symmetric;
    return HSLA_OK;
}

hsla_status hsla_pattern_set_format(hsla_pattern *p, int32_t format) {
    if (!p || (format != HSLA_FORMAT_AUTO && format != HSLA_FORMAT_CSR && format != HSLA_FORMAT_DIAGONAL))
        return HSLA_ERR_INVALID_ARG;
    p->format = format;
    return HSLA_OK;
}

hsla_status hsla_pattern_format(const hsla_pattern *p, int32_t *stencil_in_use, int32_t *num_offsets) {
    if (!p) return HSLA_ERR_INVALID_ARG;
    if (stencil_in_use) *stencil_in_use = p->use(p->stA).mask != nullptr ? 1 : 0;
    if (num_offsets) *num_offsets = p->stA.mask ? p->stA.nofs : 0;
    return HSLA_OK;
}

hsla_status hsla_pattern_signature(const hsla_pattern *p, uint64_t *signature) {
    if (!p || !signature) return HSLA_ERR_INVALID_ARG;
    *signature = p->signature;
    return HSLA_OK;
}

hsla_status hsla_pattern_get_tuning(const hsla_pattern *p, hsla_tune_state *out) {
    if (!p || !out) return HSLA_ERR_INVALID_ARG;
    *out = hsla_tune_state{p->signature, p->tuned, p->tune_dia, p->tune_dia_cu, p->tune_tile_cu, p->tune_sym,
                           p->tune_sym_cu};
    return HSLA_OK;
}

hsla_status hsla_pattern_set_tuning(hsla_pattern *p, const hsla_tune_state *in) {
    if (!p || !in || in->signature != p->signature) return HSLA_ERR_INVALID_ARG;
    auto cu_ok = [](int32_t v) { return v >= 1 && v <= 64; };
    if ((in->dia != 0 && in->dia != 1) || (in->sym != 0 && in->sym != 1) || !cu_ok(in->dia_cu) ||
        !cu_ok(in->tile_cu) || !cu_ok(in->sym_cu) || (in->tuned != 0 && in->tuned != 1))
        return HSLA_ERR_INVALID_ARG;
    p->tune_dia = in->dia;
    p->tune_dia_cu = in->dia_cu;
    p->tune_tile_cu = in->tile_cu;
    p->tune_sym = in->sym;
    p->tune_sym_cu = in->sym_cu;
    p->tuned = in->tuned;
    return HSLA_OK;
}

hsla_status hsla_pattern_lower(hsla_handle *h, const hsla_pattern *p, int32_t *d_row_ptr_L, int32_t *d_col_L,
                               int32_t *d_pos, void *stream) {
    if (!h || !p) return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "null handle or pattern");
    hsla_status st = hsla::enter(h, (hipStream_t)stream);
    if (st != HSLA_OK) return st;
    hipStream_t s = h->stream;
    if (d_row_ptr_L)
        HSLA_HIP(h, hipMemcpyAsync(d_row_ptr_L, p->rpL, sizeof(int32_t) * (p->n + 1), hipMemcpyDeviceToDevice, s));
    if (p->nnz_lower > 0) {
        if (d_col_L)
            HSLA_HIP(h, hipMemcpyAsync(d_col_L, p->colL, sizeof(int32_t) * p->nnz_lower, hipMemcpyDeviceToDevice, s));
        if (d_pos) HSLA_HIP(h, hipMemcpyAsync(d_pos, p->posL, sizeof(int32_t) * p->nnz_lower, hipMemcpyDeviceToDevice, s));
    }
    HSLA_HIP(h, hipStreamSynchronize(s));
    return HSLA_OK;
}

hsla_status hsla_pattern_colors(hsla_handle *h, const hsla_pattern *p, int32_t *d_color, int32_t *ncolors,
                                void *stream) {
    if (!h || !p || !ncolors) return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "null handle, pattern or output");
    hsla_status st = hsla::enter(h, (hipStream_t)stream);
    if (st != HSLA_OK) return st;
    hipStream_t s = h->stream;
    const int32_t n = p->n;
    const int64_t nnz = p->nnz;
    std::vector<int32_t> rp((size_t)n + 1), col(nnz > 0 ? (size_t)nnz : 1);
    HSLA_HIP(h, hipMemcpyAsync(rp.data(), p->row_ptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost, s));
    if (nnz > 0) HSLA_HIP(h, hipMemcpyAsync(col.data(), p->col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, s));
    HSLA_HIP(h, hipStreamSynchronize(s));
    // rows holding each column (counting sort)
    std::vector<int32_t> cp((size_t)n + 1, 0), rows(nnz > 0 ? (size_t)nnz : 1);
    for (int64_t k = 0; k < nnz; ++k) ++cp[col[k] + 1];
    for (int32_t j = 0; j < n; ++j) cp[j + 1] += cp[j];
    {
        std::vector<int32_t> next(cp.begin(), cp.end() - 1);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k) rows[next[col[k]]++] = i;
    }
    // greedy, columns in order: the smallest color no column sharing a row
    // with column j has taken (mark[c] == j: taken)
    std::vector<int32_t> color((size_t)n, -1), mark;
    int32_t nc = 0;
    for (int32_t j = 0; j < n; ++j) {
        for (int32_t t = cp[j]; t < cp[j + 1]; ++t) {
            const int32_t i = rows[t];
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
                const int32_t c = color[col[k]];
                if (c >= 0) mark[c] = j;
            }
        }
        int32_t c = 0;
        while (c < (int32_t)mark.size() && mark[c] == j) ++c;
        if (c == (int32_t)mark.size()) mark.push_back(-1);
        color[j] = c;
        if (c + 1 > nc) nc = c + 1;
    }
    *ncolors = nc;
    if (d_color && n > 0) {
        HSLA_HIP(h, hipMemcpyAsync(d_color, color.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
        HSLA_HIP(h, hipStreamSynchronize(s));
    }
    return HSLA_OK;
}

hsla_status hsla_pattern_transpose(hsla_handle *h, const hsla_pattern *p, int32_t *d_row_ptr_T, int32_t *d_col_T,
                                   int32_t *d_src, void *stream) {
    if (!h || !p) return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "null handle or pattern");
    hsla_status st = hsla::enter(h, (hipStream_t)stream);
    if (st != HSLA_OK) return st;
    hipStream_t s = h->stream;
    if (d_row_ptr_T)
        HSLA_HIP(h, hipMemcpyAsync(d_row_ptr_T, p->rpT, sizeof(int32_t) * (p->n + 1), hipMemcpyDeviceToDevice, s));
    if (p->nnz > 0) {
        if (d_col_T) HSLA_HIP(h, hipMemcpyAsync(d_col_T, p->colT, sizeof(int32_t) * p->nnz, hipMemcpyDeviceToDevice, s));
        if (d_src) HSLA_HIP(h, hipMemcpyAsync(d_src, p->srcT, sizeof(int32_t) * p->nnz, hipMemcpyDeviceToDevice, s));
    }
    HSLA_HIP(h, hipStreamSynchronize(s));
    return HSLA_OK;
}

}  // extern "C"
