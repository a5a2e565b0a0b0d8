// Persistent one-workgroup-per-system Jacobi-PCG: ragged batches (B systems
// with distinct sparsity patterns and sizes, the paper's list of matrices
// with distinct patterns, Sec. "Typed sparse-tensor hierarchy") and small
// systems that share one pattern, solved in a single launch.
//
// Ragged layout (all device memory, caller-owned): system s owns rows
// [row_off[s], row_off[s+1]) of the concatenated vectors b and x and entries
// [nnz_off[s], nnz_off[s+1]) of the concatenated col/values; its local
// row pointer (n_s + 1 entries, starting at 0) starts at row_ptr[row_off[s]
// + s]; column indices are local (0 <= col < n_s).  Shared layout: one
// pattern, values [B][nnz], vectors [B][n].
//
// Each workgroup pops systems from an atomic queue (ragged: longest first by
// stored entries) and runs the whole recurrence of one system with
// workgroup-level reductions; the queue gives every workgroup an exit once
// B systems have been handed out, and max_iter bounds every solve.  The
// SpMV streams each 64-row block's entries in coalesced chunks staged in LDS
// and adds each row's products in ascending column order, as the sequential
// definition does.  A system's reductions use a fixed thread count and
// order, so its result does not depend on which workgroup solved it.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "common.h"

namespace hsla {
namespace rg {

constexpr int kRB = 1024;  // threads per workgroup of the general kernel
constexpr int kRW = kRB / kWave;
constexpr int kSB = 1024;  // threads per workgroup of the small-system kernel
constexpr int kSW = kSB / kWave;
constexpr int kChunk = 256;  // entries staged per wave and step

struct RInfo {  // per-system result record (device)
    int64_t iters;
    int32_t status;
    int32_t pad;
    double rel_residual, true_residual;
    uint64_t t_begin, t_end;  // persistent kernels: device wall clock when the system was taken and finished
};

struct Args {
    int32_t B;
    int64_t shared_n, shared_nnz;  // >= 0: one shared pattern (row_off/nnz_off unused)
    const int64_t *row_off, *nnz_off;
    const int32_t *rp, *col;
    const double *val, *b;
    double *x;
    double *r, *p, *q, *dinv;  // work vectors, concatenated like b
    double *u, *w;             // single-reduction kernel: M^{-1} r and A u
    const int32_t *order;      // systems in queue order (nullptr: 0..B-1)
    int32_t *queue;            // next queue slot
    int32_t *bad;              // first invalid system (validation)
    RInfo *info;
    double rtol, atol;
    int64_t max_iter;
    int jacobi;
};

// Workgroup (NW waves) sum of NV values in a fixed order; result in every
// thread.
// TAIL = false leaves out the closing barrier: the caller then guarantees
// that `sh` is not written again before every wave has passed another
// barrier (e.g. by alternating buffers between consecutive sums).
template <int NW, int NV, bool TAIL = true>
__device__ __forceinline__ void wg_sum(double (&v)[NV], double *sh) {
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = wave_sum(v[j]);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) sh[j * NW + w] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double s = 0.0;
#pragma unroll 4
        for (int q = 0; q < NW; ++q) s += sh[j * NW + q];
        v[j] = s;
    }
    if (TAIL) __syncthreads();
}

// y = A v for one system, by the whole workgroup (NW waves): wave w takes
// the 64-row blocks w, w + NW, ...; a block's entries are loaded in
// coalesced chunks of kChunk, their products staged in the wave's LDS slice,
// and each lane adds the products of its row in ascending order.  The next
// block's row pointers, and the next chunk's values and column indices, are
// loaded while the current block or chunk is processed.
// epi(i, y_i) runs on the lane that owns row i.  NT: the values and column
// indices are read with nontemporal loads (a pass over a whole batch that
// the caches cannot hold; the persistent kernels, which re-read one system's
// matrix every iteration, keep the default policy).
template <int NW, class Epi, bool NT = false>
__device__ __forceinline__ void wg_spmv(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                        const double *__restrict__ val, const double *__restrict__ v, double *lds,
                                        Epi &&epi) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    double *L = lds + w * kChunk;
    int32_t r0 = w * kWave;
    int32_t e0 = 0, e1 = 0, ka = 0, kb = 0;
    auto fetch = [&](int32_t b0, int32_t &f0, int32_t &f1, int32_t &fa, int32_t &fb) {
        const int32_t row = b0 + lane;
        const int32_t rend = b0 + kWave < n ? b0 + kWave : n;
        f0 = rp[b0];
        f1 = rp[rend];
        fa = row < n ? rp[row] : 0;
        fb = row < n ? rp[row + 1] : 0;
        if (row >= n) fa = fb = f1;
    };
    if (r0 < n) fetch(r0, e0, e1, ka, kb);
    constexpr int U = kChunk / kWave;
    // entries of the chunk to process next; each step loads the following
    // chunk's values and column indices (the next block's first chunk after
    // a block's last) before it gathers and stages this one
    double vv[U];
    int32_t cv[U];
    bool have = false;  // vv, cv hold the current block's first chunk
    for (; r0 < n; r0 += NW * kWave) {
        const int32_t rn = r0 + NW * kWave;
        int32_t n0 = 0, n1 = 0, na = 0, nb = 0;
        if (rn < n) fetch(rn, n0, n1, na, nb);
        const int32_t row = r0 + lane;
        double acc = 0.0;
        if (!have) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t e = e0 + u * kWave + lane;
                vv[u] = e < e1 ? (NT ? __builtin_nontemporal_load(&val[e]) : val[e]) : 0.0;
                cv[u] = e < e1 ? (NT ? __builtin_nontemporal_load(&col[e]) : col[e]) : 0;
            }
        }
        have = false;
        for (int32_t c0 = e0; c0 < e1; c0 += kChunk) {
            const int32_t cnt = e1 - c0 < kChunk ? e1 - c0 : kChunk;
            double xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) xv[u] = u * kWave + lane < cnt ? v[cv[u]] : 0.0;
            const bool last = c0 + kChunk >= e1;
            const int32_t ns = last ? n0 : c0 + kChunk, ne = last ? n1 : e1;
            have = last;
            double nv[U];
            int32_t nc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t e = ns + u * kWave + lane;
                nv[u] = e < ne ? (NT ? __builtin_nontemporal_load(&val[e]) : val[e]) : 0.0;
                nc[u] = e < ne ? (NT ? __builtin_nontemporal_load(&col[e]) : col[e]) : 0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t e = u * kWave + lane;
                if (e < cnt) L[e] = vv[u] * xv[u];
                vv[u] = nv[u];
                cv[u] = nc[u];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int32_t lo = ka > c0 ? ka : c0;
            const int32_t hi = kb < c0 + cnt ? kb : c0 + cnt;
            for (int32_t k = lo; k < hi; ++k) acc += L[k - c0];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (row < n) epi(row, acc);
        e0 = n0;
        e1 = n1;
        ka = na;
        kb = nb;
    }
}

// Canonical-CSR check of every system's local pattern; reads a row only
// after its bounds are known to lie inside the system's entries.
__global__ __launch_bounds__(256) void k_ragged_validate(Args a) {
    for (int64_t s = blockIdx.x; s < a.B; s += gridDim.x) {
        const int64_t r0 = a.row_off[s], r1 = a.row_off[s + 1];
        const int64_t k0 = a.nnz_off[s], k1 = a.nnz_off[s + 1];
        const int64_t n = r1 - r0, nnz = k1 - k0;
        if (n < 0 || nnz < 0 || n >= INT32_MAX) {
            if (threadIdx.x == 0) atomicMin(a.bad, (int32_t)s);
            continue;
        }
        const int32_t *rp = a.rp + r0 + s;
        const int32_t *col = a.col + k0;
        bool ok = true;
        if (threadIdx.x == 0) ok = rp[0] == 0 && (int64_t)rp[n] == nnz;
        for (int64_t i = threadIdx.x; i < n && ok; i += blockDim.x) {
            const int32_t lo = rp[i], hi = rp[i + 1];
            if (lo < 0 || lo > hi || (int64_t)hi > nnz) {
                ok = false;
                break;
            }
            int32_t prev = -1;
            for (int32_t k = lo; k < hi; ++k) {
                const int32_t c = col[k];
                if (c < 0 || (int64_t)c >= n || c <= prev) {
                    ok = false;
                    break;
                }
                prev = c;
            }
        }
        if (!ok) atomicMin(a.bad, (int32_t)s);
    }
}

__global__ __launch_bounds__(kRB) void k_ragged_pcg(Args a) {
    __shared__ double sh[3 * kRW];
    __shared__ double lds[kRW * kChunk];
    __shared__ int32_t slot;
    for (;;) {
        if (threadIdx.x == 0) slot = atomicAdd(a.queue, 1);
        __syncthreads();
        const int32_t qs = slot;
        __syncthreads();
        if (qs >= a.B) return;
        const uint64_t t_begin = threadIdx.x == 0 ? wall_clock64() : 0;
        const int32_t s = a.order ? a.order[qs] : qs;
        const bool shared = a.shared_n >= 0;
        const int64_t r0 = shared ? (int64_t)s * a.shared_n : a.row_off[s];
        const int32_t n = (int32_t)(shared ? a.shared_n : a.row_off[s + 1] - r0);
        const int64_t k0 = shared ? (int64_t)s * a.shared_nnz : a.nnz_off[s];
        const int32_t *rp = shared ? a.rp : a.rp + r0 + s;
        const int32_t *col = shared ? a.col : a.col + k0;
        const double *__restrict__ val = a.val + k0;
        const double *__restrict__ b = a.b + r0;
        double *__restrict__ x = a.x + r0;
        double *__restrict__ r = a.r + r0;
        double *__restrict__ p = a.p + r0;
        double *__restrict__ q = a.q + r0;
        double *__restrict__ dinv = a.dinv + r0;
        // set-up: x = 0, r = b, z = D^{-1} r, p = z
        double acc3[3] = {0.0, 0.0, 0.0};
        int bad_diag = 0, neg_diag = 0;
        for (int32_t i = threadIdx.x; i < n; i += kRB) {
            double d = 0.0;
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
                if (col[k] == i) d = val[k];
            if (a.jacobi && d == 0.0) bad_diag = 1;
            if (a.jacobi && d < 0.0) neg_diag = 1;
            const double di = a.jacobi ? 1.0 / d : 1.0;
            const double bi = b[i];
            dinv[i] = di;
            x[i] = 0.0;
            r[i] = bi;
            p[i] = di * bi;
            acc3[0] += bi * bi;
            acc3[1] += bi * bi;
            acc3[2] += bi * (di * bi);
        }
        double bd[2] = {(double)bad_diag, (double)neg_diag};
        wg_sum<kRW, 2>(bd, sh);
        wg_sum<kRW, 3>(acc3, sh);
        const double bn = sqrt(acc3[0]);
        double tol = a.rtol * bn;
        if (a.atol > tol) tol = a.atol;
        double rho = acc3[2], rr = acc3[1];
        int32_t status = HSLA_NOT_CONVERGED;
        int64_t it = 0;
        if (bd[0] > 0.0) {
            status = HSLA_ERR_ZERO_DIAGONAL;
        } else if (!isfinite(bn)) {
            status = HSLA_ERR_NONFINITE;
        } else if (sqrt(rr) <= tol) {
            status = HSLA_OK;
        } else if (bd[1] > 0.0) {
            status = HSLA_BREAKDOWN;  // negative Jacobi diagonal: x stays 0
        } else {
            while (it < a.max_iter) {
                // q = A p, sigma = p.q (each row summed in ascending order)
                double acc1[1] = {0.0};
                wg_spmv<kRW>(n, rp, col, val, p, lds, [&](int32_t i, double sum) {
                    q[i] = sum;
                    acc1[0] += p[i] * sum;
                });
                wg_sum<kRW, 1>(acc1, sh);
                const double sigma = acc1[0];
                if (!isfinite(sigma)) { status = HSLA_ERR_NONFINITE; break; }
                if (!(sigma > 0.0)) { status = HSLA_BREAKDOWN; break; }
                const double alpha = rho / sigma;
                double acc2[2] = {0.0, 0.0};
                for (int32_t i0 = threadIdx.x; i0 < n; i0 += 2 * kRB) {
                    double xv[2], pv[2], rv[2], qv[2], dv[2];
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int32_t i = i0 + u * kRB;
                        if (i < n) {
                            xv[u] = x[i];
                            pv[u] = p[i];
                            rv[u] = r[i];
                            qv[u] = q[i];
                            dv[u] = dinv[i];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int32_t i = i0 + u * kRB;
                        if (i < n) {
                            x[i] = xv[u] + alpha * pv[u];
                            const double ri = rv[u] - alpha * qv[u];
                            r[i] = ri;
                            acc2[0] += ri * ri;
                            acc2[1] += ri * (dv[u] * ri);
                        }
                    }
                }
                wg_sum<kRW, 2>(acc2, sh);
                ++it;
                rr = acc2[0];
                const double rn = sqrt(rr);
                if (!isfinite(rn)) { status = HSLA_ERR_NONFINITE; break; }
                if (rn <= tol) { status = HSLA_OK; break; }
                const double beta = acc2[1] / rho;
                rho = acc2[1];
                for (int32_t i0 = threadIdx.x; i0 < n; i0 += 4 * kRB) {
                    double dv[4], rv[4], pv[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int32_t i = i0 + u * kRB;
                        if (i < n) {
                            dv[u] = dinv[i];
                            rv[u] = r[i];
                            pv[u] = p[i];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int32_t i = i0 + u * kRB;
                        if (i < n) p[i] = dv[u] * rv[u] + beta * pv[u];
                    }
                }
                __syncthreads();
            }
        }
        // true residual ||b - A x||
        double accr[2] = {0.0, 0.0};
        __syncthreads();
        wg_spmv<kRW>(n, rp, col, val, x, lds, [&](int32_t i, double sum) {
            const double e = b[i] - sum;
            accr[0] += e * e;
            accr[1] += b[i] * b[i];
        });
        wg_sum<kRW, 2>(accr, sh);
        if (threadIdx.x == 0) {
            RInfo f;
            f.iters = it;
            f.status = n == 0 ? HSLA_OK : status;
            f.pad = 0;
            f.rel_residual = bn > 0 ? sqrt(rr) / bn : sqrt(rr);
            f.true_residual = accr[1] > 0 ? sqrt(accr[0]) / sqrt(accr[1]) : sqrt(accr[0]);
            f.t_begin = t_begin;
            f.t_end = wall_clock64();
            a.info[s] = f;
        }
        __syncthreads();
    }
}

// The same persistent launch with the single-reduction recurrence of
// Chronopoulos and Gear (preconditioned: u = M^{-1} r, w = A u,
// gamma = r.u, delta = w.u; beta = gamma / gamma_old,
// alpha = gamma / (delta - beta gamma / alpha_old); p = u + beta p,
// s = w + beta s, x += alpha p, r -= alpha s): per iteration one pass with
// the SpMV and one workgroup reduction of gamma, delta and the previous
// sweep's ||r||^2 (the stop test), then one vector pass -- against three
// passes and two reductions in k_ragged_pcg.  `q` holds s.
__global__ __launch_bounds__(kRB) void k_ragged_pcg_sr(Args a) {
    __shared__ double sh[3 * kRW];
    __shared__ double lds[kRW * kChunk];
    __shared__ int32_t slot;
    for (;;) {
        if (threadIdx.x == 0) slot = atomicAdd(a.queue, 1);
        __syncthreads();
        const int32_t qs = slot;
        __syncthreads();
        if (qs >= a.B) return;
        const uint64_t t_begin = threadIdx.x == 0 ? wall_clock64() : 0;
        const int32_t s = a.order ? a.order[qs] : qs;
        const bool shared = a.shared_n >= 0;
        const int64_t r0 = shared ? (int64_t)s * a.shared_n : a.row_off[s];
        const int32_t n = (int32_t)(shared ? a.shared_n : a.row_off[s + 1] - r0);
        const int64_t k0 = shared ? (int64_t)s * a.shared_nnz : a.nnz_off[s];
        const int32_t *rp = shared ? a.rp : a.rp + r0 + s;
        const int32_t *col = shared ? a.col : a.col + k0;
        const double *__restrict__ val = a.val + k0;
        const double *__restrict__ b = a.b + r0;
        double *__restrict__ x = a.x + r0;
        double *__restrict__ r = a.r + r0;
        double *__restrict__ p = a.p + r0;
        double *__restrict__ sv = a.q + r0;
        double *__restrict__ u = a.u + r0;
        double *__restrict__ w = a.w + r0;
        double *__restrict__ dinv = a.dinv + r0;
        // set-up: x = 0, r = b, u = D^{-1} r
        double acc1[1] = {0.0};
        int bad_diag = 0, neg_diag = 0;
        for (int32_t i = threadIdx.x; i < n; i += kRB) {
            double d = 0.0;
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
                if (col[k] == i) d = val[k];
            if (a.jacobi && d == 0.0) bad_diag = 1;
            if (a.jacobi && d < 0.0) neg_diag = 1;
            const double di = a.jacobi ? 1.0 / d : 1.0;
            const double bi = b[i];
            dinv[i] = di;
            x[i] = 0.0;
            r[i] = bi;
            u[i] = di * bi;
            acc1[0] += bi * bi;
        }
        double bd[2] = {(double)bad_diag, (double)neg_diag};
        wg_sum<kRW, 2>(bd, sh);
        wg_sum<kRW, 1>(acc1, sh);
        const double bn = sqrt(acc1[0]);
        double tol = a.rtol * bn;
        if (a.atol > tol) tol = a.atol;
        double rr = acc1[0];
        int32_t status = HSLA_NOT_CONVERGED;
        int64_t it = 0;
        if (bd[0] > 0.0) {
            status = HSLA_ERR_ZERO_DIAGONAL;
        } else if (!isfinite(bn)) {
            status = HSLA_ERR_NONFINITE;
        } else if (sqrt(rr) <= tol) {
            status = HSLA_OK;
        } else if (bd[1] > 0.0) {
            status = HSLA_BREAKDOWN;  // negative Jacobi diagonal: x stays 0
        } else if (a.max_iter > 0) {
            double gamma_old = 1.0, alpha_old = 1.0;
            for (;;) {
                __syncthreads();  // u of the last sweep complete
                // w = A u with gamma = r.u, delta = w.u, and ||r||^2 of the last sweep
                double acc3[3] = {0.0, 0.0, 0.0};
                wg_spmv<kRW>(n, rp, col, val, u, lds, [&](int32_t i, double sum) {
                    const double ri = r[i], ui = u[i];
                    w[i] = sum;
                    acc3[0] += ri * ui;
                    acc3[1] += sum * ui;
                    acc3[2] += ri * ri;
                });
                wg_sum<kRW, 3>(acc3, sh);
                if (it > 0) {
                    rr = acc3[2];
                    const double rn = sqrt(rr);
                    if (!isfinite(rn)) { status = HSLA_ERR_NONFINITE; break; }
                    if (rn <= tol) { status = HSLA_OK; break; }
                    if (it >= a.max_iter) break;
                }
                const double gamma = acc3[0], delta = acc3[1];
                const double beta = it > 0 ? gamma / gamma_old : 0.0;
                const double sigma = it > 0 ? delta - beta * gamma / alpha_old : delta;
                if (!isfinite(sigma) || !isfinite(gamma)) { status = HSLA_ERR_NONFINITE; break; }
                if (!(sigma > 0.0)) { status = HSLA_BREAKDOWN; break; }
                const double alpha = gamma / sigma;
                const bool first = it == 0;
                for (int32_t i0 = threadIdx.x; i0 < n; i0 += 2 * kRB) {
                    double xv[2], pv[2], sq[2], rv[2], uv[2], wv[2], dv[2];
#pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        const int32_t i = i0 + k * kRB;
                        if (i < n) {
                            xv[k] = x[i];
                            pv[k] = first ? 0.0 : p[i];
                            sq[k] = first ? 0.0 : sv[i];
                            rv[k] = r[i];
                            uv[k] = u[i];
                            wv[k] = w[i];
                            dv[k] = dinv[i];
                        }
                    }
#pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        const int32_t i = i0 + k * kRB;
                        if (i < n) {
                            const double pn = uv[k] + beta * pv[k];
                            const double sn = wv[k] + beta * sq[k];
                            const double rn = rv[k] - alpha * sn;
                            p[i] = pn;
                            sv[i] = sn;
                            x[i] = xv[k] + alpha * pn;
                            r[i] = rn;
                            u[i] = dv[k] * rn;
                        }
                    }
                }
                gamma_old = gamma;
                alpha_old = alpha;
                ++it;
            }
        }
        // true residual ||b - A x||
        double accr[2] = {0.0, 0.0};
        __syncthreads();
        wg_spmv<kRW>(n, rp, col, val, x, lds, [&](int32_t i, double sum) {
            const double e = b[i] - sum;
            accr[0] += e * e;
            accr[1] += b[i] * b[i];
        });
        wg_sum<kRW, 2>(accr, sh);
        if (threadIdx.x == 0) {
            RInfo f;
            f.iters = it;
            f.status = n == 0 ? HSLA_OK : status;
            f.pad = 0;
            f.rel_residual = bn > 0 ? sqrt(rr) / bn : sqrt(rr);
            f.true_residual = accr[1] > 0 ? sqrt(accr[0]) / sqrt(accr[1]) : sqrt(accr[0]);
            f.t_begin = t_begin;
            f.t_end = wall_clock64();
            a.info[s] = f;
        }
        __syncthreads();
    }
}

// Small systems (n <= kSmallMaxN rows of at most K entries, one shared
// pattern): one workgroup per system keeps the whole recurrence on chip.
// Thread t owns rows t, t + kSB, ... (R of them): their x, r, D^-1, q and p
// live in registers, p is mirrored in LDS for the SpMV gathers, and the
// matrix rows are re-read from L2 every iteration as R x K independent
// loads.  Each row adds its products in ascending column order, products
// rounded before the add.
constexpr int kSmallMaxN = 4096;
constexpr int kSmallMaxRow = 16;

template <int K>
__device__ __forceinline__ double small_row(int32_t lo, int32_t len, const int32_t *__restrict__ col,
                                            const double *__restrict__ val, const double *v) {
#pragma clang fp contract(off)
    const double *__restrict__ vr = val + lo;
    const int32_t *__restrict__ cr = col + lo;
    double vv[K];
    int32_t cc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        vv[k] = 0.0;
        cc[k] = 0;
        if (k < len) {
            vv[k] = vr[k];
            cc[k] = cr[k];
        }
    }
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (k < len) {
            const double prd = vv[k] * v[cc[k]];
            sum = sum + prd;
        }
    return sum;
}

// SR: the single-reduction recurrence of Chronopoulos and Gear (1989) --
// the same iterates as Algorithm "Distributed CG" in exact arithmetic, with
// s = A p carried as a vector so that r.u, (A u).u and r.r of an iteration
// are one workgroup reduction (three barriers per iteration instead of
// five).  Breakdown when the step's curvature delta - beta gamma / alpha is
// not positive.
template <int R, int K, bool SR>
__global__ __launch_bounds__(kSB) void k_small_pcg(Args a) {
    __shared__ double ps[kSmallMaxN];
    __shared__ double sh[3 * kSW];
    __shared__ int32_t slot;
    const int32_t n = (int32_t)a.shared_n;
    const int32_t *rp = a.rp, *col = a.col;
    for (;;) {
        if (threadIdx.x == 0) slot = atomicAdd(a.queue, 1);
        __syncthreads();
        const int32_t s = slot;
        __syncthreads();
        if (s >= a.B) return;
        const uint64_t t_begin = threadIdx.x == 0 ? wall_clock64() : 0;
        const double *val = a.val + (int64_t)s * a.shared_nnz;
        const double *b = a.b + (int64_t)s * n;
        double *x = a.x + (int64_t)s * n;
        int32_t lo[R], len[R];
        double xr[R], rv[R], dv[R], pv[R], qv[R];
        double acc3[3] = {0.0, 0.0, 0.0};
        int bad_diag = 0, neg_diag = 0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int32_t i = threadIdx.x + j * kSB;
            lo[j] = 0;
            len[j] = 0;
            xr[j] = rv[j] = pv[j] = qv[j] = 0.0;
            dv[j] = 1.0;
            if (i < n) {
                lo[j] = rp[i];
                len[j] = rp[i + 1] - lo[j];
                double d = 0.0;
                for (int32_t k = 0; k < len[j]; ++k)
                    if (col[lo[j] + k] == i) d = val[lo[j] + k];
                if (a.jacobi && d == 0.0) bad_diag = 1;
                if (a.jacobi && d < 0.0) neg_diag = 1;
                const double di = a.jacobi ? 1.0 / d : 1.0;
                const double bi = b[i];
                dv[j] = di;
                rv[j] = bi;
                pv[j] = di * bi;
                ps[i] = pv[j];
                acc3[0] += bi * bi;
                acc3[1] += bi * bi;
                acc3[2] += bi * (di * bi);
            }
        }
        double bd[2] = {(double)bad_diag, (double)neg_diag};
        wg_sum<kSW, 2>(bd, sh);
        wg_sum<kSW, 3>(acc3, sh);
        const double bn = sqrt(acc3[0]);
        double tol = a.rtol * bn;
        if (a.atol > tol) tol = a.atol;
        double rho = acc3[2], rr = acc3[1];
        int32_t status = HSLA_NOT_CONVERGED;
        int64_t it = 0;
        if (bd[0] > 0.0) {
            status = HSLA_ERR_ZERO_DIAGONAL;
        } else if (!isfinite(bn)) {
            status = HSLA_ERR_NONFINITE;
        } else if (sqrt(rr) <= tol) {
            status = HSLA_OK;
        } else if (bd[1] > 0.0) {
            status = HSLA_BREAKDOWN;  // negative Jacobi diagonal: x stays 0
        } else if (SR) {
            // u = D^{-1} r is p at the start (in LDS); w = A u, s = w
            double gamma = rho, alpha = 0.0;
            {
                double d1[1] = {0.0};
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    qv[j] = small_row<K>(lo[j], len[j], col, val, ps);  // s = w = A u
                    d1[0] += qv[j] * pv[j];
                    if (j % 2 == 1) __builtin_amdgcn_sched_barrier(0);
                }
                wg_sum<kSW, 1>(d1, sh);
                if (!isfinite(d1[0])) {
                    status = HSLA_ERR_NONFINITE;
                } else if (!(d1[0] > 0.0)) {
                    status = HSLA_BREAKDOWN;
                } else {
                    alpha = gamma / d1[0];
                }
            }
            while (status == HSLA_NOT_CONVERGED && it < a.max_iter) {
                // x += alpha p, r -= alpha s, u = D^{-1} r (to LDS)
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int32_t i = threadIdx.x + j * kSB;
                    xr[j] = xr[j] + alpha * pv[j];
                    rv[j] = rv[j] - alpha * qv[j];
                    if (i < n) ps[i] = dv[j] * rv[j];
                }
                ++it;
                __syncthreads();
                // w = A u; r.u, w.u, r.r in one reduction
                double w[R];
                double d3[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    w[j] = small_row<K>(lo[j], len[j], col, val, ps);
                    const double u = dv[j] * rv[j];
                    d3[0] += rv[j] * u;
                    d3[1] += w[j] * u;
                    d3[2] += rv[j] * rv[j];
                    if (j % 2 == 1) __builtin_amdgcn_sched_barrier(0);
                }
                wg_sum<kSW, 3>(d3, sh);
                rr = d3[2];
                const double rn = sqrt(rr);
                if (!isfinite(rn) || !isfinite(d3[0]) || !isfinite(d3[1])) { status = HSLA_ERR_NONFINITE; break; }
                if (rn <= tol) { status = HSLA_OK; break; }
                const double beta = d3[0] / gamma;
                const double curv = d3[1] - beta * d3[0] / alpha;
                if (!(curv > 0.0)) { status = HSLA_BREAKDOWN; break; }
                alpha = d3[0] / curv;
                gamma = d3[0];
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    pv[j] = dv[j] * rv[j] + beta * pv[j];
                    qv[j] = w[j] + beta * qv[j];
                }
            }
        } else {
            while (it < a.max_iter) {
                // q = A p from the LDS copy of p (visible after the barriers
                // of the last reduction), sigma = p.q
                // rows in pairs, so at most 2 K loads are in flight per thread
                double acc1[1] = {0.0};
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    qv[j] = small_row<K>(lo[j], len[j], col, val, ps);
                    acc1[0] += pv[j] * qv[j];
                    if (j % 2 == 1) __builtin_amdgcn_sched_barrier(0);
                }
                wg_sum<kSW, 1>(acc1, sh);
                const double sigma = acc1[0];
                if (!isfinite(sigma)) { status = HSLA_ERR_NONFINITE; break; }
                if (!(sigma > 0.0)) { status = HSLA_BREAKDOWN; break; }
                const double alpha = rho / sigma;
                double acc2[2] = {0.0, 0.0};
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    xr[j] = xr[j] + alpha * pv[j];
                    rv[j] = rv[j] - alpha * qv[j];
                    acc2[0] += rv[j] * rv[j];
                    acc2[1] += rv[j] * (dv[j] * rv[j]);
                }
                wg_sum<kSW, 2>(acc2, sh);
                ++it;
                rr = acc2[0];
                const double rn = sqrt(rr);
                if (!isfinite(rn)) { status = HSLA_ERR_NONFINITE; break; }
                if (rn <= tol) { status = HSLA_OK; break; }
                const double beta = acc2[1] / rho;
                rho = acc2[1];
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int32_t i = threadIdx.x + j * kSB;
                    pv[j] = dv[j] * rv[j] + beta * pv[j];
                    if (i < n) ps[i] = pv[j];
                }
                __syncthreads();
            }
        }
        // x out, and the true residual ||b - A x|| from an LDS copy of x
        __syncthreads();
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int32_t i = threadIdx.x + j * kSB;
            if (i < n) {
                x[i] = xr[j];
                ps[i] = xr[j];
            }
        }
        __syncthreads();
        double accr[2] = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int32_t i = threadIdx.x + j * kSB;
            if (i < n) {
                const double bi = b[i];
                const double e = bi - small_row<K>(lo[j], len[j], col, val, ps);
                accr[0] += e * e;
                accr[1] += bi * bi;
            }
            if (j % 2 == 1) __builtin_amdgcn_sched_barrier(0);
        }
        wg_sum<kSW, 2>(accr, sh);
        if (threadIdx.x == 0) {
            RInfo f;
            f.iters = it;
            f.status = status;
            f.pad = 0;
            f.rel_residual = bn > 0 ? sqrt(rr) / bn : sqrt(rr);
            f.true_residual = accr[1] > 0 ? sqrt(accr[0]) / sqrt(accr[1]) : sqrt(accr[0]);
            f.t_begin = t_begin;
            f.t_end = wall_clock64();
            a.info[s] = f;
        }
        __syncthreads();
    }
}

// Small systems with short rows (at most K = 5 entries, or K = 8 with
// n <= 2048): the same recurrence as k_small_pcg (plain CG or Jacobi-PCG,
// Algorithm "Distributed CG" on one workgroup) with the matrix itself held in
// registers.  512 threads; thread t owns rows t + 512 j (R of them) and
// keeps their columns (as LDS byte offsets, two 16-bit offsets per
// register, loaded once per launch: the pattern is shared) and the current
// system's values (loaded once per system), so an iteration reads nothing
// but the LDS copy of p.  Each row adds its products in ascending column
// order, products rounded before the add; the K - len slots past a row's
// entries hold value 0 at offset 0, and their products (0 times a finite
// p) leave the sum as it is, so the row loop has no branches.
constexpr int kRT = 512;
constexpr int kRTW = kRT / kWave;
static_assert(kSmallMaxN * 8 <= 65536, "column byte offsets are packed in 16 bits");

template <int K>
__device__ __forceinline__ double reg_row(const double (&vv)[K], const uint32_t (&cc)[(K + 1) / 2],
                                          const double *v) {
#pragma clang fp contract(off)
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t off = (k & 1) ? cc[k / 2] >> 16 : cc[k / 2] & 0xffffu;
        const double prd = vv[k] * *(const double *)((const char *)v + off);
        sum = sum + prd;
    }
    return sum;
}

// SR: the single-reduction recurrence (as in k_small_pcg): s = A p is kept
// in registers, r.u, (A u).u and r.r are one workgroup sum, and an iteration
// has two barriers instead of three.
template <int R, int K, bool SR>
__global__ __launch_bounds__(kRT) void k_small_reg(Args a) {
    __shared__ double ps[kSmallMaxN];
    __shared__ double xs[kSmallMaxN];  // x of the thread's own rows (keeps registers for the matrix)
    static_assert(!SR || R <= 4, "the single-reduction recurrence keeps s in registers: at most 4 rows");
    __shared__ double sh[2][3 * kRTW];
    __shared__ int32_t slot;
    const int32_t n = (int32_t)a.shared_n;
    // this thread's rows of the shared pattern
    // (row starts are re-read per system and the diagonal found in cc, so
    // only the lengths and the packed columns stay in registers)
    int32_t len[R];
    uint32_t cc[R][(K + 1) / 2];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int32_t i = threadIdx.x + j * kRT;
        len[j] = 0;
#pragma unroll
        for (int u = 0; u < (K + 1) / 2; ++u) cc[j][u] = 0u;
        if (i < n) {
            const int32_t lo = a.rp[i];
            len[j] = a.rp[i + 1] - lo;
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (k < len[j]) cc[j][k / 2] |= (uint32_t)a.col[lo + k] * 8u << (16 * (k & 1));
        }
    }
    for (;;) {
        if (threadIdx.x == 0) slot = atomicAdd(a.queue, 1);
        __syncthreads();
        const int32_t s = slot;
        __syncthreads();
        if (s >= a.B) return;
        const uint64_t t_begin = threadIdx.x == 0 ? wall_clock64() : 0;
        const double *val = a.val + (int64_t)s * a.shared_nnz;
        const double *b = a.b + (int64_t)s * n;
        double *x = a.x + (int64_t)s * n;
        double vv[R][K];
        double rv[R], dv[R], pv[R], qv[R];
        double acc3[3] = {0.0, 0.0, 0.0};
        int bad_diag = 0, neg_diag = 0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int32_t i = threadIdx.x + j * kRT;
            const int32_t lo = i < n ? a.rp[i] : 0;
#pragma unroll
            for (int k = 0; k < K; ++k) vv[j][k] = k < len[j] ? val[lo + k] : 0.0;
            rv[j] = pv[j] = qv[j] = 0.0;
            dv[j] = 1.0;
            if (i < n) {
                xs[i] = 0.0;
                double d = 0.0;
#pragma unroll
                for (int k = 0; k < K; ++k)
                    if (k < len[j] && (int32_t)((cc[j][k / 2] >> (16 * (k & 1))) & 0xffffu) == 8 * i) d = vv[j][k];
                if (a.jacobi && d == 0.0) bad_diag = 1;
                if (a.jacobi && d < 0.0) neg_diag = 1;
                const double di = a.jacobi ? 1.0 / d : 1.0;
                const double bi = b[i];
                dv[j] = di;
                rv[j] = bi;
                pv[j] = di * bi;
                ps[i] = pv[j];
                acc3[0] += bi * bi;
                acc3[1] += bi * bi;
                acc3[2] += bi * (di * bi);
            }
        }
        double bd[2] = {(double)bad_diag, (double)neg_diag};
        wg_sum<kRTW, 2>(bd, sh[0]);
        wg_sum<kRTW, 3>(acc3, sh[0]);
        const double bn = sqrt(acc3[0]);
        double tol = a.rtol * bn;
        if (a.atol > tol) tol = a.atol;
        double rho = acc3[2], rr = acc3[1];
        int32_t status = HSLA_NOT_CONVERGED;
        int64_t it = 0;
        if (bd[0] > 0.0) {
            status = HSLA_ERR_ZERO_DIAGONAL;
        } else if (!isfinite(bn)) {
            status = HSLA_ERR_NONFINITE;
        } else if (sqrt(rr) <= tol) {
            status = HSLA_OK;
        } else if (bd[1] > 0.0) {
            status = HSLA_BREAKDOWN;  // negative Jacobi diagonal: x stays 0
        } else if (SR) {
            // u = D^{-1} r is p at the start (in LDS); w = A u, s = w
            double gamma = rho, alpha = 0.0;
            {
                double d1[1] = {0.0};
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int32_t i = threadIdx.x + j * kRT;
                    const double wj = reg_row<K>(vv[j], cc[j], ps);
                    qv[j] = wj;
                    d1[0] += wj * pv[j];
                }
                wg_sum<kRTW, 1>(d1, sh[0]);
                if (!isfinite(d1[0])) {
                    status = HSLA_ERR_NONFINITE;
                } else if (!(d1[0] > 0.0)) {
                    status = HSLA_BREAKDOWN;
                } else {
                    alpha = gamma / d1[0];
                }
            }
            while (status == HSLA_NOT_CONVERGED && it < a.max_iter) {
                // x += alpha p, r -= alpha s, u = D^{-1} r (to LDS)
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int32_t i = threadIdx.x + j * kRT;
                    rv[j] = rv[j] - alpha * qv[j];
                    if (i < n) {
                        xs[i] = xs[i] + alpha * pv[j];
                        ps[i] = dv[j] * rv[j];
                    }
                }
                ++it;
                __syncthreads();
                // w = A u; r.u, w.u, r.r in one sum (the barrier before the
                // next update separates consecutive sums: no closing barrier)
                double w[R];
                double d3[3] = {0.0, 0.0, 0.0};
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int32_t i = threadIdx.x + j * kRT;
                    w[j] = reg_row<K>(vv[j], cc[j], ps);
                    const double u = i < n ? ps[i] : 0.0;  // D^{-1} r of the own row
                    d3[0] += rv[j] * u;
                    d3[1] += w[j] * u;
                    d3[2] += rv[j] * rv[j];
                }
                wg_sum<kRTW, 3, false>(d3, sh[it & 1]);
                rr = d3[2];
                const double rn = sqrt(rr);
                if (!isfinite(rn) || !isfinite(d3[0]) || !isfinite(d3[1])) { status = HSLA_ERR_NONFINITE; break; }
                if (rn <= tol) { status = HSLA_OK; break; }
                const double beta = d3[0] / gamma;
                const double curv = d3[1] - beta * d3[0] / alpha;
                if (!(curv > 0.0)) { status = HSLA_BREAKDOWN; break; }
                alpha = d3[0] / curv;
                gamma = d3[0];
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    // u of the own rows is re-read from LDS rather than kept
                    // live across the sum
                    const int32_t i = threadIdx.x + j * kRT;
                    pv[j] = (i < n ? ps[i] : 0.0) + beta * pv[j];
                    qv[j] = w[j] + beta * qv[j];
                }
            }
        } else {
            while (it < a.max_iter) {
                // q = A p from the LDS copy of p, sigma = p.q
                double acc1[1] = {0.0};
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    qv[j] = reg_row<K>(vv[j], cc[j], ps);
                    acc1[0] += pv[j] * qv[j];
                }
                // sh[0] and sh[1] alternate, and every iteration ends with a
                // barrier, so the sums need no closing barrier of their own
                wg_sum<kRTW, 1, false>(acc1, sh[0]);
                const double sigma = acc1[0];
                if (!isfinite(sigma)) { status = HSLA_ERR_NONFINITE; break; }
                if (!(sigma > 0.0)) { status = HSLA_BREAKDOWN; break; }
                const double alpha = rho / sigma;
                double acc2[2] = {0.0, 0.0};
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int32_t i = threadIdx.x + j * kRT;
                    if (i < n) xs[i] = xs[i] + alpha * pv[j];
                    rv[j] = rv[j] - alpha * qv[j];
                    acc2[0] += rv[j] * rv[j];
                    acc2[1] += rv[j] * (dv[j] * rv[j]);
                }
                wg_sum<kRTW, 2, false>(acc2, sh[1]);
                ++it;
                rr = acc2[0];
                const double rn = sqrt(rr);
                if (!isfinite(rn)) { status = HSLA_ERR_NONFINITE; break; }
                if (rn <= tol) { status = HSLA_OK; break; }
                const double beta = acc2[1] / rho;
                rho = acc2[1];
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int32_t i = threadIdx.x + j * kRT;
                    pv[j] = dv[j] * rv[j] + beta * pv[j];
                    if (i < n) ps[i] = pv[j];
                }
                __syncthreads();
            }
        }
        // x out, and the true residual ||b - A x|| from an LDS copy of x
        __syncthreads();
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int32_t i = threadIdx.x + j * kRT;
            if (i < n) {
                x[i] = xs[i];
                ps[i] = xs[i];
            }
        }
        __syncthreads();
        double accr[2] = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int32_t i = threadIdx.x + j * kRT;
            if (i < n) {
                const double bi = b[i];
                const double e = bi - reg_row<K>(vv[j], cc[j], ps);
                accr[0] += e * e;
                accr[1] += bi * bi;
            }
        }
        wg_sum<kRTW, 2>(accr, sh[0]);
        if (threadIdx.x == 0) {
            RInfo f;
            f.iters = it;
            f.status = status;
            f.pad = 0;
            f.rel_residual = bn > 0 ? sqrt(rr) / bn : sqrt(rr);
            f.true_residual = accr[1] > 0 ? sqrt(accr[0]) / sqrt(accr[1]) : sqrt(accr[0]);
            f.t_begin = t_begin;
            f.t_end = wall_clock64();
            a.info[s] = f;
        }
        __syncthreads();
    }
}

// Carves the work vectors, launches the persistent kernel and returns the
// per-system records.  `a` arrives with the system description set; `order`
// (host, may be empty = identity) is the queue order.
static hsla_status run_persistent(hsla_handle *h, Args a, const hsla_opts &o, int64_t rows, int64_t entries,
                                  int64_t max_n, const std::vector<int32_t> &order, hsla_info *infos,
                                  hipStream_t s, int small_rows = 0, int small_k = 0,
                                  bool single_reduction = false, bool small_reg = false) {
    const int32_t B = a.B;
    // the general kernel's single-reduction form keeps two more vectors
    const bool sr_general = single_reduction && small_rows == 0;
    const int nvec = sr_general ? 6 : 4;
    size_t bytes = 0;
    auto add = [&](size_t v) { bytes += (v + 255) / 256 * 256; };
    add(sizeof(double) * nvec * (rows > 0 ? rows : 1));
    add(sizeof(int32_t) * B);
    add(sizeof(RInfo) * B);
    add(256);
    hsla_status st = ensure_workspace(h, bytes);
    if (st != HSLA_OK) return st;
    char *ws = (char *)h->ws;
    size_t off = 0;
    auto take = [&](size_t v) {
        char *p = ws + off;
        off += (v + 255) / 256 * 256;
        return p;
    };
    double *vec = (double *)take(sizeof(double) * nvec * (rows > 0 ? rows : 1));
    a.r = vec;
    a.p = vec + rows;
    a.q = vec + 2 * rows;
    a.dinv = vec + 3 * rows;
    a.u = sr_general ? vec + 4 * rows : nullptr;
    a.w = sr_general ? vec + 5 * rows : nullptr;
    int32_t *dorder = (int32_t *)take(sizeof(int32_t) * B);
    a.order = order.empty() ? nullptr : dorder;
    a.info = (RInfo *)take(sizeof(RInfo) * B);
    int32_t *flags = (int32_t *)take(256);
    a.queue = flags;
    a.bad = flags + 1;
    a.rtol = o.rtol;
    a.atol = o.atol;
    a.max_iter = o.max_iter > 0 ? o.max_iter : std::min<int64_t>(10 * std::max<int64_t>(max_n, 1), 100000);
    a.jacobi = o.precond == HSLA_PRECOND_JACOBI;
    const int32_t init_flags[2] = {0, INT32_MAX};
    HSLA_HIP(h, hipMemcpyAsync(flags, init_flags, sizeof init_flags, hipMemcpyHostToDevice, s));
    if (!order.empty())
        HSLA_HIP(h, hipMemcpyAsync(dorder, order.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice, s));
    // every pointer the kernels dereference must be set (rows/entries > 0)
    const bool shared = a.shared_n >= 0;
    if (!a.rp || !a.queue || !a.bad || !a.info || (!shared && (!a.row_off || !a.nnz_off || !a.order)) ||
        (rows > 0 && (!a.b || !a.x || !a.r || !a.p || !a.q || !a.dinv)) || (entries > 0 && (!a.col || !a.val)) ||
        (sr_general && rows > 0 && (!a.u || !a.w)))
        return set_error(h, HSLA_ERR_INTERNAL, "persistent solve: unset kernel argument");
    if (!shared) {
        k_ragged_validate<<<std::min(B, 4096), 256, 0, s>>>(a);
        int32_t bad = INT32_MAX;
        HSLA_HIP(h, hipMemcpyAsync(&bad, a.bad, sizeof bad, hipMemcpyDeviceToHost, s));
        HSLA_HIP(h, hipStreamSynchronize(s));
        if (bad != INT32_MAX) return set_error(h, HSLA_ERR_INVALID_CSR, "system %d is not canonical CSR", bad);
    }
    // workgroups beyond the resident ones find the queue empty and exit
    const int gs = (int)std::min<int64_t>(B, 2 * (int64_t)h->dev.num_cu);
    const int gr = gs;
#define SMALL_LAUNCH(SRV)                                                    \
    if (small_rows == 1 && small_k == 8)                                     \
        k_small_pcg<1, 8, SRV><<<gs, kSB, 0, s>>>(a);                        \
    else if (small_rows == 1)                                                \
        k_small_pcg<1, 16, SRV><<<gs, kSB, 0, s>>>(a);                       \
    else if (small_rows == 2 && small_k == 8)                                \
        k_small_pcg<2, 8, SRV><<<gs, kSB, 0, s>>>(a);                        \
    else if (small_rows == 2)                                                \
        k_small_pcg<2, 16, SRV><<<gs, kSB, 0, s>>>(a);                       \
    else if (small_rows == 4 && small_k == 8)                                \
        k_small_pcg<4, 8, SRV><<<gs, kSB, 0, s>>>(a);                        \
    else if (small_rows == 4)                                                \
        k_small_pcg<4, 16, SRV><<<gs, kSB, 0, s>>>(a);
    if (small_reg && single_reduction) {
        if (small_k == 5 && small_rows == 1)
            k_small_reg<1, 5, true><<<gs, kRT, 0, s>>>(a);
        else if (small_k == 5 && small_rows == 2)
            k_small_reg<2, 5, true><<<gs, kRT, 0, s>>>(a);
        else if (small_k == 5)
            k_small_reg<4, 5, true><<<gs, kRT, 0, s>>>(a);
        else if (small_rows == 1)
            k_small_reg<1, 8, true><<<gs, kRT, 0, s>>>(a);
        else if (small_rows == 2)
            k_small_reg<2, 8, true><<<gs, kRT, 0, s>>>(a);
        else
            k_small_reg<4, 8, true><<<gs, kRT, 0, s>>>(a);
    } else if (small_reg) {
        if (small_k == 5 && small_rows == 1)
            k_small_reg<1, 5, false><<<gs, kRT, 0, s>>>(a);
        else if (small_k == 5 && small_rows == 2)
            k_small_reg<2, 5, false><<<gs, kRT, 0, s>>>(a);
        else if (small_k == 5 && small_rows == 4)
            k_small_reg<4, 5, false><<<gs, kRT, 0, s>>>(a);
        else if (small_k == 5)
            k_small_reg<8, 5, false><<<gs, kRT, 0, s>>>(a);
        else if (small_rows == 1)
            k_small_reg<1, 8, false><<<gs, kRT, 0, s>>>(a);
        else if (small_rows == 2)
            k_small_reg<2, 8, false><<<gs, kRT, 0, s>>>(a);
        else
            k_small_reg<4, 8, false><<<gs, kRT, 0, s>>>(a);
    } else if (small_rows > 0 && single_reduction) {
        SMALL_LAUNCH(true)
    } else if (small_rows > 0) {
        SMALL_LAUNCH(false)
    } else if (sr_general) {
        k_ragged_pcg_sr<<<gr, kRB, 0, s>>>(a);
    } else {
        k_ragged_pcg<<<gr, kRB, 0, s>>>(a);
    }
#undef SMALL_LAUNCH
    HSLA_HIP(h, hipGetLastError());
    std::vector<RInfo> hi(B);
    HSLA_HIP(h, hipMemcpyAsync(hi.data(), a.info, sizeof(RInfo) * B, hipMemcpyDeviceToHost, s));
    HSLA_HIP(h, hipStreamSynchronize(s));
    int worst = HSLA_OK;
    uint64_t t0 = UINT64_MAX;
    for (int i = 0; i < B; ++i) t0 = std::min(t0, hi[i].t_begin);
    const double tick_ms = 1.0 / (double)h->dev.wall_khz;
    for (int i = 0; i < B; ++i) {
        const int sst = hi[i].status;
        if (sst < 0 || worst < 0)
            worst = std::min(worst, sst);
        else
            worst = std::max(worst, sst);
        if (infos) {
            infos[i].t_start_ms = (double)(hi[i].t_begin - t0) * tick_ms;
            infos[i].t_end_ms = (double)(hi[i].t_end - t0) * tick_ms;
            infos[i].workgroups = small_rows > 0 ? gs : gr;
            infos[i].reserved = 0;
            infos[i].iters = hi[i].iters;
            infos[i].status = sst;
            infos[i].method = single_reduction ? HSLA_METHOD_CG_SR : HSLA_METHOD_CG;
            infos[i].rel_residual = hi[i].rel_residual;
            infos[i].true_residual = hi[i].true_residual;
            infos[i].spmv_ms = 0.0;
            infos[i].spmv_launches = 0;
            infos[i].spmv_form = 3;
            infos[i].spmv_paired = 0;
        }
    }
    return (hsla_status)worst;
}

// ---------------------------------------------------------------------------
// Segmented ragged solve: the systems of a large ragged batch are treated as
// one block-diagonal operator streamed by per-iteration kernels over the
// whole chip, with each system's reductions and CG scalars kept apart.  The
// rows are cut into chunks of kSegRows that never span two systems; every
// reducing kernel writes one partial per chunk, and a one-block-per-system
// finalize adds a system's chunk partials in chunk order and advances its
// recurrence (the same scalar steps as the batched solver).  Chunks follow
// the system's own rows, so a system's result does not depend on the batch.
// ---------------------------------------------------------------------------
constexpr int kSegRows = 512;
constexpr int kSegW = kBlock / kWave;
constexpr int kSegSlots = 5;  // partials per chunk (the set-up kernel writes five)
// Batches of at least kSegMinRows rows with a system above kSegMinN rows run
// segmented (one workgroup streams a large system slower than the chip
// streams it); smaller ones run persistent.
constexpr int64_t kSegMinRows = 1 << 20;
constexpr int64_t kSegMinN = 8192;

struct Seg {
    Args a;
    const int32_t *csys;    // chunk -> system
    const int32_t *crow;    // chunk -> its first row, local to the system
    const int32_t *cfirst;  // system -> its first chunk ([B + 1])
    SysState *st;           // [B]
    double *part;           // [chunks][kSegSlots]
};

struct SegChunk {
    int32_t s, lo, hi;  // system, local rows [lo, hi)
    int64_t r0, k0;     // the system's first row and entry
    const int32_t *rp;  // the system's local row pointer
};

__device__ __forceinline__ SegChunk seg_chunk(const Seg &g, int32_t c) {
    SegChunk k;
    k.s = g.csys[c];
    k.r0 = g.a.row_off[k.s];
    k.k0 = g.a.nnz_off[k.s];
    const int32_t n = (int32_t)(g.a.row_off[k.s + 1] - k.r0);
    k.lo = g.crow[c];
    k.hi = k.lo + kSegRows < n ? k.lo + kSegRows : n;
    k.rp = g.a.rp + k.r0 + k.s;
    return k;
}

// Sum of a system's chunk partials (value j), fixed order; thread 0.
template <int NV>
__device__ __forceinline__ void seg_reduce(const Seg &g, int32_t s, double (&tot)[NV]) {
    __shared__ double sh[NV * kWavesPerBlock];
#pragma unroll
    for (int j = 0; j < NV; ++j) tot[j] = 0.0;
    for (int32_t c = g.cfirst[s] + threadIdx.x; c < g.cfirst[s + 1]; c += blockDim.x) {
#pragma unroll
        for (int j = 0; j < NV; ++j) tot[j] += g.part[(int64_t)c * kSegSlots + j];
    }
    block_sum<NV>(tot, sh);
}

template <int NV>
__device__ __forceinline__ void seg_partial(const Seg &g, int32_t c, double (&v)[NV]) {
    __shared__ double sh[NV * kWavesPerBlock];
    block_sum<NV>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) g.part[(int64_t)c * kSegSlots + j] = v[j];
    }
}

__global__ void k_seg_reset(SysState *st, int32_t B, int64_t max_iter, int32_t stall) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < B; i += gridDim.x * blockDim.x) {
        SysState z;
        memset(&z, 0, sizeof z);
        z.max_iter = max_iter;
        z.stall = stall;
        z.rho = z.alpha = z.omega = 1.0;
        st[i] = z;
    }
}

// x = 0, r = b, D^{-1} (1 without Jacobi), p = D^{-1} r; partials of b.b,
// r.r, r.D^{-1}r, a missing-or-zero-diagonal flag and a negative-diagonal
// flag (Jacobi).
__global__ __launch_bounds__(kBlock) void k_seg_init(Seg g) {
    const int32_t c = blockIdx.x;
    const SegChunk k = seg_chunk(g, c);
    const Args &a = g.a;
    const int32_t *col = a.col + k.k0;
    const double *val = a.val + k.k0;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int32_t i = k.lo + threadIdx.x; i < k.hi; i += kBlock) {
        double d = 0.0;
        for (int32_t e = k.rp[i]; e < k.rp[i + 1]; ++e)
            if (col[e] == i) d = val[e];
        if (a.jacobi && d == 0.0) acc[3] = 1.0;
        if (a.jacobi && d < 0.0) acc[4] = 1.0;
        const double di = a.jacobi ? 1.0 / d : 1.0;
        const int64_t gi = k.r0 + i;
        const double bi = a.b[gi];
        a.dinv[gi] = di;
        a.x[gi] = 0.0;
        a.r[gi] = bi;
        a.p[gi] = di * bi;
        acc[0] += bi * bi;
        acc[1] += bi * bi;
        acc[2] += bi * (di * bi);
    }
    seg_partial<5>(g, c, acc);
}

// A negative Jacobi diagonal (D^{-1} is then no SPD preconditioner) ends the
// solve with BREAKDOWN before the first iteration, x = 0, as on the batched
// path; a zero or missing one is an error and takes precedence.
__global__ __launch_bounds__(kBlock) void k_seg_fin_init(Seg g) {
    const int32_t s = blockIdx.x;
    double tot[5];
    seg_reduce<5>(g, s, tot);
    if (threadIdx.x != 0) return;
    SysState &st = g.st[s];
    if (tot[3] > 0.0) st.bad_diag = 1;
    cg_step_init(st, tot[0], tot[1], tot[2], g.a.rtol, g.a.atol);
    if (tot[4] > 0.0 && !st.done) {
        st.status = HSLA_BREAKDOWN;
        st.done = 1;
    }
}

// q = A p for the chunk's rows (ascending per-row sums); partial of p.q.
__global__ __launch_bounds__(kBlock) void k_seg_spmv_dot(Seg g) {
    __shared__ double lds[kSegW * kChunk];
    const int32_t c = blockIdx.x;
    const SegChunk k = seg_chunk(g, c);
    if (g.st[k.s].done) return;
    const Args &a = g.a;
    const double *p = a.p + k.r0;
    double *q = a.q + k.r0;
    double acc[1] = {0.0};
    auto epi = [&](int32_t i, double sum) {
        const int32_t row = k.lo + i;
        __builtin_nontemporal_store(sum, &q[row]);
        acc[0] += p[row] * sum;
    };
    wg_spmv<kSegW, decltype(epi) &, true>(k.hi - k.lo, k.rp + k.lo, a.col + k.k0, a.val + k.k0, p, lds, epi);
    seg_partial<1>(g, c, acc);
}

__global__ __launch_bounds__(kBlock) void k_seg_fin_alpha(Seg g) {
    const int32_t s = blockIdx.x;
    SysState &st = g.st[s];
    if (st.done) return;
    double tot[1];
    seg_reduce<1>(g, s, tot);
    if (threadIdx.x == 0) cg_step_alpha(st, tot[0]);
}

// r -= alpha q; partials of r.r and r.D^{-1}r.
__global__ __launch_bounds__(kBlock) void k_seg_update(Seg g) {
    const int32_t c = blockIdx.x;
    const SegChunk k = seg_chunk(g, c);
    const SysState &st = g.st[k.s];
    if (st.done) return;
    const double alpha = st.alpha;
    const Args &a = g.a;
    double acc[2] = {0.0, 0.0};
    for (int32_t i = k.lo + threadIdx.x; i < k.hi; i += 2 * kBlock) {
        double rv[2], qv[2], dv[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int32_t j = i + u * kBlock;
            if (j < k.hi) {
                rv[u] = __builtin_nontemporal_load(&a.r[k.r0 + j]);
                qv[u] = __builtin_nontemporal_load(&a.q[k.r0 + j]);
                dv[u] = __builtin_nontemporal_load(&a.dinv[k.r0 + j]);
            }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int32_t j = i + u * kBlock;
            if (j < k.hi) {
                const double ri = rv[u] - alpha * qv[u];
                __builtin_nontemporal_store(ri, &a.r[k.r0 + j]);
                acc[0] += ri * ri;
                acc[1] += ri * (dv[u] * ri);
            }
        }
    }
    seg_partial<2>(g, c, acc);
}

__global__ __launch_bounds__(kBlock) void k_seg_fin_beta(Seg g) {
    const int32_t s = blockIdx.x;
    SysState &st = g.st[s];
    if (st.done) {
        if (threadIdx.x == 0) st.xpend = 0;
        return;
    }
    double tot[2];
    seg_reduce<2>(g, s, tot);
    if (threadIdx.x == 0) cg_step_beta(st, tot[0], tot[1], true);
}

// x += alpha p, then p = D^{-1} r + beta p (only the x update for a system
// that stopped in this iteration).
__global__ __launch_bounds__(kBlock) void k_seg_direction(Seg g) {
    const int32_t c = blockIdx.x;
    const SegChunk k = seg_chunk(g, c);
    const SysState &st = g.st[k.s];
    const bool xonly = st.done != 0;
    if (xonly && !st.xpend) return;
    const double alpha = st.alpha, beta = st.beta;
    const Args &a = g.a;
    for (int32_t i = k.lo + threadIdx.x; i < k.hi; i += 2 * kBlock) {
        double xv[2], pv[2], rv[2], dv[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int32_t j = i + u * kBlock;
            if (j < k.hi) {
                xv[u] = __builtin_nontemporal_load(&a.x[k.r0 + j]);
                pv[u] = __builtin_nontemporal_load(&a.p[k.r0 + j]);
                if (!xonly) {
                    rv[u] = __builtin_nontemporal_load(&a.r[k.r0 + j]);
                    dv[u] = __builtin_nontemporal_load(&a.dinv[k.r0 + j]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int32_t j = i + u * kBlock;
            if (j < k.hi) {
                __builtin_nontemporal_store(xv[u] + alpha * pv[u], &a.x[k.r0 + j]);
                if (!xonly) __builtin_nontemporal_store(dv[u] * rv[u] + beta * pv[u], &a.p[k.r0 + j]);
            }
        }
    }
}

// Partials of ||b - A x||^2 and ||b||^2.
__global__ __launch_bounds__(kBlock) void k_seg_residual(Seg g) {
    __shared__ double lds[kSegW * kChunk];
    const int32_t c = blockIdx.x;
    const SegChunk k = seg_chunk(g, c);
    const Args &a = g.a;
    const double *b = a.b + k.r0;
    double acc[2] = {0.0, 0.0};
    wg_spmv<kSegW>(k.hi - k.lo, k.rp + k.lo, a.col + k.k0, a.val + k.k0, a.x + k.r0, lds,
                   [&](int32_t i, double sum) {
                       const double bi = b[k.lo + i];
                       const double e = bi - sum;
                       acc[0] += e * e;
                       acc[1] += bi * bi;
                   });
    seg_partial<2>(g, c, acc);
}

__global__ __launch_bounds__(kBlock) void k_seg_fin_residual(Seg g) {
    const int32_t s = blockIdx.x;
    double tot[2];
    seg_reduce<2>(g, s, tot);
    if (threadIdx.x != 0) return;
    const SysState &st = g.st[s];
    RInfo f;
    f.iters = st.iters;
    f.status = st.done ? st.status : HSLA_ERR_INTERNAL;
    f.pad = 0;
    const double rn = sqrt(st.rnorm2);
    f.rel_residual = st.bnorm > 0 ? rn / st.bnorm : rn;
    f.true_residual = tot[1] > 0 ? sqrt(tot[0]) / sqrt(tot[1]) : sqrt(tot[0]);
    f.t_begin = f.t_end = 0;
    g.a.info[s] = f;
}

// Host side of the segmented solve; `a` has the ragged system description,
// `ro` the host copy of its row offsets.
static hsla_status run_segmented(hsla_handle *h, Args a, const hsla_opts &o, const std::vector<int64_t> &ro,
                                 int64_t max_n, hsla_info *infos, hipStream_t s) {
    const int32_t B = a.B;
    const int64_t rows = ro[B];
    std::vector<int32_t> cfirst(B + 1), csys, crow;
    for (int32_t i = 0; i < B; ++i) {
        cfirst[i] = (int32_t)csys.size();
        const int64_t n = ro[i + 1] - ro[i];
        for (int64_t r = 0; r < n; r += kSegRows) {
            csys.push_back(i);
            crow.push_back((int32_t)r);
        }
    }
    const int32_t nch = (int32_t)csys.size();
    cfirst[B] = nch;
    size_t bytes = 0;
    auto add = [&](size_t v) { bytes += (v + 255) / 256 * 256; };
    add(sizeof(double) * 4 * (size_t)(rows > 0 ? rows : 1));
    add(sizeof(int32_t) * (size_t)(nch > 0 ? nch : 1) * 2);
    add(sizeof(int32_t) * (B + 1));
    add(sizeof(SysState) * B);
    add(sizeof(double) * kSegSlots * (size_t)(nch > 0 ? nch : 1));
    add(sizeof(RInfo) * B);
    add(256);
    hsla_status st = ensure_workspace(h, bytes);
    if (st != HSLA_OK) return st;
    st = ensure_host_state(h, B);
    if (st != HSLA_OK) return st;
    char *ws = (char *)h->ws;
    size_t off = 0;
    auto take = [&](size_t v) {
        char *q = ws + off;
        off += (v + 255) / 256 * 256;
        return q;
    };
    double *vec = (double *)take(sizeof(double) * 4 * (size_t)(rows > 0 ? rows : 1));
    a.r = vec;
    a.p = vec + rows;
    a.q = vec + 2 * rows;
    a.dinv = vec + 3 * rows;
    int32_t *tab = (int32_t *)take(sizeof(int32_t) * (size_t)(nch > 0 ? nch : 1) * 2);
    int32_t *dfirst = (int32_t *)take(sizeof(int32_t) * (B + 1));
    Seg g{};
    g.st = (SysState *)take(sizeof(SysState) * B);
    g.part = (double *)take(sizeof(double) * kSegSlots * (size_t)(nch > 0 ? nch : 1));
    a.info = (RInfo *)take(sizeof(RInfo) * B);
    a.bad = (int32_t *)take(256);
    a.queue = nullptr;
    a.order = nullptr;
    a.rtol = o.rtol;
    a.atol = o.atol;
    a.max_iter = o.max_iter > 0 ? o.max_iter : std::min<int64_t>(10 * std::max<int64_t>(max_n, 1), 100000);
    a.jacobi = o.precond == HSLA_PRECOND_JACOBI;
    // every pointer the kernels dereference must be set (rows/entries > 0)
    if (!a.rp || !a.row_off || !a.nnz_off || !a.info || !a.bad ||
        (rows > 0 && (!a.b || !a.x || !a.r || !a.p || !a.q || !a.dinv)))
        return set_error(h, HSLA_ERR_INTERNAL, "segmented solve: unset kernel argument");
    const int32_t no_bad = INT32_MAX;
    HSLA_HIP(h, hipMemcpyAsync(a.bad, &no_bad, sizeof no_bad, hipMemcpyHostToDevice, s));
    k_ragged_validate<<<std::min(B, 4096), 256, 0, s>>>(a);
    int32_t bad = INT32_MAX;
    HSLA_HIP(h, hipMemcpyAsync(&bad, a.bad, sizeof bad, hipMemcpyDeviceToHost, s));
    HSLA_HIP(h, hipStreamSynchronize(s));
    if (bad != INT32_MAX) return set_error(h, HSLA_ERR_INVALID_CSR, "system %d is not canonical CSR", bad);
    g.a = a;
    g.csys = tab;
    g.crow = tab + nch;
    g.cfirst = dfirst;
    if (nch > 0) {
        HSLA_HIP(h, hipMemcpyAsync(tab, csys.data(), sizeof(int32_t) * nch, hipMemcpyHostToDevice, s));
        HSLA_HIP(h, hipMemcpyAsync(tab + nch, crow.data(), sizeof(int32_t) * nch, hipMemcpyHostToDevice, s));
    }
    HSLA_HIP(h, hipMemcpyAsync(dfirst, cfirst.data(), sizeof(int32_t) * (B + 1), hipMemcpyHostToDevice, s));
    k_seg_reset<<<(B + kBlock - 1) / kBlock, kBlock, 0, s>>>(g.st, B, a.max_iter,
                                                             o.stall_window > 0 ? o.stall_window : 0);
    if (nch > 0) k_seg_init<<<nch, kBlock, 0, s>>>(g);
    k_seg_fin_init<<<B, kBlock, 0, s>>>(g);
    HSLA_HIP(h, hipGetLastError());
    // chunks of 8 iterations between host checks; every system stops by
    // max_iter, so the loop ends
    SysState *hs = h->h_state;
    for (;;) {
        HSLA_HIP(h, hipMemcpyAsync(hs, g.st, sizeof(SysState) * B, hipMemcpyDeviceToHost, s));
        HSLA_HIP(h, hipStreamSynchronize(s));
        bool all = true;
        for (int32_t i = 0; i < B && all; ++i) all = hs[i].done != 0;
        if (all || nch == 0) break;
        for (int k = 0; k < 8; ++k) {
            k_seg_spmv_dot<<<nch, kBlock, 0, s>>>(g);
            k_seg_fin_alpha<<<B, kBlock, 0, s>>>(g);
            k_seg_update<<<nch, kBlock, 0, s>>>(g);
            k_seg_fin_beta<<<B, kBlock, 0, s>>>(g);
            k_seg_direction<<<nch, kBlock, 0, s>>>(g);
        }
        HSLA_HIP(h, hipGetLastError());
    }
    if (nch > 0) k_seg_residual<<<nch, kBlock, 0, s>>>(g);
    k_seg_fin_residual<<<B, kBlock, 0, s>>>(g);
    HSLA_HIP(h, hipGetLastError());
    std::vector<RInfo> hi(B);
    HSLA_HIP(h, hipMemcpyAsync(hi.data(), a.info, sizeof(RInfo) * B, hipMemcpyDeviceToHost, s));
    HSLA_HIP(h, hipStreamSynchronize(s));
    int worst = HSLA_OK;
    for (int i = 0; i < B; ++i) {
        const int sst = hi[i].status;
        if (sst < 0 || worst < 0)
            worst = std::min(worst, sst);
        else
            worst = std::max(worst, sst);
        if (infos) {
            infos[i].iters = hi[i].iters;
            infos[i].status = sst;
            infos[i].method = HSLA_METHOD_CG;
            infos[i].rel_residual = hi[i].rel_residual;
            infos[i].true_residual = hi[i].true_residual;
            infos[i].spmv_ms = 0.0;
            infos[i].spmv_launches = 0;
            infos[i].spmv_form = 0;
            infos[i].spmv_paired = 0;
            infos[i].t_start_ms = infos[i].t_end_ms = 0.0;
            infos[i].workgroups = 0;
            infos[i].reserved = 0;
        }
    }
    return (hsla_status)worst;
}

}  // namespace rg

// The register-resident kernel wins for every small system; the general
// shared-mode kernel only once the batch gives every CU a system (one
// workgroup streams a mid-size system slower than the per-iteration kernels
// stream it over the whole chip).
bool persistent_eligible(const hsla_handle *h, const hsla_pattern *p, int B, int method, const hsla_opts &o) {
    if (method != HSLA_METHOD_CG || (o.precond != HSLA_PRECOND_JACOBI && o.precond != HSLA_PRECOND_NONE) ||
        o.use_x0 || o.profile || o.stall_window > 0 || B < 1 || p->n < 1)
        return false;
    if (p->n <= rg::kSmallMaxN && p->max_row <= rg::kSmallMaxRow) return true;
    return B >= h->dev.num_cu && p->nnz <= kPersistentMaxNnz;
}

hsla_status persistent_solve(hsla_handle *h, const hsla_pattern *p, int B, const double *values, const double *b,
                             double *x, const hsla_opts &o, hsla_info *infos, hipStream_t s, bool single_reduction) {
    rg::Args a{};
    a.B = B;
    a.shared_n = p->n;
    a.shared_nnz = p->nnz;
    a.rp = p->row_ptr;
    a.col = p->col;
    a.val = values;
    a.b = b;
    a.x = x;
    int rows = 0, k = 0;
    bool reg = false;
    if (p->n <= rg::kSmallMaxN && p->max_row <= rg::kSmallMaxRow) {
        rows = p->n <= rg::kSB ? 1 : p->n <= 2 * rg::kSB ? 2 : 4;
        k = p->max_row <= 8 ? 8 : 16;
        // rows short enough to keep the matrix in registers (the
        // single-reduction recurrence, which keeps s = A p there as well, at
        // up to 4 rows per thread)
        if ((p->max_row <= 5 || (p->max_row <= 8 && p->n <= 4 * rg::kRT)) &&
            !(single_reduction && p->n > 4 * rg::kRT)) {
            reg = true;
            k = p->max_row <= 5 ? 5 : 8;
            rows = p->n <= rg::kRT ? 1 : p->n <= 2 * rg::kRT ? 2 : p->n <= 4 * rg::kRT ? 4 : 8;
        }
    }
    return rg::run_persistent(h, a, o, (int64_t)B * p->n, p->nnz, p->n, {}, infos, s, rows, k, single_reduction,
                              reg);
}

}  // namespace hsla

extern "C" hsla_status hsla_solve_ragged(hsla_handle *h, int32_t B, const int64_t *d_row_off,
                                         const int64_t *d_nnz_off, const int32_t *d_row_ptr, const int32_t *d_col,
                                         const double *d_values, const double *d_b, double *d_x,
                                         const hsla_opts *opts, hsla_info *infos, void *stream) {
    using namespace hsla;
    using namespace hsla::rg;
    if (!h) return HSLA_ERR_INVALID_ARG;
    if (B < 0) return set_error(h, HSLA_ERR_INVALID_ARG, "negative batch");
    hsla_opts o;
    if (opts)
        o = *opts;
    else
        hsla_opts_default(&o);
    if (o.method == HSLA_METHOD_BICGSTAB || o.precond == HSLA_PRECOND_FSAI || o.use_x0)
        return set_error(h, HSLA_ERR_INVALID_ARG, "ragged batches run CG with Jacobi or no preconditioner from x0 = 0");
    if (!(o.rtol >= 0) || !(o.atol >= 0)) return set_error(h, HSLA_ERR_INVALID_ARG, "negative or NaN tolerance");
    hsla_status st = enter(h, (hipStream_t)stream);
    if (st != HSLA_OK) return st;
    if (B == 0) return HSLA_OK;
    if (!d_row_off || !d_nnz_off || !d_row_ptr) return set_error(h, HSLA_ERR_INVALID_ARG, "null pointer");
    hipStream_t s = h->stream;
    std::vector<int64_t> ro(B + 1), no(B + 1);
    HSLA_HIP(h, hipMemcpyAsync(ro.data(), d_row_off, sizeof(int64_t) * (B + 1), hipMemcpyDeviceToHost, s));
    HSLA_HIP(h, hipMemcpyAsync(no.data(), d_nnz_off, sizeof(int64_t) * (B + 1), hipMemcpyDeviceToHost, s));
    HSLA_HIP(h, hipStreamSynchronize(s));
    if (ro[0] != 0 || no[0] != 0) return set_error(h, HSLA_ERR_INVALID_CSR, "offsets must start at 0");
    int64_t max_n = 0;
    for (int i = 0; i < B; ++i) {
        if (ro[i + 1] < ro[i] || no[i + 1] < no[i])
            return set_error(h, HSLA_ERR_INVALID_CSR, "offsets of system %d decrease", i);
        max_n = std::max(max_n, ro[i + 1] - ro[i]);
    }
    const int64_t rows = ro[B];
    if (rows > 0 && (!d_b || !d_x)) return set_error(h, HSLA_ERR_INVALID_ARG, "null b or x");
    if (no[B] > 0 && (!d_col || !d_values)) return set_error(h, HSLA_ERR_INVALID_ARG, "null col or values");
    // longest (most entries) first
    std::vector<int32_t> order(B);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return no[a + 1] - no[a] > no[b + 1] - no[b]; });
    Args a{};
    a.B = B;
    a.shared_n = -1;
    a.shared_nnz = -1;
    a.row_off = d_row_off;
    a.nnz_off = d_nnz_off;
    a.rp = d_row_ptr;
    a.col = d_col;
    a.val = d_values;
    a.b = d_b;
    a.x = d_x;
    if (!o.persistent || o.stall_window > 0 || (o.persistent != 2 && rows >= kSegMinRows && max_n > kSegMinN))
        return run_segmented(h, a, o, ro, max_n, infos, s);
    return run_persistent(h, a, o, rows, no[B], max_n, order, infos, s, 0, 0, o.method == HSLA_METHOD_CG_SR);
}
