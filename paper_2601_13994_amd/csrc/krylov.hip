// Krylov solvers on CSR for MI355X: tile SpMV, Jacobi/FSAI-preconditioned CG
// and right-Jacobi BiCGStab, the true-residual check and the adjoint
// gradient assembly.  All recurrences run in FP64.
//
// One iteration is a short chain of kernels on one stream; every dot
// product is folded into the kernel that produces its operands and reduced
// in a single pass: blocks store partials, and a one-block finalize kernel
// per system adds them in a fixed order and advances the scalar recurrence
// (alpha, beta, omega, stop test) in device memory.  Kernels of a stopped
// system return at entry, so chunks of K iterations are enqueued (and
// replayed as a HIP graph) with one host check per chunk.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace hsla {

// ---------------------------------------------------------------------------
// Kernel argument bundles
// ---------------------------------------------------------------------------
struct Pat {
    const int32_t *rp, *col, *diag;
    const int2 *meta;
    int32_t ntiles, n;
    int64_t nnz;
    Stencil sn;  // offset-mask form in use (mask == nullptr: CSR)
};

struct FPat {  // pattern + values of one FSAI factor (float32 values)
    const int32_t *rp, *col;
    const int2 *meta;
    int32_t ntiles;
    int64_t nnz;
    const float *val;
    Stencil sn;
    const float *dia;  // diagonal-major copy of val ([B][nofs][n]) when sn is used
};

static Pat pat_of(const hsla_pattern *p) {
    return Pat{p->row_ptr, p->col, p->diag, p->meta, p->ntiles, p->n, p->nnz, p->use(p->stA)};
}

static Pat pat_T_of(const hsla_pattern *p) {
    return Pat{p->rpT, p->colT, p->diagT, p->metaT, p->ntilesT, p->n, p->nnz, p->use(p->stT)};
}

struct Sys {
    const double *val;  // [B][nnz]
    const double *aval; // [B][nnz] values of the operator iterated on: val, or for right-Jacobi
                        // BiCGStab the column-scaled A D^{-1} (tile form)
    const double *dia;  // [B][nofs][n] diagonal-major copy of val (offset-mask patterns)
    const double *b;    // [B][n]
    double *x;          // [B][n]
    // work vectors, [B][n] each
    double *r, *p, *q, *dinv, *z, *w;
    double *rh, *y, *v, *s, *t;  // BiCGStab: y accumulates the iterate of A M^{-1} y = b - A x0
    SysState *st;       // [B]
    double *part;       // [B][3][G] block partials of the last producing kernel
    double *part2;      // [B][G] block partials of the single-reduction sweep (kept past the next SpMV)
    // s-step CG: basis vectors past p and r ([2s-1][B][n]), Gram partials
    // ([B][2 NG][G]) and the coordinates of x, r, p ([B][3][2s+1])
    double *ssb, *ssp, *ssc;
};

#define SYS_OFFSETS(S, A)                                               \
    const int sidx = blockIdx.y;                                        \
    const int64_t vo = (int64_t)sidx * (A).n;                           \
    SysState &st = (S).st[sidx];                                        \
    double *part = (S).part + (int64_t)sidx * 3 * gridDim.x;

// y = A v for system sidx through the form the solve uses: the
// diagonal-major copy of the values (NS > 0, offset-mask patterns) or the
// tile walk over CSR / row masks.
template <int NS, class Epi>
__device__ __forceinline__ void spmv_A(const Pat &A, const Sys &S, int sidx, const double *v, double *lds,
                                       Epi &&epi) {
    if constexpr (NS > 0)
        spmv_dia<NS>(A.sn, S.dia + (int64_t)sidx * dia_stored(NS, A.sn.nofs) * dia_chunks(A.n) * kDiaChunk,
                     (int64_t)A.n, v, epi);
    else
        spmv_tiles(A.rp, A.col, A.sn, S.aval + (int64_t)sidx * A.nnz, v, A.meta, A.ntiles, lds, epi);
}

// y = F v for an FSAI factor (float32 values), same two forms.
template <int NS, class Epi>
__device__ __forceinline__ void spmv_F(const FPat &F, int64_t n, int sidx, const double *v, double *lds,
                                       Epi &&epi) {
    if constexpr (NS > 0)
        spmv_dia<NS>(F.sn, F.dia + (int64_t)sidx * F.sn.nofs * dia_chunks(n) * kDiaChunk, n, v, epi);
    else
        spmv_tiles(F.rp, F.col, F.sn, F.val + (int64_t)sidx * F.nnz, v, F.meta, F.ntiles, lds, epi);
}

// Chunked diagonal-major copy of the values of an offset-mask pattern (see
// kDiaChunk): the entry of row i on diagonal s at dia_index(i, s), 0 where
// the row has none and for the padding rows of the last chunk.  With
// `cscale` ([B][n]) the entry (i, j) is multiplied by cscale[j] (the
// operator A D^{-1} of right-Jacobi BiCGStab) or, with `sym`, by
// cscale[i] cscale[j] (S A S of Jacobi CG).
// `unit`: the diagonal of the scaled operator is 1 and is left out (slots
// past it move down by one; needs a diagonal slot).
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_to_dia(int32_t n, const int32_t *__restrict__ rp, Stencil sn,
                                                   int64_t nnz, const VT *__restrict__ vals, VT *__restrict__ dia,
                                                   const double *__restrict__ cscale = nullptr, int sym = 0,
                                                   int unit = 0) {
    const int sidx = blockIdx.y;
    const int64_t rows = dia_chunks(n) * kDiaChunk;
    const int nst = unit ? sn.nofs - 1 : sn.nofs;
    const VT *v = vals + (int64_t)sidx * nnz;
    VT *d = dia + (int64_t)sidx * nst * rows;
    const double *cs = cscale ? cscale + (int64_t)sidx * n : nullptr;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < rows; i += (int64_t)gridDim.x * kBlock) {
        const uint32_t m = i < n ? (uint32_t)sn.mask[i] : 0u;
        int32_t k = i < n ? rp[i] : 0;
        for (int s = 0; s < sn.nofs; ++s) {
            VT val = VT(0);
            if ((m >> s) & 1u) {
                val = v[k++];
                if (cs && sym && sn.ofs[s] == 0)
                    val = VT(1);  // the diagonal of S A S is 1 by construction
                else if (cs)
                    val = VT((double)val * (sym ? cs[i] * cs[i + sn.ofs[s]] : cs[i + sn.ofs[s]]));
            }
            if (unit && s == sn.diag_slot) continue;
            d[dia_index(i, unit && s > sn.diag_slot ? s - 1 : s, nst)] = val;
        }
    }
}

// The same column scaling on the CSR values (tile form): out = val D^{-1},
// the diagonal 1 by construction.
__global__ __launch_bounds__(kBlock) void k_scale_cols(int32_t n, int64_t nnz, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col,
                                                       const double *__restrict__ val,
                                                       const double *__restrict__ cscale, double *__restrict__ out) {
    const int sidx = blockIdx.y;
    const double *v = val + (int64_t)sidx * nnz;
    const double *cs = cscale + (int64_t)sidx * n;
    double *o = out + (int64_t)sidx * nnz;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) o[k] = col[k] == i ? 1.0 : v[k] * cs[col[k]];
}

// The half form's copy (see kSymNS): the main and upper diagonals only, at
// stored slot s - nofs/2.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_to_dia_sym(int32_t n, const int32_t *__restrict__ rp, Stencil sn,
                                                       int64_t nnz, const VT *__restrict__ vals,
                                                       VT *__restrict__ dia, const double *__restrict__ sc = nullptr,
                                                       int unit = 0) {
    const int sidx = blockIdx.y;
    const int ds = sn.nofs / 2, nh = unit ? ds : ds + 1, u0 = unit ? ds + 1 : ds;
    const int64_t rows = dia_chunks(n) * kDiaChunk;
    const VT *v = vals + (int64_t)sidx * nnz;
    VT *d = dia + (int64_t)sidx * nh * rows;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < rows; i += (int64_t)gridDim.x * kBlock) {
        const uint32_t m = i < n ? (uint32_t)sn.mask[i] : 0u;
        int32_t k = i < n ? rp[i] + __popc(m & ((1u << ds) - 1u)) : 0;
        const double *cs = sc ? sc + (int64_t)sidx * n : nullptr;
        for (int s = ds; s < sn.nofs; ++s) {
            VT val = VT(0);
            if ((m >> s) & 1u) {
                val = v[k++];
                if (cs) val = VT((double)val * (cs[i] * cs[i + sn.ofs[s]]));
            }
            if (s >= u0) d[dia_index(i, s - u0, nh)] = val;
        }
    }
}

// Finalize kernels run one block per system (grid = B).
#define FIN_OFFSETS(S, G)                                               \
    const int sidx = blockIdx.x;                                        \
    SysState &st = (S).st[sidx];                                        \
    const double *part = (S).part + (int64_t)sidx * 3 * (G);

__device__ __forceinline__ bool stopped(const SysState &st) { return st.done != 0; }

// Grid-stride element loops: each thread takes 4 elements per trip
// (i, i+S, i+2S, i+3S with S the grid's thread count) so that all their
// loads are in flight together; the per-thread summation order is the
// plain grid-stride order.
#define GRID_LOOP_BEGIN(n)                                                           \
    {                                                                                \
        const int64_t n_ = (n);                                                      \
        const int64_t S_ = (int64_t)gridDim.x * kBlock;                              \
        int64_t i_ = (int64_t)blockIdx.x * kBlock + threadIdx.x;                     \
        for (; i_ + 3 * S_ < n_; i_ += 4 * S_) {
#define GRID_LOOP_TAIL \
        }              \
        for (; i_ < n_; i_ += S_) {
#define GRID_LOOP_END \
        }             \
    }

// The same over pairs of elements (2 i_, 2 i_ + 1), for vectors that are all
// 16-byte aligned: each access is one 16-byte load or store for two
// elements, two pairs per thread per step.
#define PAIR_LOOP_BEGIN(np)                                                          \
    {                                                                                \
        const int64_t n_ = (np);                                                     \
        const int64_t S_ = (int64_t)gridDim.x * kBlock;                              \
        int64_t i_ = (int64_t)blockIdx.x * kBlock + threadIdx.x;                     \
        for (; i_ + S_ < n_; i_ += 2 * S_) {
#define PAIR_LOOP_TAIL GRID_LOOP_TAIL
#define PAIR_LOOP_END GRID_LOOP_END

__device__ __forceinline__ bool al16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
// Vector sweeps touch every element once per kernel, and every SpMV output is
// written once and read by the next sweep: nontemporal loads and stores keep
// a pass over hundreds of MB from cycling the caches, and leave no dirty
// lines to be written back under the next kernel.  Measured on the 256^3
// Jacobi-CG: 0.395 -> 0.358 ms per iteration, its SpMV 163 -> 134 us.
__device__ __forceinline__ dpair ldp(const double *p) { return __builtin_nontemporal_load((const dpair *)p); }
__device__ __forceinline__ void stp(double *p, dpair v) { __builtin_nontemporal_store(v, (dpair *)p); }
__device__ __forceinline__ void st_nt(double *p, double v) { __builtin_nontemporal_store(v, p); }

// ---------------------------------------------------------------------------
// State reset
// ---------------------------------------------------------------------------
__global__ void k_reset(SysState *st, int B, int64_t max_iter, int32_t stall) {
    for (int i = threadIdx.x; i < B; i += blockDim.x) {
        SysState z;
        memset(&z, 0, sizeof z);
        z.max_iter = max_iter;
        z.stall = stall;
        z.rho = z.alpha = z.omega = 1.0;
        st[i] = z;
    }
}

// ---------------------------------------------------------------------------
// SpMV
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_spmv(Pat A, const double *__restrict__ val, const double *__restrict__ x,
                                                 double *__restrict__ y) {
    __shared__ double lds[kWavesPerBlock][kTileCap];
    const int64_t sidx = blockIdx.y;
    val += sidx * A.nnz;
    x += sidx * A.n;
    y += sidx * A.n;
    spmv_tiles(A.rp, A.col, A.sn, val, x, A.meta, A.ntiles, lds[threadIdx.x / kWave],
               [&](int32_t row, double yv) {
                   st_nt(&y[row], yv);
               });
}

// y = A x on a diagonal-major copy of the values (offset-mask patterns).
template <int NS>
__global__ __launch_bounds__(kBlock) void k_spmv_dia(Pat A, const double *__restrict__ dia,
                                                     const double *__restrict__ x, double *__restrict__ y) {
    const int64_t sidx = blockIdx.y;
    x += sidx * A.n;
    y += sidx * A.n;
    spmv_dia<NS>(A.sn, dia + sidx * dia_stored(NS, A.sn.nofs) * dia_chunks(A.n) * kDiaChunk, (int64_t)A.n, x,
                 [&](int64_t row, double yv) { st_nt(&y[row], yv); });
}

// ---------------------------------------------------------------------------
// CG / PCG
// ---------------------------------------------------------------------------
enum { PRE_NONE = 0, PRE_JACOBI = 1, PRE_FSAI = 2 };

// x = 0 or x0, r = b - A x0 (q holds A x0), z = M^{-1} r (none / FSAI),
// p = z; partials of b.b, r.r, r.z.
// Jacobi runs as CG on the scaled system S A S y = S r0 with S = D^{-1/2}
// (the same iterates as Jacobi-PCG in exact arithmetic: x = x0 + S y, the
// scaled residual is S r and its inner product the PCG's r.D^{-1}r): the
// work vectors hold S r, S^{-1} x and the scaled p, the dinv slot holds
// S, and the operator's values are scaled once per solve.  The stop test
// stays on the unscaled ||r||.  A negative diagonal (no real S; Jacobi is
// then not a valid CG preconditioner) stops the solve with BREAKDOWN before
// the first iteration.
template <int PRE>
__global__ __launch_bounds__(kBlock) void k_cg_init(Pat A, Sys S, int use_x0) {
    SYS_OFFSETS(S, A)
    const double *val = S.val + sidx * A.nnz;
    double acc[3] = {0.0, 0.0, 0.0};  // b.b, r.r, r.z
    bool bad = false, neg = false;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < A.n; i += (int64_t)gridDim.x * kBlock) {
        const double bi = S.b[vo + i];
        const double ri = use_x0 ? bi - S.q[vo + i] : bi;
        double zi = ri;
        if (PRE == PRE_JACOBI) {
            const int32_t d = A.diag[i];
            const double a = d >= 0 ? val[d] : 0.0;
            if (a == 0.0) bad = true;
            if (a < 0.0) neg = true;
            const double si = a > 0.0 ? 1.0 / sqrt(a) : 1.0;
            S.dinv[vo + i] = si;
            // the stop test's weights 1/S_i^2 = a_ii, in FP32 (z slot)
            reinterpret_cast<float *>(S.z)[vo + i] = a > 0.0 ? (float)a : 1.0f;
            zi = si * ri;  // the scaled residual S r
            S.r[vo + i] = zi;
            S.x[vo + i] = use_x0 ? S.x[vo + i] / si : 0.0;
            acc[2] += zi * zi;
        } else {
            if (!use_x0) S.x[vo + i] = 0.0;
            S.r[vo + i] = ri;
            acc[2] += ri * zi;
        }
        S.p[vo + i] = PRE == PRE_FSAI ? 0.0 : zi;
        acc[0] += bi * bi;
        acc[1] += ri * ri;
    }
    // bit 0: a missing or zero diagonal, bit 1: a negative one
    const int any_bad = __syncthreads_or(bad ? 1 : 0);
    const int any_neg = __syncthreads_or(neg ? 1 : 0);
    const int flags = (any_bad ? 1 : 0) | (any_neg ? 2 : 0);
    if (threadIdx.x == 0 && flags) atomicOr(&st.bad_diag, flags);
    block_partial<3>(acc, part);
}

// ||b||, tol = max(rtol ||b||, atol), initial stop test, rho = r.z.
template <int PRE>
__global__ __launch_bounds__(kBlock) void k_fin_cg_init(Sys S, int G, double rtol, double atol) {
    FIN_OFFSETS(S, G)
    double tot[3];
    reduce_partials<3>(part, G, tot);
    if (threadIdx.x != 0) return;
    // bit 0: missing or zero Jacobi diagonal, bit 1: negative one, bit 2:
    // invalid FSAI factor
    const bool neg = (st.bad_diag & 6) != 0;
    st.bad_diag &= 1;
    cg_step_init(st, tot[0], tot[1], PRE == PRE_FSAI ? 0.0 : tot[2], rtol, atol);
    if (neg && !st.done) {
        st.status = HSLA_BREAKDOWN;
        st.done = 1;
    }
}

// q = A p and partials of sigma = p.q.
template <int NS>
__global__ __launch_bounds__(kBlock) void k_cg_spmv_dot(Pat A, Sys S) {
    __shared__ double lds[kWavesPerBlock][kTileCap];
    SYS_OFFSETS(S, A)
    if (stopped(st)) return;
    const double *p = S.p + vo;
    double *q = S.q + vo;
    double acc[1] = {0.0};
    if constexpr (NS > 0) {
        // p of the row itself comes with the SpMV's gathers
        spmv_dia<NS>(A.sn, S.dia + (int64_t)sidx * dia_stored(NS, A.sn.nofs) * dia_chunks(A.n) * kDiaChunk,
                     (int64_t)A.n, p,
                     [&](int64_t row, double yv, double prow) {
                         st_nt(&q[row], yv);
                         acc[0] += prow * yv;
                     });
    } else {
        spmv_tiles(A.rp, A.col, A.sn, S.aval + (int64_t)sidx * A.nnz, p, A.meta, A.ntiles, lds[threadIdx.x / kWave],
                   [&](int64_t row, double yv) {
                       st_nt(&q[row], yv);
                       acc[0] += p[row] * yv;
                   });
    }
    block_partial<1>(acc, part);
}

// alpha = rho / sigma, or breakdown if sigma <= 0.
__global__ __launch_bounds__(kBlock) void k_fin_alpha(Sys S, int G) {
    FIN_OFFSETS(S, G)
    if (stopped(st)) return;
    double tot[1];
    reduce_partials<1>(part, G, tot);
    if (threadIdx.x != 0) return;
    cg_step_alpha(st, tot[0]);
}

// r -= alpha q; partials of r.r and r.z (Jacobi, scaled system: r holds
// S r, so the unscaled r.r is the sum of r_i^2 / S_i^2 = r_i^2 a_ii, with
// a_ii read as FP32 -- the norm only decides when to stop, and the 4-byte
// weights take an eighth off the sweep's bytes -- and r.z = r.r of the
// scaled vector).  x += alpha p of the same iteration is applied by the
// direction kernel, which reads p anyway, so p is read once per iteration.
template <int PRE>
__global__ __launch_bounds__(kBlock) void k_cg_update(Pat A, Sys S) {
    SYS_OFFSETS(S, A)
    if (stopped(st)) return;
    const double alpha = st.alpha;
    double *__restrict__ r = S.r + vo;
    const double *__restrict__ q = S.q + vo;
    const float *__restrict__ wt = reinterpret_cast<const float *>(S.z) + vo;
    double acc[2] = {0.0, 0.0};  // r.r, r.z
    auto elem = [&](double rv, double qv, float wv) {
        const double ri = rv - alpha * qv;
        if (PRE == PRE_JACOBI) {
            const double rr = ri * ri;
            acc[0] += rr * (double)wv;
            acc[1] += rr;
        } else {
            acc[0] += ri * ri;
        }
        return ri;
    };
    typedef float fpair __attribute__((ext_vector_type(2)));
    if (al16(r) && al16(q) && (PRE != PRE_JACOBI || ((uintptr_t)wt & 7u) == 0)) {
        const fpair one = {1.0f, 1.0f};
        PAIR_LOOP_BEGIN(A.n / 2)
                dpair rv[2], qv[2];
                fpair wv[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int64_t e = 2 * (i_ + j * S_);
                    rv[j] = ldp(r + e);
                    qv[j] = ldp(q + e);
                    wv[j] = PRE == PRE_JACOBI ? __builtin_nontemporal_load((const fpair *)(wt + e)) : one;
                }
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    dpair o;
                    o.x = elem(rv[j].x, qv[j].x, wv[j].x);
                    o.y = elem(rv[j].y, qv[j].y, wv[j].y);
                    stp(r + 2 * (i_ + j * S_), o);
                }
        PAIR_LOOP_TAIL
                const int64_t e = 2 * i_;
                const dpair rv = ldp(r + e), qv = ldp(q + e);
                const fpair wv = PRE == PRE_JACOBI ? __builtin_nontemporal_load((const fpair *)(wt + e)) : one;
                dpair o;
                o.x = elem(rv.x, qv.x, wv.x);
                o.y = elem(rv.y, qv.y, wv.y);
                stp(r + e, o);
        PAIR_LOOP_END
        if ((A.n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
            const int64_t e = A.n - 1;
            r[e] = elem(r[e], q[e], PRE == PRE_JACOBI ? wt[e] : 1.0f);
        }
    } else {
        GRID_LOOP_BEGIN(A.n)
                double rv[4], qv[4];
                float wv[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t e = i_ + j * S_;
                    rv[j] = r[e];
                    qv[j] = q[e];
                    wv[j] = PRE == PRE_JACOBI ? wt[e] : 1.0f;
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) r[i_ + j * S_] = elem(rv[j], qv[j], wv[j]);
        GRID_LOOP_TAIL
                r[i_] = elem(r[i_], q[i_], PRE == PRE_JACOBI ? wt[i_] : 1.0f);
        GRID_LOOP_END
    }
    if (PRE == PRE_NONE) acc[1] = acc[0];
    block_partial<2>(acc, part);
}

// Stop test on ||r||, then (Jacobi / none) rho' = r.z, beta = rho'/rho.  A
// system that stops here still has this iteration's x += alpha p to apply
// (xpend); one already stopped clears it.
template <int PRE>
__global__ __launch_bounds__(kBlock) void k_fin_beta(Sys S, int G) {
    FIN_OFFSETS(S, G)
    if (stopped(st)) {
        if (threadIdx.x == 0) st.xpend = 0;
        return;
    }
    double tot[2];
    reduce_partials<2>(part, G, tot);
    if (threadIdx.x != 0) return;
    cg_step_beta(st, tot[0], tot[1], PRE != PRE_FSAI);
}

// x += alpha p, then p = z + beta p with z = r (none, and Jacobi on the
// scaled system; FSAI runs its direction update inside the second half of
// its apply); a system that stopped in this iteration takes only the x
// update.  XUP = false: no x update.
template <int PRE, bool XUP = true>
__global__ __launch_bounds__(kBlock) void k_cg_direction(Pat A, Sys S) {
    SYS_OFFSETS(S, A)
    (void)part;
    const bool xonly = stopped(st);
    if (xonly && (!XUP || !st.xpend)) return;
    const double alpha = st.alpha, beta = st.beta;
    double *__restrict__ x = S.x + vo;
    double *__restrict__ p = S.p + vo;
    const double *__restrict__ r = S.r + vo;
    const double *__restrict__ z = S.z + vo;
    const double *__restrict__ zz = PRE == PRE_FSAI ? z : r;
    if (al16(x) && al16(p) && al16(zz)) {
        PAIR_LOOP_BEGIN(A.n / 2)
                dpair zv[2], pv[2], xv[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int64_t e = 2 * (i_ + j * S_);
                    pv[j] = ldp(p + e);
                    if (XUP) xv[j] = ldp(x + e);
                    if (!xonly) zv[j] = ldp(zz + e);
                }
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int64_t e = 2 * (i_ + j * S_);
                    if (XUP) stp(x + e, xv[j] + alpha * pv[j]);
                    if (!xonly) stp(p + e, zv[j] + beta * pv[j]);
                }
        PAIR_LOOP_TAIL
                const int64_t e = 2 * i_;
                const dpair pv = ldp(p + e);
                if (XUP) stp(x + e, ldp(x + e) + alpha * pv);
                if (!xonly) stp(p + e, ldp(zz + e) + beta * pv);
        PAIR_LOOP_END
        if ((A.n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
            const int64_t e = A.n - 1;
            const double pi = p[e];
            if (XUP) x[e] = x[e] + alpha * pi;
            if (!xonly) p[e] = zz[e] + beta * pi;
        }
        return;
    }
    if (xonly) {
        GRID_LOOP_BEGIN(A.n)
                double xv[4], pv[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t e = i_ + j * S_;
                    xv[j] = x[e];
                    pv[j] = p[e];
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) x[i_ + j * S_] = xv[j] + alpha * pv[j];
        GRID_LOOP_TAIL
                x[i_] = x[i_] + alpha * p[i_];
        GRID_LOOP_END
        return;
    }
    GRID_LOOP_BEGIN(A.n)
            double zv[4], pv[4], xv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t e = i_ + j * S_;
                zv[j] = zz[e];
                pv[j] = p[e];
                if (XUP) xv[j] = x[e];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t e = i_ + j * S_;
                if (XUP) x[e] = xv[j] + alpha * pv[j];
                p[e] = zv[j] + beta * pv[j];
            }
    GRID_LOOP_TAIL
            const double pi = p[i_];
            if (XUP) x[i_] = x[i_] + alpha * pi;
            p[i_] = zz[i_] + beta * pi;
    GRID_LOOP_END
}

// Jacobi on the scaled system: x = S x_scaled after the last iteration.
__global__ __launch_bounds__(kBlock) void k_cg_unscale(Pat A, Sys S) {
    SYS_OFFSETS(S, A)
    (void)part;
    (void)st;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < A.n; i += (int64_t)gridDim.x * kBlock)
        S.x[vo + i] = S.dinv[vo + i] * S.x[vo + i];
}

// ---------------------------------------------------------------------------
// Single-reduction CG (Chronopoulos and Gear), the roadmap the paper gives
// after its Algorithm "Distributed CG" for cutting synchronisation points
// (appendix "Distributed Conjugate Gradient and Halo Exchange").  With
// w = A r, gamma = r.r and delta = w.r of the same residual:
//   beta = gamma / gamma_old,  sigma = delta - beta gamma / alpha_old
//   (= p.Ap of the new direction),  alpha = gamma / sigma,
//   p = r + beta p,  s = w + beta s  (s = A p),  x += alpha p,  r -= alpha s.
// The same iterates as CG in exact arithmetic.  One iteration is three
// launches: the SpMV with both sums, one finalize, one vector sweep.  The
// sweep's ||r||^2 partials go to part2 and are read by the next finalize,
// which takes the stop test there (a stopped system's x is already final,
// one SpMV later).  Jacobi runs on the scaled system S A S as in CG.
// ---------------------------------------------------------------------------

// w = A r and partials of gamma = r.r, delta = w.r.
template <int NS>
__global__ __launch_bounds__(kBlock) void k_sr_spmv_dot(Pat A, Sys S) {
    __shared__ double lds[kWavesPerBlock][kTileCap];
    SYS_OFFSETS(S, A)
    if (stopped(st)) return;
    const double *r = S.r + vo;
    double *w = S.w + vo;
    double acc[2] = {0.0, 0.0};
    if constexpr (NS > 0) {
        spmv_dia<NS>(A.sn, S.dia + (int64_t)sidx * dia_stored(NS, A.sn.nofs) * dia_chunks(A.n) * kDiaChunk,
                     (int64_t)A.n, r,
                     [&](int64_t row, double yv, double rrow) {
                         st_nt(&w[row], yv);
                         acc[0] += rrow * rrow;
                         acc[1] += rrow * yv;
                     });
    } else {
        spmv_tiles(A.rp, A.col, A.sn, S.aval + (int64_t)sidx * A.nnz, r, A.meta, A.ntiles, lds[threadIdx.x / kWave],
                   [&](int64_t row, double yv) {
                       const double rv = r[row];
                       st_nt(&w[row], yv);
                       acc[0] += rv * rv;
                       acc[1] += rv * yv;
                   });
    }
    block_partial<2>(acc, part);
}

// Stop test on the last sweep's ||r|| (from part2, Gv partials; none before
// the first sweep), then beta, sigma and alpha from gamma and delta (Gs
// partials); sigma <= 0 is BREAKDOWN, as p.Ap <= 0 in CG.
__global__ __launch_bounds__(kBlock) void k_fin_sr(Sys S, int Gs, int Gv) {
    FIN_OFFSETS(S, Gs)
    if (stopped(st)) return;
    double tot[2];
    reduce_partials<2>(part, Gs, tot);
    double rr[1] = {0.0};
    const bool swept = st.sr_swept != 0;
    if (swept) reduce_partials<1>(S.part2 + (int64_t)sidx * Gv, Gv, rr);
    if (threadIdx.x != 0) return;
    if (swept) {
        cg_step_beta(st, rr[0], 0.0, false);
        if (st.done) return;
    }
    const double gamma = tot[0], delta = tot[1];
    double beta = 0.0, sigma = delta;
    if (swept) {
        beta = gamma / st.rho;
        sigma = delta - beta * gamma / st.alpha;
    }
    if (!isfinite(sigma) || !isfinite(gamma)) {
        st.status = HSLA_ERR_NONFINITE;
        st.done = 1;
    } else if (!(sigma > 0.0)) {
        st.status = HSLA_BREAKDOWN;
        st.done = 1;
    } else {
        st.beta = beta;
        st.alpha = gamma / sigma;
        st.rho = gamma;
        st.sr_swept = swept ? 2 : 1;  // 1: the coming sweep is the first
    }
}

// p = r + beta p; s = w + beta s; x += alpha p; r -= alpha s; partials of
// the unscaled ||r||^2 into part2 (Jacobi: r holds S r).
template <int PRE>
__global__ __launch_bounds__(kBlock) void k_sr_sweep(Pat A, Sys S) {
    SYS_OFFSETS(S, A)
    (void)part;
    if (stopped(st)) return;
    const double alpha = st.alpha, beta = st.beta;
    // the first sweep sets p = r and s = w without reading them (the work
    // vectors hold whatever an earlier call left there)
    const bool first = st.sr_swept == 1;
    double *__restrict__ x = S.x + vo;
    double *__restrict__ p = S.p + vo;
    double *__restrict__ sv = S.q + vo;
    double *__restrict__ r = S.r + vo;
    const double *__restrict__ w = S.w + vo;
    const double *__restrict__ dinv = S.dinv + vo;
    double acc[1] = {0.0};
    auto elem = [&](double &xv, double &pv, double &s_, double &rv, double wv, double dv) {
        pv = first ? rv : rv + beta * pv;
        s_ = first ? wv : wv + beta * s_;
        xv = xv + alpha * pv;
        rv = rv - alpha * s_;
        const double u = PRE == PRE_JACOBI ? rv / dv : rv;
        acc[0] += u * u;
    };
    auto pair_elem = [&](dpair &xv, dpair &pv, dpair &s_, dpair &rv, dpair wv, dpair dv) {
        double x0 = xv.x, p0 = pv.x, s0 = s_.x, r0 = rv.x, x1 = xv.y, p1 = pv.y, s1 = s_.y, r1 = rv.y;
        elem(x0, p0, s0, r0, wv.x, dv.x);
        elem(x1, p1, s1, r1, wv.y, dv.y);
        xv = dpair{x0, x1};
        pv = dpair{p0, p1};
        s_ = dpair{s0, s1};
        rv = dpair{r0, r1};
    };
    if (al16(x) && al16(p) && al16(sv) && al16(r) && al16(w) && (PRE != PRE_JACOBI || al16(dinv))) {
        const dpair one = {1.0, 1.0};
        PAIR_LOOP_BEGIN(A.n / 2)
                dpair xv[2], pv[2], sq[2], rv[2], wv[2], dv[2];
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int64_t e = 2 * (i_ + j * S_);
                    xv[j] = ldp(x + e);
                    pv[j] = ldp(p + e);
                    sq[j] = ldp(sv + e);
                    rv[j] = ldp(r + e);
                    wv[j] = ldp(w + e);
                    dv[j] = PRE == PRE_JACOBI ? ldp(dinv + e) : one;
                }
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int64_t e = 2 * (i_ + j * S_);
                    pair_elem(xv[j], pv[j], sq[j], rv[j], wv[j], dv[j]);
                    stp(x + e, xv[j]);
                    stp(p + e, pv[j]);
                    stp(sv + e, sq[j]);
                    stp(r + e, rv[j]);
                }
        PAIR_LOOP_TAIL
                const int64_t e = 2 * i_;
                dpair xv = ldp(x + e), pv = ldp(p + e), sq = ldp(sv + e), rv = ldp(r + e);
                const dpair wv = ldp(w + e), dv = PRE == PRE_JACOBI ? ldp(dinv + e) : one;
                pair_elem(xv, pv, sq, rv, wv, dv);
                stp(x + e, xv);
                stp(p + e, pv);
                stp(sv + e, sq);
                stp(r + e, rv);
        PAIR_LOOP_END
        if ((A.n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
            const int64_t e = A.n - 1;
            double xv = x[e], pv = p[e], sq = sv[e], rv = r[e];
            elem(xv, pv, sq, rv, w[e], PRE == PRE_JACOBI ? dinv[e] : 1.0);
            x[e] = xv;
            p[e] = pv;
            sv[e] = sq;
            r[e] = rv;
        }
    } else {
        GRID_LOOP_BEGIN(A.n)
                double xv[4], pv[4], sq[4], rv[4], wv[4], dv[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t e = i_ + j * S_;
                    xv[j] = x[e];
                    pv[j] = p[e];
                    sq[j] = sv[e];
                    rv[j] = r[e];
                    wv[j] = w[e];
                    dv[j] = PRE == PRE_JACOBI ? dinv[e] : 1.0;
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t e = i_ + j * S_;
                    elem(xv[j], pv[j], sq[j], rv[j], wv[j], dv[j]);
                    x[e] = xv[j];
                    p[e] = pv[j];
                    sv[e] = sq[j];
                    r[e] = rv[j];
                }
        GRID_LOOP_TAIL
                double xv = x[i_], pv = p[i_], sq = sv[i_], rv = r[i_];
                elem(xv, pv, sq, rv, w[i_], PRE == PRE_JACOBI ? dinv[i_] : 1.0);
                x[i_] = xv;
                p[i_] = pv;
                sv[i_] = sq;
                r[i_] = rv;
        GRID_LOOP_END
    }
    __shared__ double sh[kWavesPerBlock];
    block_sum<1>(acc, sh);
    if (threadIdx.x == 0) S.part2[(int64_t)sidx * gridDim.x + blockIdx.x] = acc[0];
}

// ---------------------------------------------------------------------------
// s-step CG: the communication-avoiding CG the paper names after Algorithm
// "Distributed CG" (appendix "Distributed Conjugate Gradient and Halo
// Exchange"), in Carson and Demmel's formulation of the s-step method of
// Chronopoulos and Gear, on the Jacobi-scaled operator S A S (unit
// diagonal).  One outer iteration: 2 SS - 1 SpMVs build the Chebyshev basis
// on [0, 2] of the Krylov spaces of p (T_0..T_SS) and r (T_0..T_{SS-1});
// one pass forms the Gram matrices Y^T Y and Y^T S^{-2} Y (the outer
// iteration's only reduction); one finalize block per system takes SS CG
// steps on coordinate vectors, with the stop test on the unscaled residual
// after every step; one sweep recovers x, r and p from the basis.
// ---------------------------------------------------------------------------
template <int SS>
struct SStep {
    static constexpr int NB = 2 * SS + 1;         // basis vectors
    static constexpr int NG = NB * (NB + 1) / 2;  // Gram entries, upper triangle by rows
    static constexpr int NGT = 2 * NG;            // plain and S^{-2}-weighted
};

// Basis vector k: 0 = p, 1..SS = T_k(p), SS + 1 = r, SS + 2..2 SS =
// T_{k-SS-1}(r); each a [B][n] array (Bn = B n).
template <int SS>
__device__ __forceinline__ const double *ss_vec(const Sys &S, int k, int64_t Bn) {
    return k == 0 ? S.p : k == SS + 1 ? S.r : S.ssb + (int64_t)(k <= SS ? k - 1 : k - 2) * Bn;
}

// out = (A - I) in (first), else 2 (A - I) in - prev: one step of the
// Chebyshev recurrence.
template <int NS>
__global__ __launch_bounds__(kBlock) void k_ss_basis(Pat A, Sys S, const double *in, const double *prev,
                                                     double *out, int first) {
    __shared__ double lds[kWavesPerBlock][kTileCap];
    SYS_OFFSETS(S, A)
    (void)part;
    if (stopped(st)) return;
    in += vo;
    prev += vo;
    out += vo;
    if constexpr (NS > 0) {
        spmv_A<NS>(A, S, sidx, in, lds[threadIdx.x / kWave], [&](int64_t row, double yv, double vrow) {
            const double t = yv - vrow;
            out[row] = first ? t : 2.0 * t - prev[row];
        });
    } else {
        spmv_A<NS>(A, S, sidx, in, lds[threadIdx.x / kWave], [&](int64_t row, double yv) {
            const double t = yv - in[row];
            out[row] = first ? t : 2.0 * t - prev[row];
        });
    }
}

// Partials of the Gram matrices over the basis (entry (a, b), a <= b, at
// a NB - a (a - 1) / 2 + b - a; the weighted ones NG further).
template <int SS>
__global__ __launch_bounds__(kBlock) void k_ss_gram(Pat A, Sys S) {
    using Q = SStep<SS>;
    const int sidx = blockIdx.y;
    const int64_t n = A.n, vo = (int64_t)sidx * n, Bn = (int64_t)gridDim.y * n;
    if (stopped(S.st[sidx])) return;
    const double *y[Q::NB];
#pragma unroll
    for (int k = 0; k < Q::NB; ++k) y[k] = ss_vec<SS>(S, k, Bn) + vo;
    const double *sc = S.dinv + vo;
    double acc[Q::NGT];
#pragma unroll
    for (int g = 0; g < Q::NGT; ++g) acc[g] = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        double v[Q::NB];
#pragma unroll
        for (int k = 0; k < Q::NB; ++k) v[k] = y[k][i];
        const double si = sc[i];
        const double wt = 1.0 / (si * si);  // r = S^{-1} r^: weight of the unscaled norm
        int g = 0;
#pragma unroll
        for (int a = 0; a < Q::NB; ++a) {
#pragma unroll
            for (int b = a; b < Q::NB; ++b) {
                const double pr = v[a] * v[b];
                acc[g] += pr;
                acc[Q::NG + g] += pr * wt;
                ++g;
            }
        }
    }
    block_partial<Q::NGT>(acc, S.ssp + (int64_t)sidx * Q::NGT * gridDim.x);
}

// u^T M v for the packed symmetric M (tot + off), fixed order.
template <int NB>
__device__ __forceinline__ double ss_form(const double *tot, int off, const double (&u)[NB], const double (&v)[NB]) {
    double acc = 0.0;
#pragma unroll
    for (int a = 0; a < NB; ++a) {
        double row = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int lo = a < b ? a : b, hi = a < b ? b : a;
            row += tot[off + lo * NB - lo * (lo - 1) / 2 + hi - lo] * v[b];
        }
        acc += u[a] * row;
    }
    return acc;
}

// out = B c: coordinates of A (Y c) (A T_0 = T_0 + T_1, A T_j = (T_{j-1} +
// T_{j+1}) / 2 + T_j in each block; a block's last vector is never mapped).
template <int SS>
__device__ __forceinline__ void ss_bmul(const double (&c)[SStep<SS>::NB], double (&out)[SStep<SS>::NB]) {
    constexpr int NB = SStep<SS>::NB;
#pragma unroll
    for (int k = 0; k < NB; ++k) out[k] = 0.0;
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
        const int start = blk == 0 ? 0 : SS + 1, len = blk == 0 ? SS + 1 : SS;
#pragma unroll
        for (int j = 0; j + 1 < len; ++j) {
            const int k = start + j;
            const double v = c[k];
            if (j == 0) {
                out[k] += v;
                out[k + 1] += v;
            } else {
                out[k - 1] += 0.5 * v;
                out[k] += v;
                out[k + 1] += 0.5 * v;
            }
        }
    }
}

// The SS inner steps of one outer iteration, on coordinates (thread 0 of a
// block per system); leaves the coordinates of x (increment), r and p.
template <int SS>
__global__ __launch_bounds__(kBlock) void k_fin_ss(Sys S, int G) {
    using Q = SStep<SS>;
    constexpr int NB = Q::NB;
    const int sidx = blockIdx.x;
    SysState &st = S.st[sidx];
    if (stopped(st)) {
        if (threadIdx.x == 0) st.xpend = 0;
        return;
    }
    double tot[Q::NGT];
    reduce_partials<Q::NGT>(S.ssp + (int64_t)sidx * Q::NGT * G, G, tot);
    if (threadIdx.x != 0) return;
    double pc[NB], rc[NB], xc[NB], bp[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) pc[k] = rc[k] = xc[k] = 0.0;
    pc[0] = 1.0;
    rc[SS + 1] = 1.0;
    double rho = ss_form<NB>(tot, 0, rc, rc);
    bool stop = false;
#pragma unroll
    for (int j = 0; j < SS; ++j) {
        if (stop) break;
        ss_bmul<SS>(pc, bp);
        const double sigma = ss_form<NB>(tot, 0, pc, bp);
        if (!isfinite(sigma)) {
            st.status = HSLA_ERR_NONFINITE;
            stop = true;
            break;
        }
        if (!(sigma > 0.0)) {
            st.status = HSLA_BREAKDOWN;
            stop = true;
            break;
        }
        const double alpha = rho / sigma;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            xc[k] = xc[k] + alpha * pc[k];
            rc[k] = rc[k] - alpha * bp[k];
        }
        st.iters += 1;
        const double rr = ss_form<NB>(tot, Q::NG, rc, rc);
        st.rnorm2 = rr > 0.0 ? rr : 0.0;
        if (!isfinite(rr)) {
            st.status = HSLA_ERR_NONFINITE;
            stop = true;
        } else if (sqrt(st.rnorm2) <= st.tol) {
            st.status = HSLA_OK;
            stop = true;
        } else if (st.iters >= st.max_iter) {
            st.status = HSLA_NOT_CONVERGED;
            stop = true;
        } else {
            const double rho_new = ss_form<NB>(tot, 0, rc, rc);
            const double beta = rho_new / rho;
            rho = rho_new;
#pragma unroll
            for (int k = 0; k < NB; ++k) pc[k] = rc[k] + beta * pc[k];
        }
    }
    if (stop) st.done = 1;
    st.xpend = 1;  // this outer iteration's recovery sweep applies x (and r, p)
    double *cf = S.ssc + (int64_t)sidx * 3 * NB;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        cf[k] = xc[k];
        cf[NB + k] = rc[k];
        cf[2 * NB + k] = pc[k];
    }
}

// x += Y x_c; r = Y r_c, p = Y p_c (a system that stopped takes x only).
template <int SS>
__global__ __launch_bounds__(kBlock) void k_ss_recover(Pat A, Sys S) {
    using Q = SStep<SS>;
    constexpr int NB = Q::NB;
    const int sidx = blockIdx.y;
    const int64_t n = A.n, vo = (int64_t)sidx * n, Bn = (int64_t)gridDim.y * n;
    const SysState &st = S.st[sidx];
    if (st.done && !st.xpend) return;
    const bool full = !st.done;
    const double *cf = S.ssc + (int64_t)sidx * 3 * NB;
    double xc[NB], rc[NB], pc[NB];
    const double *y[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        xc[k] = cf[k];
        rc[k] = cf[NB + k];
        pc[k] = cf[2 * NB + k];
        y[k] = ss_vec<SS>(S, k, Bn) + vo;
    }
    double *x = S.x + vo, *r = S.r + vo, *p = S.p + vo;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        double v[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) v[k] = y[k][i];
        double xs = 0.0, rs = 0.0, ps = 0.0;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            xs += xc[k] * v[k];
            rs += rc[k] * v[k];
            ps += pc[k] * v[k];
        }
        x[i] = x[i] + xs;
        if (full) {
            r[i] = rs;
            p[i] = ps;
        }
    }
}

// The operator S A S of the scaled system on CSR values (tile form): each
// entry times S_row S_col, the diagonal 1 by construction.
__global__ __launch_bounds__(kBlock) void k_scale_sym(int32_t n, int64_t nnz, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ col, const double *__restrict__ val,
                                                      const double *__restrict__ sc, double *__restrict__ out) {
    const int sidx = blockIdx.y;
    const double *v = val + (int64_t)sidx * nnz;
    const double *sv = sc + (int64_t)sidx * n;
    double *o = out + (int64_t)sidx * nnz;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) o[k] = col[k] == i ? 1.0 : v[k] * (sv[i] * sv[col[k]]);
}

// FSAI apply, first half: w = G r (G lower, float32 values, FP64 products)
// and partials of r.z = r^T G^T G r = w.w, so the second half needs no r.
template <int NS>
__global__ __launch_bounds__(kBlock) void k_fsai_lower_dot(Pat A, FPat L, Sys S) {
    __shared__ double lds[kWavesPerBlock][kTileCap];
    SYS_OFFSETS(S, A)
    if (stopped(st)) return;
    const double *r = S.r + vo;
    double *w = S.w + vo;
    double acc[1] = {0.0};
    spmv_F<NS>(L, A.n, sidx, r, lds[threadIdx.x / kWave],
               [&](int64_t row, double yv) {
                   st_nt(&w[row], yv);
                   acc[0] += yv * yv;
               });
    block_partial<1>(acc, part);
}

// The FSAI factor of each system must have finite values and end every
// row of its lower pattern with a positive diagonal entry (G nonsingular, so
// M^{-1} = G^T G is SPD); a system whose factor fails is flagged (bit 2 of
// bad_diag) and stops with BREAKDOWN before its first iteration.
__global__ __launch_bounds__(kBlock) void k_fsai_check(FPat L, Sys S, int32_t n) {
    const int sidx = blockIdx.y;
    const float *__restrict__ g = L.val + (int64_t)sidx * L.nnz;
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const int32_t lo = L.rp[i], hi = L.rp[i + 1];
        if (hi <= lo || L.col[hi - 1] != i || !(g[hi - 1] > 0.0f)) bad = true;
        for (int32_t k = lo; k < hi; ++k)
            if (!isfinite(g[k])) bad = true;
    }
    if (__syncthreads_or(bad ? 1 : 0) && threadIdx.x == 0) atomicOr(&S.st[sidx].bad_diag, 4);
}

// FSAI apply, second half, with CG's direction update: z = G^T w, then
// x += alpha p and p = z + beta p row by row (z itself is never stored).
// beta = (r.z)'/(r.z) is known by then: r.z = w.w comes from the first half.
// XUP = false (the start, p = z): no x update.  A system that stopped with
// its last x update pending takes only that.
template <bool XUP>
struct UpperDirEpi : OwnRowsEpi {
    double *__restrict__ x;
    double *__restrict__ p;
    double alpha, beta;
    struct One {
        double x, p;
    };
    __device__ One load_one(int64_t i) const {
        return {XUP ? __builtin_nontemporal_load(x + i) : 0.0, __builtin_nontemporal_load(p + i)};
    }
    __device__ void one(int64_t i, double z, const One &o) const {
        if (XUP) st_nt(&x[i], o.x + alpha * o.p);
        st_nt(&p[i], z + beta * o.p);
    }
    __device__ void operator()(int64_t i, double z) const { one(i, z, load_one(i)); }
};

template <int NS, bool XUP>
__device__ __forceinline__ void fsai_upper_dir(const Pat &A, const FPat &U, const Sys &S) {
    __shared__ double lds[kWavesPerBlock][kTileCap];
    SYS_OFFSETS(S, A)
    (void)part;
    const bool xonly = stopped(st);
    if (xonly && (!XUP || !st.xpend)) return;
    double *x = S.x + vo;
    double *p = S.p + vo;
    const double alpha = st.alpha;
    if (xonly) {
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < A.n; i += (int64_t)gridDim.x * kBlock)
            x[i] = x[i] + alpha * p[i];
        return;
    }
    spmv_F<NS>(U, A.n, sidx, S.w + vo, lds[threadIdx.x / kWave], UpperDirEpi<XUP>{{}, x, p, alpha, st.beta});
}

template <int NS>
__global__ __launch_bounds__(kBlock) void k_fsai_upper_dir(Pat A, FPat U, Sys S) {
    fsai_upper_dir<NS, true>(A, U, S);
}

template <int NS>
__global__ __launch_bounds__(kBlock) void k_fsai_upper_start(Pat A, FPat U, Sys S) {
    fsai_upper_dir<NS, false>(A, U, S);
}

// Set-up: rho = r.z (p = z follows from beta = 0 and p = 0); iteration:
// beta = rho'/rho, rho = rho'.
__global__ __launch_bounds__(kBlock) void k_fin_fsai(Sys S, int G, int setup) {
    FIN_OFFSETS(S, G)
    if (stopped(st)) return;
    double tot[1];
    reduce_partials<1>(part, G, tot);
    if (threadIdx.x != 0) return;
    if (!isfinite(tot[0])) {
        st.status = HSLA_ERR_NONFINITE;
        st.done = 1;
        st.xpend = setup ? 0 : 1;
    } else if (setup) {
        st.rho = tot[0];
        st.beta = 0.0;
    } else {
        st.beta = tot[0] / st.rho;
        st.rho = tot[0];
    }
}

// ---------------------------------------------------------------------------
// BiCGStab (right preconditioning with D^{-1} or none)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void bicg_breakdown(SysState &st) {
    if (st.restarts == 0) {
        // restart from the current iterate: r_hat = r, p = v = 0,
        // rho = alpha = omega = 1, so rho' = r.r and p = r next
        st.restarts = 1;
        st.restart_pending = 1;
        st.rho = 1.0;
        st.alpha = 1.0;
        st.omega = 1.0;
        st.rho_new = st.rnorm2;
        if (st.rho_new == 0.0) {
            st.status = HSLA_BREAKDOWN;
            st.done = 1;
        }
    } else {
        st.status = HSLA_BREAKDOWN;
        st.done = 1;
    }
}

template <int PRE>
__global__ __launch_bounds__(kBlock) void k_bicg_init(Pat A, Sys S, int use_x0) {
    SYS_OFFSETS(S, A)
    const double *val = S.val + sidx * A.nnz;
    double acc[2] = {0.0, 0.0};  // b.b, r.r
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < A.n; i += (int64_t)gridDim.x * kBlock) {
        const int64_t j = vo + i;
        const double bi = S.b[j];
        const double ri = use_x0 ? bi - S.q[j] : bi;
        if (!use_x0) S.x[j] = 0.0;
        S.r[j] = ri;
        S.rh[j] = ri;
        S.p[j] = 0.0;
        S.v[j] = 0.0;
        S.y[j] = 0.0;
        if (PRE == PRE_JACOBI) {
            const int32_t d = A.diag[i];
            const double a = d >= 0 ? val[d] : 0.0;
            if (a == 0.0) bad = true;
            S.dinv[j] = 1.0 / a;
        }
        acc[0] += bi * bi;
        acc[1] += ri * ri;
    }
    if (bad) st.bad_diag = 1;
    block_partial<2>(acc, part);
}

__global__ __launch_bounds__(kBlock) void k_fin_bicg_init(Sys S, int G, double rtol, double atol) {
    FIN_OFFSETS(S, G)
    double tot[2];
    reduce_partials<2>(part, G, tot);
    if (threadIdx.x != 0) return;
    const double bn = sqrt(tot[0]);
    double tol = rtol * bn;
    if (atol > tol) tol = atol;
    st.bnorm = bn;
    st.tol = tol;
    st.rnorm2 = tot[1];
    st.win_rr = tot[1];
    st.win_it = 0;
    const double rn = sqrt(tot[1]);
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
        st.rho_new = tot[1];  // r_hat.r with r_hat = r
        st.beta = (st.rho_new / st.rho) * (st.alpha / st.omega);
    }
}

// Right preconditioning runs on the operator A M^{-1} (M = D for Jacobi, I
// otherwise; its values are copied once per solve with the columns scaled
// by D^{-1}): the recurrence iterates y for A M^{-1} y = b - A x0 with
// v = (A M^{-1}) p and t = (A M^{-1}) s, so p_hat = M^{-1} p and s_hat =
// M^{-1} s are never formed, and x = x0 + M^{-1} y once at the end.

// p = r + beta (p - omega v) (after a restart: r_hat = r, p = r).
__global__ __launch_bounds__(kBlock) void k_bicg_dir(Pat A, Sys S) {
    SYS_OFFSETS(S, A)
    (void)part;
    if (stopped(st)) return;
    const double beta = st.beta, omega = st.omega;
    const int restart = st.restart_pending;
    const double *__restrict__ r = S.r + vo;
    const double *__restrict__ v = S.v + vo;
    double *__restrict__ p = S.p + vo;
    double *__restrict__ rh = S.rh + vo;
    if (restart) {
        GRID_LOOP_BEGIN(A.n)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t e = i_ + j * S_;
                    const double ri = r[e];
                    rh[e] = ri;
                    p[e] = ri;
                }
        GRID_LOOP_TAIL
                const double ri = r[i_];
                rh[i_] = ri;
                p[i_] = ri;
        GRID_LOOP_END
        return;
    }
    GRID_LOOP_BEGIN(A.n)
            double rv[4], pv[4], vv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t e = i_ + j * S_;
                rv[j] = r[e]; pv[j] = p[e]; vv[j] = v[e];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) p[i_ + j * S_] = rv[j] + beta * (pv[j] - omega * vv[j]);
    GRID_LOOP_TAIL
            p[i_] = r[i_] + beta * (p[i_] - omega * v[i_]);
    GRID_LOOP_END
}

// v = (A M^{-1}) p and partials of r_hat.v.
template <int NS>
__global__ __launch_bounds__(kBlock) void k_bicg_spmv_v(Pat A, Sys S) {
    __shared__ double lds[kWavesPerBlock][kTileCap];
    SYS_OFFSETS(S, A)
    if (stopped(st)) return;
    const double *p = S.p + vo;
    const double *rh = S.rh + vo;
    double *v = S.v + vo;
    double acc[1] = {0.0};
    spmv_A<NS>(A, S, sidx, p, lds[threadIdx.x / kWave],
               [&](int64_t row, double yv) {
                   st_nt(&v[row], yv);
                   acc[0] += rh[row] * yv;
               });
    block_partial<1>(acc, part);
}

// alpha = rho' / (r_hat.v); clears a pending restart (it ran in k_bicg_dir).
__global__ __launch_bounds__(kBlock) void k_fin_bicg_v(Sys S, int G) {
    FIN_OFFSETS(S, G)
    if (stopped(st)) return;
    double tot[1];
    reduce_partials<1>(part, G, tot);
    if (threadIdx.x != 0) return;
    st.restart_pending = 0;
    const double rv = tot[0];
    if (!isfinite(rv)) {
        st.status = HSLA_ERR_NONFINITE;
        st.done = 1;
    } else if (rv == 0.0) {
        bicg_breakdown(st);
    } else {
        st.alpha = st.rho_new / rv;
    }
}

// s = r - alpha v and partials of s.s.
__global__ __launch_bounds__(kBlock) void k_bicg_s(Pat A, Sys S) {
    SYS_OFFSETS(S, A)
    if (stopped(st) || st.restart_pending) return;
    const double alpha = st.alpha;
    const double *__restrict__ r = S.r + vo;
    const double *__restrict__ v = S.v + vo;
    double *__restrict__ s = S.s + vo;
    double acc[1] = {0.0};
    GRID_LOOP_BEGIN(A.n)
            double rv[4], vv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t e = i_ + j * S_;
                rv[j] = r[e]; vv[j] = v[e];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double si = rv[j] - alpha * vv[j];
                s[i_ + j * S_] = si;
                acc[0] += si * si;
            }
    GRID_LOOP_TAIL
            const double si = r[i_] - alpha * v[i_];
            s[i_] = si;
            acc[0] += si * si;
    GRID_LOOP_END
    block_partial<1>(acc, part);
}

// Counts the iteration; ||s|| <= tol finishes the solve in the update kernel
// with y += alpha p.
__global__ __launch_bounds__(kBlock) void k_fin_bicg_s(Sys S, int G) {
    FIN_OFFSETS(S, G)
    if (stopped(st) || st.restart_pending) return;
    double tot[1];
    reduce_partials<1>(part, G, tot);
    if (threadIdx.x != 0) return;
    st.iters += 1;
    st.snorm2 = tot[0];
    const double sn = sqrt(tot[0]);
    if (!isfinite(sn)) {
        st.status = HSLA_ERR_NONFINITE;
        st.done = 1;
    } else if (sn <= st.tol) {
        st.s_exit = 1;
    }
}

// t = (A M^{-1}) s and partials of t.s, t.t (the diagonal-major walk hands
// over s of the row itself with its gathers).
template <int NS>
__global__ __launch_bounds__(kBlock) void k_bicg_spmv_t(Pat A, Sys S) {
    __shared__ double lds[kWavesPerBlock][kTileCap];
    SYS_OFFSETS(S, A)
    if (stopped(st) || st.restart_pending || st.s_exit) return;
    const double *s = S.s + vo;
    double *t = S.t + vo;
    double acc[2] = {0.0, 0.0};
    if constexpr (NS > 0) {
        spmv_A<NS>(A, S, sidx, s, lds[threadIdx.x / kWave],
                   [&](int64_t row, double yv, double srow) {
                       st_nt(&t[row], yv);
                       acc[0] += yv * srow;
                       acc[1] += yv * yv;
                   });
    } else {
        spmv_A<NS>(A, S, sidx, s, lds[threadIdx.x / kWave],
                   [&](int64_t row, double yv) {
                       st_nt(&t[row], yv);
                       acc[0] += yv * s[row];
                       acc[1] += yv * yv;
                   });
    }
    block_partial<2>(acc, part);
}

// omega = t.s / t.t.
__global__ __launch_bounds__(kBlock) void k_fin_bicg_t(Sys S, int G) {
    FIN_OFFSETS(S, G)
    if (stopped(st) || st.restart_pending || st.s_exit) return;
    double tot[2];
    reduce_partials<2>(part, G, tot);
    if (threadIdx.x != 0) return;
    if (!isfinite(tot[0]) || !isfinite(tot[1])) {
        st.status = HSLA_ERR_NONFINITE;
        st.done = 1;
    } else if (tot[1] == 0.0) {
        bicg_breakdown(st);
    } else {
        st.omega = tot[0] / tot[1];
    }
}

// y += alpha p + omega s, r = s - omega t (or, after the s test, y += alpha
// p, r = s); partials of r.r and r_hat.r.
__global__ __launch_bounds__(kBlock) void k_bicg_update(Pat A, Sys S) {
    SYS_OFFSETS(S, A)
    if (stopped(st) || st.restart_pending) return;
    const double alpha = st.alpha, omega = st.omega;
    const int sx = st.s_exit;
    double *__restrict__ y = S.y + vo;
    double *__restrict__ r = S.r + vo;
    const double *__restrict__ p = S.p + vo;
    const double *__restrict__ s = S.s + vo;
    const double *__restrict__ t = S.t + vo;
    const double *__restrict__ rh = S.rh + vo;
    double acc[2] = {0.0, 0.0};  // r.r, r_hat.r
    if (sx) {
        GRID_LOOP_BEGIN(A.n)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t e = i_ + j * S_;
                    y[e] = y[e] + alpha * p[e];
                    r[e] = s[e];
                }
        GRID_LOOP_TAIL
                y[i_] = y[i_] + alpha * p[i_];
                r[i_] = s[i_];
        GRID_LOOP_END
    } else {
        GRID_LOOP_BEGIN(A.n)
                double yv[4], pv[4], sv[4], tv[4], rhv[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t e = i_ + j * S_;
                    yv[j] = y[e]; pv[j] = p[e]; sv[j] = s[e]; tv[j] = t[e]; rhv[j] = rh[e];
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int64_t e = i_ + j * S_;
                    y[e] = yv[j] + (alpha * pv[j] + omega * sv[j]);
                    const double ri = sv[j] - omega * tv[j];
                    r[e] = ri;
                    acc[0] += ri * ri;
                    acc[1] += rhv[j] * ri;
                }
        GRID_LOOP_TAIL
                y[i_] = y[i_] + (alpha * p[i_] + omega * s[i_]);
                const double ri = s[i_] - omega * t[i_];
                r[i_] = ri;
                acc[0] += ri * ri;
                acc[1] += rh[i_] * ri;
        GRID_LOOP_END
    }
    block_partial<2>(acc, part);
}

// x = x0 + M^{-1} y after the last iteration.
template <int PRE>
__global__ __launch_bounds__(kBlock) void k_bicg_finish(Pat A, Sys S) {
    SYS_OFFSETS(S, A)
    (void)part;
    (void)st;
    double *__restrict__ x = S.x + vo;
    const double *__restrict__ y = S.y + vo;
    const double *__restrict__ dinv = S.dinv + vo;
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < A.n; i += (int64_t)gridDim.x * kBlock)
        x[i] = x[i] + (PRE == PRE_JACOBI ? dinv[i] * y[i] : y[i]);
}

// Stop test on ||r||, then rho' = r_hat.r and beta = (rho'/rho)(alpha/omega).
__global__ __launch_bounds__(kBlock) void k_fin_bicg_update(Sys S, int G) {
    FIN_OFFSETS(S, G)
    if (stopped(st) || st.restart_pending) return;
    double tot[2];
    reduce_partials<2>(part, G, tot);
    if (threadIdx.x != 0) return;
    const double omega = st.omega;
    st.rnorm2 = tot[0];
    const double rn = sqrt(tot[0]);
    if (st.s_exit) {
        st.status = HSLA_OK;
        st.done = 1;
        st.rnorm2 = st.snorm2;
    } else if (!isfinite(rn)) {
        st.status = HSLA_ERR_NONFINITE;
        st.done = 1;
    } else if (rn <= st.tol) {
        st.status = HSLA_OK;
        st.done = 1;
    } else if (omega == 0.0) {
        bicg_breakdown(st);
    } else if (st.iters >= st.max_iter) {
        st.status = HSLA_NOT_CONVERGED;
        st.done = 1;
    } else if (stall_step(st, tot[0])) {
        st.status = HSLA_STAGNATED;
        st.done = 1;
    } else {
        st.rho = st.rho_new;
        st.rho_new = tot[1];
        if (!isfinite(st.rho_new)) {
            st.status = HSLA_ERR_NONFINITE;
            st.done = 1;
        } else if (st.rho_new == 0.0) {
            bicg_breakdown(st);
        } else {
            st.beta = (st.rho_new / st.rho) * (st.alpha / st.omega);
        }
    }
}

// ---------------------------------------------------------------------------
// Residual, symmetry and adjoint helpers
// ---------------------------------------------------------------------------

// Partials of ||b - A x||^2 and ||b||^2 per system.
__global__ __launch_bounds__(kBlock) void k_residual(Pat A, Sys S) {
    __shared__ double lds[kWavesPerBlock][kTileCap];
    SYS_OFFSETS(S, A)
    (void)st;
    const double *val = S.val + sidx * A.nnz;
    const double *x = S.x + vo;
    const double *b = S.b + vo;
    double acc[2] = {0.0, 0.0};
    spmv_tiles(A.rp, A.col, A.sn, val, x, A.meta, A.ntiles, lds[threadIdx.x / kWave],
               [&](int32_t row, double yv) {
                   const double e = b[row] - yv;
                   acc[0] += e * e;
                   acc[1] += b[row] * b[row];
               });
    block_partial<2>(acc, part);
}

__global__ __launch_bounds__(kBlock) void k_fin_residual(Sys S, int G, double *out) {
    FIN_OFFSETS(S, G)
    (void)st;
    double tot[2];
    reduce_partials<2>(part, G, tot);
    if (threadIdx.x != 0) return;
    out[2 * sidx] = tot[0];
    out[2 * sidx + 1] = tot[1];
}

// flag = 1 if val[s][src[k]] != val[s][k] for some system and entry.
__global__ __launch_bounds__(kBlock) void k_value_asym(int64_t nnz, int B, const double *__restrict__ val,
                                                       const int32_t *__restrict__ src, int32_t *flag) {
    const int64_t total = nnz * B;
    bool diff = false;
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBlock) {
        const int64_t s = e / nnz, k = e - s * nnz;
        if (!(val[s * nnz + src[k]] == val[e])) diff = true;
    }
    if (diff) *flag = 1;
}

// out[s][k] = in[s][src[k]]
__global__ __launch_bounds__(kBlock) void k_gather_values(int64_t nnz, int B, const double *__restrict__ in,
                                                          const int32_t *__restrict__ src, double *__restrict__ out) {
    const int64_t total = nnz * B;
    for (int64_t e = blockIdx.x * (int64_t)kBlock + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBlock) {
        const int64_t s = e / nnz, k = e - s * nnz;
        out[e] = in[s * nnz + src[k]];
    }
}

// Eq. adjoint_linear on the pattern: gA[s][k] = -lambda[s][row(k)] * x[s][col(k)].
__global__ __launch_bounds__(kBlock) void k_outer(int32_t n, int64_t nnz, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col, const double *__restrict__ lam,
                                                  const double *__restrict__ x, double *__restrict__ gA) {
    const int64_t sidx = blockIdx.y;
    lam += sidx * n;
    x += sidx * n;
    gA += sidx * nnz;
    for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        const double li = -lam[i];
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) gA[k] = li * x[col[k]];
    }
}

// ---------------------------------------------------------------------------
// Host drivers
// ---------------------------------------------------------------------------

struct Layout {
    size_t off_state, off_part, off_vec, off_res, off_extra, total;
    int gmax;  // partials per value and system; part2 starts 3 gmax B doubles past off_part
};

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static Layout make_layout(int B, int64_t n, int nvec, int G, size_t extra = 0) {
    Layout L{};
    size_t o = 0;
    L.off_state = o;
    o = align_up(o + sizeof(SysState) * B, 256);
    L.off_part = o;
    L.gmax = G;
    o = align_up(o + sizeof(double) * 4 * (size_t)G * B, 256);
    L.off_res = o;
    o = align_up(o + sizeof(double) * 2 * (size_t)B, 256);
    L.off_vec = o;
    o = align_up(o + sizeof(double) * (size_t)nvec * B * (size_t)n, 256);
    L.off_extra = o;
    o = align_up(o + extra, 256);
    L.total = o;
    return L;
}

__global__ __launch_bounds__(kBlock) void k_fill_f64(double *__restrict__ a, int64_t m, double v) {
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < m; i += (int64_t)gridDim.x * kBlock) a[i] = v;
}

// Launches K<NS> for the diagonal-major slot count `ns` (0 = tile walk).
#define NS_LAUNCH(K, ns, grid, ...)                                       \
    switch (ns) {                                                         \
        case 0: K<0><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break;         \
        case 4: K<4><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break;         \
        case 5: K<5><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break;         \
        case 7: K<7><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break;         \
        case 8: K<8><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break;         \
        case 9: K<9><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break;         \
        case 12: K<12><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break;       \
        default: K<16><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break;       \
    }

// NS_LAUNCH plus the half form's slot counts, for the SpMV kernels on A.
#define NS_LAUNCH_A(K, ns, grid, ...)                                           \
    switch (ns) {                                                               \
        case kSymNS + 5: K<kSymNS + 5><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break; \
        case kSymNS + 7: K<kSymNS + 7><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break; \
        case kSymNS + 9: K<kSymNS + 9><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break; \
        case kUnitNS + 5: K<kUnitNS + 5><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break; \
        case kUnitNS + 7: K<kUnitNS + 7><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break; \
        case kUnitNS + 9: K<kUnitNS + 9><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break; \
        case kUnitFullNS + 5: K<kUnitFullNS + 5><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break; \
        case kUnitFullNS + 7: K<kUnitFullNS + 7><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break; \
        case kUnitFullNS + 9: K<kUnitFullNS + 9><<<grid, kBlock, 0, s>>>(__VA_ARGS__); break; \
        default: NS_LAUNCH(K, ns, grid, __VA_ARGS__);                          \
    }

static hsla_status values_symmetric(hsla_handle *h, const hsla_pattern *p, int B, const double *values, hipStream_t s,
                                    bool *sym);

hsla_status launch_spmv(hsla_handle *h, const hsla_pattern *p, int B, const double *values, const double *x,
                        double *y, hipStream_t s) {
    if (p->n == 0 || B == 0) return HSLA_OK;
    Pat A = pat_of(p);
    if (p->format == HSLA_FORMAT_DIAGONAL && A.sn.mask) {
        // the half form where the values allow it, else the full copy
        bool half = false;
        if (stencil_half_ok(A.sn)) {
            const hsla_status st = values_symmetric(h, p, B, values, s, &half);
            if (st != HSLA_OK) return st;
        }
        const int ns = half ? kSymNS + A.sn.nofs : dia_slots_for(A.sn.nofs);
        const size_t rows = (size_t)dia_chunks(A.n) * kDiaChunk;
        const hsla_status st = ensure_workspace(h, sizeof(double) * (size_t)B * dia_stored(ns, A.sn.nofs) * rows);
        if (st != HSLA_OK) return st;
        double *dia = (double *)h->ws;
        const int Gv = grid_blocks(h, kBlock * 4, A.n, B, 8);
        A.sn.pencil = pencil_len(A.sn, A.n, B, h->dev.num_cu);
        const int Gd = grid_blocks(h, half ? (int64_t)kDiaChunk * A.sn.pencil : kDiaChunk, A.n, B, 8);
        if (half)
            k_to_dia_sym<double><<<dim3(Gv, B), kBlock, 0, s>>>(A.n, A.rp, A.sn, A.nnz, values, dia);
        else
            k_to_dia<double><<<dim3(Gv, B), kBlock, 0, s>>>(A.n, A.rp, A.sn, A.nnz, values, dia);
        const dim3 gd(Gd, B);
        NS_LAUNCH_A(k_spmv_dia, ns, gd, A, dia, x, y);
        HSLA_HIP(h, hipGetLastError());
        return HSLA_OK;
    }
    const int G = grid_blocks(h, kWavesPerBlock, p->ntiles, B, 16);
    k_spmv<<<dim3(G, B), kBlock, 0, s>>>(A, values, x, y);
    HSLA_HIP(h, hipGetLastError());
    return HSLA_OK;
}

struct SolveCall {
    Pat A;
    FPat L, U;
    Sys S;
    int B;
    int method;   // HSLA_METHOD_CG / BICGSTAB
    int precond;  // PRE_*
    int Gt, Gv;   // blocks per system: SpMV-based kernels, vector kernels
    int nsA, nsF; // slot counts of the diagonal-major SpMV of A and of the FSAI factors (0: tiles)
    int Gs, Gf;   // blocks per system of the A-SpMV and FSAI kernels
    int sr;       // CG with the single-reduction recurrence (no or Jacobi preconditioner)
    int ss;       // s-step CG: inner steps per outer iteration (0: off; Jacobi only)
};



// Enqueues `iters` iterations.  With `ev` (profile mode) the SpMV(+dot)
// launch of iteration k is bracketed by ev[2k], ev[2k+1].  Every reducing
// kernel is followed by its one-block-per-system finalize kernel.
static void enqueue_iterations(const SolveCall &c, int iters, hipStream_t s, hipEvent_t *ev) {
    const dim3 gs(c.Gs, c.B), gfs(c.Gf, c.B), gv(c.Gv, c.B), gf(c.B);
    const int Gs = c.Gs, Gfs = c.Gf, Gv = c.Gv;
    for (int k = 0; k < iters; ++k) {
        if (c.method == HSLA_METHOD_CG && c.ss) {
            // one outer iteration (c.ss inner steps)
            const Sys &S = c.S;
            const int64_t Bn = (int64_t)c.B * c.A.n;
            for (int blk = 0; blk < 2; ++blk) {
                const double *v0 = blk == 0 ? S.p : S.r;
                double *base = S.ssb + (blk == 0 ? 0 : (int64_t)c.ss * Bn);
                const int len = blk == 0 ? c.ss + 1 : c.ss;
                for (int j = 1; j < len; ++j) {
                    const double *in = j == 1 ? v0 : base + (int64_t)(j - 2) * Bn;
                    const double *prev = j == 1 ? v0 : j == 2 ? v0 : base + (int64_t)(j - 3) * Bn;
                    double *out = base + (int64_t)(j - 1) * Bn;
                    NS_LAUNCH_A(k_ss_basis, c.nsA, gs, c.A, c.S, in, prev, out, j == 1 ? 1 : 0);
                }
            }
            switch (c.ss) {
                case 2:
                    k_ss_gram<2><<<gv, kBlock, 0, s>>>(c.A, c.S);
                    k_fin_ss<2><<<gf, kBlock, 0, s>>>(c.S, Gv);
                    k_ss_recover<2><<<gv, kBlock, 0, s>>>(c.A, c.S);
                    break;
                case 3:
                    k_ss_gram<3><<<gv, kBlock, 0, s>>>(c.A, c.S);
                    k_fin_ss<3><<<gf, kBlock, 0, s>>>(c.S, Gv);
                    k_ss_recover<3><<<gv, kBlock, 0, s>>>(c.A, c.S);
                    break;
                default:
                    k_ss_gram<4><<<gv, kBlock, 0, s>>>(c.A, c.S);
                    k_fin_ss<4><<<gf, kBlock, 0, s>>>(c.S, Gv);
                    k_ss_recover<4><<<gv, kBlock, 0, s>>>(c.A, c.S);
                    break;
            }
        } else if (c.method == HSLA_METHOD_CG && c.sr) {
            if (ev) (void)hipEventRecord(ev[2 * k], s);
            NS_LAUNCH_A(k_sr_spmv_dot, c.nsA, gs, c.A, c.S);
            if (ev) (void)hipEventRecord(ev[2 * k + 1], s);
            k_fin_sr<<<gf, kBlock, 0, s>>>(c.S, Gs, Gv);
            if (c.precond == PRE_JACOBI)
                k_sr_sweep<PRE_JACOBI><<<gv, kBlock, 0, s>>>(c.A, c.S);
            else
                k_sr_sweep<PRE_NONE><<<gv, kBlock, 0, s>>>(c.A, c.S);
        } else if (c.method == HSLA_METHOD_CG) {
            if (ev) (void)hipEventRecord(ev[2 * k], s);
            NS_LAUNCH_A(k_cg_spmv_dot, c.nsA, gs, c.A, c.S);
            if (ev) (void)hipEventRecord(ev[2 * k + 1], s);
            k_fin_alpha<<<gf, kBlock, 0, s>>>(c.S, Gs);
            switch (c.precond) {
                case PRE_NONE:
                    k_cg_update<PRE_NONE><<<gv, kBlock, 0, s>>>(c.A, c.S);
                    k_fin_beta<PRE_NONE><<<gf, kBlock, 0, s>>>(c.S, Gv);
                    k_cg_direction<PRE_NONE><<<gv, kBlock, 0, s>>>(c.A, c.S);
                    break;
                case PRE_JACOBI:
                    k_cg_update<PRE_JACOBI><<<gv, kBlock, 0, s>>>(c.A, c.S);
                    k_fin_beta<PRE_JACOBI><<<gf, kBlock, 0, s>>>(c.S, Gv);
                    k_cg_direction<PRE_JACOBI><<<gv, kBlock, 0, s>>>(c.A, c.S);
                    break;
                default:
                    k_cg_update<PRE_FSAI><<<gv, kBlock, 0, s>>>(c.A, c.S);
                    k_fin_beta<PRE_FSAI><<<gf, kBlock, 0, s>>>(c.S, Gv);
                    NS_LAUNCH(k_fsai_lower_dot, c.nsF, gfs, c.A, c.L, c.S);
                    k_fin_fsai<<<gf, kBlock, 0, s>>>(c.S, Gfs, 0);
                    NS_LAUNCH(k_fsai_upper_dir, c.nsF, gfs, c.A, c.U, c.S);
                    break;
            }
        } else {
            k_bicg_dir<<<gv, kBlock, 0, s>>>(c.A, c.S);
            if (ev) (void)hipEventRecord(ev[2 * k], s);
            NS_LAUNCH_A(k_bicg_spmv_v, c.nsA, gs, c.A, c.S);
            if (ev) (void)hipEventRecord(ev[2 * k + 1], s);
            k_fin_bicg_v<<<gf, kBlock, 0, s>>>(c.S, Gs);
            k_bicg_s<<<gv, kBlock, 0, s>>>(c.A, c.S);
            k_fin_bicg_s<<<gf, kBlock, 0, s>>>(c.S, Gv);
            NS_LAUNCH_A(k_bicg_spmv_t, c.nsA, gs, c.A, c.S);
            k_fin_bicg_t<<<gf, kBlock, 0, s>>>(c.S, Gs);
            k_bicg_update<<<gv, kBlock, 0, s>>>(c.A, c.S);
            k_fin_bicg_update<<<gf, kBlock, 0, s>>>(c.S, Gv);
        }
    }
}

static uint64_t fnv(const void *data, size_t len, uint64_t hsh = 1469598103934665603ull) {
    const unsigned char *b = (const unsigned char *)data;
    for (size_t i = 0; i < len; ++i) hsh = (hsh ^ b[i]) * 1099511628211ull;
    return hsh;
}

// Runs `iters` iterations.  Without profiling they are replayed from a
// cached graph of `unit` iterations (8 when `iters` is a multiple of 8), so
// every chunk length of a solve reuses one captured graph.
static hsla_status run_chunk(hsla_handle *h, const SolveCall &c, int iters, bool use_graph, hipStream_t s,
                             hipEvent_t *ev) {
    if (!use_graph || ev) {
        enqueue_iterations(c, iters, s, ev);
        HSLA_HIP(h, hipGetLastError());
        return HSLA_OK;
    }
    const int unit = iters % 8 == 0 ? 8 : iters;
    uint64_t key = fnv(&c, sizeof c);
    key = fnv(&unit, sizeof unit, key);
    int slot = -1;
    for (int i = 0; i < hsla_handle::kGraphCache; ++i)
        if (h->graph_exec[i] && h->graph_key[i] == key) slot = i;
    if (slot < 0) {
        slot = 0;
        for (int i = 1; i < hsla_handle::kGraphCache; ++i)
            if (h->graph_use[i] < h->graph_use[slot]) slot = i;
        if (h->graph_exec[slot]) {
            HSLA_HIP(h, hipGraphExecDestroy(h->graph_exec[slot]));
            h->graph_exec[slot] = nullptr;
            h->graph_key[slot] = 0;
        }
        hipGraph_t g = nullptr;
        HSLA_HIP(h, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        enqueue_iterations(c, unit, s, nullptr);
        const hipError_t le = hipGetLastError();
        const hipError_t ce = hipStreamEndCapture(s, &g);
        if (le != hipSuccess || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return set_error(h, HSLA_ERR_HIP, "graph capture failed: %s",
                             hipGetErrorString(le != hipSuccess ? le : ce));
        }
        const hipError_t ie = hipGraphInstantiate(&h->graph_exec[slot], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            h->graph_exec[slot] = nullptr;
            return set_error(h, HSLA_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(ie));
        }
        h->graph_key[slot] = key;
    }
    h->graph_use[slot] = ++h->graph_clock;
    for (int done = 0; done < iters; done += unit) HSLA_HIP(h, hipGraphLaunch(h->graph_exec[slot], s));
    return HSLA_OK;
}

static hsla_status ensure_prof_events(hsla_handle *h, int pairs) {
    if (2 * pairs <= h->prof_cap) return HSLA_OK;
    for (int i = 0; i < h->prof_cap; ++i) (void)hipEventDestroy(h->prof_ev[i]);
    delete[] h->prof_ev;
    h->prof_ev = new hipEvent_t[2 * pairs];
    h->prof_cap = 0;
    for (int i = 0; i < 2 * pairs; ++i) {
        HSLA_HIP(h, hipEventCreate(&h->prof_ev[i]));
        h->prof_cap = i + 1;
    }
    return HSLA_OK;
}

static int worst_status(int a, int b) {
    if (a < 0 || b < 0) return a < b ? a : b;
    return a > b ? a : b;
}

// Shared solve driver for the single, batched and transposed (adjoint)
// paths.  `A` is the operator actually iterated on.
// SpMV configuration of a solve (the pattern's autotuned choice).
// `half`: this solve's values are symmetric and the half form applies.
struct Tune {
    int dia, tile_cu, dia_cu, sym, sym_cu;
    bool half;
};

static Tune tune_of(const hsla_pattern *p) {
    return Tune{p->tune_dia, p->tune_tile_cu, p->tune_dia_cu, p->tune_sym, p->tune_sym_cu, false};
}

// Sets tn.half for a solve on p's own pattern: the half form is enabled for
// p, applies to its stencil, and the values are symmetric (`sym` < 0:
// unknown, checked here).
static hsla_status decide_half(hsla_handle *h, const hsla_pattern *p, const Pat &A, int B, const double *values,
                               int sym, hipStream_t s, Tune *tn) {
    tn->half = false;
    if (!tn->sym || !p->pattern_symmetric || !stencil_half_ok(A.sn)) return HSLA_OK;
    if (sym < 0) {
        bool v = false;
        const hsla_status st = values_symmetric(h, p, B, values, s, &v);
        if (st != HSLA_OK) return st;
        sym = v ? 1 : 0;
    }
    tn->half = sym == 1;
    return HSLA_OK;
}

// Grid sizes, SpMV forms and workspace layout of one solve.
struct Plan {
    int nvec, Gt, Gv, nsA, nsF, Gd, Gs, Gf, pencil;
    size_t diaA, diaL, diaU, sval, ssp, ssc;
    Layout lay;
};

// Gram partials per block of s-step CG (plain and weighted upper triangles).
static int ss_partials(int ss) { return ss > 0 ? (2 * ss + 1) * (2 * ss + 2) : 0; }

static Plan plan_solve(hsla_handle *h, const Tune &tn, const Pat &A, const FPat *L, const FPat *U, int B, int method,
                       int pre, int ss = 0) {
    Plan pl{};
    const int64_t n = A.n;
    // s-step CG keeps its 2 ss - 1 basis vectors past p and r after the six
    pl.nvec = method == HSLA_METHOD_CG ? 6 + (ss > 0 ? 2 * ss - 1 : 0) : 8;
    // SpMV-based kernels: up to 16 blocks per CU; vector kernels: up to 8,
    // shared by the systems of a batch (fewer, longer-running blocks each)
    pl.Gt = grid_blocks(h, kWavesPerBlock, A.ntiles, B, tn.tile_cu);
    pl.Gv = grid_blocks(h, kBlock * 4, n, B, 8);
    // offset-mask patterns run their SpMVs on diagonal-major copies of the
    // values made once per solve (row per thread, two rows per step) unless
    // the autotuner found the row tiles faster (the tuning covers A's SpMV;
    // the FSAI factors always use their diagonal-major copies where they
    // have one)
    auto dia_slots = [](const Stencil &sn) { return sn.mask ? dia_slots_for(sn.nofs) : 0; };
    // right-Jacobi BiCGStab iterates on A D^{-1}, which is not symmetric;
    // Jacobi CG on S A S, which is
    const bool cscaled = method == HSLA_METHOD_BICGSTAB && pre == PRE_JACOBI;
    const bool scaled = cscaled || (method == HSLA_METHOD_CG && pre == PRE_JACOBI);
    const bool half = tn.half && !cscaled;
    const bool unit = half && scaled;  // Jacobi CG: S A S has a unit diagonal
    // right-Jacobi BiCGStab: A D^{-1} has a unit diagonal, left out of the full copy
    const bool unit_full = cscaled && tn.dia && A.sn.mask && A.sn.diag_slot >= 0 &&
                           (A.sn.nofs == 5 || A.sn.nofs == 7 || A.sn.nofs == 9);
    pl.nsA = half ? (unit ? kUnitNS : kSymNS) + A.sn.nofs : unit_full ? kUnitFullNS + A.sn.nofs
             : tn.dia                                  ? dia_slots(A.sn)
                                                       : 0;
    const bool fsai = pre == PRE_FSAI && L && U;
    pl.nsF = fsai && L->sn.mask && U->sn.mask ? std::max(dia_slots(L->sn), dia_slots(U->sn)) : 0;
    pl.pencil = half ? pencil_len(A.sn, n, B, h->dev.num_cu) : 1;
    pl.Gd = half ? grid_blocks(h, (int64_t)kDiaChunk * pl.pencil, n, B, tn.sym_cu)
                 : grid_blocks(h, kDiaChunk, n, B, tn.dia_cu);
    pl.Gs = pl.nsA ? pl.Gd : pl.Gt;
    pl.Gf = pl.nsF ? grid_blocks(h, kDiaChunk, n, B, 8) : pl.Gt;
    const size_t drows = (size_t)dia_chunks(n) * kDiaChunk;
    pl.diaA = pl.nsA ? sizeof(double) * (size_t)B * dia_stored(pl.nsA, A.sn.nofs) * drows : 0;
    pl.diaL = pl.nsF ? sizeof(float) * (size_t)B * L->sn.nofs * drows : 0;
    pl.diaU = pl.nsF ? sizeof(float) * (size_t)B * U->sn.nofs * drows : 0;
    pl.sval = scaled && !pl.nsA ? sizeof(double) * (size_t)B * (size_t)A.nnz : 0;
    pl.ssp = sizeof(double) * (size_t)ss_partials(ss) * pl.Gv * B;
    pl.ssc = ss > 0 ? sizeof(double) * 3 * (2 * ss + 1) * (size_t)B : 0;
    const size_t extra = align_up(pl.diaA, 256) + align_up(pl.diaL, 256) + align_up(pl.diaU, 256) +
                         align_up(pl.sval, 256) + align_up(pl.ssp, 256) + align_up(pl.ssc, 256);
    const int Gmax = std::max(std::max(pl.Gt, pl.Gv), std::max(pl.Gd, pl.Gf));
    pl.lay = make_layout(B, n, pl.nvec, Gmax, extra);
    return pl;
}

static hsla_status solve_core(hsla_handle *h, const Tune &tn, const Pat &A, const FPat *L, const FPat *U, int B,
                              const double *values,
                              const double *b, double *x, const hsla_opts &o, int method, hsla_info *infos,
                              hipStream_t s, bool sr = false, int ss = 0) {
    const int64_t n = A.n;
    const int pre = o.precond == HSLA_PRECOND_NONE ? PRE_NONE : o.precond == HSLA_PRECOND_FSAI ? PRE_FSAI : PRE_JACOBI;
    if (method == HSLA_METHOD_BICGSTAB && pre == PRE_FSAI)
        return set_error(h, HSLA_ERR_INVALID_ARG, "FSAI preconditioning is for CG only");
    if (ss > 0 && (method != HSLA_METHOD_CG || pre != PRE_JACOBI))
        return set_error(h, HSLA_ERR_INVALID_ARG, "s-step CG runs on the Jacobi-scaled operator (precond JACOBI)");
    const Plan pl = plan_solve(h, tn, A, L, U, B, method, pre, ss);
    const int nvec = pl.nvec, Gt = pl.Gt, Gv = pl.Gv, nsA = pl.nsA, nsF = pl.nsF, Gs = pl.Gs, Gf = pl.Gf;
    const size_t diaA = pl.diaA, diaL = pl.diaL;
    const Layout lay = pl.lay;
    hsla_status st = ensure_workspace(h, lay.total);
    if (st != HSLA_OK) return st;
    st = ensure_host_state(h, B);
    if (st != HSLA_OK) return st;
    char *ws = (char *)h->ws;
    SolveCall c{};
    c.A = A;
    c.A.sn.pencil = pl.pencil;
    if (L) c.L = *L;
    if (U) c.U = *U;
    c.B = B;
    c.method = method;
    c.precond = pre;
    c.Gt = Gt;
    c.Gv = Gv;
    c.nsA = nsA;
    c.nsF = nsF;
    c.Gs = Gs;
    c.Gf = Gf;
    c.sr = sr && method == HSLA_METHOD_CG && (pre == PRE_NONE || pre == PRE_JACOBI);
    c.ss = ss;
    Sys &S = c.S;
    S.val = values;
    S.b = b;
    S.x = x;
    S.st = (SysState *)(ws + lay.off_state);
    S.part = (double *)(ws + lay.off_part);
    S.part2 = S.part + 3 * (size_t)lay.gmax * B;
    double *vec = (double *)(ws + lay.off_vec);
    const size_t vs = (size_t)B * n;
    double **cg_slots[] = {&S.r, &S.p, &S.q, &S.dinv, &S.z, &S.w};
    double **bicg_slots[] = {&S.r, &S.p, &S.t, &S.dinv, &S.rh, &S.y, &S.v, &S.s};
    double ***slots = method == HSLA_METHOD_CG ? cg_slots : bicg_slots;
    const int nslots = method == HSLA_METHOD_CG ? 6 : 8;
    for (int k = 0; k < nslots && k < nvec; ++k) *slots[k] = vec + k * vs;
    S.ssb = ss > 0 ? vec + 6 * vs : nullptr;
    S.aval = values;
    // right-Jacobi BiCGStab iterates on A D^{-1}: its values are scaled
    // below, once D^{-1} is known
    const bool cscaled = method == HSLA_METHOD_BICGSTAB && pre == PRE_JACOBI;
    const bool sscaled = method == HSLA_METHOD_CG && pre == PRE_JACOBI;
    const bool scaled = cscaled || sscaled;
    const int64_t max_iter = o.max_iter > 0 ? o.max_iter : (10 * n < 100000 ? 10 * n : 100000);
    const dim3 gt(Gt, B), gv(Gv, B), gf(B), gfs(Gf, B);
    {
        char *ex = ws + lay.off_extra;
        if (nsA) {
            double *d = (double *)ex;
            if (!scaled && nsA > kSymNS)
                k_to_dia_sym<double><<<dim3(Gv, B), kBlock, 0, s>>>((int32_t)n, A.rp, A.sn, A.nnz, values, d);
            else if (!scaled)
                k_to_dia<double><<<dim3(Gv, B), kBlock, 0, s>>>((int32_t)n, A.rp, A.sn, A.nnz, values, d);
            S.dia = d;
            ex += align_up(diaA, 256);
        } else if (scaled) {
            S.aval = (const double *)ex;
            ex += align_up(pl.sval, 256);
        }
        if (nsF) {
            float *dl = (float *)ex;
            float *du = (float *)(ex + align_up(diaL, 256));
            k_to_dia<float><<<dim3(Gv, B), kBlock, 0, s>>>((int32_t)n, L->rp, L->sn, L->nnz, L->val, dl);
            k_to_dia<float><<<dim3(Gv, B), kBlock, 0, s>>>((int32_t)n, U->rp, U->sn, U->nnz, U->val, du);
            c.L.dia = dl;
            c.U.dia = du;
            ex += align_up(diaL, 256) + align_up(pl.diaU, 256);
        }
        if (ss > 0) {
            S.ssp = (double *)ex;
            ex += align_up(pl.ssp, 256);
            S.ssc = (double *)ex;
        }
    }
    k_reset<<<1, kBlock, 0, s>>>(S.st, B, max_iter, o.stall_window > 0 ? o.stall_window : 0);
    if (o.use_x0) k_spmv<<<gt, kBlock, 0, s>>>(A, values, x, S.q);
    if (method == HSLA_METHOD_CG) {
        switch (pre) {
            case PRE_NONE:
                k_cg_init<PRE_NONE><<<gv, kBlock, 0, s>>>(A, S, o.use_x0);
                k_fin_cg_init<PRE_NONE><<<gf, kBlock, 0, s>>>(S, Gv, o.rtol, o.atol);
                break;
            case PRE_JACOBI:
                k_cg_init<PRE_JACOBI><<<gv, kBlock, 0, s>>>(A, S, o.use_x0);
                k_fin_cg_init<PRE_JACOBI><<<gf, kBlock, 0, s>>>(S, Gv, o.rtol, o.atol);
                // S A S, once S is known
                if (nsA > kSymNS)
                    k_to_dia_sym<double><<<dim3(Gv, B), kBlock, 0, s>>>((int32_t)n, A.rp, A.sn, A.nnz, values,
                                                                        (double *)S.dia, S.dinv, nsA > kUnitNS);
                else if (nsA)
                    k_to_dia<double><<<dim3(Gv, B), kBlock, 0, s>>>((int32_t)n, A.rp, A.sn, A.nnz, values,
                                                                    (double *)S.dia, S.dinv, 1);
                else
                    k_scale_sym<<<dim3(Gv, B), kBlock, 0, s>>>((int32_t)n, A.nnz, A.rp, A.col, values, S.dinv,
                                                               (double *)S.aval);
                break;
            default:
                k_cg_init<PRE_FSAI><<<gv, kBlock, 0, s>>>(A, S, o.use_x0);
                k_fsai_check<<<gv, kBlock, 0, s>>>(c.L, S, (int32_t)n);
                k_fin_cg_init<PRE_FSAI><<<gf, kBlock, 0, s>>>(S, Gv, o.rtol, o.atol);
                NS_LAUNCH(k_fsai_lower_dot, nsF, gfs, A, c.L, S);
                k_fin_fsai<<<gf, kBlock, 0, s>>>(S, Gf, 1);
                NS_LAUNCH(k_fsai_upper_start, nsF, gfs, A, c.U, S);
                break;
        }
    } else {
        if (pre == PRE_JACOBI)
            k_bicg_init<PRE_JACOBI><<<gv, kBlock, 0, s>>>(A, S, o.use_x0);
        else
            k_bicg_init<PRE_NONE><<<gv, kBlock, 0, s>>>(A, S, o.use_x0);
        k_fin_bicg_init<<<gf, kBlock, 0, s>>>(S, Gv, o.rtol, o.atol);
        if (scaled && nsA)
            k_to_dia<double><<<dim3(Gv, B), kBlock, 0, s>>>((int32_t)n, A.rp, A.sn, A.nnz, values,
                                                            (double *)S.dia, S.dinv, 0, nsA > kUnitFullNS);
        else if (scaled)
            k_scale_cols<<<dim3(Gv, B), kBlock, 0, s>>>((int32_t)n, A.nnz, A.rp, A.col, values, S.dinv,
                                                        (double *)S.aval);
    }
    HSLA_HIP(h, hipGetLastError());

    // chunks of iterations, one host check per chunk
    int chunk = o.check_every > 0 ? o.check_every : 8;
    const int chunk_cap = o.check_every > 0 ? o.check_every : 64;
    hipEvent_t *ev = nullptr;
    if (o.profile && !c.ss) {  // (s-step CG runs unprofiled)
        st = ensure_prof_events(h, chunk_cap > chunk ? chunk_cap : chunk);
        if (st != HSLA_OK) return st;
        ev = h->prof_ev;
    }
    double prof_ms = 0.0;
    int64_t prof_n = 0;
    SysState *hs = h->h_state;
    int64_t run = 0, last_iters = 0;
    int pending = 0;  // launches of the previous chunk not yet accounted
    for (;;) {
        HSLA_HIP(h, hipMemcpyAsync(hs, S.st, sizeof(SysState) * B, hipMemcpyDeviceToHost, s));
        HSLA_HIP(h, hipStreamSynchronize(s));
        if (ev && pending > 0) {
            // launches that did work: the largest per-system iteration advance
            int64_t most = 0;
            for (int i = 0; i < B; ++i) most = hs[i].iters > most ? hs[i].iters : most;
            const int64_t worked = most - last_iters;
            last_iters = most;
            for (int64_t k = 0; k < worked && k < pending; ++k) {
                float ms = 0.f;
                HSLA_HIP(h, hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]));
                prof_ms += ms;
                ++prof_n;
            }
            pending = 0;
        }
        bool all_done = true;
        for (int i = 0; i < B; ++i)
            if (!hs[i].done) {
                all_done = false;
                break;
            }
        if (all_done || run >= max_iter + 2) break;
        if (chunk > chunk_cap) chunk = chunk_cap;
        st = run_chunk(h, c, chunk, o.use_graph != 0, s, ev);
        if (st != HSLA_OK) return st;
        run += (int64_t)chunk * (c.ss > 0 ? c.ss : 1);
        pending = chunk;
        if (chunk < chunk_cap) chunk *= 2;
    }
    if (method == HSLA_METHOD_BICGSTAB) {
        if (pre == PRE_JACOBI)
            k_bicg_finish<PRE_JACOBI><<<gv, kBlock, 0, s>>>(A, S);
        else
            k_bicg_finish<PRE_NONE><<<gv, kBlock, 0, s>>>(A, S);
    } else if (sscaled) {
        k_cg_unscale<<<gv, kBlock, 0, s>>>(A, S);
    }
    // true residual ||b - A x|| / ||b||
    double *res = (double *)(ws + lay.off_res);
    k_residual<<<gt, kBlock, 0, s>>>(A, S);
    k_fin_residual<<<gf, kBlock, 0, s>>>(S, Gt, res);
    HSLA_HIP(h, hipGetLastError());
    std::vector<double> hres(2 * (size_t)B);
    HSLA_HIP(h, hipMemcpyAsync(hres.data(), res, sizeof(double) * 2 * B, hipMemcpyDeviceToHost, s));
    HSLA_HIP(h, hipStreamSynchronize(s));
    int worst = HSLA_OK;
    for (int i = 0; i < B; ++i) {
        const int sst = hs[i].done ? hs[i].status : HSLA_ERR_INTERNAL;
        worst = worst_status(worst, sst);
        if (infos) {
            hsla_info &f = infos[i];
            f.iters = hs[i].iters;
            f.status = sst;
            f.method = c.ss ? HSLA_METHOD_CG_SSTEP : c.sr ? HSLA_METHOD_CG_SR : method;
            const double bn = hs[i].bnorm;
            const double rn = std::sqrt(hs[i].rnorm2);
            f.rel_residual = bn > 0 ? rn / bn : rn;
            const double tr = std::sqrt(hres[2 * i]), tb = std::sqrt(hres[2 * i + 1]);
            f.true_residual = tb > 0 ? tr / tb : tr;
            f.spmv_ms = prof_ms;
            f.spmv_launches = prof_n;
            f.spmv_form = nsA > kUnitFullNS ? 5 : nsA > kUnitNS ? 4 : nsA > kSymNS ? 2 : nsA > 0 ? 1 : 0;
            // the diagonal forms' SpMV operands (p, and BiCGStab's s) share
            // p's alignment: every work vector is B n doubles past the last
            f.spmv_paired = nsA > 0 && pairable_stencil(A.sn, n) && ((uintptr_t)S.p & 15u) == 0 ? 1 : 0;
            f.t_start_ms = f.t_end_ms = 0.0;
            f.workgroups = 0;
            f.reserved = 0;
        }
    }
    return (hsla_status)worst;
}

static hsla_status check_common(hsla_handle *h, const hsla_pattern *p, int B, hipStream_t user) {
    if (!h) return HSLA_ERR_INVALID_ARG;
    if (!p) return set_error(h, HSLA_ERR_INVALID_ARG, "null pattern");
    if (p->device != h->device) return set_error(h, HSLA_ERR_INVALID_ARG, "pattern on another device");
    if (B < 0) return set_error(h, HSLA_ERR_INVALID_ARG, "negative batch");
    return enter(h, user);
}

// True when the pattern equals its transpose and every system's values are
// symmetric bit for bit (the paper detects symmetry on the values).
static hsla_status values_symmetric(hsla_handle *h, const hsla_pattern *p, int B, const double *values, hipStream_t s,
                                    bool *sym) {
    if (!p->pattern_symmetric) {
        *sym = false;
        return HSLA_OK;
    }
    HSLA_HIP(h, hipMemsetAsync(h->d_flags, 0, sizeof(int32_t), s));
    if (p->nnz > 0 && B > 0) {
        const int64_t tot = p->nnz * B;
        int blocks = (int)((tot + kBlock - 1) / kBlock);
        if (blocks > 8192) blocks = 8192;
        k_value_asym<<<blocks, kBlock, 0, s>>>(p->nnz, B, values, p->srcT, h->d_flags);
        HSLA_HIP(h, hipGetLastError());
    }
    int32_t hf = 0;
    HSLA_HIP(h, hipMemcpyAsync(&hf, h->d_flags, sizeof hf, hipMemcpyDeviceToHost, s));
    HSLA_HIP(h, hipStreamSynchronize(s));
    *sym = hf == 0;
    return HSLA_OK;
}

static hsla_status read_opts(hsla_handle *h, const hsla_opts *opts, hsla_opts *o) {
    if (opts)
        *o = *opts;
    else
        hsla_opts_default(o);
    if (!(o->rtol >= 0) || !(o->atol >= 0)) return set_error(h, HSLA_ERR_INVALID_ARG, "negative or NaN tolerance");
    if (o->method < HSLA_METHOD_AUTO || o->method > HSLA_METHOD_CG_SSTEP)
        return set_error(h, HSLA_ERR_INVALID_ARG, "unknown method %d", o->method);
    if (o->method == HSLA_METHOD_CG_SSTEP && (o->s_step < 2 || o->s_step > 4))
        return set_error(h, HSLA_ERR_INVALID_ARG, "s_step must be 2, 3 or 4 (got %d)", o->s_step);
    if (o->precond < HSLA_PRECOND_NONE || o->precond > HSLA_PRECOND_FSAI)
        return set_error(h, HSLA_ERR_INVALID_ARG, "unknown preconditioner %d", o->precond);
    return HSLA_OK;
}

static void trivial_infos(hsla_info *infos, int B) {
    for (int i = 0; infos && i < B; ++i) {
        std::memset(&infos[i], 0, sizeof infos[i]);
        infos[i].method = HSLA_METHOD_CG;
    }
}

hsla_status solve_entry(hsla_handle *h, const hsla_pattern *p, int B, const double *values, const double *b, double *x,
                        const hsla_opts *opts, hsla_info *infos, hipStream_t user) {
    hsla_status st = check_common(h, p, B, user);
    if (st != HSLA_OK) return st;
    hipStream_t s = h->stream;
    hsla_opts o;
    st = read_opts(h, opts, &o);
    if (st != HSLA_OK) return st;
    if (B == 0) return HSLA_OK;
    if (p->n == 0) {
        trivial_infos(infos, B);
        return HSLA_OK;
    }
    if (!values || !b || !x) return set_error(h, HSLA_ERR_INVALID_ARG, "null values, b or x");
    int method = o.method;
    const bool sr = method == HSLA_METHOD_CG_SR;  // single-reduction CG where it applies
    const int ss = method == HSLA_METHOD_CG_SSTEP ? o.s_step : 0;  // s-step CG (per-iteration kernels)
    if (sr || ss) method = HSLA_METHOD_CG;
    int symv = -1;  // values symmetric: -1 not checked
    if (method == HSLA_METHOD_AUTO) {
        bool sym = false;
        st = values_symmetric(h, p, B, values, s, &sym);
        if (st != HSLA_OK) return st;
        method = sym ? HSLA_METHOD_CG : HSLA_METHOD_BICGSTAB;
        symv = sym ? 1 : 0;
    }
    if (!ss && o.persistent && persistent_eligible(h, p, B, method, o))
        return persistent_solve(h, p, B, values, b, x, o, infos, s, sr);
    const Pat A = pat_of(p);
    FPat L{}, U{};
    if (o.precond == HSLA_PRECOND_FSAI) {
        if (!o.d_G || !o.d_GT) return set_error(h, HSLA_ERR_INVALID_ARG, "FSAI needs d_G and d_GT");
        L = FPat{p->rpL, p->colL, p->metaL, p->ntilesL, p->nnz_lower, o.d_G, p->use(p->stL)};
        U = FPat{p->rpU, p->colU, p->metaU, p->ntilesU, p->nnz_lower, o.d_GT, p->use(p->stU)};
    }
    Tune tn = tune_of(p);
    st = decide_half(h, p, A, B, values, symv, s, &tn);
    if (st != HSLA_OK) return st;
    return solve_core(h, tn, A, &L, &U, B, values, b, x, o, method, infos, s, sr, ss);
}

// Eq. adjoint_linear: A^T lambda = gx, gb = lambda, gA = -lambda x^T on the
// pattern.  A symmetric A is iterated on directly; otherwise the values are
// permuted into the transpose's entry order and the transpose's pattern is
// iterated on.
hsla_status adjoint_entry(hsla_handle *h, const hsla_pattern *p, int B, const double *values, const double *x,
                          const double *gx, double *gA, double *gb, const hsla_opts *opts, hsla_info *infos,
                          hipStream_t user) {
    hsla_status st = check_common(h, p, B, user);
    if (st != HSLA_OK) return st;
    hipStream_t s = h->stream;
    hsla_opts o;
    st = read_opts(h, opts, &o);
    if (st != HSLA_OK) return st;
    if (o.use_x0) return set_error(h, HSLA_ERR_INVALID_ARG, "use_x0 is not supported by the adjoint");
    if (o.precond == HSLA_PRECOND_FSAI) return set_error(h, HSLA_ERR_INVALID_ARG, "the adjoint uses Jacobi or none");
    if (B == 0) return HSLA_OK;
    if (p->n == 0) {
        trivial_infos(infos, B);
        return HSLA_OK;
    }
    if (!values || !x || !gx) return set_error(h, HSLA_ERR_INVALID_ARG, "null values, x or gx");
    bool sym = false;
    st = values_symmetric(h, p, B, values, s, &sym);
    if (st != HSLA_OK) return st;
    const bool sr = o.method == HSLA_METHOD_CG_SR;
    const int ss = o.method == HSLA_METHOD_CG_SSTEP ? o.s_step : 0;
    const int method = o.method == HSLA_METHOD_AUTO ? (sym ? HSLA_METHOD_CG : HSLA_METHOD_BICGSTAB)
                       : sr || ss                   ? HSLA_METHOD_CG
                                                    : o.method;
    const int64_t n = p->n;
    double *lam = gb, *lam_own = nullptr, *valT = nullptr;
    if (!lam) {
        HSLA_HIP(h, dev_alloc(h, (void **)&lam_own, sizeof(double) * (size_t)B * n));
        lam = lam_own;
    }
    hsla_status res;
    if (sym) {
        const Pat A = pat_of(p);
        if (!ss && o.persistent && persistent_eligible(h, p, B, method, o)) {
            res = persistent_solve(h, p, B, values, gx, lam, o, infos, s, sr);
        } else {
            Tune tn = tune_of(p);
            res = decide_half(h, p, A, B, values, 1, s, &tn);
            if (res == HSLA_OK)
                res = solve_core(h, tn, A, nullptr, nullptr, B, values, gx, lam, o, method, infos, s, sr, ss);
        }
    } else {
        if (dev_alloc(h, (void **)&valT, sizeof(double) * (size_t)B * (p->nnz > 0 ? p->nnz : 1)) != hipSuccess) {
            dev_free(h, lam_own);
            return set_error(h, HSLA_ERR_NO_MEMORY, "transposed values");
        }
        const int64_t tot = p->nnz * B;
        int blocks = (int)((tot + kBlock - 1) / kBlock);
        if (blocks > 8192) blocks = 8192;
        if (tot > 0) k_gather_values<<<blocks, kBlock, 0, s>>>(p->nnz, B, values, p->srcT, valT);
        const Pat AT = pat_T_of(p);
        res = solve_core(h, tune_of(p), AT, nullptr, nullptr, B, valT, gx, lam, o, method, infos, s, sr, ss);
    }
    if (res >= 0 && gA) {
        int Gr = (int)((n + kBlock - 1) / kBlock);
        if (Gr > 4096) Gr = 4096;
        k_outer<<<dim3(Gr, B), kBlock, 0, s>>>(p->n, p->nnz, p->row_ptr, p->col, lam, x, gA);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) res = set_error(h, HSLA_ERR_HIP, "outer product: %s", hipGetErrorString(e));
    }
    const hipError_t se = hipStreamSynchronize(s);
    dev_free(h, valT);
    dev_free(h, lam_own);
    if (se != hipSuccess) return set_error(h, HSLA_ERR_HIP, "adjoint: %s", hipGetErrorString(se));
    return res;
}

// Workspace bytes of a solve (hsla_workspace_size).
hsla_status workspace_size(hsla_handle *h, const hsla_pattern *p, int B, const hsla_opts &o, size_t *bytes) {
    const Pat A = pat_of(p);
    const int pre = o.precond == HSLA_PRECOND_NONE ? PRE_NONE : o.precond == HSLA_PRECOND_FSAI ? PRE_FSAI : PRE_JACOBI;
    FPat L{p->rpL, p->colL, p->metaL, p->ntilesL, p->nnz_lower, nullptr, p->use(p->stL)};
    FPat U{p->rpU, p->colU, p->metaU, p->ntilesU, p->nnz_lower, nullptr, p->use(p->stU)};
    size_t need = 0;
    // the single-reduction and s-step recurrences are CG solves
    const int om = o.method == HSLA_METHOD_CG_SR || o.method == HSLA_METHOD_CG_SSTEP ? HSLA_METHOD_CG : o.method;
    const int ss = o.method == HSLA_METHOD_CG_SSTEP ? o.s_step : 0;
    for (int method : {HSLA_METHOD_CG, HSLA_METHOD_BICGSTAB}) {
        if (om != HSLA_METHOD_AUTO && om != method) continue;
        if (method == HSLA_METHOD_BICGSTAB && pre == PRE_FSAI) continue;
        const Plan pl = plan_solve(h, tune_of(p), A, &L, &U, B, method, pre, method == HSLA_METHOD_CG ? ss : 0);
        need = std::max(need, pl.lay.total);
        if (o.persistent && persistent_eligible(h, p, B, method, o))
            need = std::max(need, sizeof(double) * 4 * (size_t)B * p->n + 1024 + 40 * (size_t)B);
    }
    *bytes = need + need / 8 + 4096;  // the growth margin ensure_workspace adds
    return HSLA_OK;
}

// Autotuner: times the solvers' SpMV forms and grid densities on the device
// (synthetic values 1, x = 1) and keeps the fastest in the pattern.  The
// half form is timed where the pattern allows it (the synthetic values are
// symmetric); it is used only by solves whose values are symmetric, so the
// full copy and the tiles are ranked among themselves for the others.
hsla_status autotune(hsla_handle *h, hsla_pattern *p, int B, int effort, hsla_tuning *out, hipStream_t s) {
    Pat A = pat_of(p);
    const int64_t n = p->n, nnz = p->nnz;
    const bool dia_ok = A.sn.mask != nullptr;
    const bool half_ok = dia_ok && p->pattern_symmetric && stencil_half_ok(A.sn);
    if (half_ok) A.sn.pencil = pencil_len(A.sn, n, B, h->dev.num_cu);
    const size_t rows = dia_ok ? (size_t)dia_chunks(n) * kDiaChunk : 0;
    const size_t nv = align_up(sizeof(double) * (size_t)B * (nnz > 0 ? nnz : 1), 256);
    const size_t nx = align_up(sizeof(double) * (size_t)B * n, 256);
    const size_t nd = dia_ok ? align_up(sizeof(double) * (size_t)B * A.sn.nofs * rows, 256) : 0;
    const size_t nh = half_ok ? align_up(sizeof(double) * (size_t)B * (A.sn.nofs / 2 + 1) * rows, 256) : 0;
    hsla_status st = ensure_workspace(h, nv + 2 * nx + nd + nh);
    if (st != HSLA_OK) return st;
    char *ws = (char *)h->ws;
    double *val = (double *)ws, *x = (double *)(ws + nv), *y = (double *)(ws + nv + nx);
    double *dia = dia_ok ? (double *)(ws + nv + 2 * nx) : nullptr;
    double *diah = half_ok ? (double *)(ws + nv + 2 * nx + nd) : nullptr;
    k_fill_f64<<<4096, kBlock, 0, s>>>(val, (int64_t)B * nnz, 1.0);
    k_fill_f64<<<4096, kBlock, 0, s>>>(x, (int64_t)B * n, 1.0);
    if (dia_ok) {
        const int Gv = grid_blocks(h, kBlock * 4, n, B, 8);
        k_to_dia<double><<<dim3(Gv, B), kBlock, 0, s>>>((int32_t)n, A.rp, A.sn, nnz, val, dia);
        if (half_ok) k_to_dia_sym<double><<<dim3(Gv, B), kBlock, 0, s>>>((int32_t)n, A.rp, A.sn, nnz, val, diah);
    }
    HSLA_HIP(h, hipGetLastError());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HSLA_HIP(h, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(h, HSLA_ERR_HIP, "autotune: event creation failed");
    }
    enum { F_DIA = 0, F_TILES = 1, F_HALF = 2 };
    auto time = [&](int form, int cu, double *us) -> hipError_t {
        const int ns = form == F_HALF ? kSymNS + A.sn.nofs : dia_slots_for(A.sn.nofs);
        const int gx = form == F_HALF  ? grid_blocks(h, (int64_t)kDiaChunk * A.sn.pencil, n, B, cu)
                       : form == F_DIA ? grid_blocks(h, kDiaChunk, n, B, cu)
                                       : grid_blocks(h, kWavesPerBlock, p->ntiles, B, cu);
        const dim3 g(gx, B);
        for (int r = -1; r < effort; ++r) {
            if (r == 0) {
                const hipError_t e = hipEventRecord(e0, s);
                if (e != hipSuccess) return e;
            }
            if (form == F_TILES) {
                k_spmv<<<g, kBlock, 0, s>>>(A, val, x, y);
            } else {
                NS_LAUNCH_A(k_spmv_dia, ns, g, A, form == F_HALF ? diah : dia, x, y);
            }
        }
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        *us = 1e3 * ms / effort;
        return e;
    };
    struct Cand {
        int form;
        int cu;
        double us;
    };
    std::vector<Cand> cands;
    if (half_ok)
        for (int cu : {1, 2, 3, 4, 8, 16}) cands.push_back({F_HALF, cu, 0.0});
    if (dia_ok)
        for (int cu : {1, 2, 4, 8, 16}) cands.push_back({F_DIA, cu, 0.0});
    for (int cu : {4, 8, 16, 32}) cands.push_back({F_TILES, cu, 0.0});
    hipError_t err = hipSuccess;
    for (Cand &c : cands)
        if (err == hipSuccess) err = time(c.form, c.cu, &c.us);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return set_error(h, HSLA_ERR_HIP, "autotune: %s", hipGetErrorString(err));
    const Cand *best = nullptr, *best_other = nullptr, *best_tiles = nullptr, *best_half = nullptr, *dflt = nullptr;
    const int dflt_form = half_ok ? F_HALF : dia_ok ? F_DIA : F_TILES;
    for (const Cand &c : cands) {
        if (!best || c.us < best->us) best = &c;
        if (c.form != F_HALF && (!best_other || c.us < best_other->us)) best_other = &c;
        if (c.form == F_TILES && (!best_tiles || c.us < best_tiles->us)) best_tiles = &c;
        if (c.form == F_HALF && (!best_half || c.us < best_half->us)) best_half = &c;
        if (c.form == dflt_form && c.cu == (dflt_form == F_TILES ? 16 : 8)) dflt = &c;
    }
    p->tune_dia = best_other->form == F_DIA ? 1 : 0;
    if (best_other->form == F_DIA) p->tune_dia_cu = best_other->cu;
    p->tune_tile_cu = best_tiles->cu;
    p->tune_sym = best_half && best_half->us < best_other->us ? 1 : 0;
    if (best_half) p->tune_sym_cu = best_half->cu;
    p->tuned = 1;
    if (out) {
        out->form = best->form;
        out->blocks_per_cu = best->cu;
        out->best_us = best->us;
        out->default_us = dflt ? dflt->us : best->us;
    }
    return HSLA_OK;
}

}  // namespace hsla

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

hsla_status hsla_workspace_size(hsla_handle *h, const hsla_pattern *p, int32_t B, const hsla_opts *opts,
                                size_t *bytes) {
    if (!h || !p || !bytes) return HSLA_ERR_INVALID_ARG;
    if (B < 0) return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "negative batch");
    hsla_opts o;
    if (opts)
        o = *opts;
    else
        hsla_opts_default(&o);
    return hsla::workspace_size(h, p, B, o, bytes);
}

hsla_status hsla_autotune(hsla_handle *h, hsla_pattern *p, int32_t B, int32_t effort, hsla_tuning *out,
                          void *stream) {
    hsla_status st = hsla::check_common(h, p, B, (hipStream_t)stream);
    if (st != HSLA_OK) return st;
    if (B < 1 || B > 65535 || effort < 1 || effort > 100)
        return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "autotune needs 1 <= B <= 65535 and 1 <= effort <= 100");
    if (p->n == 0) {
        if (out) *out = hsla_tuning{p->stA.mask ? 0 : 1, 0, 0.0, 0.0};
        return HSLA_OK;
    }
    st = hsla::autotune(h, p, B, effort, out, h->stream);
    if (st != HSLA_OK) return st;
    HSLA_HIP(h, hipStreamSynchronize(h->stream));
    return HSLA_OK;
}


hsla_status hsla_spmv(hsla_handle *h, const hsla_pattern *p, int32_t B, const double *d_values, const double *d_x,
                      double *d_y, void *stream) {
    hsla_status st = hsla::check_common(h, p, B, (hipStream_t)stream);
    if (st != HSLA_OK) return st;
    if (B > 0 && p->n > 0 && (!d_values || !d_x || !d_y))
        return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "null pointer");
    st = hsla::launch_spmv(h, p, B, d_values, d_x, d_y, h->stream);
    if (st != HSLA_OK) return st;
    HSLA_HIP(h, hipStreamSynchronize(h->stream));
    return HSLA_OK;
}

hsla_status hsla_solve(hsla_handle *h, const hsla_pattern *p, const double *d_values, const double *d_b, double *d_x,
                       const hsla_opts *opts, hsla_info *info, void *stream) {
    return hsla::solve_entry(h, p, 1, d_values, d_b, d_x, opts, info, (hipStream_t)stream);
}

hsla_status hsla_solve_batched(hsla_handle *h, const hsla_pattern *p, int32_t B, const double *d_values,
                               const double *d_b, double *d_x, const hsla_opts *opts, hsla_info *infos, void *stream) {
    return hsla::solve_entry(h, p, B, d_values, d_b, d_x, opts, infos, (hipStream_t)stream);
}

hsla_status hsla_adjoint(hsla_handle *h, const hsla_pattern *p, const double *d_values, const double *d_x,
                         const double *d_gx, double *d_gA, double *d_gb, const hsla_opts *opts, hsla_info *info,
                         void *stream) {
    return hsla::adjoint_entry(h, p, 1, d_values, d_x, d_gx, d_gA, d_gb, opts, info, (hipStream_t)stream);
}

hsla_status hsla_adjoint_batched(hsla_handle *h, const hsla_pattern *p, int32_t B, const double *d_values,
                                 const double *d_x, const double *d_gx, double *d_gA, double *d_gb,
                                 const hsla_opts *opts, hsla_info *infos, void *stream) {
    return hsla::adjoint_entry(h, p, B, d_values, d_x, d_gx, d_gA, d_gb, opts, infos, (hipStream_t)stream);
}

hsla_status hsla_outer_on_pattern(hsla_handle *h, const hsla_pattern *p, int32_t B, const double *d_lambda,
                                  const double *d_x, double *d_gA, void *stream) {
    hsla_status st = hsla::check_common(h, p, B, (hipStream_t)stream);
    if (st != HSLA_OK) return st;
    if (B == 0 || p->n == 0) return HSLA_OK;
    if (!d_lambda || !d_x || !d_gA) return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "null pointer");
    int G = (int)((p->n + hsla::kBlock - 1) / hsla::kBlock);
    if (G > 4096) G = 4096;
    hsla::k_outer<<<dim3(G, B), hsla::kBlock, 0, h->stream>>>(p->n, p->nnz, p->row_ptr, p->col, d_lambda, d_x, d_gA);
    HSLA_HIP(h, hipGetLastError());
    HSLA_HIP(h, hipStreamSynchronize(h->stream));
    return HSLA_OK;
}

hsla_status hsla_residual_norms(hsla_handle *h, const hsla_pattern *p, int32_t B, const double *d_values,
                                const double *d_b, const double *d_x, double *res_norm, double *b_norm, void *stream) {
    hsla_status st = hsla::check_common(h, p, B, (hipStream_t)stream);
    if (st != HSLA_OK) return st;
    if (B == 0) return HSLA_OK;
    if (p->n > 0 && (!d_values || !d_b || !d_x)) return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "null pointer");
    hipStream_t s = h->stream;
    const int G = hsla::grid_blocks(h, hsla::kWavesPerBlock, p->ntiles, B, 16);
    const hsla::Layout lay = hsla::make_layout(B, p->n, 0, G);
    st = hsla::ensure_workspace(h, lay.total);
    if (st != HSLA_OK) return st;
    char *ws = (char *)h->ws;
    hsla::Sys S{};
    S.val = d_values;
    S.aval = d_values;
    S.b = d_b;
    S.x = const_cast<double *>(d_x);
    S.st = (hsla::SysState *)(ws + lay.off_state);
    S.part = (double *)(ws + lay.off_part);
    hsla::k_reset<<<1, hsla::kBlock, 0, s>>>(S.st, B, 1, 0);
    const hsla::Pat A = hsla::pat_of(p);
    double *res = (double *)(ws + lay.off_res);
    std::vector<double> hr(2 * (size_t)B, 0.0);
    if (p->n > 0) {
        hsla::k_residual<<<dim3(G, B), hsla::kBlock, 0, s>>>(A, S);
        hsla::k_fin_residual<<<dim3(B), hsla::kBlock, 0, s>>>(S, G, res);
        HSLA_HIP(h, hipGetLastError());
        HSLA_HIP(h, hipMemcpyAsync(hr.data(), res, sizeof(double) * 2 * B, hipMemcpyDeviceToHost, s));
    }
    HSLA_HIP(h, hipStreamSynchronize(s));
    for (int i = 0; i < B; ++i) {
        if (res_norm) res_norm[i] = std::sqrt(hr[2 * i]);
        if (b_norm) b_norm[i] = std::sqrt(hr[2 * i + 1]);
    }
    return HSLA_OK;
}

}  // extern "C"
