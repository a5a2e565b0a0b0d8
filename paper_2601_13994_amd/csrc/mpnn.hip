// Learned factorized sparse approximate inverse: the message-passing network
// that maps A to G^ on A's lower pattern, its backward pass, the probe loss
// ||G^ A^ G^^T z - z||^2 with its gradient, Adam, and the conversion of G^ to
// the factors the FSAI-preconditioned CG applies (G = G^ D^{-1/2} and G^T).
//
// Network (hidden 64, three message-passing layers, bf16 weights and
// activations, fp32 accumulation; dense layers on the matrix cores with
// gfx950's v_mfma_f32_16x16x32_bf16, K in steps of 32):
//   f_k   = [a^_k, [j<i], [j>i], [j=i]],  a^_k = a_k / sqrt(a_ii a_jj)
//   h0_i  = relu(sum_{k in row i} f_k W0 + b0)
//   m_i   = sum_{k in row i} (f_k C_l) * h_{col k}            l = 1..3
//   h_i   = relu([h_i, m_i] W_l + b_l)
//   g^_k  = head([h_i, h_j, f_k]) for lower entries k = (i, j), j <= i:
//           z = relu(x H1 + c1), t = z.H2 + c2, g^ = softplus(t) on the
//           diagonal (positive, so G^T G stays SPD) and t elsewhere.
// The paper lists learned preconditioners as future work; this network is
// this project's design.
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace hsla {
namespace mp {

constexpr int HID = 64, HEAD = 32, NF = 4, LAYERS = 3;
constexpr int KH = 2 * HID + NF;  // 132 head inputs
constexpr int KHP = 160;          // padded to 5 k-steps of 32
constexpr int KHT = 144;          // 9 row tiles of 16 cover the 132 inputs (weight gradient)

// Packed fp32 parameter layout (master copy, Adam state, gradients).
constexpr int OFF_W0 = 0, OFF_B0 = OFF_W0 + NF * HID;
constexpr int LAYER0 = OFF_B0 + HID;
constexpr int L_C = 0, L_W = NF * HID, L_B = L_W + 2 * HID * HID, L_SIZE = L_B + HID;
constexpr int OFF_H1 = LAYER0 + LAYERS * L_SIZE;
constexpr int OFF_C1 = OFF_H1 + KH * HEAD;
constexpr int OFF_H2 = OFF_C1 + HEAD;
constexpr int OFF_C2 = OFF_H2 + HEAD;
constexpr int NPARAM = OFF_C2 + 1;
__host__ __device__ constexpr int off_layer(int l) { return LAYER0 + (l - 1) * L_SIZE; }

typedef short short8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// One 16x16x32 product on the matrix cores: lane (i, q) = (l % 16, l / 16)
// brings A[i][8q + t] and B[8q + t][i] (t = 0..7) and holds
// C[4q + t][i] (t = 0..3) of the accumulator.
__device__ __forceinline__ float4_t mfma32(short8_t a, short8_t b, float4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                   c, 0, 0, 0);
}
__device__ __forceinline__ short8_t ld8(const uint16_t *p) { return *reinterpret_cast<const short8_t *>(p); }

// float -> bfloat16 bits, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float rbf(float x) { return bf2f(f2bf(x)); }

// Swizzled B operand of a K x N bf16 matrix (K a multiple of 32) for the
// 16x16x32 product: fragment (ks, nt) holds, for lane l,
// B[32 ks + 8 (l/16) + t][16 nt + l%16], t = 0..7, stored as 8 consecutive
// bf16 (one 16-byte load) at ((ks * NT + nt) * 64 + l) * 8.
__device__ __forceinline__ void put_bfrag(uint16_t *dst, int NT, int k, int n, float v) {
    const int ks = k / 32, kr = k % 32, q = kr / 8, t = kr % 8;
    const int nt = n / 16, i = n % 16;
    dst[((size_t)(ks * NT + nt) * 64 + q * 16 + i) * 8 + t] = f2bf(v);
}

// Device copies of the weights derived from the fp32 master.
struct Weights {
    float *wq;        // [NPARAM] master with every matrix rounded to bf16
    uint16_t *Wf[3];  // W_l   as B fragments: K = 128, N = 64
    uint16_t *WTf[3]; // W_l^T as B fragments: K = 64,  N = 128
    uint16_t *H1f;    // H1 (padded to K = 160) as B fragments, N = 32
    uint16_t *H1Tf;   // H1^T restricted to its first 128 columns: K = 32, N = 128
};

__global__ void k_mp_weights(const float *__restrict__ P, Weights w) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nth = gridDim.x * blockDim.x;
    for (int e = tid; e < NPARAM; e += nth) {
        bool mat = (e < OFF_B0) || (e >= OFF_H1 && e < OFF_C1) || (e >= OFF_H2 && e < OFF_C2);
        for (int l = 1; l <= LAYERS; ++l) {
            const int o = off_layer(l);
            if (e >= o && e < o + L_B) mat = true;
        }
        w.wq[e] = mat ? rbf(P[e]) : P[e];
    }
    for (int l = 1; l <= LAYERS; ++l) {
        const float *W = P + off_layer(l) + L_W;  // [128][64]
        for (int e = tid; e < 2 * HID * HID; e += nth) {
            const int k = e / HID, n = e % HID;
            put_bfrag(w.Wf[l - 1], HID / 16, k, n, W[e]);
            put_bfrag(w.WTf[l - 1], 2 * HID / 16, n, k, W[e]);  // W^T[n][k]
        }
    }
    const float *H1 = P + OFF_H1;  // [132][32]
    for (int e = tid; e < KHP * HEAD; e += nth) {
        const int k = e / HEAD, n = e % HEAD;
        put_bfrag(w.H1f, HEAD / 16, k, n, k < KH ? H1[k * HEAD + n] : 0.0f);
    }
    for (int e = tid; e < HEAD * 2 * HID; e += nth) {
        const int k = e / (2 * HID), n = e % (2 * HID);  // H1^T[k][n] = H1[n][k]
        put_bfrag(w.H1Tf, 2 * HID / 16, k, n, H1[n * HEAD + k]);
    }
}

// ---------------------------------------------------------------------------
// Generic bf16 GEMM on the matrix cores: C[M x 16NT] = A[M x 32KS] B.
// A row r is the concatenation of A0[r][0:K0] and A1[r][0:K-K0] (bf16,
// leading dimensions lda0/lda1 multiples of 8, K0 a multiple of 8, so that
// each lane's 8 operands are one aligned 16-byte load from one of them).  Each wave computes 16
// rows; rows past M are clamped on load and skipped on store.  The epilogue
// gets (row, col, accumulated value) for every valid element.
// ---------------------------------------------------------------------------
template <int KS, int NT, class Epi>
__global__ __launch_bounds__(kBlock) void k_gemm(int64_t M, const uint16_t *__restrict__ A0, int lda0,
                                                 const uint16_t *__restrict__ A1, int lda1, int K0,
                                                 const uint16_t *__restrict__ Bf, Epi epi) {
    const int lane = threadIdx.x & 63, i = lane & 15, q = lane >> 4;
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; tile * 16 < M; tile += waves) {
        const int64_t row0 = tile * 16;
        int64_t ra = row0 + i;
        if (ra >= M) ra = M - 1;
        float4_t acc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int k = ks * 32 + 8 * q;
            const short8_t a = ld8(k < K0 ? A0 + ra * lda0 + k : A1 + ra * lda1 + (k - K0));
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[nt] = mfma32(a, ld8(Bf + ((size_t)(ks * NT + nt) * 64 + lane) * 8), acc[nt]);
        }
        epi(row0, q, i, acc);
    }
}

// Epilogue: + bias, relu, store bf16 (row-major, ld = 16 NT).
template <int NT>
struct EpiBiasReluBf16 {
    const float *bias;
    uint16_t *out;
    int64_t M;
    __device__ void operator()(int64_t row0, int q, int i, float4_t (&acc)[NT]) const {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t r = row0 + 4 * q + t;
            if (r >= M) continue;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int c = nt * 16 + i;
                out[r * (16 * NT) + c] = f2bf(fmaxf(acc[nt][t] + bias[c], 0.f));
            }
        }
    }
};

// Epilogue: store fp32 (row-major, ld = 16 NT).
template <int NT>
struct EpiStoreF32 {
    float *out;
    int64_t M;
    __device__ void operator()(int64_t row0, int q, int i, float4_t (&acc)[NT]) const {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t r = row0 + 4 * q + t;
            if (r >= M) continue;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) out[r * (16 * NT) + nt * 16 + i] = acc[nt][t];
        }
    }
};

// Head epilogue: z = relu(acc + c1) (bf16, saved), t = z.H2 + c2, and
// g^ = softplus(t) on diagonal entries, t elsewhere.  The 32 z values of a
// row sit on the 16 lanes sharing q (two column tiles); their dot product
// with H2 is a butterfly over those lanes.
struct EpiHead {
    const float *wq;  // rounded parameters (c1, H2, c2)
    uint16_t *z;      // [M][32]
    float *t;         // [M]
    float *g;         // [M]
    const uint8_t *isdiag;  // [nnzL] (entry within one system)
    int64_t nL, M;
    __device__ void operator()(int64_t row0, int q, int i, float4_t (&acc)[2]) const {
        const float *c1 = wq + OFF_C1, *H2 = wq + OFF_H2;
        const float c2 = wq[OFF_C2];
#pragma unroll
        for (int tt = 0; tt < 4; ++tt) {
            const int64_t r = row0 + 4 * q + tt;
            float part = 0.f;
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                const int c = nt * 16 + i;
                const float zz = rbf(fmaxf(acc[nt][tt] + c1[c], 0.f));
                if (z && r < M) z[r * HEAD + c] = f2bf(zz);
                part += zz * H2[c];
            }
            // sum over the 16 lanes of this q (fixed butterfly)
            part += __shfl_xor(part, 1, 16);
            part += __shfl_xor(part, 2, 16);
            part += __shfl_xor(part, 4, 16);
            part += __shfl_xor(part, 8, 16);
            if (i == 0 && r < M) {
                const float tv = part + c2;
                if (t) t[r] = tv;
                const bool d = isdiag[r % nL] != 0;
                g[r] = d ? (tv > 20.f ? tv : log1pf(expf(tv))) : tv;
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Weight gradients: C[K x N] += A^T B with A [M x K] (two column blocks as
// in k_gemm) and B [M x N] (bf16).  Block b sums rows of its own contiguous
// chunk, 32 at a time, with MFMA (A^T fragment: lane (i, q) holds
// A[m + 8q + t][16 kt + i], t = 0..7)
// and writes a partial; k_sum_partials adds the partials in block order.
// Wave w of the block owns output fragments f = w, w + 4, ... of the
// (K/16) x (N/16) grid.
// ---------------------------------------------------------------------------
template <int KT, int NT>
__global__ __launch_bounds__(kBlock) void k_gemm_tn(int64_t M, const uint16_t *__restrict__ A0, int lda0,
                                                    const uint16_t *__restrict__ A1, int lda1, int K0,
                                                    const uint16_t *__restrict__ Bm, int ldb,
                                                    float *__restrict__ part) {
    constexpr int NFRAG = KT * NT;
    constexpr int PER = (NFRAG + kWavesPerBlock - 1) / kWavesPerBlock;
    constexpr int KW = KT * 16, NW = NT * 16;  // columns of A and B the product uses
    // 32 rows of A and B per step, staged with 16-byte coalesced loads; the
    // MFMA operands (8 consecutive rows of one column per lane) are then
    // read from LDS.  Rows padded by 8 elements: 16-byte aligned, and
    // consecutive rows start on different banks.
    __shared__ __attribute__((aligned(16))) uint16_t sa[32][KW + 8];
    __shared__ __attribute__((aligned(16))) uint16_t sb[32][NW + 8];
    const int lane = threadIdx.x & 63, i = lane & 15, q = lane >> 4, w = threadIdx.x / kWave;
    const int64_t chunk = (M + gridDim.x - 1) / gridDim.x;
    const int64_t m_lo = (int64_t)blockIdx.x * chunk;
    int64_t m_hi = m_lo + chunk;
    if (m_hi > M) m_hi = M;
    float4_t acc[PER];
#pragma unroll
    for (int f = 0; f < PER; ++f) acc[f] = float4_t{0.f, 0.f, 0.f, 0.f};
    // The wave's fragments share one column tile (NT divides the wave
    // count), so its B operand is read once per step.
    static_assert(kWavesPerBlock % NT == 0, "a wave's fragments must share their column tile");
    const int nt = w % NT;
    const short8_t zero8 = short8_t{0, 0, 0, 0, 0, 0, 0, 0};
    // the next step's rows are loaded into registers while the current
    // step's products run (a block has few waves to hide the latency with)
    constexpr int EA = 32 * (KW / 8), EB = 32 * (NW / 8);
    constexpr int RA = (EA + kBlock - 1) / kBlock, RB = (EB + kBlock - 1) / kBlock;
    short8_t ra[RA], rb[RB];
    auto fetch = [&](int64_t m) {
#pragma unroll
        for (int u = 0; u < RA; ++u) {
            const int e = threadIdx.x + u * kBlock;
            const int r = e / (KW / 8), k = (e % (KW / 8)) * 8;
            const int64_t row = m + r;
            ra[u] = zero8;
            if (e < EA && row < m_hi) ra[u] = ld8(k < K0 ? A0 + row * lda0 + k : A1 + row * lda1 + (k - K0));
        }
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const int e = threadIdx.x + u * kBlock;
            const int r = e / (NW / 8), k = (e % (NW / 8)) * 8;
            const int64_t row = m + r;
            rb[u] = zero8;
            if (e < EB && row < m_hi) rb[u] = ld8(Bm + row * ldb + k);
        }
    };
    if (m_lo < m_hi) fetch(m_lo);
    for (int64_t m = m_lo; m < m_hi; m += 32) {
#pragma unroll
        for (int u = 0; u < RA; ++u) {
            const int e = threadIdx.x + u * kBlock;
            if (e < EA) *reinterpret_cast<short8_t *>(&sa[e / (KW / 8)][(e % (KW / 8)) * 8]) = ra[u];
        }
#pragma unroll
        for (int u = 0; u < RB; ++u) {
            const int e = threadIdx.x + u * kBlock;
            if (e < EB) *reinterpret_cast<short8_t *>(&sb[e / (NW / 8)][(e % (NW / 8)) * 8]) = rb[u];
        }
        __syncthreads();
        if (m + 32 < m_hi) fetch(m + 32);
        short8_t bv;
#pragma unroll
        for (int t = 0; t < 8; ++t) bv[t] = (short)sb[8 * q + t][nt * 16 + i];
#pragma unroll
        for (int f = 0; f < PER; ++f) {
            const int fr = w + f * kWavesPerBlock;
            if (fr >= NFRAG) continue;
            const int k = (fr / NT) * 16 + i;
            short8_t av;
#pragma unroll
            for (int t = 0; t < 8; ++t) av[t] = (short)sa[8 * q + t][k];
            acc[f] = mfma32(av, bv, acc[f]);
        }
        __syncthreads();
    }
    float *out = part + (size_t)blockIdx.x * (KT * 16) * (NT * 16);
#pragma unroll
    for (int f = 0; f < PER; ++f) {
        const int fr = w + f * kWavesPerBlock;
        if (fr >= NFRAG) continue;
        const int kt = fr / NT;
#pragma unroll
        for (int t = 0; t < 4; ++t) out[(size_t)(kt * 16 + 4 * q + t) * (NT * 16) + nt * 16 + i] = acc[f][t];
    }
}

// dst[e] (+)= sum_b part[b][e]: four running sums over b mod 4 (sixteen
// loads in flight per step), combined as (s0 + s1) + (s2 + s3) -- a fixed
// order, so the result is deterministic; rows >= rows_valid of a
// [rows x cols] partial are dropped (padding of the head's K).
__global__ void k_sum_partials(const float *__restrict__ part, int nb, int rows, int cols, int rows_valid,
                               float *__restrict__ dst, int accumulate) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows_valid * cols) return;
    const size_t stride = (size_t)rows * cols;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    int b = 0;
    for (; b + 16 <= nb; b += 16) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = part[(size_t)(b + u) * stride + e];
#pragma unroll
        for (int u = 0; u < 16; ++u) s[u & 3] += v[u];
    }
    for (; b < nb; ++b) s[b & 3] += part[(size_t)b * stride + e];
    const double t = (s[0] + s[1]) + (s[2] + s[3]);
    dst[e] = accumulate ? dst[e] + (float)t : (float)t;
}

// ---------------------------------------------------------------------------
// Graph kernels (VALU)
// ---------------------------------------------------------------------------
struct Graph {
    int32_t n;
    int64_t nnz, nL;
    const int32_t *rp, *col, *diag;     // A
    const int32_t *rpT, *colT, *srcT;   // A^T (srcT: position in A)
    const int32_t *rpL, *colL, *posL;   // lower triangle (posL: position in A)
    const int32_t *rpU, *colU, *srcU;   // L^T (srcU: position in L)
    const int32_t *rowL;                // row of each lower entry
    const uint8_t *isdiag;              // lower entry on the diagonal
};

// Scaled values a^ = a / sqrt(a_ii a_jj): fp64 (probe loss) and fp32 (features).
// Sixteen lanes per node, one entry of its row per lane (rows longer than 16
// take further turns), so that the column -> diagonal -> value loads of a
// row's entries are in flight together.
__global__ void k_mp_scale(Graph g, int B, const double *__restrict__ val, double *__restrict__ ah64,
                           float *__restrict__ ah32, int32_t *bad) {
    const int l16 = threadIdx.x & 15;
    const int64_t total = (int64_t)B * g.n;
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / 16);
    for (int64_t e = (int64_t)blockIdx.x * (blockDim.x / 16) + threadIdx.x / 16; e < total; e += groups) {
        const int64_t s = e / g.n;
        const int32_t i = (int32_t)(e - s * g.n);
        const double *v = val + s * g.nnz;
        const int32_t di = g.diag[i];
        const double aii = di >= 0 ? v[di] : 0.0;
        if (!(aii > 0.0)) {
            if (l16 == 0) *bad = 1;
            continue;
        }
        for (int32_t k = g.rp[i] + l16; k < g.rp[i + 1]; k += 16) {
            const int32_t j = g.col[k];
            const int32_t dj = g.diag[j];
            const double ajj = dj >= 0 ? v[dj] : 0.0;
            const double a = v[k] / (sqrt(aii) * sqrt(ajj));
            ah64[s * g.nnz + k] = a;
            ah32[s * g.nnz + k] = (float)a;
        }
    }
}

__device__ __forceinline__ void feats(const Graph &g, const float *ah, int64_t k, int32_t i, float f[4]) {
    const int32_t j = g.col[k];
    f[0] = ah[k];
    f[1] = j < i ? 1.f : 0.f;
    f[2] = j > i ? 1.f : 0.f;
    f[3] = j == i ? 1.f : 0.f;
}

// h0 = relu(s W0 + b0), s_i = sum_{k in row i} f_k.  Four nodes per wave,
// 16 lanes per node, 4 channels per lane; a row's entries are loaded 8 at
// a time and their features summed in order.
__global__ __launch_bounds__(kBlock) void k_mp_init(Graph g, int B, const float *__restrict__ wq,
                                                    const float *__restrict__ ah, uint16_t *__restrict__ h0) {
    const int lane = threadIdx.x & 63;
    const int c0 = (lane & 15) * 4;
    const int64_t total = (int64_t)B * g.n;
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t node = wave * 4 + (lane >> 4); node < total; node += nwaves * 4) {
        const int64_t s = node / g.n;
        const int32_t i = (int32_t)(node - s * g.n);
        const float *a = ah + s * g.nnz;
        float sf[4] = {0.f, 0.f, 0.f, 0.f};
        const int32_t lo = g.rp[i], hi = g.rp[i + 1];
        for (int32_t k0 = lo; k0 < hi; k0 += 8) {
            int32_t cj[8];
            float av[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                cj[u] = i;
                av[u] = 0.f;
                if (k0 + u < hi) {
                    cj[u] = g.col[k0 + u];
                    av[u] = a[k0 + u];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 + u < hi) {
                    sf[0] += av[u];
                    sf[1] += cj[u] < i ? 1.f : 0.f;
                    sf[2] += cj[u] > i ? 1.f : 0.f;
                    sf[3] += cj[u] == i ? 1.f : 0.f;
                }
        }
        uint16_t hb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + u;
            float acc = wq[OFF_B0 + c];
#pragma unroll
            for (int t = 0; t < 4; ++t) acc += sf[t] * wq[OFF_W0 + t * HID + c];
            hb[u] = f2bf(fmaxf(acc, 0.f));
        }
        uint2 out;
        out.x = (uint32_t)hb[0] | ((uint32_t)hb[1] << 16);
        out.y = (uint32_t)hb[2] | ((uint32_t)hb[3] << 16);
        *reinterpret_cast<uint2 *>(h0 + node * HID + c0) = out;
    }
}

// m_i = sum_{k in row i} (f_k C_l) * h_{col k}.  Four nodes per wave: 16
// lanes per node, 4 channels per lane (one 8-byte load of h per neighbour);
// a row's column indices, features and neighbour rows are loaded 8 entries
// at a time, then summed in ascending entry order.
__global__ __launch_bounds__(kBlock) void k_mp_aggregate(Graph g, int B, const float *__restrict__ C,
                                                         const float *__restrict__ ah, const uint16_t *__restrict__ h,
                                                         uint16_t *__restrict__ m) {
    const int lane = threadIdx.x & 63;
    const int c0 = (lane & 15) * 4;
    float Cc[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) Cc[t][u] = C[t * HID + c0 + u];
    const int64_t total = (int64_t)B * g.n;
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t node = wave * 4 + (lane >> 4); node < total; node += nwaves * 4) {
        const int64_t s = node / g.n;
        const int32_t i = (int32_t)(node - s * g.n);
        const float *a = ah + s * g.nnz;
        const uint16_t *hs = h + s * (int64_t)g.n * HID + c0;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        const int32_t lo = g.rp[i], hi = g.rp[i + 1];
        for (int32_t k0 = lo; k0 < hi; k0 += 8) {
            int32_t cj[8];
            float av[8];
            uint2 hv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                cj[u] = i;
                av[u] = 0.f;
                if (k0 + u < hi) {
                    cj[u] = g.col[k0 + u];
                    av[u] = a[k0 + u];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 + u < hi) hv[u] = *reinterpret_cast<const uint2 *>(hs + (int64_t)cj[u] * HID);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (k0 + u < hi) {
                    const float f[4] = {av[u], cj[u] < i ? 1.f : 0.f, cj[u] > i ? 1.f : 0.f, cj[u] == i ? 1.f : 0.f};
                    const uint16_t hb[4] = {(uint16_t)(hv[u].x & 0xffffu), (uint16_t)(hv[u].x >> 16),
                                            (uint16_t)(hv[u].y & 0xffffu), (uint16_t)(hv[u].y >> 16)};
#pragma unroll
                    for (int ch = 0; ch < 4; ++ch) {
                        const float gate = f[0] * Cc[0][ch] + f[1] * Cc[1][ch] + f[2] * Cc[2][ch] + f[3] * Cc[3][ch];
                        acc[ch] += gate * bf2f(hb[ch]);
                    }
                }
            }
        }
        uint2 out;
        out.x = (uint32_t)f2bf(acc[0]) | ((uint32_t)f2bf(acc[1]) << 16);
        out.y = (uint32_t)f2bf(acc[2]) | ((uint32_t)f2bf(acc[3]) << 16);
        *reinterpret_cast<uint2 *>(m + node * HID + c0) = out;
    }
}

// Head inputs x_k = [h3_i, h3_j, f_k, 0...] (bf16, 160 wide) for lower
// entries.  Four entries per wave, 16 lanes per entry, 8-byte copies.
__global__ __launch_bounds__(kBlock) void k_mp_head_gather(Graph g, int B, const float *__restrict__ ah,
                                                           const uint16_t *__restrict__ h3, uint16_t *__restrict__ X) {
    const int lane = threadIdx.x & 63;
    const int l16 = lane & 15;
    const int64_t total = (int64_t)B * g.nL;
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t e = wave * 4 + (lane >> 4); e < total; e += nwaves * 4) {
        const int64_t s = e / g.nL, kl = e - s * g.nL;
        const int32_t i = g.rowL[kl], j = g.colL[kl];
        const uint16_t *hs = h3 + s * (int64_t)g.n * HID + l16 * 4;
        uint16_t *x = X + e * KHP;
        const uint2 vi = *reinterpret_cast<const uint2 *>(hs + (int64_t)i * HID);
        const uint2 vj = *reinterpret_cast<const uint2 *>(hs + (int64_t)j * HID);
        *reinterpret_cast<uint2 *>(x + l16 * 4) = vi;
        *reinterpret_cast<uint2 *>(x + HID + l16 * 4) = vj;
        float f[4];
        feats(g, ah + s * g.nnz, g.posL[kl], i, f);
        // columns 128..159: the features, then zeros (two per lane)
        const int c = 2 * l16;
        const uint32_t lo = c < NF ? f2bf(f[c < NF ? c : 0]) : 0u;
        const uint32_t hi = c + 1 < NF ? f2bf(f[c + 1 < NF ? c + 1 : 0]) : 0u;
        *reinterpret_cast<uint32_t *>(x + 2 * HID + c) = lo | (hi << 16);
    }
}

// Inference head without the x_k buffer: the GEMM's A operand is fetched
// straight from h3 (rows i and j of the entry) and the features, giving the
// same bf16 operand values as k_mp_head_gather + k_gemm<5, 2>.
__global__ __launch_bounds__(kBlock) void k_mp_head_fused(Graph g, int64_t M, const float *__restrict__ ah,
                                                          const uint16_t *__restrict__ h3,
                                                          const uint16_t *__restrict__ Bf, EpiHead epi) {
    const int lane = threadIdx.x & 63, i = lane & 15, q = lane >> 4;
    const int64_t waves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; tile * 16 < M; tile += waves) {
        const int64_t row0 = tile * 16;
        int64_t ra = row0 + i;
        if (ra >= M) ra = M - 1;
        const int64_t s = ra / g.nL, kl = ra - s * g.nL;
        const int32_t ni = g.rowL[kl], nj = g.colL[kl];
        const uint16_t *hs = h3 + s * (int64_t)g.n * HID + 8 * q;
        short8_t fa = short8_t{0, 0, 0, 0, 0, 0, 0, 0};
        if (q == 0) {
            float f[4];
            feats(g, ah + s * g.nnz, g.posL[kl], ni, f);
            fa = short8_t{(short)f2bf(f[0]), (short)f2bf(f[1]), (short)f2bf(f[2]), (short)f2bf(f[3]), 0, 0, 0, 0};
        }
        float4_t acc[2];
        acc[0] = acc[1] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 5; ++ks) {
            short8_t a;
            if (ks < 2)
                a = ld8(hs + (int64_t)ni * HID + ks * 32);
            else if (ks < 4)
                a = ld8(hs + (int64_t)nj * HID + (ks - 2) * 32);
            else
                a = fa;
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) acc[nt] = mfma32(a, ld8(Bf + ((size_t)(ks * 2 + nt) * 64 + lane) * 8), acc[nt]);
        }
        epi(row0, q, i, acc);
    }
}

// Head backward, per lower entry: dt = dg * (sigmoid(t) on the diagonal, 1
// elsewhere), dz = bf16(dt H2 * [z > 0]); block partials laid out like the
// parameters [c1 (32), H2 (32), c2]: dc1 = sum dz, dH2 = sum z dt, dc2 = sum dt.
// Eight entries per wave, 8 lanes per entry, 4 channels per lane (8-byte
// accesses of z and dz).
__global__ __launch_bounds__(kBlock) void k_mp_head_bwd(Graph g, int64_t M, const float *__restrict__ wq,
                                                        const float *__restrict__ dg, const float *__restrict__ t,
                                                        const uint16_t *__restrict__ z, uint16_t *__restrict__ dz,
                                                        float *__restrict__ part) {
    __shared__ float sh[kWavesPerBlock][2 * HEAD + 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x / kWave;
    const int c0 = (lane & 7) * 4, sub = lane >> 3;
    float H2c[4], pH2[4], pc1[4], pc2 = 0.f;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        H2c[u] = wq[OFF_H2 + c0 + u];
        pH2[u] = pc1[u] = 0.f;
    }
    for (int64_t e = ((int64_t)blockIdx.x * kWavesPerBlock + w) * 8 + sub; e < M;
         e += (int64_t)gridDim.x * kWavesPerBlock * 8) {
        const bool d = g.isdiag[e % g.nL] != 0;
        const float tv = t[e];
        const float dt = d ? dg[e] / (1.f + expf(-tv)) : dg[e];
        const uint2 zv = *reinterpret_cast<const uint2 *>(z + e * HEAD + c0);
        const float zz[4] = {bf2f((uint16_t)(zv.x & 0xffffu)), bf2f((uint16_t)(zv.x >> 16)),
                             bf2f((uint16_t)(zv.y & 0xffffu)), bf2f((uint16_t)(zv.y >> 16))};
        uint16_t db[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            db[u] = f2bf(zz[u] > 0.f ? dt * H2c[u] : 0.f);
            pH2[u] += zz[u] * dt;
            pc1[u] += bf2f(db[u]);
        }
        uint2 o;
        o.x = (uint32_t)db[0] | ((uint32_t)db[1] << 16);
        o.y = (uint32_t)db[2] | ((uint32_t)db[3] << 16);
        *reinterpret_cast<uint2 *>(dz + e * HEAD + c0) = o;
        if ((lane & 7) == 0) pc2 += dt;
    }
    // the eight entries of a wave share channels (fixed butterfly), then
    // the waves of the block in order
#pragma unroll
    for (int x = 8; x < 64; x *= 2) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pH2[u] += __shfl_xor(pH2[u], x);
            pc1[u] += __shfl_xor(pc1[u], x);
        }
        pc2 += __shfl_xor(pc2, x);
    }
    if (lane < 8) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            sh[w][c0 + u] = pc1[u];
            sh[w][HEAD + c0 + u] = pH2[u];
        }
    }
    if (lane == 0) sh[w][2 * HEAD] = pc2;
    __syncthreads();
    if (threadIdx.x < 2 * HEAD + 1) {
        float s = 0.f;
        for (int q = 0; q < kWavesPerBlock; ++q) s += sh[q][threadIdx.x];
        part[(size_t)blockIdx.x * (2 * HEAD + 1) + threadIdx.x] = s;
    }
}

// dh3_i = sum over lower entries k of row i of dX[k][0:64]
//       + sum over lower entries k with column i of dX[k][64:128]
// (the second sum walks row i of L^T, whose src gives the entry in L).
// Four nodes per wave, 16 lanes per node, 4 channels per lane (16-byte
// loads); each sum's entries are loaded 8 at a time and added in order.
__global__ __launch_bounds__(kBlock) void k_mp_head_dh(Graph g, int B, const float *__restrict__ dX,
                                                       float *__restrict__ dh) {
    const int lane = threadIdx.x & 63;
    const int c0 = (lane & 15) * 4;
    const int64_t total = (int64_t)B * g.n;
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t node = wave * 4 + (lane >> 4); node < total; node += nwaves * 4) {
        const int64_t s = node / g.n;
        const int32_t i = (int32_t)(node - s * g.n);
        const float *d = dX + s * g.nL * (2 * HID) + c0;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        auto walk = [&](int32_t lo, int32_t hi, const int32_t *src, int off) {
            for (int32_t k0 = lo; k0 < hi; k0 += 8) {
                float4 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (k0 + u < hi) {
                        const int64_t e = src ? src[k0 + u] : k0 + u;
                        v[u] = *reinterpret_cast<const float4 *>(d + e * 2 * HID + off);
                    }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (k0 + u < hi) {
                        acc[0] += v[u].x;
                        acc[1] += v[u].y;
                        acc[2] += v[u].z;
                        acc[3] += v[u].w;
                    }
            }
        };
        walk(g.rpL[i], g.rpL[i + 1], nullptr, 0);
        walk(g.rpU[i], g.rpU[i + 1], g.srcU, HID);
        *reinterpret_cast<float4 *>(dh + node * HID + c0) = float4{acc[0], acc[1], acc[2], acc[3]};
    }
}

// dpre = bf16(dh * [h > 0]) and block partials of db = sum dpre.
__global__ __launch_bounds__(kBlock) void k_mp_relu_bwd(int64_t rows, const float *__restrict__ dh,
                                                        const uint16_t *__restrict__ h, uint16_t *__restrict__ dpre,
                                                        float *__restrict__ part) {
    __shared__ float sh[kWavesPerBlock][HID];
    const int c = threadIdx.x & 63, w = threadIdx.x / kWave;
    float pb = 0.f;
    for (int64_t r = (int64_t)blockIdx.x * kWavesPerBlock + w; r < rows; r += (int64_t)gridDim.x * kWavesPerBlock) {
        const float v = bf2f(h[r * HID + c]) > 0.f ? dh[r * HID + c] : 0.f;
        const uint16_t b = f2bf(v);
        dpre[r * HID + c] = b;
        pb += bf2f(b);
    }
    sh[w][c] = pb;
    __syncthreads();
    if (threadIdx.x < HID) {
        float s = 0.f;
        for (int q = 0; q < kWavesPerBlock; ++q) s += sh[q][threadIdx.x];
        part[(size_t)blockIdx.x * HID + threadIdx.x] = s;
    }
}

// Aggregation backward: dh_prev_j = dhm[j][0:64] + sum_{k: col k = j} gate_k *
// dm_{row k}, walking row j of A^T; block partials of dC = sum_k f_k^T
// (dm_{row k} * h_{col k}) (4 x 64).  Laid out like k_mp_aggregate: four
// nodes per wave, 16 lanes per node, 4 channels per lane (16-byte loads of
// dm); a row's transposed entries are loaded 8 at a time, then summed in
// ascending order.  An entry of row j of A^T has column j in A, so its
// features need only its row i and value.
__global__ __launch_bounds__(kBlock) void k_mp_aggregate_bwd(Graph g, int B, const float *__restrict__ C,
                                                             const float *__restrict__ ah,
                                                             const uint16_t *__restrict__ hprev,
                                                             const float *__restrict__ dhm, float *__restrict__ dh_out,
                                                             float *__restrict__ part) {
    __shared__ float sh[kWavesPerBlock][NF * HID];
    const int lane = threadIdx.x & 63, w = threadIdx.x / kWave;
    const int c0 = (lane & 15) * 4;
    float Cc[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) Cc[t][u] = C[t * HID + c0 + u];
    float pC[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) pC[t][u] = 0.f;
    const int64_t total = (int64_t)B * g.n;
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + w;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t node = wave * 4 + (lane >> 4); node < total; node += nwaves * 4) {
        const int64_t s = node / g.n;
        const int32_t j = (int32_t)(node - s * g.n);
        const float *a = ah + s * g.nnz;
        const float *dm = dhm + s * (int64_t)g.n * 2 * HID + HID + c0;  // dm[row][c0..] at dm[row * 128]
        const uint2 hv = *reinterpret_cast<const uint2 *>(hprev + node * HID + c0);
        const float hj[4] = {bf2f((uint16_t)(hv.x & 0xffffu)), bf2f((uint16_t)(hv.x >> 16)),
                             bf2f((uint16_t)(hv.y & 0xffffu)), bf2f((uint16_t)(hv.y >> 16))};
        const float4 d0 = *reinterpret_cast<const float4 *>(dhm + node * 2 * HID + c0);
        float acc[4] = {d0.x, d0.y, d0.z, d0.w};
        const int32_t lo = g.rpT[j], hi = g.rpT[j + 1];
        for (int32_t k0 = lo; k0 < hi; k0 += 8) {
            int32_t ri[8];
            float av[8];
            float4 dv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                ri[u] = j;
                av[u] = 0.f;
                if (k0 + u < hi) {
                    ri[u] = g.colT[k0 + u];
                    av[u] = a[g.srcT[k0 + u]];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 + u < hi) dv[u] = *reinterpret_cast<const float4 *>(dm + (int64_t)ri[u] * 2 * HID);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (k0 + u < hi) {
                    // features of entry (i, j): value, j < i, j > i, j = i
                    const float f[4] = {av[u], j < ri[u] ? 1.f : 0.f, j > ri[u] ? 1.f : 0.f, j == ri[u] ? 1.f : 0.f};
                    const float dmi[4] = {dv[u].x, dv[u].y, dv[u].z, dv[u].w};
#pragma unroll
                    for (int ch = 0; ch < 4; ++ch) {
                        const float gate = f[0] * Cc[0][ch] + f[1] * Cc[1][ch] + f[2] * Cc[2][ch] + f[3] * Cc[3][ch];
                        acc[ch] += gate * dmi[ch];
                        const float prod = dmi[ch] * hj[ch];
#pragma unroll
                        for (int t = 0; t < 4; ++t) pC[t][ch] += f[t] * prod;
                    }
                }
            }
        }
        *reinterpret_cast<float4 *>(dh_out + node * HID + c0) = float4{acc[0], acc[1], acc[2], acc[3]};
    }
    // the four nodes of a wave share channels: lanes l, l + 16, l + 32, l + 48
    // (fixed butterfly), then the waves of the block in order
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pC[t][u] += __shfl_xor(pC[t][u], 16);
            pC[t][u] += __shfl_xor(pC[t][u], 32);
        }
    if (lane < 16) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int u = 0; u < 4; ++u) sh[w][t * HID + c0 + u] = pC[t][u];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NF * HID; e += blockDim.x) {
        float sum = 0.f;
        for (int q = 0; q < kWavesPerBlock; ++q) sum += sh[q][e];
        part[(size_t)blockIdx.x * NF * HID + e] = sum;
    }
}

// Init backward: block partials of dW0 = sum_i s_i^T dpre0_i (4 x 64) and
// db0 = sum dpre0 (64), dpre0 = bf16(dh0 * [h0 > 0]).  Four nodes per wave,
// 16 lanes per node, 4 channels per lane; a row's entries are loaded 8 at a
// time and their features summed in order.
__global__ __launch_bounds__(kBlock) void k_mp_init_bwd(Graph g, int B, const float *__restrict__ ah,
                                                        const uint16_t *__restrict__ h0, const float *__restrict__ dh0,
                                                        float *__restrict__ part) {
    __shared__ float sh[kWavesPerBlock][(NF + 1) * HID];
    const int lane = threadIdx.x & 63, w = threadIdx.x / kWave;
    const int c0 = (lane & 15) * 4;
    float pW[4][4], pb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        pb[u] = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) pW[t][u] = 0.f;
    }
    const int64_t total = (int64_t)B * g.n;
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + w;
    const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t node = wave * 4 + (lane >> 4); node < total; node += nwaves * 4) {
        const int64_t s = node / g.n;
        const int32_t i = (int32_t)(node - s * g.n);
        const float *a = ah + s * g.nnz;
        const uint2 hv = *reinterpret_cast<const uint2 *>(h0 + node * HID + c0);
        const float4 dv = *reinterpret_cast<const float4 *>(dh0 + node * HID + c0);
        const float hb[4] = {bf2f((uint16_t)(hv.x & 0xffffu)), bf2f((uint16_t)(hv.x >> 16)),
                             bf2f((uint16_t)(hv.y & 0xffffu)), bf2f((uint16_t)(hv.y >> 16))};
        const float dd[4] = {dv.x, dv.y, dv.z, dv.w};
        float sf[4] = {0.f, 0.f, 0.f, 0.f};
        const int32_t lo = g.rp[i], hi = g.rp[i + 1];
        for (int32_t k0 = lo; k0 < hi; k0 += 8) {
            int32_t cj[8];
            float av[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                cj[u] = i;
                av[u] = 0.f;
                if (k0 + u < hi) {
                    cj[u] = g.col[k0 + u];
                    av[u] = a[k0 + u];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 + u < hi) {
                    sf[0] += av[u];
                    sf[1] += cj[u] < i ? 1.f : 0.f;
                    sf[2] += cj[u] > i ? 1.f : 0.f;
                    sf[3] += cj[u] == i ? 1.f : 0.f;
                }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const float dp = rbf(hb[u] > 0.f ? dd[u] : 0.f);
#pragma unroll
            for (int t = 0; t < 4; ++t) pW[t][u] += sf[t] * dp;
            pb[u] += dp;
        }
    }
    // the four nodes of a wave share channels (fixed butterfly), then the
    // waves of the block in order
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        pb[u] += __shfl_xor(pb[u], 16);
        pb[u] += __shfl_xor(pb[u], 32);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            pW[t][u] += __shfl_xor(pW[t][u], 16);
            pW[t][u] += __shfl_xor(pW[t][u], 32);
        }
    }
    if (lane < 16) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int t = 0; t < 4; ++t) sh[w][t * HID + c0 + u] = pW[t][u];
            sh[w][NF * HID + c0 + u] = pb[u];
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < (NF + 1) * HID; e += blockDim.x) {
        float sum = 0.f;
        for (int q = 0; q < kWavesPerBlock; ++q) sum += sh[q][e];
        part[(size_t)blockIdx.x * (NF + 1) * HID + e] = sum;
    }
}

// Adam (fp32 master), bias-corrected: p -= lr mhat / (sqrt(vhat) + eps).
__global__ void k_adam(int n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gi;
    const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// Probe loss  sum_p ||G^ A^ G^^T z - z||^2  and its gradient on G^'s pattern
// ---------------------------------------------------------------------------

// GT[s][k'] = G[s][srcU[k']] (values of L^T in its CSR order).
__global__ void k_perm_f32(int64_t nL, int B, const float *__restrict__ G, const int32_t *__restrict__ src,
                           float *__restrict__ GT) {
    const int64_t total = nL * B;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = e / nL, k = e - s * nL;
        GT[e] = G[s * nL + src[k]];
    }
}

struct SpPat {
    const int32_t *rp, *col;
    const int2 *meta;
    int32_t ntiles;
    int64_t nnz;
};

// y[bp] = M_s x[bp] for bp = system s * P + probe, values of system s.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_bspmv(SpPat A, int P, int32_t n, const VT *__restrict__ val,
                                                  const double *__restrict__ x, double *__restrict__ y) {
    __shared__ double lds[kWavesPerBlock][kTileCap];
    const int64_t bp = blockIdx.y;
    const VT *v = val + (bp / P) * A.nnz;
    const double *xb = x + bp * n;
    double *yb = y + bp * n;
    spmv_tiles(A.rp, A.col, Stencil{}, v, xb, A.meta, A.ntiles, lds[threadIdx.x / kWave],
               [&](int32_t row, double yv) { yb[row] = yv; });
}

// e = v - z and per-(system, probe) block partials of ||e||^2.
__global__ __launch_bounds__(kBlock) void k_probe_err(int32_t n, const double *__restrict__ v,
                                                      const double *__restrict__ z, double *__restrict__ e,
                                                      double *__restrict__ part) {
    const int64_t bp = blockIdx.y;
    double acc[1] = {0.0};
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const double d = v[bp * n + i] - z[bp * n + i];
        e[bp * n + i] = d;
        acc[0] += d * d;
    }
    block_partial<1>(acc, part + bp * gridDim.x);
}

__global__ void k_probe_loss_fin(int B, int P, int G, const double *__restrict__ part, double *__restrict__ loss) {
    const int s = blockIdx.x;
    double tot = 0.0;
    if (threadIdx.x == 0) {
        for (int p = 0; p < P; ++p)
            for (int b = 0; b < G; ++b) tot += part[((int64_t)s * P + p) * G + b];
        loss[s] = tot;
    }
}

// dG^[s][k] = scale * sum_p 2 (e_i u_j + z_i y_j) for lower entry k = (i, j).
__global__ void k_probe_grad(int64_t nL, int B, int P, int32_t n, const int32_t *__restrict__ rowL,
                             const int32_t *__restrict__ colL, const double *__restrict__ e,
                             const double *__restrict__ u, const double *__restrict__ z, const double *__restrict__ y,
                             double scale, float *__restrict__ dG) {
    const int64_t total = nL * B;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = q / nL, k = q - s * nL;
        const int32_t i = rowL[k], j = colL[k];
        double acc = 0.0;
        for (int p = 0; p < P; ++p) {
            const int64_t o = (s * P + p) * n;
            acc += 2.0 * (e[o + i] * u[o + j] + z[o + i] * y[o + j]);
        }
        dG[q] = (float)(scale * acc);
    }
}

// FSAI factors for the solver: G[s][k] = G^[s][k] / sqrt(a_jj), GT = G in L^T order.
__global__ void k_fsai_factor(Graph g, int B, const double *__restrict__ val, const float *__restrict__ Gh,
                              float *__restrict__ G) {
    const int64_t total = g.nL * B;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = q / g.nL, k = q - s * g.nL;
        const int32_t j = g.colL[k];
        const double ajj = val[s * g.nnz + g.diag[j]];
        G[q] = (float)((double)Gh[q] / sqrt(ajj));
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

static Graph make_graph(const hsla_pattern *p) {
    Graph g;
    g.n = p->n;
    g.nnz = p->nnz;
    g.nL = p->nnz_lower;
    g.rp = p->row_ptr; g.col = p->col; g.diag = p->diag;
    g.rpT = p->rpT; g.colT = p->colT; g.srcT = p->srcT;
    g.rpL = p->rpL; g.colL = p->colL; g.posL = p->posL;
    g.rpU = p->rpU; g.colU = p->colU; g.srcU = p->srcU;
    g.rowL = p->rowL; g.isdiag = p->isdiagL;
    return g;
}

// Bump allocator over the handle's network workspace.
struct Bump {
    char *base;
    size_t off, cap;
    template <typename T>
    T *take(size_t count) {
        off = (off + 255) / 256 * 256;
        T *r = reinterpret_cast<T *>(base + off);
        off += sizeof(T) * (count > 0 ? count : 1);
        return r;
    }
};

struct Fwd {  // tensors of one kept forward
    Weights w;
    float *ah32;
    double *ah64;
    uint16_t *h[LAYERS + 1], *m[LAYERS];
    uint16_t *X, *z;
    float *t;
    int32_t *bad;
};

static size_t fwd_bytes(int B, const hsla_pattern *p) {
    const size_t n = p->n, nnz = p->nnz, nL = p->nnz_lower;
    size_t b = 0;
    auto add = [&](size_t bytes) { b += (bytes + 255) / 256 * 256 + 256; };
    add(sizeof(float) * NPARAM);
    for (int l = 0; l < LAYERS; ++l) { add(2 * 2 * HID * HID); add(2 * 2 * HID * HID); }
    add(2 * KHP * HEAD);
    add(2 * HEAD * 2 * HID);
    add(sizeof(float) * B * nnz);
    add(sizeof(double) * B * nnz);
    for (int l = 0; l < 2 * LAYERS + 1; ++l) add(2 * B * n * HID);
    add(2 * B * nL * KHP);
    add(2 * B * nL * HEAD);
    add(sizeof(float) * B * nL);
    add(64);
    return b;
}

static Fwd carve_fwd(Bump &bp, int B, const hsla_pattern *p) {
    const size_t n = p->n, nnz = p->nnz, nL = p->nnz_lower;
    Fwd f;
    f.w.wq = bp.take<float>(NPARAM);
    for (int l = 0; l < LAYERS; ++l) {
        f.w.Wf[l] = bp.take<uint16_t>(2 * HID * HID);
        f.w.WTf[l] = bp.take<uint16_t>(2 * HID * HID);
    }
    f.w.H1f = bp.take<uint16_t>(KHP * HEAD);
    f.w.H1Tf = bp.take<uint16_t>(HEAD * 2 * HID);
    f.ah32 = bp.take<float>(B * nnz);
    f.ah64 = bp.take<double>(B * nnz);
    for (int l = 0; l <= LAYERS; ++l) f.h[l] = bp.take<uint16_t>(B * n * HID);
    for (int l = 0; l < LAYERS; ++l) f.m[l] = bp.take<uint16_t>(B * n * HID);
    f.X = bp.take<uint16_t>(B * nL * KHP);
    f.z = bp.take<uint16_t>(B * nL * HEAD);
    f.t = bp.take<float>(B * nL);
    f.bad = bp.take<int32_t>(16);
    return f;
}

static hsla_status ensure_mp_ws(hsla_handle *h, size_t bytes) {
    if (bytes <= h->mp_ws_bytes) return HSLA_OK;
    if (h->mp_ws) {
        HSLA_HIP(h, hipStreamSynchronize(h->stream));
        dev_free(h, h->mp_ws);
        h->mp_ws = nullptr;
        h->mp_ws_bytes = 0;
        h->mp_keep_B = 0;
        h->mp_keep_pattern = nullptr;
    }
    const size_t want = bytes + bytes / 8 + 4096;
    if (dev_alloc(h, &h->mp_ws, want) != hipSuccess) {
        h->mp_ws = nullptr;
        return set_error(h, HSLA_ERR_NO_MEMORY, "network workspace of %zu bytes", want);
    }
    h->mp_ws_bytes = want;
    return HSLA_OK;
}

static int nblocks(int64_t work, int per, int cap) {
    int64_t b = (work + per - 1) / per;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

constexpr int NB_TN = 512;   // blocks of the weight-gradient GEMMs
constexpr int NB_V = 1024;   // blocks of the VALU kernels that write partials

struct Bwd {
    uint16_t *dz, *dpre;
    float *dX, *dh, *dhm, *part;
};

static size_t bwd_reserve(int B, const hsla_pattern *p) {
    const size_t n = p->n, nL = p->nnz_lower;
    size_t b = 0;
    auto add = [&](size_t bytes) { b += (bytes + 255) / 256 * 256 + 256; };
    add(2 * B * nL * HEAD);
    add(2 * B * n * HID);
    add(4 * B * nL * 2 * HID);
    add(4 * B * n * HID);
    add(4 * B * n * 2 * HID);
    add(4 * (size_t)NB_TN * KHP * 2 * HID);
    return b;
}

static Bwd carve_bwd(Bump &bp, int B, const hsla_pattern *p) {
    const size_t n = p->n, nL = p->nnz_lower;
    Bwd w;
    w.dz = bp.take<uint16_t>(B * nL * HEAD);
    w.dpre = bp.take<uint16_t>(B * n * HID);
    w.dX = bp.take<float>(B * nL * 2 * HID);
    w.dh = bp.take<float>(B * n * HID);
    w.dhm = bp.take<float>(B * n * 2 * HID);
    w.part = bp.take<float>((size_t)NB_TN * KHP * 2 * HID);
    return w;
}

static hsla_status forward(hsla_handle *h, const hsla_pattern *p, int B, const double *values, const float *params,
                           float *Ghat, bool keep, hipStream_t s) {
    if (B <= 0) return HSLA_OK;
    const size_t fb = fwd_bytes(B, p);
    hsla_status st = ensure_mp_ws(h, fb + (keep ? bwd_reserve(B, p) : 0));
    if (st != HSLA_OK) return st;
    Bump bp{(char *)h->mp_ws, 0, h->mp_ws_bytes};
    Fwd f = carve_fwd(bp, B, p);
    const Graph g = make_graph(p);
    const int64_t n = p->n, nL = p->nnz_lower;
    HSLA_HIP(h, hipMemsetAsync(f.bad, 0, sizeof(int32_t), s));
    k_mp_weights<<<64, kBlock, 0, s>>>(params, f.w);
    k_mp_scale<<<nblocks(B * n, kBlock / 16, 16384), kBlock, 0, s>>>(g, B, values, f.ah64, f.ah32, f.bad);
    const int ga = nblocks(B * n, 4 * kWavesPerBlock, 16384);
    k_mp_init<<<ga, kBlock, 0, s>>>(g, B, f.w.wq, f.ah32, f.h[0]);
    for (int l = 1; l <= LAYERS; ++l) {
        k_mp_aggregate<<<ga, kBlock, 0, s>>>(g, B, f.w.wq + off_layer(l) + L_C, f.ah32, f.h[l - 1], f.m[l - 1]);
        const int64_t M = B * n;
        EpiBiasReluBf16<4> epi{f.w.wq + off_layer(l) + L_B, f.h[l], M};
        k_gemm<4, 4><<<nblocks((M + 15) / 16, kWavesPerBlock, 8192), kBlock, 0, s>>>(
            M, f.h[l - 1], HID, f.m[l - 1], HID, HID, f.w.Wf[l - 1], epi);
    }
    if (keep) {
        // training: keep x_k, z and t for the backward
        k_mp_head_gather<<<nblocks(B * nL, 4 * kWavesPerBlock, 16384), kBlock, 0, s>>>(g, B, f.ah32, f.h[LAYERS],
                                                                                        f.X);
        const int64_t M = B * nL;
        EpiHead epi{f.w.wq, f.z, f.t, Ghat, p->isdiagL, nL, M};
        k_gemm<5, 2><<<nblocks((M + 15) / 16, kWavesPerBlock, 8192), kBlock, 0, s>>>(M, f.X, KHP, f.X, KHP, KHP,
                                                                                   f.w.H1f, epi);
    } else {
        const int64_t M = B * nL;
        EpiHead epi{f.w.wq, nullptr, nullptr, Ghat, p->isdiagL, nL, M};
        k_mp_head_fused<<<nblocks((M + 15) / 16, kWavesPerBlock, 8192), kBlock, 0, s>>>(g, M, f.ah32, f.h[LAYERS],
                                                                                        f.w.H1f, epi);
    }
    HSLA_HIP(h, hipGetLastError());
    int32_t bad = 0;
    HSLA_HIP(h, hipMemcpyAsync(&bad, f.bad, sizeof bad, hipMemcpyDeviceToHost, s));
    HSLA_HIP(h, hipStreamSynchronize(s));
    if (bad) return set_error(h, HSLA_ERR_ZERO_DIAGONAL, "the network needs a positive stored diagonal");
    h->mp_keep_B = keep ? B : 0;
    h->mp_keep_pattern = keep ? p : nullptr;
    return HSLA_OK;
}

static void sum_into(const float *part, int nb, int rows, int cols, int rows_valid, float *dst, hipStream_t s) {
    const int tot = rows_valid * cols;
    k_sum_partials<<<(tot + 255) / 256, 256, 0, s>>>(part, nb, rows, cols, rows_valid, dst, 0);
}

static hsla_status backward(hsla_handle *h, const hsla_pattern *p, int B, const float *dG, float *grads, hipStream_t s) {
    if (h->mp_keep_B != B || h->mp_keep_pattern != p || B <= 0)
        return set_error(h, HSLA_ERR_INVALID_ARG, "backward needs a kept forward of the same pattern and batch");
    Bump bp{(char *)h->mp_ws, 0, h->mp_ws_bytes};
    Fwd f = carve_fwd(bp, B, p);
    Bwd w = carve_bwd(bp, B, p);
    if (bp.off > h->mp_ws_bytes) return set_error(h, HSLA_ERR_INTERNAL, "network workspace too small");
    const Graph g = make_graph(p);
    const int64_t n = p->n, nL = p->nnz_lower;
    const int64_t ML = B * nL, MN = B * n;
    // head
    k_mp_head_bwd<<<NB_V, kBlock, 0, s>>>(g, ML, f.w.wq, dG, f.t, f.z, w.dz, w.part);
    sum_into(w.part, NB_V, 1, 2 * HEAD + 1, 1, grads + OFF_C1, s);
    k_gemm_tn<KHT / 16, 2><<<NB_TN, kBlock, 0, s>>>(ML, f.X, KHP, f.X, KHP, KHP, w.dz, HEAD, w.part);
    sum_into(w.part, NB_TN, KHT, HEAD, KH, grads + OFF_H1, s);
    k_gemm<1, 8><<<nblocks((ML + 15) / 16, kWavesPerBlock, 8192), kBlock, 0, s>>>(
        ML, w.dz, HEAD, w.dz, HEAD, HEAD, f.w.H1Tf, EpiStoreF32<8>{w.dX, ML});
    k_mp_head_dh<<<nblocks(MN, 4 * kWavesPerBlock, 16384), kBlock, 0, s>>>(g, B, w.dX, w.dh);
    // message-passing layers
    for (int l = LAYERS; l >= 1; --l) {
        k_mp_relu_bwd<<<NB_V, kBlock, 0, s>>>(MN, w.dh, f.h[l], w.dpre, w.part);
        sum_into(w.part, NB_V, 1, HID, 1, grads + off_layer(l) + L_B, s);
        k_gemm_tn<8, 4><<<NB_TN, kBlock, 0, s>>>(MN, f.h[l - 1], HID, f.m[l - 1], HID, HID, w.dpre, HID, w.part);
        sum_into(w.part, NB_TN, 2 * HID, HID, 2 * HID, grads + off_layer(l) + L_W, s);
        k_gemm<2, 8><<<nblocks((MN + 15) / 16, kWavesPerBlock, 8192), kBlock, 0, s>>>(
            MN, w.dpre, HID, w.dpre, HID, HID, f.w.WTf[l - 1], EpiStoreF32<8>{w.dhm, MN});
        k_mp_aggregate_bwd<<<NB_V, kBlock, 0, s>>>(g, B, f.w.wq + off_layer(l) + L_C, f.ah32, f.h[l - 1], w.dhm,
                                                   w.dh, w.part);
        sum_into(w.part, NB_V, 1, NF * HID, 1, grads + off_layer(l) + L_C, s);
    }
    k_mp_init_bwd<<<NB_V, kBlock, 0, s>>>(g, B, f.ah32, f.h[0], w.dh, w.part);
    sum_into(w.part, NB_V, 1, (NF + 1) * HID, 1, grads + OFF_W0, s);
    HSLA_HIP(h, hipGetLastError());
    HSLA_HIP(h, hipStreamSynchronize(s));
    return HSLA_OK;
}

__global__ void k_perm_f64(int64_t nnz, int B, const double *__restrict__ in, const int32_t *__restrict__ src,
                           double *__restrict__ out) {
    const int64_t total = nnz * B;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = e / nnz, k = e - s * nnz;
        out[e] = in[s * nnz + src[k]];
    }
}

static hsla_status ensure_pr_ws(hsla_handle *h, size_t bytes) {
    if (bytes <= h->pr_ws_bytes) return HSLA_OK;
    if (h->pr_ws) {
        HSLA_HIP(h, hipStreamSynchronize(h->stream));
        dev_free(h, h->pr_ws);
        h->pr_ws = nullptr;
        h->pr_ws_bytes = 0;
    }
    const size_t want = bytes + bytes / 8 + 4096;
    if (dev_alloc(h, &h->pr_ws, want) != hipSuccess) {
        h->pr_ws = nullptr;
        return set_error(h, HSLA_ERR_NO_MEMORY, "probe workspace of %zu bytes", want);
    }
    h->pr_ws_bytes = want;
    return HSLA_OK;
}

static hsla_status probe_loss(hsla_handle *h, const hsla_pattern *p, int B, const double *values, const float *Gh,
                              int P, const double *Z, double scale, double *loss, float *dG, hipStream_t s) {
    const int64_t n = p->n, nnz = p->nnz, nL = p->nnz_lower;
    const int64_t BP = (int64_t)B * P;
    if (BP > 65535) return set_error(h, HSLA_ERR_INVALID_ARG, "systems x probes must be <= 65535");
    const int Gt = grid_blocks(h, kWavesPerBlock, p->ntiles, (int)BP, 16);
    const int Gp = grid_blocks(h, kBlock * 4, n, (int)BP, 4);
    size_t need = 0;
    auto add = [&](size_t bytes) { need += (bytes + 255) / 256 * 256 + 256; };
    add(8 * B * nnz); add(4 * B * nnz); add(8 * B * nnz); add(4 * B * nL);
    for (int k = 0; k < 6; ++k) add(8 * BP * n);
    add(8 * BP * Gp); add(8 * B); add(64);
    hsla_status st = ensure_pr_ws(h, need);
    if (st != HSLA_OK) return st;
    Bump bp{(char *)h->pr_ws, 0, h->pr_ws_bytes};
    double *ah64 = bp.take<double>(B * nnz);
    float *ah32 = bp.take<float>(B * nnz);
    double *ahT = bp.take<double>(B * nnz);
    float *GhT = bp.take<float>(B * nL);
    double *w = bp.take<double>(BP * n), *u = bp.take<double>(BP * n), *v = bp.take<double>(BP * n);
    double *e = bp.take<double>(BP * n), *t1 = bp.take<double>(BP * n), *y = bp.take<double>(BP * n);
    double *part = bp.take<double>(BP * Gp);
    double *dloss = bp.take<double>(B);
    int32_t *bad = bp.take<int32_t>(16);
    const Graph g = make_graph(p);
    HSLA_HIP(h, hipMemsetAsync(bad, 0, sizeof(int32_t), s));
    k_mp_scale<<<nblocks(B * n, kBlock / 16, 16384), kBlock, 0, s>>>(g, B, values, ah64, ah32, bad);
    k_perm_f64<<<nblocks(B * nnz, kBlock, 8192), kBlock, 0, s>>>(nnz, B, ah64, p->srcT, ahT);
    k_perm_f32<<<nblocks(B * nL, kBlock, 8192), kBlock, 0, s>>>(nL, B, Gh, p->srcU, GhT);
    const SpPat A{p->row_ptr, p->col, p->meta, p->ntiles, nnz};
    const SpPat AT{p->rpT, p->colT, p->metaT, p->ntilesT, nnz};
    const SpPat L{p->rpL, p->colL, p->metaL, p->ntilesL, nL};
    const SpPat U{p->rpU, p->colU, p->metaU, p->ntilesU, nL};
    const dim3 gs(Gt, (unsigned)BP), gv(Gp, (unsigned)BP);
    k_bspmv<float><<<gs, kBlock, 0, s>>>(U, P, (int32_t)n, GhT, Z, w);
    k_bspmv<double><<<gs, kBlock, 0, s>>>(A, P, (int32_t)n, ah64, w, u);
    k_bspmv<float><<<gs, kBlock, 0, s>>>(L, P, (int32_t)n, Gh, u, v);
    k_probe_err<<<gv, kBlock, 0, s>>>((int32_t)n, v, Z, e, part);
    k_probe_loss_fin<<<B, 64, 0, s>>>(B, P, Gp, part, dloss);
    if (dG) {
        k_bspmv<float><<<gs, kBlock, 0, s>>>(U, P, (int32_t)n, GhT, e, t1);
        k_bspmv<double><<<gs, kBlock, 0, s>>>(AT, P, (int32_t)n, ahT, t1, y);
        k_probe_grad<<<nblocks(B * nL, kBlock, 8192), kBlock, 0, s>>>(nL, B, P, (int32_t)n, p->rowL, p->colL, e, u,
                                                                      Z, y, scale, dG);
    }
    HSLA_HIP(h, hipGetLastError());
    std::vector<double> hl(B);
    int32_t hbad = 0;
    HSLA_HIP(h, hipMemcpyAsync(hl.data(), dloss, sizeof(double) * B, hipMemcpyDeviceToHost, s));
    HSLA_HIP(h, hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, s));
    HSLA_HIP(h, hipStreamSynchronize(s));
    if (hbad) return set_error(h, HSLA_ERR_ZERO_DIAGONAL, "the probe loss needs a positive stored diagonal");
    for (int i = 0; i < B; ++i) loss[i] = scale * hl[i];
    return HSLA_OK;
}

}  // namespace mp
}  // namespace hsla

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int32_t hsla_mpnn_num_params(void) { return hsla::mp::NPARAM; }

static hsla_status mp_check(hsla_handle *h, const hsla_pattern *p, int32_t B, void *stream) {
    if (!h) return HSLA_ERR_INVALID_ARG;
    if (!p) return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "null pattern");
    if (B < 0 || B > 65535) return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "batch out of range");
    if (p->device != h->device) return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "pattern on another device");
    return hsla::enter(h, (hipStream_t)stream);
}

hsla_status hsla_mpnn_forward(hsla_handle *h, const hsla_pattern *p, int32_t B, const double *d_values,
                              const float *d_params, float *d_Ghat, int32_t keep, void *stream) {
    hsla_status st = mp_check(h, p, B, stream);
    if (st != HSLA_OK) return st;
    if (B > 0 && (!d_values || !d_params || !d_Ghat)) return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "null pointer");
    if (B == 0 || p->n == 0) return HSLA_OK;
    return hsla::mp::forward(h, p, B, d_values, d_params, d_Ghat, keep != 0, h->stream);
}

hsla_status hsla_mpnn_backward(hsla_handle *h, const hsla_pattern *p, int32_t B, const float *d_dGhat,
                               float *d_grads, void *stream) {
    hsla_status st = mp_check(h, p, B, stream);
    if (st != HSLA_OK) return st;
    if (!d_dGhat || !d_grads) return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "null pointer");
    return hsla::mp::backward(h, p, B, d_dGhat, d_grads, h->stream);
}

hsla_status hsla_probe_loss(hsla_handle *h, const hsla_pattern *p, int32_t B, const double *d_values,
                            const float *d_Ghat, int32_t P, const double *d_Z, double scale, double *loss,
                            float *d_dGhat, void *stream) {
    hsla_status st = mp_check(h, p, B, stream);
    if (st != HSLA_OK) return st;
    if (P <= 0 || !loss) return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "bad probes or loss output");
    if (B == 0 || p->n == 0) return HSLA_OK;
    if (!d_values || !d_Ghat || !d_Z) return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "null pointer");
    return hsla::mp::probe_loss(h, p, B, d_values, d_Ghat, P, d_Z, scale, loss, d_dGhat, h->stream);
}

hsla_status hsla_adam_step(hsla_handle *h, int64_t n, float *d_params, const float *d_grads, float *d_m, float *d_v,
                           float lr, float beta1, float beta2, float eps, int64_t step, void *stream) {
    if (!h) return HSLA_ERR_INVALID_ARG;
    if (n < 0 || step < 1 || n > INT32_MAX) return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "bad Adam arguments");
    hsla_status st = hsla::enter(h, (hipStream_t)stream);
    if (st != HSLA_OK) return st;
    if (n == 0) return HSLA_OK;
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hsla::mp::k_adam<<<(unsigned)((n + 255) / 256), 256, 0, h->stream>>>((int)n, d_params, d_grads, d_m, d_v, lr,
                                                                       beta1, beta2, eps, c1, c2);
    HSLA_HIP(h, hipGetLastError());
    HSLA_HIP(h, hipStreamSynchronize(h->stream));
    return HSLA_OK;
}

hsla_status hsla_fsai_factors(hsla_handle *h, const hsla_pattern *p, int32_t B, const double *d_values,
                              const float *d_Ghat, float *d_G, float *d_GT, void *stream) {
    hsla_status st = mp_check(h, p, B, stream);
    if (st != HSLA_OK) return st;
    if (B == 0 || p->n == 0) return HSLA_OK;
    if (!d_values || !d_Ghat || !d_G || !d_GT) return hsla::set_error(h, HSLA_ERR_INVALID_ARG, "null pointer");
    const hsla::mp::Graph g = hsla::mp::make_graph(p);
    const int64_t tot = (int64_t)B * p->nnz_lower;
    const int blocks = hsla::mp::nblocks(tot, 256, 8192);
    hsla::mp::k_fsai_factor<<<blocks, 256, 0, h->stream>>>(g, B, d_values, d_Ghat, d_G);
    hsla::mp::k_perm_f32<<<blocks, 256, 0, h->stream>>>(p->nnz_lower, B, d_G, p->srcU, d_GT);
    HSLA_HIP(h, hipGetLastError());
    HSLA_HIP(h, hipStreamSynchronize(h->stream));
    return HSLA_OK;
}

}  // extern "C"
