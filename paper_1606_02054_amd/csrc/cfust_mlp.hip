// cfust_mlp.hip -- the surrogate network: a 16 -> 256 -> 256 -> 256 -> 256 -> 16
// perceptron with tanh-form GELU, BF16 weights and activations, FP32
// accumulation on the matrix cores (gfx950's v_mfma_f32_16x16x32_bf16), FP32
// master weights and Adam.  Forward, backward, loss and optimiser kernels.
//
// GEMM convention: C[M][N] = P[M][K] * Q[N][K]^T with P, Q row-major BF16
// (K contiguous).  One 256-thread block computes a 64 x 64 tile of C; each
// wave a 32 x 32 quarter as 2 x 2 MFMA tiles of 16 x 16, stepping K by 32.
// 64 x 64 slices of P and Q are staged in LDS with coalesced 16-byte loads;
// operand fragments (16 bytes per lane: eight consecutive K values) are read
// from there in the layout the 16x16x32 BF16 MFMA expects:
//   lane l holds P[row0 + l%16][k0 + 8(l/16) + 0..7] and Q[col0 + l%16][k0 + 8(l/16) + 0..7],
//   and receives C[row0 + 4(l/16) + i][col0 + l%16], i = 0..3.
// A K of 16 (the input layer) is zero-padded to 32.
#include "cfust_kernels.h"

namespace cfust {

typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma32(v8s a, v8s b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr float GELU_C = 0.7978845608028654f;   // sqrt(2/pi)
constexpr float GELU_A = 0.044715f;

// tanh u = 1 - 2 / (e^(2u) + 1): one exp2 and one reciprocal.  Its absolute
// error (a few 1e-8) is far below the BF16 rounding of the activations; the
// limits +-1 come out exactly when e^(2u) overflows or underflows.
__device__ __forceinline__ float fast_tanh(float u) {
    const float e = __builtin_amdgcn_exp2f(2.8853900817779268f * u);     // e^(2u)
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

__device__ __forceinline__ float gelu(float z) {
    const float u = GELU_C * (z + GELU_A * z * z * z);
    return 0.5f * z * (1.0f + fast_tanh(u));
}
__device__ __forceinline__ float gelu_grad(float z) {
    const float u = GELU_C * (z + GELU_A * z * z * z);
    const float t = fast_tanh(u);
    return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * GELU_C * (1.0f + 3.0f * GELU_A * z * z);
}

// Epilogue of a GEMM tile element: add bias, apply the activation, store.
struct GemmOut {
    const float *bias;      // [N] or null
    float *Cf;              // [M][N] FP32 (pre-activation) or null
    uint16_t *Cb;           // [M][N] BF16 after activation, or null
    uint16_t *CbT;          // [N][M] BF16 after activation (transposed), or null
    float *Cpart;           // split-K partials [split][M][N] or null
    int act;                // 0: identity, 1: GELU
};

// C = P Q^T in BF16 with FP32 accumulation (P [M][K], Q [N][K] row-major),
// block tile 64 x 64 over 4 waves, each 32 x 32 in 16 x 16 MFMA tiles (K 32 per MFMA).
// 64 x 64 slices of P and Q are staged in LDS per step with 16-byte loads;
// the next slice's loads are issued before the current slice's MFMAs, so
// their latency is hidden.  Rows past M or N and K past the chunk are zero,
// which adds exact zeros to the same MFMA sequence (K ascending by 32) as
// fragments read straight from memory.  (A 128 x 128 tile was no faster: the
// forward products are bound by their epilogue writes, FP32 pre-activations
// and two BF16 layouts, not by feeding the MFMAs.)
__global__ __launch_bounds__(256) void k_gemm_bf16(const uint16_t *__restrict__ P, const uint16_t *__restrict__ Q,
                                                   int M, int N, int K, int kchunk, GemmOut o) {
    constexpr int BT = 64;                       // block tile
    constexpr int TW = BT / 32;                  // 16 x 16 tiles per wave and dimension
    constexpr int NLD = BT / 32;                 // 16-byte loads per thread and operand
    constexpr int KC = 64, KP = KC + 8;          // pitch: 144-byte rows spread over the banks
    __shared__ __align__(16) uint16_t ps[BT * KP], qs[BT * KP];
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int wr = (BT / 2) * (wave >> 1), wc = (BT / 2) * (wave & 1);   // the wave's quarter of the tile
    const int row_w = blockIdx.y * BT + wr;
    const int col_w = blockIdx.x * BT + wc;
    const int k_beg = blockIdx.z * kchunk;
    const int k_end = min(K, k_beg + kchunk);
    v4f acc[TW][TW];
#pragma unroll
    for (int a = 0; a < TW; ++a)
#pragma unroll
        for (int b = 0; b < TW; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    bool colok[TW], rowok[TW];
#pragma unroll
    for (int a = 0; a < TW; ++a) { colok[a] = col_w + 16 * a < N; rowok[a] = row_w + 16 * a < M; }
    const int lr = l & 15, lk = 8 * (l >> 4), lo = 4 * (l >> 4);
    uint4 pv[NLD], qv[NLD];
    // load i of this thread: slice row (t + 256 i) / 8, K offset 8 ((t + 256 i) % 8);
    // K, kchunk multiples of 16: a load that starts before k_end has its 8 values in range,
    // and the K past k_end in the slice is zero
    auto fetch = [&](int k0) {
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int u = threadIdx.x + 256 * i, srow = u >> 3, kq = k0 + 8 * (u & 7);
            const int prow = blockIdx.y * BT + srow, qrow = blockIdx.x * BT + srow;
            pv[i] = make_uint4(0, 0, 0, 0);
            qv[i] = make_uint4(0, 0, 0, 0);
            if (kq < k_end) {
                if (prow < M) pv[i] = *reinterpret_cast<const uint4 *>(P + (size_t)prow * K + kq);
                if (qrow < N) qv[i] = *reinterpret_cast<const uint4 *>(Q + (size_t)qrow * K + kq);
            }
        }
    };
    if (k_beg < k_end) fetch(k_beg);
    for (int k0 = k_beg; k0 < k_end; k0 += KC) {
#pragma unroll
        for (int i = 0; i < NLD; ++i) {
            const int u = threadIdx.x + 256 * i, srow = u >> 3, sk = 8 * (u & 7);
            *reinterpret_cast<uint4 *>(ps + srow * KP + sk) = pv[i];
            *reinterpret_cast<uint4 *>(qs + srow * KP + sk) = qv[i];
        }
        __syncthreads();
        if (k0 + KC < k_end) fetch(k0 + KC);
#pragma unroll
        for (int kk = 0; kk < KC; kk += 32) {
            if (k0 + kk >= k_end) break;
            v8s pa[TW], qb[TW];
#pragma unroll
            for (int a = 0; a < TW; ++a) {
                pa[a] = *reinterpret_cast<const v8s *>(ps + (wr + 16 * a + lr) * KP + kk + lk);
                qb[a] = *reinterpret_cast<const v8s *>(qs + (wc + 16 * a + lr) * KP + kk + lk);
            }
#pragma unroll
            for (int a = 0; a < TW; ++a)
#pragma unroll
                for (int b = 0; b < TW; ++b) acc[a][b] = mfma32(pa[a], qb[b], acc[a][b]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < TW; ++a)
#pragma unroll
        for (int b = 0; b < TW; ++b) {
            if (!rowok[a] || !colok[b]) continue;
            const int col = col_w + 16 * b + lr;
            const int r0 = row_w + 16 * a + lo;
            if (o.Cpart) {
                float *dst = o.Cpart + (size_t)blockIdx.z * M * N;
#pragma unroll
                for (int i = 0; i < 4; ++i) dst[(size_t)(r0 + i) * N + col] = acc[a][b][i];
                continue;
            }
            const float bias = o.bias ? o.bias[col] : 0.0f;
            uint16_t ob[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float z = acc[a][b][i] + bias;
                if (o.Cf) o.Cf[(size_t)(r0 + i) * N + col] = z;
                const float y = o.act ? gelu(z) : z;
                ob[i] = f2bf(y);
                if (o.Cb) o.Cb[(size_t)(r0 + i) * N + col] = ob[i];
            }
            if (o.CbT) {
                // four consecutive rows = four consecutive entries of the transposed row
                uint2 pk;
                pk.x = (uint32_t)ob[0] | ((uint32_t)ob[1] << 16);
                pk.y = (uint32_t)ob[2] | ((uint32_t)ob[3] << 16);
                *reinterpret_cast<uint2 *>(o.CbT + (size_t)col * M + r0) = pk;
            }
        }
}

// Sum split-K partials: dst[i] = sum_s part[s][i].
__global__ void k_sum_split(const float *__restrict__ part, int nsplit, size_t count, float *__restrict__ dst) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float s = 0.0f;
    for (int k = 0; k < nsplit; ++k) s += part[(size_t)k * count + i];
    dst[i] = s;
}

// dZ = dY * gelu'(Z) (or dY when the layer has no activation), written as BF16
// in both layouts, and the bias gradient by a column reduction.
// dZ = dY * GELU'(Z) (or dY) in BF16, row-major and transposed.  One block
// per 64 x 64 tile: coalesced row-major reads and writes, the transposed copy
// written through an LDS tile so its stores are coalesced too.
__global__ __launch_bounds__(256) void k_act_back(const float *__restrict__ dY, const float *__restrict__ Z, int M,
                                                  int N, int act, uint16_t *__restrict__ dZb,
                                                  uint16_t *__restrict__ dZbT) {
    __shared__ uint16_t tile[64][66];            // odd dword pitch: column reads hit distinct banks
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
#pragma unroll 4
    for (int j = 0; j < 16; ++j) {
        const int rr = ty + 4 * j, r = r0 + rr, c = c0 + tx;
        if (r < M && c < N) {
            const size_t i = (size_t)r * N + c;
            const float g = act ? dY[i] * gelu_grad(Z[i]) : dY[i];
            const uint16_t h = f2bf(g);
            dZb[i] = h;
            tile[rr][tx] = h;
        }
    }
    __syncthreads();
#pragma unroll 4
    for (int j = 0; j < 16; ++j) {
        const int cc = ty + 4 * j, c = c0 + cc, r = r0 + tx;
        if (r < M && c < N) dZbT[(size_t)c * M + r] = tile[tx][cc];
    }
}

__global__ void k_col_sum(const uint16_t *__restrict__ dZbT, int M, int N, float *__restrict__ db) {
    // one block per column, rows reduced in a fixed order
    __shared__ float red[256];
    const int c = blockIdx.x;
    float s = 0.0f;
    // 8 values per 16-byte load (M is a multiple of 64)
    for (int r = 8 * threadIdx.x; r < M; r += 8 * blockDim.x) {
        const uint4 v = *reinterpret_cast<const uint4 *>(dZbT + (size_t)c * M + r);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            s += bf2f((uint16_t)(w[k] & 0xffffu));
            s += bf2f((uint16_t)(w[k] >> 16));
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[c] = red[0];
}

// Adam on FP32 master weights (one launch per parameter array), refreshing
// the BF16 copies in both layouts for weight matrices.
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, size_t count, int rows, int cols, float lr, float b1,
                       float b2, float eps, float c1, float c2, uint16_t *__restrict__ wb,
                       uint16_t *__restrict__ wbT) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) {
        const uint16_t h = f2bf(wi);
        wb[i] = h;
        const int r = (int)(i / cols), c = (int)(i % cols);
        wbT[(size_t)c * rows + r] = h;
    }
}

// Loss of the two heads and the gradient w.r.t. the network output.
// out[b][0]: prediction of the scaled log-probability, out[b][1]: predicted
// log10 of its absolute error.  Rows b >= nvalid are padding.
__global__ __launch_bounds__(256) void k_mlp_loss(const float *__restrict__ out, const float *__restrict__ label,
                                                  int B, int nvalid, float lam, float *__restrict__ dout,
                                                  float *__restrict__ part) {
    __shared__ float red[256];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    float loss = 0.0f;
    if (b < B) {
        for (int c = 0; c < CFUST_MLP_OUT; ++c) dout[(size_t)b * CFUST_MLP_OUT + c] = 0.0f;
        if (b < nvalid) {
            const float o0 = out[(size_t)b * CFUST_MLP_OUT], o1 = out[(size_t)b * CFUST_MLP_OUT + 1];
            const float r = o0 - label[b];
            const float tgt = log10f(fabsf(r) + 1e-6f);
            const float r1 = o1 - tgt;
            loss = r * r + lam * r1 * r1;
            dout[(size_t)b * CFUST_MLP_OUT] = 2.0f * r / nvalid;
            dout[(size_t)b * CFUST_MLP_OUT + 1] = 2.0f * lam * r1 / nvalid;
        }
    }
    red[threadIdx.x] = loss;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Copy of the network input in both layouts ([B][16] and [16][B]).
__global__ void k_transpose_in(const uint16_t *__restrict__ X0, int B, uint16_t *__restrict__ X,
                               uint16_t *__restrict__ XT) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * CFUST_MLP_IN) return;
    const int r = i / CFUST_MLP_IN, c = i % CFUST_MLP_IN;
    const uint16_t v = X0[i];
    X[i] = v;
    XT[(size_t)c * B + r] = v;
}

// --------------------------------------------------------------- launch ----

static const int LAYER_K[CFUST_MLP_LAYERS] = {CFUST_MLP_IN, CFUST_MLP_HIDDEN, CFUST_MLP_HIDDEN, CFUST_MLP_HIDDEN,
                                              CFUST_MLP_HIDDEN};
static const int LAYER_N[CFUST_MLP_LAYERS] = {CFUST_MLP_HIDDEN, CFUST_MLP_HIDDEN, CFUST_MLP_HIDDEN, CFUST_MLP_HIDDEN,
                                              CFUST_MLP_OUT};

int mlp_layer_k(int l) { return LAYER_K[l]; }
int mlp_layer_n(int l) { return LAYER_N[l]; }

static hipError_t gemm(const uint16_t *P, const uint16_t *Q, int M, int N, int K, int nsplit, const GemmOut &o,
                       hipStream_t s) {
    const int kchunk = ((K / nsplit + 31) / 32) * 32;
    dim3 grid((N + 63) / 64, (M + 63) / 64, nsplit);
    hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, P, Q, M, N, K, kchunk, o);
    return hipGetLastError();
}

// Inference (no activations saved): the whole network for a tile of 64 rows
// in one block, the tile's activations staying in LDS between layers.  Each
// wave computes 64 rows x 64 output columns of a hidden layer (4 x 4 MFMA
// tiles; weight fragments read straight from global memory, so every block
// reads each weight matrix once), then, after every wave has read the layer's
// input, writes its BF16 outputs back over it.  The operands, the K order,
// the bias, GELU and BF16 rounding are those of k_gemm_bf16, so the results
// equal the layer-by-layer pass bit for bit.
constexpr int FU_ROWS = 64;
constexpr int FU_STRIDE = CFUST_MLP_HIDDEN + 8;     // LDS row pitch (BF16): rows fall in different banks

// Weights in MFMA fragment order for the fused pass: for layer l (N x K, K
// padded to KP = 32 for the input layer),
// element (column tile ct, K step ks, lane, j) = W_l[16 ct + lane % 16][32 ks + 8 (lane / 16) + j]
// (0 past K), at offset ((ct (KP/32) + ks) 64 + lane) 8 + j of the layer's
// block, so each wave-wide fragment load reads 1024 contiguous bytes.  Layer
// blocks follow one another (N_l KP_l elements each).
constexpr int FU_K0 = 32;                        // input layer K, padded
constexpr int FU_OFF[CFUST_MLP_LAYERS + 1] = {
    0, CFUST_MLP_HIDDEN * FU_K0, CFUST_MLP_HIDDEN * FU_K0 + CFUST_MLP_HIDDEN * CFUST_MLP_HIDDEN,
    CFUST_MLP_HIDDEN * FU_K0 + 2 * CFUST_MLP_HIDDEN * CFUST_MLP_HIDDEN,
    CFUST_MLP_HIDDEN * FU_K0 + 3 * CFUST_MLP_HIDDEN * CFUST_MLP_HIDDEN,
    CFUST_MLP_HIDDEN * FU_K0 + 3 * CFUST_MLP_HIDDEN * CFUST_MLP_HIDDEN + CFUST_MLP_OUT * CFUST_MLP_HIDDEN};

__global__ __launch_bounds__(256) void k_mlp_pack(cfust_mlp_weights W, uint16_t *__restrict__ Wp) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= FU_OFF[CFUST_MLP_LAYERS]) return;
    int l = 0;
    while (t >= FU_OFF[l + 1]) ++l;
    const int K = l == 0 ? CFUST_MLP_IN : CFUST_MLP_HIDDEN;
    const int KP = l == 0 ? FU_K0 : CFUST_MLP_HIDDEN;
    const int e = t - FU_OFF[l];
    const int j = e & 7, lane = (e >> 3) & 63, tile = e >> 9;     // tile = ct (KP/32) + ks
    const int ct = tile / (KP / 32), ks = tile % (KP / 32);
    const int k = 32 * ks + 8 * (lane >> 4) + j;
    Wp[t] = k < K ? ((const uint16_t *)W.W[l])[(size_t)(16 * ct + (lane & 15)) * K + k] : (uint16_t)0;
}

// One hidden layer of the fused pass (K inputs, zero-padded to a multiple of
// 32, 256 outputs), in place in xs.
template <int K>
__device__ __forceinline__ void fused_hidden_layer(uint16_t *xs, const uint16_t *__restrict__ Wl,
                                                   const float *__restrict__ bl, int wave, int l, int lr, int lk,
                                                   int lo) {
    const int col_w = 64 * wave;
    v4f acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    constexpr int KS = (K + 31) / 32;
#pragma unroll 4
    for (int ks = 0; ks < KS; ++ks) {
        v8s pa[4], qb[4];
#pragma unroll
        for (int b = 0; b < 4; ++b)
            qb[b] = *reinterpret_cast<const v8s *>(Wl + ((size_t)((4 * wave + b) * KS + ks) * 64 + l) * 8);
#pragma unroll
        for (int a = 0; a < 4; ++a)
            pa[a] = *reinterpret_cast<const v8s *>(xs + (16 * a + lr) * FU_STRIDE + 32 * ks + lk);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = mfma32(pa[a], qb[b], acc[a][b]);
    }
    __syncthreads();                                                       // the layer's input is read
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int col = col_w + 16 * b + lr;
        const float bias = bl[col];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                xs[(16 * a + lo + i) * FU_STRIDE + col] = f2bf(gelu(acc[a][b][i] + bias));
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_mlp_fwd_fused(const uint16_t *__restrict__ X0, cfust_mlp_weights W,
                                                       const uint16_t *__restrict__ Wp, float *__restrict__ out) {
    __shared__ __align__(16) uint16_t xs[FU_ROWS * FU_STRIDE];
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int lr = l & 15, lk = 8 * (l >> 4), lo = 4 * (l >> 4);
    const size_t row0 = (size_t)blockIdx.x * FU_ROWS;
    // the input tile, its columns CFUST_MLP_IN .. FU_K0 - 1 zeroed (the padded K)
    for (int t = threadIdx.x; t < FU_ROWS * FU_K0; t += blockDim.x) {
        const int r = t / FU_K0, c = t % FU_K0;
        xs[r * FU_STRIDE + c] = c < CFUST_MLP_IN ? X0[(row0 + r) * CFUST_MLP_IN + c] : (uint16_t)0;
    }
    __syncthreads();
    fused_hidden_layer<CFUST_MLP_IN>(xs, Wp + FU_OFF[0], W.b[0], wave, l, lr, lk, lo);
    for (int layer = 1; layer < CFUST_MLP_LAYERS - 1; ++layer)
        fused_hidden_layer<CFUST_MLP_HIDDEN>(xs, Wp + FU_OFF[layer], W.b[layer], wave, l, lr, lk, lo);
    // output layer, 256 -> 16: wave w takes rows 16 w .. 16 w + 15
    const int L = CFUST_MLP_LAYERS - 1;
    const uint16_t *Wl = Wp + FU_OFF[L];                                    // one column tile
    v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < CFUST_MLP_HIDDEN / 32; ++ks) {
        const v8s pa = *reinterpret_cast<const v8s *>(xs + (16 * wave + lr) * FU_STRIDE + 32 * ks + lk);
        const v8s qb = *reinterpret_cast<const v8s *>(Wl + ((size_t)ks * 64 + l) * 8);
        acc = mfma32(pa, qb, acc);
    }
    const float bias = W.b[L][lr];
#pragma unroll
    for (int i = 0; i < 4; ++i) out[(row0 + 16 * wave + lo + i) * CFUST_MLP_OUT + lr] = acc[i] + bias;
}

size_t mlp_packed_elems() { return (size_t)FU_OFF[CFUST_MLP_LAYERS]; }

hipError_t launch_mlp_forward(const cfust_mlp_weights &W, const uint16_t *X0, int B, float *out,
                              const cfust_mlp_acts *acts, uint16_t *scratch_a, uint16_t *scratch_b,
                              hipStream_t s) {
    if (!acts) {                                 // inference: the fused kernel (B is a multiple of 64)
        // scratch_a receives the weights in fragment order (mlp_packed_elems() BF16)
        hipLaunchKernelGGL(k_mlp_pack, dim3((FU_OFF[CFUST_MLP_LAYERS] + 255) / 256), dim3(256), 0, s, W, scratch_a);
        hipLaunchKernelGGL(k_mlp_fwd_fused, dim3(B / FU_ROWS), dim3(256), 0, s, X0, W, scratch_a, out);
        return hipGetLastError();
    }
    const uint16_t *x = X0;
    hipError_t e = hipSuccess;
    for (int l = 0; l < CFUST_MLP_LAYERS && e == hipSuccess; ++l) {
        GemmOut o{};
        o.bias = W.b[l];
        const bool last = l == CFUST_MLP_LAYERS - 1;
        o.act = last ? 0 : 1;
        if (last) {
            o.Cf = out;
        } else {
            o.Cf = acts ? acts->Z[l] : nullptr;
            uint16_t *next = acts ? acts->X[l + 1] : ((l & 1) ? scratch_b : scratch_a);
            o.Cb = next;
            o.CbT = acts ? acts->XT[l + 1] : nullptr;
        }
        e = gemm(x, (const uint16_t *)W.W[l], B, LAYER_N[l], LAYER_K[l], 1, o, s);
        // the forward pass of layer l + 1 reads the BF16 activation just written
        if (!last) x = o.Cb;
    }
    return e;
}

hipError_t launch_mlp_backward(const cfust_mlp_weights &W, const cfust_mlp_acts &A, const float *dout, int B,
                               const cfust_mlp_grads &G, float *part, float *dY, uint16_t *dZb, uint16_t *dZbT,
                               hipStream_t s) {
    hipError_t e = hipSuccess;
    const float *dy = dout;
    for (int l = CFUST_MLP_LAYERS - 1; l >= 0 && e == hipSuccess; --l) {
        const int N = LAYER_N[l], K = LAYER_K[l];
        const bool last = l == CFUST_MLP_LAYERS - 1;
        hipLaunchKernelGGL(k_act_back, dim3((N + 63) / 64, (B + 63) / 64), dim3(256), 0, s, dy,
                           last ? nullptr : A.Z[l], B, N, last ? 0 : 1, dZb, dZbT);
        hipLaunchKernelGGL(k_col_sum, dim3(N), dim3(256), 0, s, dZbT, B, N, G.db[l]);
        // dW[N][K] = dZ^T X : P = dZ^T [N][B], Q = X^T [K][B], split over the batch
        const int nsplit = B >= 1024 ? 16 : 1;
        GemmOut o{};
        o.Cpart = part;
        e = gemm(dZbT, A.XT[l], N, K, B, nsplit, o, s);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_sum_split, dim3((unsigned)(((size_t)N * K + 255) / 256)), dim3(256), 0, s, part,
                           nsplit, (size_t)N * K, G.dW[l]);
        if (l > 0) {
            // dX[B][K] = dZ W : P = dZ [B][N], Q = W^T [K][N]
            GemmOut ox{};
            ox.Cf = dY;
            e = gemm(dZb, (const uint16_t *)W.Wt[l], B, K, N, 1, ox, s);
            dy = dY;
            // dY is consumed by the next k_act_back before being overwritten
        }
    }
    return e == hipSuccess ? hipGetLastError() : e;
}

hipError_t launch_mlp_adam(const cfust_mlp_master &Mst, const cfust_mlp_grads &G, const cfust_mlp_weights &W,
                           float lr, float b1, float b2, float eps, int step, hipStream_t s) {
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    for (int l = 0; l < CFUST_MLP_LAYERS; ++l) {
        const int N = LAYER_N[l], K = LAYER_K[l];
        const size_t nw = (size_t)N * K;
        hipLaunchKernelGGL(k_adam, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, Mst.W[l], Mst.mW[l],
                           Mst.vW[l], G.dW[l], nw, N, K, lr, b1, b2, eps, c1, c2, (uint16_t *)W.W[l],
                           (uint16_t *)W.Wt[l]);
        hipLaunchKernelGGL(k_adam, dim3((N + 255) / 256), dim3(256), 0, s, Mst.b[l], Mst.mb[l], Mst.vb[l],
                           G.db[l], (size_t)N, 1, N, lr, b1, b2, eps, c1, c2, (uint16_t *)nullptr,
                           (uint16_t *)nullptr);
    }
    return hipGetLastError();
}

hipError_t launch_mlp_loss(const float *out, const float *label, int B, int nvalid, float lam, float *dout,
                           float *part, float *loss, hipStream_t s) {
    const int nb = (B + 255) / 256;
    hipLaunchKernelGGL(k_mlp_loss, dim3(nb), dim3(256), 0, s, out, label, B, nvalid, lam, dout, part);
    hipLaunchKernelGGL(k_sum_split, dim3(1), dim3(1), 0, s, part, nb, (size_t)1, loss);
    return hipGetLastError();
}

hipError_t launch_transpose_in(const uint16_t *X0, int B, uint16_t *X, uint16_t *XT, hipStream_t s) {
    const int cnt = B * CFUST_MLP_IN;
    hipLaunchKernelGGL(k_transpose_in, dim3((cnt + 255) / 256), dim3(256), 0, s, X0, B, X, XT);
    return hipGetLastError();
}

}  // namespace cfust
