// Learned proposal network: 16 -> 256 -> 256 -> 1 perceptron (ReLU, sigmoid),
// BF16 weights and activations on the matrix cores with FP32 accumulation,
// trained on the GPU with binary cross-entropy and Adam.
//
// Precision contract (every rounding is round-to-nearest-even to bfloat16):
//   forward  xb = bf16(x); a1 = xb W1b^T + b1; h1b = bf16(relu(a1));
//            a2 = h1b W2b^T + b2; h2b = bf16(relu(a2)); z = h2b . w3b + b3; p = sigmoid(z)
//   backward dz = (p - y)/B; dw3 = sum dz h2b; db3 = sum dz;
//            dh2 = dz w3b [h2b > 0]; dW2 = bf16(dh2)^T h1b; db2 = sum dh2;
//            dh1 = (bf16(dh2) W2b) [h1b > 0]; dW1 = bf16(dh1)^T xb; db1 = sum dh1
// All products of two matrices go through one "NT" GEMM, C[m][n] =
// sum_k A[m][k] B[n][k], with bf16 operands stored k-contiguous, on
// v_mfma_f32_32x32x16_bf16 (wave64: lane l holds A[l%32][8(l/32)+0..7],
// B[8(l/32)+0..7][l%32]; accumulator v is C[8(v/4)+4(l/32)+v%4][l%32]).
#include <algorithm>
#include <cmath>

#include <hipcub/hipcub.hpp>

#include "common.h"

namespace laue {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr int kIn = 16;
constexpr int kHid = 256;

// parameter layout of the FP32 masters
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + kHid * kIn;
constexpr int64_t kOffW2 = kOffB1 + kHid;
constexpr int64_t kOffB2 = kOffW2 + kHid * kHid;
constexpr int64_t kOffW3 = kOffB2 + kHid;
constexpr int64_t kOffB3 = kOffW3 + kHid;
constexpr int64_t kNParams = kOffB3 + 1;
// bf16 copies: W1b [256][16], W2b [256][256], W2bT [256][256], w3b [256]
constexpr int64_t kBfW1 = 0;
constexpr int64_t kBfW2 = kBfW1 + kHid * kIn;
constexpr int64_t kBfW2T = kBfW2 + kHid * kHid;
constexpr int64_t kBfW3 = kBfW2T + kHid * kHid;
constexpr int64_t kNBf = kBfW3 + kHid;

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

// C[M][N] (FP32, row stride ldc) = A[M][K] * B[N][K]^T; A, B bf16 with row
// stride K; K % 16 == 0.  One wave per 32x32 tile of C, 4 waves per block.
__global__ __launch_bounds__(256) void k_gemm_nt(const uint16_t *__restrict__ A,
                                                 const uint16_t *__restrict__ B,
                                                 float *__restrict__ Cm, int M, int N, int K,
                                                 int64_t ldc) {
    const int wave = threadIdx.x / 64, l = threadIdx.x % 64;
    const int tiles_n = (N + 31) / 32;
    const int tile = blockIdx.x * 4 + wave;
    const int tm = tile / tiles_n, tn = tile % tiles_n;
    if (tm * 32 >= M) return;
    const int m = tm * 32 + l % 32, n = tn * 32 + l % 32, kq = 8 * (l / 32);
    const bool mv = m < M, nv = n < N;
    f32x16 acc = {};
    const uint16_t *pa = A + static_cast<int64_t>(mv ? m : 0) * K + kq;
    const uint16_t *pb = B + static_cast<int64_t>(nv ? n : 0) * K + kq;
    for (int k0 = 0; k0 < K; k0 += 16) {
        uint4 va = mv ? *reinterpret_cast<const uint4 *>(pa + k0) : make_uint4(0, 0, 0, 0);
        uint4 vb = nv ? *reinterpret_cast<const uint4 *>(pb + k0) : make_uint4(0, 0, 0, 0);
        bf16x8 a, b;
        __builtin_memcpy(&a, &va, 16);
        __builtin_memcpy(&b, &vb, 16);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    const int col = tn * 32 + l % 32;
    if (col >= N) return;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = tm * 32 + 8 * (v / 4) + 4 * (l / 32) + v % 4;
        if (row < M) Cm[static_cast<int64_t>(row) * ldc + col] = acc[v];
    }
}

int gemm_nt(const uint16_t *A, const uint16_t *B, float *C, int M, int N, int K, int64_t ldc,
            hipStream_t s) {
    const int64_t tiles = static_cast<int64_t>((M + 31) / 32) * ((N + 31) / 32);
    k_gemm_nt<<<static_cast<unsigned>((tiles + 3) / 4), 256, 0, s>>>(A, B, C, M, N, K, ldc);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

// masters -> bf16 copies (W1b, W2b, W2b^T, w3b)
__global__ void k_mlp_to_bf16(const float *__restrict__ p, uint16_t *__restrict__ wb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kHid * kIn) wb[kBfW1 + i] = f2bf(p[kOffW1 + i]);
    if (i < kHid * kHid) {
        const int r = i / kHid, c = i % kHid;
        const uint16_t v = f2bf(p[kOffW2 + i]);
        wb[kBfW2 + i] = v;
        wb[kBfW2T + static_cast<int64_t>(c) * kHid + r] = v;
    }
    if (i < kHid) wb[kBfW3 + i] = f2bf(p[kOffW3 + i]);
}

// x [n][16] FP32 -> xb [n][16] bf16 and (optionally) xbT [16][ldt]
__global__ void k_mlp_in(const float *__restrict__ x, int64_t n, uint16_t *__restrict__ xb,
                         uint16_t *__restrict__ xbT, int64_t ldt) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n * kIn) return;
    const uint16_t v = f2bf(x[i]);
    xb[i] = v;
    if (xbT) xbT[(i % kIn) * ldt + i / kIn] = v;
}

// a [n][256] FP32 -> h = bf16(relu(a + b)) row-major and (optionally) transposed
__global__ void k_mlp_act(const float *__restrict__ a, const float *__restrict__ bias, int64_t n,
                          uint16_t *__restrict__ h, uint16_t *__restrict__ hT, int64_t ldt) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n * kHid) return;
    const int c = static_cast<int>(i % kHid);
    const uint16_t v = f2bf(fmaxf(a[i] + bias[c], 0.0f));
    h[i] = v;
    if (hT) hT[static_cast<int64_t>(c) * ldt + i / kHid] = v;
}

// z = h2b . w3b + b3, p = sigmoid(z): one wave per row, fixed-order reduction
__global__ __launch_bounds__(64) void k_mlp_out(const uint16_t *__restrict__ h2,
                                                const uint16_t *__restrict__ wb,
                                                const float *__restrict__ p, int64_t n,
                                                float *__restrict__ prob) {
    const int64_t r = blockIdx.x;
    if (r >= n) return;
    float s = 0.0f;
    for (int c = threadIdx.x; c < kHid; c += 64)
        s = fmaf(bf2f(h2[r * kHid + c]), bf2f(wb[kBfW3 + c]), s);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x == 0) prob[r] = 1.0f / (1.0f + __expf(-(s + p[kOffB3])));
}

struct MlpFwdWs {
    uint16_t *xb, *xbT, *h1, *h1T, *h2;
    float *acc;
};

int mlp_forward_chunk(const float *params, const uint16_t *wb, const float *x, int64_t n,
                      float *prob, MlpFwdWs &w, bool keep_t, int64_t ldt, hipStream_t s) {
    const unsigned g16 = static_cast<unsigned>((n * kIn + 255) / 256);
    const unsigned g256 = static_cast<unsigned>((n * kHid + 255) / 256);
    k_mlp_in<<<g16, 256, 0, s>>>(x, n, w.xb, keep_t ? w.xbT : nullptr, ldt);
    int rc;
    if ((rc = gemm_nt(w.xb, wb + kBfW1, w.acc, static_cast<int>(n), kHid, kIn, kHid, s))) return rc;
    k_mlp_act<<<g256, 256, 0, s>>>(w.acc, params + kOffB1, n, w.h1, keep_t ? w.h1T : nullptr, ldt);
    if ((rc = gemm_nt(w.h1, wb + kBfW2, w.acc, static_cast<int>(n), kHid, kHid, kHid, s))) return rc;
    k_mlp_act<<<g256, 256, 0, s>>>(w.acc, params + kOffB2, n, w.h2, nullptr, 0);
    k_mlp_out<<<static_cast<unsigned>(n), 64, 0, s>>>(w.h2, wb, params, n, prob);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

// ---------------------------------------------------------------- training

// dz and the per-row loss terms: one thread per row
__global__ __launch_bounds__(256) void k_mlp_dz(const float *__restrict__ prob,
                                               const float *__restrict__ y, int64_t n,
                                               float *__restrict__ dz, double *__restrict__ lrow) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const float p = prob[r];
    dz[r] = (p - y[r]) / static_cast<float>(n);
    const double pc = fmin(fmax(static_cast<double>(p), 1e-12), 1.0 - 1e-12);
    lrow[r] = -(y[r] * log(pc) + (1.0 - y[r]) * log(1.0 - pc));
}

// per column c of h2: dh2 = dz w3b[c] [h2b > 0] stored as bf16 row-major and
// transposed; per block of kDh2Rows rows, the partial sums of
// dw3[c] = sum_r dz_r h2b[r][c] and db2[c] = sum_r dh2 (FP32), and of db3.
constexpr int kDh2Rows = 256;

__global__ __launch_bounds__(256) void k_mlp_dh2(const float *__restrict__ dz,
                                                 const uint16_t *__restrict__ h2,
                                                 const uint16_t *__restrict__ wb, int64_t n,
                                                 float *__restrict__ part, uint16_t *__restrict__ dh2,
                                                 uint16_t *__restrict__ dh2T) {
    const int c = threadIdx.x;
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kDh2Rows;
    const int64_t r1 = min(r0 + kDh2Rows, n);
    const float w3 = bf2f(wb[kBfW3 + c]);
    float sw = 0.0f, sb = 0.0f, sz = 0.0f;
    for (int64_t r = r0; r < r1; ++r) {
        const float z = dz[r];
        const float hv = bf2f(h2[r * kHid + c]);
        sw = fmaf(z, hv, sw);
        const float d = hv > 0.0f ? z * w3 : 0.0f;
        sb += d;
        sz += z;
        const uint16_t db = f2bf(d);
        dh2[r * kHid + c] = db;
        dh2T[static_cast<int64_t>(c) * n + r] = db;
    }
    float *p = part + static_cast<int64_t>(blockIdx.x) * (2 * kHid + 1);
    p[c] = sw;
    p[kHid + c] = sb;
    if (c == 0) p[2 * kHid] = sz;
}

// Sum of the partials over the row blocks, in block order.
__global__ __launch_bounds__(256) void k_mlp_dh2_sum(const float *__restrict__ part, int nblk,
                                                     float *__restrict__ g) {
    const int c = threadIdx.x;
    float sw = 0.0f, sb = 0.0f, sz = 0.0f;
    for (int k = 0; k < nblk; ++k) {
        const float *p = part + static_cast<int64_t>(k) * (2 * kHid + 1);
        sw += p[c];
        sb += p[kHid + c];
        if (c == 0) sz += p[2 * kHid];
    }
    g[kOffW3 + c] = sw;
    g[kOffB2 + c] = sb;
    if (c == 0) g[kOffB3] = sz;
}

// dh1^T [256][n] (FP32, from the GEMM) -> mask with h1b > 0 -> bf16 dh1b^T, db1
__global__ __launch_bounds__(256) void k_mlp_dh1(const float *__restrict__ dh1T,
                                                 const uint16_t *__restrict__ h1T, int64_t n,
                                                 float *__restrict__ g, uint16_t *__restrict__ dh1bT) {
    const int c = blockIdx.x;
    float sb = 0.0f;
    __shared__ float part[256];
    for (int64_t r = threadIdx.x; r < n; r += 256) {
        const int64_t i = static_cast<int64_t>(c) * n + r;
        const float d = bf2f(h1T[i]) > 0.0f ? dh1T[i] : 0.0f;
        sb += d;
        dh1bT[i] = f2bf(d);
    }
    part[threadIdx.x] = sb;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int k = 0; k < 256; ++k) s += part[k];
        g[kOffB1 + c] = s;
    }
}

// dW1[c][j] = sum_r dh1b[r][c] xb[r][j]  (FP32 accumulate of exact bf16 products)
__global__ __launch_bounds__(256) void k_mlp_dw1(const uint16_t *__restrict__ dh1bT,
                                                 const uint16_t *__restrict__ xbT, int64_t n,
                                                 float *__restrict__ g) {
    const int c = blockIdx.x;
    const int j = threadIdx.x % kIn, part = threadIdx.x / kIn;   // 16 partial sums per output
    __shared__ float red[256];
    float s = 0.0f;
    for (int64_t r = part; r < n; r += 16)
        s = fmaf(bf2f(dh1bT[static_cast<int64_t>(c) * n + r]), bf2f(xbT[static_cast<int64_t>(j) * n + r]), s);
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < kIn) {
        float t = 0.0f;
        for (int q = 0; q < 16; ++q) t += red[q * kIn + threadIdx.x];
        g[kOffW1 + c * kIn + threadIdx.x] = t;
    }
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_sum_d(const double *__restrict__ v, int64_t n, double *__restrict__ out) {
    __shared__ double part[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += v[i];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < 256; ++k) t += part[k];
        *out = t;
    }
}

// He-uniform initialisation from Philox (counter (i, 0, 0, 6)); biases 0,
// output layer scaled by 0.1.
__global__ void k_mlp_init(float *__restrict__ p, uint32_t k0, uint32_t k1) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= kNParams) return;
    uint32_t c[4] = {static_cast<uint32_t>(i), 0u, 0u, 6u};
    philox(c, k0, k1);
    const float u = (static_cast<float>(c[0]) + 0.5f) * (1.0f / 4294967296.0f) * 2.0f - 1.0f;
    float v = 0.0f;
    if (i < kOffB1) v = u * sqrtf(6.0f / kIn);
    else if (i >= kOffW2 && i < kOffB2) v = u * sqrtf(6.0f / kHid);
    else if (i >= kOffW3 && i < kOffB3) v = 0.1f * u * sqrtf(6.0f / kHid);
    p[i] = v;
}

size_t carve_fwd(Carver &cv, MlpFwdWs &w, int64_t n, bool train) {
    w.xb = cv.take<uint16_t>(n * kIn);
    w.xbT = train ? cv.take<uint16_t>(n * kIn) : nullptr;
    w.h1 = cv.take<uint16_t>(n * kHid);
    w.h1T = train ? cv.take<uint16_t>(n * kHid) : nullptr;
    w.h2 = cv.take<uint16_t>(n * kHid);
    w.acc = cv.take<float>(n * kHid);
    return cv.size();
}

struct MlpTrainWs {
    MlpFwdWs f;
    float *prob, *dz, *grad, *dh1T, *part;
    double *lrow, *lsum;
    uint16_t *dh2, *dh2T, *dh1bT;
};

size_t carve_train(Carver &cv, MlpTrainWs &w, int64_t B) {
    carve_fwd(cv, w.f, B, true);
    w.prob = cv.take<float>(B);
    w.dz = cv.take<float>(B);
    w.grad = cv.take<float>(kNParams);
    w.dh1T = cv.take<float>(B * kHid);
    w.part = cv.take<float>(((B + kDh2Rows - 1) / kDh2Rows) * (2 * kHid + 1));
    w.lrow = cv.take<double>(B);
    w.lsum = cv.take<double>(1);
    w.dh2 = cv.take<uint16_t>(B * kHid);
    w.dh2T = cv.take<uint16_t>(B * kHid);
    w.dh1bT = cv.take<uint16_t>(B * kHid);
    return cv.size();
}

int validate_mlp(const laue_mlp *m) {
    LAUE_REQUIRE(m && m->params && m->wbf16, LAUE_EINVAL, "network or its arrays are NULL");
    LAUE_REQUIRE(m->n_in == kIn && m->n_hidden == kHid, LAUE_EINVAL, "only a 16-256-256-1 network is supported");
    return LAUE_OK;
}

}  // namespace laue

using namespace laue;

constexpr int64_t kFwdChunk = 1 << 16;

extern "C" int64_t laue_mlp_n_params(int32_t n_in, int32_t n_hidden) {
    return (n_in == kIn && n_hidden == kHid) ? kNParams : -1;
}

extern "C" int64_t laue_mlp_n_bf16(int32_t n_in, int32_t n_hidden) {
    return (n_in == kIn && n_hidden == kHid) ? kNBf : -1;
}

extern "C" int laue_mlp_init(laue_mlp *m, uint64_t seed, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_mlp(m))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    k_mlp_init<<<static_cast<unsigned>((kNParams + 255) / 256), 256, 0, s>>>(
        m->params, static_cast<uint32_t>(seed & 0xffffffffu), static_cast<uint32_t>(seed >> 32));
    k_mlp_to_bf16<<<(kHid * kHid + 255) / 256, 256, 0, s>>>(m->params, m->wbf16);
    LAUE_CHECK_HIP(hipGetLastError());
    m->step = 0;
    return LAUE_OK;
}

extern "C" int laue_mlp_sync_bf16(laue_mlp *m, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_mlp(m))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    k_mlp_to_bf16<<<(kHid * kHid + 255) / 256, 256, 0, s>>>(m->params, m->wbf16);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

extern "C" size_t laue_mlp_forward_workspace_size(int64_t n) {
    if (n < 0) return 0;
    Carver cv(nullptr);
    MlpFwdWs w;
    return carve_fwd(cv, w, std::min<int64_t>(std::max<int64_t>(n, 1), kFwdChunk), false);
}

extern "C" int laue_mlp_forward(const laue_mlp *m, const float *feat, int64_t n, float *prob,
                                void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_mlp(m))) return rc;
    LAUE_REQUIRE(n >= 0 && (n == 0 || (feat && prob)), LAUE_EINVAL, "bad inputs");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    MlpFwdWs w;
    const int64_t ch = std::min<int64_t>(std::max<int64_t>(n, 1), kFwdChunk);
    size_t need = carve_fwd(cv, w, ch, false);
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    for (int64_t r0 = 0; r0 < n; r0 += ch) {
        const int64_t nn = std::min(ch, n - r0);
        if ((rc = mlp_forward_chunk(m->params, m->wbf16, feat + r0 * kIn, nn, prob + r0, w, false, 0, s)))
            return rc;
    }
    return LAUE_OK;
}

extern "C" size_t laue_mlp_train_workspace_size(int64_t batch) {
    if (batch < 1) return 0;
    Carver cv(nullptr);
    MlpTrainWs w;
    return carve_train(cv, w, batch);
}

namespace laue {
namespace {
// Forward, loss and gradient of one batch into the training workspace (the
// gradient in w.grad, the summed loss in w.lsum on the device).
int backward_core(const laue_mlp *m, const float *feat, const float *label, int64_t B, MlpTrainWs &w,
                  hipStream_t s) {
    int rc;
    if ((rc = mlp_forward_chunk(m->params, m->wbf16, feat, B, w.prob, w.f, true, B, s))) return rc;
    k_mlp_dz<<<static_cast<unsigned>((B + 255) / 256), 256, 0, s>>>(w.prob, label, B, w.dz, w.lrow);
    const int nblk = static_cast<int>((B + kDh2Rows - 1) / kDh2Rows);
    k_mlp_dh2<<<nblk, 256, 0, s>>>(w.dz, w.f.h2, m->wbf16, B, w.part, w.dh2, w.dh2T);
    k_mlp_dh2_sum<<<1, 256, 0, s>>>(w.part, nblk, w.grad);
    LAUE_CHECK_HIP(hipGetLastError());
    // dW2 = dh2b^T h1b: A = dh2b^T [256][B], B = h1b^T [256][B]
    if ((rc = gemm_nt(w.dh2T, w.f.h1T, w.grad + kOffW2, kHid, kHid, static_cast<int>(B), kHid, s))) return rc;
    // dh1^T = W2b^T dh2b^T: A = W2b^T [256][256], B = dh2b [B][256]
    if ((rc = gemm_nt(m->wbf16 + kBfW2T, w.dh2, w.dh1T, kHid, static_cast<int>(B), kHid, B, s))) return rc;
    k_mlp_dh1<<<kHid, 256, 0, s>>>(w.dh1T, w.f.h1T, B, w.grad, w.dh1bT);
    k_mlp_dw1<<<kHid, 256, 0, s>>>(w.dh1bT, w.f.xbT, B, w.grad);
    k_sum_d<<<1, 256, 0, s>>>(w.lrow, B, w.lsum);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}
}  // namespace
}  // namespace laue

extern "C" int laue_mlp_backward(const laue_mlp *m, const float *feat, const float *label,
                                 int64_t batch, float *grad, double *loss, void *ws,
                                 size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_mlp(m))) return rc;
    LAUE_REQUIRE(batch >= 16 && batch % 16 == 0 && batch <= (1 << 24) && feat && label && loss,
                 LAUE_EINVAL, "batch must be a positive multiple of 16");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    MlpTrainWs w;
    size_t need = carve_train(cv, w, batch);
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    if ((rc = backward_core(m, feat, label, batch, w, s))) return rc;
    if (grad)
        LAUE_CHECK_HIP(hipMemcpyAsync(grad, w.grad, kNParams * sizeof(float), hipMemcpyDeviceToDevice, s));
    double ls = 0.0;
    LAUE_CHECK_HIP(hipMemcpyAsync(&ls, w.lsum, sizeof(double), hipMemcpyDeviceToHost, s));
    LAUE_CHECK_HIP(hipStreamSynchronize(s));
    *loss = ls / static_cast<double>(batch);
    return LAUE_OK;
}

extern "C" int laue_mlp_adam(laue_mlp *m, const float *grad, const laue_adam_params *ap, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_mlp(m))) return rc;
    LAUE_REQUIRE(grad && ap && m->adam_m && m->adam_v, LAUE_EINVAL, "NULL argument");
    LAUE_REQUIRE(std::isfinite(ap->lr) && ap->lr >= 0 && ap->beta1 >= 0 && ap->beta1 < 1 && ap->beta2 >= 0 &&
                     ap->beta2 < 1 && ap->eps > 0,
                 LAUE_EINVAL, "bad Adam parameters");
    hipStream_t s = static_cast<hipStream_t>(stream);
    m->step += 1;
    const double c1 = 1.0 - std::pow(ap->beta1, m->step), c2 = 1.0 - std::pow(ap->beta2, m->step);
    k_adam<<<static_cast<unsigned>((kNParams + 255) / 256), 256, 0, s>>>(
        m->params, grad, m->adam_m, m->adam_v, kNParams, static_cast<float>(ap->lr),
        static_cast<float>(ap->beta1), static_cast<float>(ap->beta2), static_cast<float>(ap->eps),
        static_cast<float>(c1), static_cast<float>(c2));
    k_mlp_to_bf16<<<(kHid * kHid + 255) / 256, 256, 0, s>>>(m->params, m->wbf16);
    LAUE_CHECK_HIP(hipGetLastError());
    return LAUE_OK;
}

extern "C" int laue_mlp_train_step(laue_mlp *m, const float *feat, const float *label,
                                   int64_t batch, const laue_adam_params *ap, double *loss,
                                   void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = laue_mlp_backward(m, feat, label, batch, nullptr, loss, ws, ws_bytes, stream))) return rc;
    Carver cv(ws);
    MlpTrainWs w;
    carve_train(cv, w, batch);
    return laue_mlp_adam(m, w.grad, ap, stream);
}

// ---------------------------------------------------------------- one training epoch

namespace laue {
namespace {
// 64-bit order key of example i in epoch e: Philox4x32-10 counter (i, e, 0, 8)
__global__ void k_epoch_keys(int64_t n, int epoch, uint32_t k0, uint32_t k1, unsigned long long *__restrict__ key,
                             int *__restrict__ idx) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t c[4] = {static_cast<uint32_t>(i), static_cast<uint32_t>(epoch), 0u, 8u};
    philox(c, k0, k1);
    key[i] = (static_cast<unsigned long long>(c[0]) << 32) | c[1];
    idx[i] = static_cast<int>(i);
}

// rows perm[b0 .. b0 + B) of the examples into the batch buffers
__global__ void k_epoch_gather(const float *__restrict__ feat, const float *__restrict__ label,
                               const int *__restrict__ perm, int64_t b0, int64_t B, float *__restrict__ bf,
                               float *__restrict__ bl) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= B * 16) return;
    const int64_t r = t >> 4, k = t & 15;
    const int64_t src = perm[b0 + r];
    bf[t] = feat[src * 16 + k];
    if (k == 0) bl[r] = label[src];
}

__global__ void k_epoch_add(const double *__restrict__ v, double *__restrict__ acc, int first) {
    *acc = first ? *v : *acc + *v;
}

struct EpochWs {
    unsigned long long *key_in, *key_out;
    int *idx_in, *idx_out;
    void *tmp;
    size_t tmp_bytes;
    float *bf, *bl;
    double *acc;
    MlpTrainWs t;
};

size_t carve_epoch(Carver &cv, EpochWs &w, int64_t n, int64_t batch) {
    w.key_in = cv.take<unsigned long long>(std::max<int64_t>(n, 1));
    w.key_out = cv.take<unsigned long long>(std::max<int64_t>(n, 1));
    w.idx_in = cv.take<int>(std::max<int64_t>(n, 1));
    w.idx_out = cv.take<int>(std::max<int64_t>(n, 1));
    size_t tmp = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, static_cast<unsigned long long *>(nullptr),
                                             static_cast<unsigned long long *>(nullptr), static_cast<int *>(nullptr),
                                             static_cast<int *>(nullptr), static_cast<int>(std::max<int64_t>(n, 1)));
    w.tmp_bytes = tmp;
    w.tmp = cv.take<char>(static_cast<int64_t>(tmp));
    w.bf = cv.take<float>(batch * 16);
    w.bl = cv.take<float>(batch);
    w.acc = cv.take<double>(1);
    carve_train(cv, w.t, batch);
    return cv.size();
}
}  // namespace
}  // namespace laue

extern "C" size_t laue_mlp_epoch_workspace_size(int64_t n, int64_t batch) {
    if (n < 1 || batch < 16) return 0;
    Carver cv(nullptr);
    EpochWs w;
    return carve_epoch(cv, w, n, batch);
}

extern "C" int laue_mlp_train_epoch(laue_mlp *m, const float *feat, const float *label, int64_t n, int64_t batch,
                                    uint64_t seed, int32_t epoch, const laue_adam_params *ap, double *loss_mean,
                                    void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = validate_mlp(m))) return rc;
    LAUE_REQUIRE(batch >= 16 && batch % 16 == 0 && batch <= (1 << 24), LAUE_EINVAL,
                 "batch must be a positive multiple of 16");
    LAUE_REQUIRE(n >= batch && n < (int64_t(1) << 31) && feat && label && ap && loss_mean && epoch >= 0,
                 LAUE_EINVAL, "need at least one batch of examples (n < 2^31), features, labels and outputs");
    hipStream_t s = static_cast<hipStream_t>(stream);
    Carver cv(ws);
    EpochWs w;
    const size_t need = carve_epoch(cv, w, n, batch);
    if ((rc = check_ws(ws, ws_bytes, need))) return rc;
    const uint32_t k0 = static_cast<uint32_t>(seed & 0xffffffffu), k1 = static_cast<uint32_t>(seed >> 32);
    k_epoch_keys<<<static_cast<unsigned>((n + 255) / 256), 256, 0, s>>>(n, epoch, k0, k1, w.key_in, w.idx_in);
    LAUE_CHECK_HIP(hipGetLastError());
    size_t tb = w.tmp_bytes;
    LAUE_CHECK_HIP(hipcub::DeviceRadixSort::SortPairs(w.tmp, tb, w.key_in, w.key_out, w.idx_in, w.idx_out,
                                                     static_cast<int>(n), 0, 64, s));
    const int64_t nb = n / batch;
    for (int64_t b = 0; b < nb; ++b) {
        k_epoch_gather<<<static_cast<unsigned>((batch * 16 + 255) / 256), 256, 0, s>>>(feat, label, w.idx_out,
                                                                                      b * batch, batch, w.bf, w.bl);
        if ((rc = backward_core(m, w.bf, w.bl, batch, w.t, s))) return rc;
        k_epoch_add<<<1, 1, 0, s>>>(w.t.lsum, w.acc, b == 0);
        if ((rc = laue_mlp_adam(m, w.t.grad, ap, stream))) return rc;
    }
    LAUE_CHECK_HIP(hipGetLastError());
    double tot = 0.0;
    LAUE_CHECK_HIP(hipMemcpyAsync(&tot, w.acc, sizeof(double), hipMemcpyDeviceToHost, s));
    LAUE_CHECK_HIP(hipStreamSynchronize(s));
    *loss_mean = tot / static_cast<double>(nb * batch);
    return LAUE_OK;
}
