// Warm-start network kernels (gfx950): a 32 -> 64 -> 64 -> 3 perceptron with
// exact-erf GELU, evaluated and trained with BF16 MFMA (v_mfma_f32_16x16x32_bf16)
// accumulating in FP32.
//
// Training: one wave takes a chunk of 32 samples.  Weights, activations and
// pre-activations of the chunk sit in LDS; every product is a small GEMM
// computed tile by tile (16 x 16 output tiles, K in steps of 32).  Operands
// are rounded to BF16 (round to nearest even) when they enter an MFMA; biases,
// GELU and the loss are FP32.  Training writes one gradient row per chunk;
// a second kernel sums the rows in chunk order (deterministic) and a third
// applies Adam.
#include "snake_mlp.h"

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

namespace {

constexpr int NI = 32, NH = 64, NO = 3;
constexpr int P_W1 = 0, P_B1 = P_W1 + NH * NI, P_W2 = P_B1 + NH, P_B2 = P_W2 + NH * NH;
constexpr int P_W3 = P_B2 + NH, P_B3 = P_W3 + NO * NH, P_COUNT = P_B3 + NO;
constexpr int CH = 32;  // samples per training chunk (one wave)
constexpr int MT = CH / 16, KS = CH / 32;   // sample row tiles; sample K steps

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

thread_local std::string g_mlp_err;

int mfail(int code, const std::string& m)
{
    g_mlp_err = m;
    return code;
}

// erf(x) by Abramowitz and Stegun, Handbook of Mathematical Functions,
// formula 7.1.26: 1 - (a1 t + ... + a5 t^5) exp(-x^2), t = 1 / (1 + p |x|),
// odd in x; absolute error at most 1.5e-7 (far below the BF16 rounding of
// the activations).  exp(-x^2) also serves GELU's derivative.
__device__ __forceinline__ float erf_as(float x, float& e)
{
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.f));
    const float poly =
        t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f),
                 0.254829592f);
    e = __builtin_amdgcn_exp2f(-1.4426950408889634f * (x * x));   // exp(-x^2)
    return copysignf(fmaf(-poly, e, 1.f), x);
}

__device__ __forceinline__ float gelu(float z)
{
    float e;
    return 0.5f * z * (1.f + erf_as(z * 0.70710678118654752f, e));
}

// d GELU / dz = Phi(z) + z phi(z), phi(z) = exp(-z^2 / 2) / sqrt(2 pi)
__device__ __forceinline__ float gelu_grad(float z)
{
    float e;
    const float phi = 0.5f * (1.f + erf_as(z * 0.70710678118654752f, e));
    return phi + z * 0.39894228040143268f * e;
}

// C[M x N] = A[M x K] B[K x N] for M, N multiples of 16 and K of 32, on one
// wave.  Lane l supplies A rows l % 16 and B columns l % 16 for the k-slice
// 8 (l / 16) .. +8 and receives D rows 4 (l / 16) .. +4 of column l % 16.
template <class FA, class FB, class FS>
__device__ __forceinline__ void wave_gemm(int mtiles, int ntiles, int ktiles, FA A, FB Bm, FS store)
{
    const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
    for (int mt = 0; mt < mtiles; ++mt)
        for (int nt = 0; nt < ntiles; ++nt) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            for (int kt = 0; kt < ktiles; ++kt) {
                bf16x8 a, b;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    a[j] = A(mt * 16 + r, kt * 32 + 8 * g + j);
                    b[j] = Bm(kt * 32 + 8 * g + j, nt * 16 + r);
                }
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) store(mt * 16 + 4 * g + v, nt * 16 + r, acc[v]);
        }
}

struct Lds {
    __bf16 W1[NH][NI];
    __bf16 W2[NH][NH];
    __bf16 W3[16][NH];   // rows >= 3 are zero
    __bf16 X[CH][NI];
    __bf16 H1[CH][NH];
    __bf16 H2[CH][NH];
    float Z1[CH][NH];    // pre-activation, later d loss / d z1
    float Z2[CH][NH];
    __bf16 dY[CH][16];   // columns >= 3 are zero
    __bf16 dZ[CH][NH];
    float dYf[CH][NO];
    float red[64];
};

// Weight matrices to LDS as BF16.  Each lane loads its float4 groups before
// converting any, so the loads are in flight together.
template <int ROWS, int COLS, int PROWS>
__device__ __forceinline__ void load_matrix(__bf16 (*dst)[COLS], const float* __restrict__ src)
{
    constexpr int G = ROWS * COLS / 4;   // float4 groups of the stored rows
    constexpr int PER = (G + 63) / 64;
    const int l = threadIdx.x;
    float4 v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int gi = l + 64 * k;
        v[k] = (gi < G && 4 * gi < PROWS * COLS) ? reinterpret_cast<const float4*>(src)[gi]
                                                  : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int gi = l + 64 * k;
        if (gi < G) {
            const int e = 4 * gi;
            __bf16* d = &dst[e / COLS][e % COLS];
            d[0] = (__bf16)v[k].x;
            d[1] = (__bf16)v[k].y;
            d[2] = (__bf16)v[k].z;
            d[3] = (__bf16)v[k].w;
        }
    }
}

__device__ void load_weights(Lds& S, const float* __restrict__ p)
{
    load_matrix<NH, NI, NH>(S.W1, p + P_W1);
    load_matrix<NH, NH, NH>(S.W2, p + P_W2);
    load_matrix<16, NH, NO>(S.W3, p + P_W3);   // rows >= 3 are zero
}

// forward pass of one chunk; samples past n contribute zeros
__device__ void chunk_forward(Lds& S, const float* __restrict__ p, const float* __restrict__ ms,
                              const float* __restrict__ x, int64_t base, int64_t n, float* y_out)
{
    const int l = threadIdx.x;
    for (int e = l; e < CH * NI; e += 64) {
        const int s = e / NI, k = e % NI;
        const int64_t row = base + s;
        const float v = row < n ? (x[row * NI + k] - ms[k]) / ms[NI + k] : 0.f;
        S.X[s][k] = (__bf16)v;
    }
    __syncthreads();
    wave_gemm(MT, 4, 1, [&](int i, int k) { return S.X[i][k]; }, [&](int k, int o) { return S.W1[o][k]; },
              [&](int i, int o, float a) {
                  const float z = a + p[P_B1 + o];
                  S.Z1[i][o] = z;
                  S.H1[i][o] = (__bf16)gelu(z);
              });
    __syncthreads();
    wave_gemm(MT, 4, 2, [&](int i, int k) { return S.H1[i][k]; }, [&](int k, int o) { return S.W2[o][k]; },
              [&](int i, int o, float a) {
                  const float z = a + p[P_B2 + o];
                  S.Z2[i][o] = z;
                  S.H2[i][o] = (__bf16)gelu(z);
              });
    __syncthreads();
    wave_gemm(MT, 1, 2, [&](int i, int k) { return S.H2[i][k]; }, [&](int k, int o) { return S.W3[o][k]; },
              [&](int i, int o, float a) {
                  if (o < NO) y_out[i * NO + o] = a + p[P_B3 + o];
              });
    __syncthreads();
}

// Inference: four waves per workgroup, each taking tiles of 16 samples in a
// grid-stride loop.  The weights stay in registers as MFMA B operands for
// the whole launch; a 16 x 64 BF16 buffer per wave in LDS turns each layer's
// output (D layout: lane l holds rows 4 (l / 16) .. +4 of column l % 16) into
// the next layer's A operand (row l % 16, columns 8 (l / 16) .. +8).  Same
// arithmetic as the training pass: BF16 operands, FP32 accumulation, bias
// and GELU.
constexpr int FW_WAVES = 4, FW_ROW = NH + 8;   // padded row (144 bytes)

__global__ void __launch_bounds__(64 * FW_WAVES) __attribute__((amdgpu_waves_per_eu(4))) k_mlp_forward(const float* __restrict__ p,
                                                               const float* __restrict__ ms,
                                                               const float* __restrict__ x,
                                                               float* __restrict__ y, int64_t n)
{
    __shared__ __align__(16) __bf16 Hs[FW_WAVES][16][FW_ROW];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, r = l & 15, g = l >> 4;
    __bf16 (*H)[FW_ROW] = Hs[w];
    bf16x8 B1[4], B2[4][2], B3[2];
    float bb1[4], bb2[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int o = nt * 16 + r;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            B1[nt][j] = (__bf16)p[P_W1 + o * NI + 8 * g + j];
            B2[nt][0][j] = (__bf16)p[P_W2 + o * NH + 8 * g + j];
            B2[nt][1][j] = (__bf16)p[P_W2 + o * NH + 32 + 8 * g + j];
        }
        bb1[nt] = p[P_B1 + o];
        bb2[nt] = p[P_B2 + o];
    }
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
        for (int j = 0; j < 8; ++j) B3[kt][j] = r < NO ? (__bf16)p[P_W3 + r * NH + kt * 32 + 8 * g + j] : (__bf16)0.f;
    const float bb3 = r < NO ? p[P_B3 + r] : 0.f;
    float mu[8], is[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        mu[j] = ms[8 * g + j];
        is[j] = 1.f / ms[NI + 8 * g + j];
    }
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    const int64_t tiles = (n + 15) / 16;
    for (int64_t t = (int64_t)blockIdx.x * FW_WAVES + w; t < tiles; t += (int64_t)gridDim.x * FW_WAVES) {
        const int64_t row = t * 16 + r;
        bf16x8 a;
        if (row < n) {
            const float4* xp = reinterpret_cast<const float4*>(x + row * NI + 8 * g);
            const float4 u0 = xp[0], u1 = xp[1];
            const float xv[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = (__bf16)((xv[j] - mu[j]) * is[j]);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) a[j] = (__bf16)0.f;
        }
        // layer 1: h1 = GELU(W1 x + b1)
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, B1[nt], zero, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) H[4 * g + v][nt * 16 + r] = (__bf16)gelu(acc[v] + bb1[nt]);
        }
        // (memcpy: the vector read may not be reordered with the element stores)
        bf16x8 a2[2];
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) __builtin_memcpy(&a2[kt], &H[r][kt * 32 + 8 * g], sizeof(bf16x8));
        // layer 2: h2 = GELU(W2 h1 + b2)
        f32x4 acc2[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            acc2[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[0], B2[nt][0], zero, 0, 0, 0);
            acc2[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[1], B2[nt][1], acc2[nt], 0, 0, 0);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) H[4 * g + v][nt * 16 + r] = (__bf16)gelu(acc2[nt][v] + bb2[nt]);
        bf16x8 a3[2];
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) __builtin_memcpy(&a3[kt], &H[r][kt * 32 + 8 * g], sizeof(bf16x8));
        // layer 3: y = W3 h2 + b3 (columns >= 3 are padding)
        f32x4 acc3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3[0], B3[0], zero, 0, 0, 0);
        acc3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3[1], B3[1], acc3, 0, 0, 0);
        if (r < NO) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t rr = t * 16 + 4 * g + v;
                if (rr < n) y[rr * NO + r] = acc3[v] + bb3;
            }
        }
    }
}

// forward + backward of one chunk per workgroup; one gradient row per chunk
__global__ void __launch_bounds__(64) k_mlp_grad(const float* __restrict__ p, const float* __restrict__ ms,
                                                 const float* __restrict__ x, const float* __restrict__ t,
                                                 int64_t n, float* __restrict__ gpart,
                                                 float* __restrict__ lpart)
{
    __shared__ Lds S;
    __shared__ float Y[CH * NO];
    load_weights(S, p);
    const int l = threadIdx.x;
    const int64_t c = blockIdx.x;
    const int64_t base = c * CH;
    float* g = gpart + c * P_COUNT;
    chunk_forward(S, p, ms, x, base, n, Y);
    // d loss / d y for loss = mean over samples and outputs of (y - t)^2
    const float scale = 2.f / (float)(n * NO);
    float lsum = 0.f;
    for (int e = l; e < CH * 16; e += 64) {
        const int s = e / 16, o = e % 16;
        const int64_t row = base + s;
        float d = 0.f;
        if (o < NO && row < n) {
            const float err = Y[s * NO + o] - t[row * NO + o];
            lsum += err * err;
            d = scale * err;
        }
        if (o < NO) S.dYf[s][o] = d;
        S.dY[s][o] = (__bf16)d;
    }
    S.red[l] = lsum;
    __syncthreads();
    if (l == 0) {
        float acc = 0.f;
        for (int k = 0; k < 64; ++k) acc += S.red[k];
        lpart[c] = acc;
    }
    if (l < NO) {
        float acc = 0.f;
        for (int s = 0; s < CH; ++s) acc += S.dYf[s][l];
        g[P_B3 + l] = acc;
    }
    // dW3 = dY^T H2 (M = outputs padded to 16, K = samples)
    wave_gemm(1, 4, KS, [&](int o, int s) { return S.dY[s][o]; }, [&](int s, int k) { return S.H2[s][k]; },
              [&](int o, int k, float a) {
                  if (o < NO) g[P_W3 + o * NH + k] = a;
              });
    // dH2 = dY W3 (K = outputs padded to 32); dz2 = dH2 * GELU'(z2)
    wave_gemm(MT, 4, 1, [&](int s, int o) { return o < 16 ? S.dY[s][o] : (__bf16)0.f; },
              [&](int o, int k) { return o < 16 ? S.W3[o][k] : (__bf16)0.f; },
              [&](int s, int k, float a) {
                  const float dz = a * gelu_grad(S.Z2[s][k]);
                  S.Z2[s][k] = dz;
                  S.dZ[s][k] = (__bf16)dz;
              });
    __syncthreads();
    if (l < NH) {
        float acc = 0.f;
        for (int s = 0; s < CH; ++s) acc += S.Z2[s][l];
        g[P_B2 + l] = acc;
    }
    // dW2 = dZ2^T H1 ; dH1 = dZ2 W2
    wave_gemm(4, 4, KS, [&](int o, int s) { return S.dZ[s][o]; }, [&](int s, int k) { return S.H1[s][k]; },
              [&](int o, int k, float a) { g[P_W2 + o * NH + k] = a; });
    wave_gemm(MT, 4, 2, [&](int s, int o) { return S.dZ[s][o]; }, [&](int o, int k) { return S.W2[o][k]; },
              [&](int s, int k, float a) { S.Z1[s][k] = a * gelu_grad(S.Z1[s][k]); });
    __syncthreads();
    for (int e = l; e < CH * NH; e += 64) S.dZ[e / NH][e % NH] = (__bf16)S.Z1[e / NH][e % NH];
    if (l < NH) {
        float acc = 0.f;
        for (int s = 0; s < CH; ++s) acc += S.Z1[s][l];
        g[P_B1 + l] = acc;
    }
    __syncthreads();
    // dW1 = dZ1^T X
    wave_gemm(4, 2, KS, [&](int o, int s) { return S.dZ[s][o]; }, [&](int s, int k) { return S.X[s][k]; },
              [&](int o, int k, float a) { g[P_W1 + o * NI + k] = a; });
}

// grad[k] = sum over chunks, loss likewise, in a fixed order: eight partial
// sums over chunks c = j mod 8 (loads in flight together), then combined
// pairwise.  The same inputs give the same bits on every call.
__device__ __forceinline__ float ordered_sum(const float* __restrict__ a, int64_t stride, int64_t count)
{
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int64_t c = 0;
    for (; c + 8 <= count; c += 8) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = a[(c + j) * stride];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] += v[j];
    }
    for (int j = 0; c < count; ++c, ++j) acc[j] += a[c * stride];
    return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

__global__ void k_mlp_reduce(const float* __restrict__ gpart, const float* __restrict__ lpart, int64_t chunks,
                             int64_t n, float* __restrict__ grad, float* __restrict__ loss)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < P_COUNT) grad[k] = ordered_sum(gpart + k, P_COUNT, chunks);
    if (k == 0) *loss = ordered_sum(lpart, 1, chunks) / (float)(n * NO);
}

// Adam with bias correction (Kingma and Ba), step t counts from 1
__global__ void k_mlp_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                           const float* __restrict__ g, int t, float lr, float b1, float b2, float eps)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P_COUNT) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.f - b1) * gk;
    const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float mh = mk / (1.f - powf(b1, (float)t));
    const float vh = vk / (1.f - powf(b2, (float)t));
    p[k] -= lr * mh / (sqrtf(vh) + eps);
}

// per-feature mean and standard deviation, accumulated in double
__global__ void __launch_bounds__(256) k_mlp_stats(const float* __restrict__ x, int64_t n, float* __restrict__ ms)
{
    __shared__ double sh[256];
    const int k = blockIdx.x;   // feature
    const int l = threadIdx.x;
    double s = 0.0;
    for (int64_t r = l; r < n; r += 256) s += x[r * NI + k];
    sh[l] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (l < o) sh[l] += sh[l + o];
        __syncthreads();
    }
    const double mean = sh[0] / (double)n;
    __syncthreads();
    double q = 0.0;
    for (int64_t r = l; r < n; r += 256) {
        const double d = x[r * NI + k] - mean;
        q += d * d;
    }
    sh[l] = q;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (l < o) sh[l] += sh[l + o];
        __syncthreads();
    }
    if (l == 0) {
        ms[k] = (float)mean;
        ms[NI + k] = (float)sqrt(sh[0] / (double)n + 1e-12);
    }
}

// Fixed scratch of mlp_grad_noalloc: the gradient rows and loss partials of
// a batch of up to kNoAllocSamples samples (3.3 MB).  Every device the
// library runs on holds its own copy until the process ends.  In host code
// the array's name is only a stand-in: its device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr int64_t kNoAllocSamples = 4096;
constexpr int64_t kNoAllocChunks = (kNoAllocSamples + CH - 1) / CH;
constexpr int kMaxDevices = 64;
__device__ __align__(256) float scratch[kNoAllocChunks * (P_COUNT + 1)];

std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (nullptr on failure,
// with the message set)
float* scratch_on_current_device()
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        mfail(SIM_EDEVICE, std::string("mlp_grad_noalloc: hipGetDevice: ") + hipGetErrorString(e));
        return nullptr;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        mfail(SIM_EINVAL, "mlp_grad_noalloc: device index beyond 63");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            mfail(SIM_EDEVICE, std::string("mlp_grad_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = static_cast<float*>(ptr);
    }
    return g_scratch_ptr[dev];
}

int launch_grad(const float* params, const float* mean_std, const float* x, const float* t, int64_t n,
                float* grad, float* loss, float* buf, hipStream_t st)
{
    const int64_t chunks = (n + CH - 1) / CH;
    float* gpart = buf;
    float* lpart = buf + chunks * P_COUNT;
    hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)chunks), dim3(64), 0, st, params, mean_std, x, t, n, gpart, lpart);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((P_COUNT + 255) / 256), dim3(256), 0, st, gpart, lpart, chunks, n, grad, loss);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SIM_OK : mfail(SIM_EDEVICE, hipGetErrorString(e));
}

}  // namespace

extern "C" {

int mlp_param_count(void) { return P_COUNT; }

const char* mlp_last_error(void) { return g_mlp_err.c_str(); }

int64_t mlp_train_scratch_floats(int64_t n)
{
    const int64_t chunks = (n + CH - 1) / CH;
    return chunks * P_COUNT + chunks;
}

int mlp_norm_stats(const float* x, int64_t n, float* mean_std, void* stream)
{
    if (!x || !mean_std || n < 1) return mfail(SIM_EINVAL, "mlp_norm_stats: bad arguments");
    hipLaunchKernelGGL(k_mlp_stats, dim3(NI), dim3(256), 0, (hipStream_t)stream, x, n, mean_std);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SIM_OK : mfail(SIM_EDEVICE, hipGetErrorString(e));
}

int mlp_forward(const float* params, const float* mean_std, const float* x, float* y, int64_t n, void* stream)
{
    if (!params || !mean_std || !x || !y || n < 0) return mfail(SIM_EINVAL, "mlp_forward: bad arguments");
    if (n == 0) return SIM_OK;
    const int64_t groups = ((n + 15) / 16 + FW_WAVES - 1) / FW_WAVES;
    const int grid = (int)(groups < 2048 ? groups : 2048);
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(64 * FW_WAVES), 0, (hipStream_t)stream, params, mean_std,
                       x, y, n);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SIM_OK : mfail(SIM_EDEVICE, hipGetErrorString(e));
}

int mlp_grad(const float* params, const float* mean_std, const float* x, const float* t, int64_t n, float* grad,
             float* loss, float* scratch, int64_t scratch_floats, void* stream)
{
    if (!params || !mean_std || !x || !t || !grad || !loss || !scratch || n < 1)
        return mfail(SIM_EINVAL, "mlp_grad: bad arguments");
    if (scratch_floats < mlp_train_scratch_floats(n)) return mfail(SIM_ENOMEM, "mlp_grad: scratch too small");
    const int64_t chunks = (n + CH - 1) / CH;
    if (chunks > (1 << 30)) return mfail(SIM_EINVAL, "mlp_grad: batch too large");
    return launch_grad(params, mean_std, x, t, n, grad, loss, scratch, (hipStream_t)stream);
}

int mlp_grad_noalloc(const float* params, const float* mean_std, const float* x, const float* t, int64_t n,
                     float* grad, float* loss, void* stream)
{
    if (!params || !mean_std || !x || !t || !grad || !loss || n < 1)
        return mfail(SIM_EINVAL, "mlp_grad_noalloc: bad arguments");
    if (n > kNoAllocSamples)
        return mfail(SIM_EINVAL, "mlp_grad_noalloc: batch of " + std::to_string(n) + " samples exceeds the fixed "
                                 "scratch (at most " + std::to_string(kNoAllocSamples) + ")");
    float* buf = scratch_on_current_device();
    if (!buf) return SIM_EDEVICE;
    return launch_grad(params, mean_std, x, t, n, grad, loss, buf, (hipStream_t)stream);
}

int mlp_adam(float* params, float* m, float* v, const float* grad, int32_t t, float lr, void* stream)
{
    if (!params || !m || !v || !grad || t < 1) return mfail(SIM_EINVAL, "mlp_adam: bad arguments");
    hipLaunchKernelGGL(k_mlp_adam, dim3((P_COUNT + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, m, v,
                       grad, t, lr, 0.9f, 0.999f, 1e-8f);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SIM_OK : mfail(SIM_EDEVICE, hipGetErrorString(e));
}

}  // extern "C"
