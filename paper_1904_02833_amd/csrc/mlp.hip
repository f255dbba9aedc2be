// Warm-start network kernels (gfx950): a 32 -> 64 -> 64 -> 3 perceptron with
// GELU (mlp_device.h), evaluated and trained with BF16 MFMA
// (v_mfma_f32_16x16x32_bf16) accumulating in FP32.
//
// Training: a workgroup of four waves takes a chunk of 32 samples.  Weights,
// activations and pre-activations of the chunk sit in LDS; every product is
// a small GEMM computed tile by tile (16 x 16 output tiles, K in steps of
// 32), the tiles of one product spread over the four waves.  Operands are
// rounded to BF16 (round to nearest even) when they enter an MFMA; biases,
// GELU and the loss are FP32.  Training writes one gradient row per chunk;
// a second kernel sums the rows in chunk order (deterministic) and a third
// applies Adam.
//
// Inference for the solver's learned start (k_warm_net) computes each
// joint's inputs in registers (net_inputs.h) and feeds them to the network
// through LDS, so the inputs never travel through HBM.
#include "snake_mlp.h"

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "net_inputs.h"
#include "kernels.h"
#include "mlp_device.h"

namespace {

using namespace snake::mlp;

constexpr int CH = 32;  // samples per training chunk
constexpr int MT = CH / 16, KS = CH / 32;   // sample row tiles; sample K steps
constexpr int GW = 4;   // waves per training workgroup

thread_local std::string g_mlp_err;

int mfail(int code, const std::string& m)
{
    g_mlp_err = m;
    return code;
}

// C[M x N] = A[M x K] B[K x N] for M, N multiples of 16 and K of 32.  The
// 16 x 16 output tiles (row-major over tiles) go to the waves of the
// workgroup in turn; each tile is computed by one wave.  Lane l supplies A
// rows l % 16 and B columns l % 16 for the k-slice 8 (l / 16) .. +8 and
// receives D rows 4 (l / 16) .. +4 of column l % 16.
template <class FA, class FB, class FS>
__device__ __forceinline__ void wave_gemm(int mtiles, int ntiles, int ktiles, FA A, FB Bm, FS store)
{
    const int l = threadIdx.x & 63, r = l & 15, g = l >> 4, wv = threadIdx.x >> 6;
    for (int tile = wv; tile < mtiles * ntiles; tile += GW) {
        const int mt = tile / ntiles, nt = tile % ntiles;
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

// Weight matrices to LDS as BF16.  Each thread loads its float4 groups
// before converting any, so the loads are in flight together.
template <int ROWS, int COLS, int PROWS>
__device__ __forceinline__ void load_matrix(__bf16 (*dst)[COLS], const float* __restrict__ src)
{
    constexpr int T = 64 * GW;
    constexpr int G = ROWS * COLS / 4;   // float4 groups of the stored rows
    constexpr int PER = (G + T - 1) / T;
    const int l = threadIdx.x;
    float4 v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int gi = l + T * k;
        v[k] = (gi < G && 4 * gi < PROWS * COLS) ? reinterpret_cast<const float4*>(src)[gi]
                                                  : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int gi = l + T * k;
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
    for (int e = l; e < CH * NI; e += 64 * GW) {
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
// the whole launch; a 16 x 64 BF16 buffer per wave in LDS carries each
// layer's output to the next (forward_tile).  Same arithmetic as the
// training pass: BF16 operands, FP32 accumulation, bias and GELU.
constexpr int FW_WAVES = 4;

__global__ void __launch_bounds__(64 * FW_WAVES) __attribute__((amdgpu_waves_per_eu(4)))
k_mlp_forward(const float* __restrict__ p, const float* __restrict__ ms, const float* __restrict__ x,
              float* __restrict__ y, int64_t n)
{
    __shared__ __align__(16) __bf16 Hs[FW_WAVES][16][FW_ROW];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, r = l & 15, g = l >> 4;
    FwdWeights W;
    load_fwd_weights(p, W);
    float mu[8], is[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        mu[j] = ms[8 * g + j];
        is[j] = 1.f / ms[NI + 8 * g + j];
    }
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
        const f32x4 out = forward_tile(W, a, Hs[w]);
        if (r < NO) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t rr = t * 16 + 4 * g + v;
                if (rr < n) y[rr * NO + r] = out[v];
            }
        }
    }
}

// The solver's learned start: network outputs of every joint's two rows at
// the predicted state of the current substep, y[2 J][3] (row 2 j stretch,
// 2 j + 1 bend-twist).  A wave takes 64 joints at a time: each lane computes
// one joint's inputs (joint_features), normalises them and writes both rows
// as BF16 to the wave's 128-row buffer in LDS; then the wave runs the
// network over the buffer in eight 16-sample tiles.  The inputs, their
// normalisation and the network's arithmetic are those of k_features
// followed by k_mlp_forward, so the outputs are the same bits.
constexpr int WN_ROW = NI + 8;   // padded input row (80 bytes)

__global__ void __launch_bounds__(64 * FW_WAVES) __attribute__((amdgpu_waves_per_eu(3)))
k_warm_net(snake::KParams P, const float* __restrict__ p, const float* __restrict__ ms, float* __restrict__ y)
{
    __shared__ __align__(16) __bf16 Xs[FW_WAVES][128][WN_ROW];
    __shared__ __align__(16) __bf16 Hs[FW_WAVES][16][FW_ROW];
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6, r = l & 15, g = l >> 4;
    FwdWeights W;
    load_fwd_weights(p, W);
    const int J = P.J;
    const int64_t rows = 2 * (int64_t)J;
    for (int64_t j0 = ((int64_t)blockIdx.x * FW_WAVES + w) * 64; j0 < J; j0 += (int64_t)gridDim.x * FW_WAVES * 64) {
        const int64_t gj = j0 + l;
        __bf16* xs = Xs[w][2 * l];
        __bf16* xb = Xs[w][2 * l + 1];
        // the wave's 64 joints lie in snakes s0..s1 (searched once per wave)
        const int s0 = snake::snake_of_joint(P, __builtin_amdgcn_readfirstlane((int)j0), 0, P.n_snakes - 1);
        const int jl = (int)(j0 + 63 < J ? j0 + 63 : J - 1);
        const int s1 = snake::snake_of_joint(P, __builtin_amdgcn_readfirstlane(jl), s0, P.n_snakes - 1);
        if (gj < J) {
            float f[32];
            snake::V3 lbn;
            snake::joint_features(P, (int)gj, s0, s1, f, lbn);
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                const float mu = ms[k], is = 1.f / ms[NI + k];
                xs[k] = (__bf16)((f[k] - mu) * is);
                const float fb = k == 19 ? lbn.x : k == 20 ? lbn.y : k == 21 ? lbn.z : k == 30 ? 1.f : f[k];
                xb[k] = (__bf16)((fb - mu) * is);
            }
        } else {
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                xs[k] = (__bf16)0.f;
                xb[k] = (__bf16)0.f;
            }
        }
#pragma unroll 1
        for (int tt = 0; tt < 8; ++tt) {
            // (memcpy: the vector read may not be reordered with the element stores)
            bf16x8 a;
            __builtin_memcpy(&a, &Xs[w][16 * tt + r][8 * g], sizeof(bf16x8));
            const f32x4 out = forward_tile(W, a, Hs[w]);
            if (r < NO) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t rr = 2 * j0 + 16 * tt + 4 * g + v;
                    if (rr < rows) y[rr * NO + r] = out[v];
                }
            }
        }
    }
}

// forward + backward of one chunk per workgroup; one gradient row per chunk
__global__ void __launch_bounds__(64 * GW) k_mlp_grad(const float* __restrict__ p, const float* __restrict__ ms,
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
    if (l < 64) {   // the first wave: 64 partial sums of the loss, as in chunk order
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
    }
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
    for (int e = l; e < CH * NH; e += 64 * GW) S.dZ[e / NH][e % NH] = (__bf16)S.Z1[e / NH][e % NH];
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
// sums over chunks c = j mod 8, each in increasing c, then combined pairwise
// ((0 + 1) + (2 + 3)) + ((4 + 5) + (6 + 7)).  Eight lanes share a parameter,
// one partial sum each, and combine by lane swaps; the same inputs give the
// same bits on every call.
constexpr int RED_PARAMS = 32;   // parameters per 256-thread block

__global__ void __launch_bounds__(256) k_mlp_reduce(const float* __restrict__ gpart, const float* __restrict__ lpart,
                                                    int64_t chunks, int64_t n, float* __restrict__ grad,
                                                    float* __restrict__ loss)
{
    const int j = threadIdx.x & 7;
    const int k = blockIdx.x * RED_PARAMS + (threadIdx.x >> 3);   // k == P_COUNT: the loss
    const float* a = k < P_COUNT ? gpart + k : lpart;
    const int64_t stride = k < P_COUNT ? P_COUNT : 1;
    float acc = 0.f;
    if (k <= P_COUNT) {
        int64_t c = j;
        for (; c + 24 < chunks; c += 32) {
            const float v0 = a[c * stride], v1 = a[(c + 8) * stride], v2 = a[(c + 16) * stride],
                        v3 = a[(c + 24) * stride];
            acc += v0;
            acc += v1;
            acc += v2;
            acc += v3;
        }
        for (; c < chunks; c += 8) acc += a[c * stride];
    }
    acc += __shfl_xor(acc, 1, 8);
    acc += __shfl_xor(acc, 2, 8);
    acc += __shfl_xor(acc, 4, 8);
    if (j == 0 && k < P_COUNT) grad[k] = acc;
    if (j == 0 && k == P_COUNT) *loss = acc / (float)(n * NO);
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
    hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)chunks), dim3(64 * GW), 0, st, params, mean_std, x, t, n, gpart, lpart);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((P_COUNT + 1 + RED_PARAMS - 1) / RED_PARAMS), dim3(256), 0, st, gpart, lpart,
                       chunks, n, grad, loss);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SIM_OK : mfail(SIM_EDEVICE, hipGetErrorString(e));
}

}  // namespace

namespace snake {

hipError_t launch_warm_net(const KParams& P, const float* params, const float* mean_std, float* y,
                           hipStream_t stream)
{
    if (P.J <= 0) return hipSuccess;
    const int64_t blocks = ((int64_t)P.J + 64 * FW_WAVES - 1) / (64 * FW_WAVES);
    const int grid = (int)(blocks < 1024 ? blocks : 1024);
    hipLaunchKernelGGL(k_warm_net, dim3(grid), dim3(64 * FW_WAVES), 0, stream, P, params, mean_std, y);
    return hipGetLastError();
}

}  // namespace snake

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
