// Index work on the device: offsets, block list, degrees, greedy colouring,
// size buckets and the work order.  Integer only; results are unique, so
// they are checked bit for bit.
#include "kernels.h"

namespace snake {

namespace {

constexpr int kScanThreads = 1024;

// exclusive prefix sums of B, B-1, M and the block count, one workgroup
__global__ void __launch_bounds__(kScanThreads) k_offsets(IParams P)
{
    __shared__ int sb[kScanThreads], sm[kScanThreads], sk[kScanThreads];
    __shared__ int carry[3];
    const int t = threadIdx.x;
    if (t == 0) carry[0] = carry[1] = carry[2] = 0;
    __syncthreads();
    for (int base = 0; base < P.n_snakes; base += kScanThreads) {
        const int s = base + t;
        int b = 0, mm = 0, k = 0;
        if (s < P.n_snakes) {
            b = P.Bn[s];
            mm = P.Mn[s];
            k = 2 * (b - 1) + (P.ground ? b : 0);
        }
        sb[t] = b;
        sm[t] = mm;
        sk[t] = k;
        __syncthreads();
        // Hillis-Steele inclusive scan
        for (int off = 1; off < kScanThreads; off <<= 1) {
            int vb = 0, vm = 0, vk = 0;
            if (t >= off) {
                vb = sb[t - off];
                vm = sm[t - off];
                vk = sk[t - off];
            }
            __syncthreads();
            sb[t] += vb;
            sm[t] += vm;
            sk[t] += vk;
            __syncthreads();
        }
        if (s < P.n_snakes) {
            const int eb = carry[0] + sb[t] - b;
            P.body_off[s] = eb;
            P.joint_off[s] = eb - s;
            P.module_off[s] = carry[1] + sm[t] - mm;
            P.block_off[s] = carry[2] + sk[t] - k;
        }
        __syncthreads();
        if (t == kScanThreads - 1) {
            carry[0] += sb[t];
            carry[1] += sm[t];
            carry[2] += sk[t];
        }
        __syncthreads();
    }
    if (t == 0) {
        P.body_off[P.n_snakes] = carry[0];
        P.joint_off[P.n_snakes] = carry[0] - P.n_snakes;
        P.module_off[P.n_snakes] = carry[1];
        P.block_off[P.n_snakes] = carry[2];
    }
}

__device__ __forceinline__ int find_segment(const int* off, int n, int g)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// block list: per snake (stretch_j, bend_j) for each joint, then contacts
__global__ void k_blocks(IParams P)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.n_blocks) return;
    const int s = find_segment(P.block_off, P.n_snakes, k);
    const int local = k - P.block_off[s];
    const int B = P.Bn[s];
    const int bo = P.body_off[s];
    if (local < 2 * (B - 1)) {
        const int j = local >> 1;
        P.blk_type[k] = local & 1;
        P.blk_a[k] = bo + j;
        P.blk_b[k] = bo + j + 1;
    } else {
        P.blk_type[k] = 2;
        P.blk_a[k] = bo + (local - 2 * (B - 1));
        P.blk_b[k] = -1;
    }
}

__global__ void k_degree(IParams P)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= P.N) return;
    const int s = find_segment(P.body_off, P.n_snakes, g);
    const int i = g - P.body_off[s];
    const int B = P.Bn[s];
    P.degree[g] = P.ground + (i > 0 ? 2 : 0) + (i + 1 < B ? 2 : 0);
    P.color_scratch[g] = 0;
}

// Greedy colouring in block-list order: each block takes the smallest colour
// not used by an earlier block sharing a body.  Snakes share no body, so each
// snake is coloured independently by one thread, in order.
__global__ void k_color(IParams P)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= P.n_snakes) return;
    const int k0 = P.block_off[s], k1 = P.block_off[s + 1];
    for (int k = k0; k < k1; ++k) {
        const int a = P.blk_a[k], b = P.blk_b[k];
        unsigned used = (unsigned)P.color_scratch[a];
        if (b >= 0) used |= (unsigned)P.color_scratch[b];
        const int col = __builtin_ctz(~used);
        P.blk_color[k] = col;
        P.color_scratch[a] = (int)((unsigned)P.color_scratch[a] | (1u << col));
        if (b >= 0) P.color_scratch[b] = (int)((unsigned)P.color_scratch[b] | (1u << col));
    }
}

// bucket = ceil(log2 B); work order position = number of snakes that come
// before s under (B descending, id ascending)
constexpr int kOrderTile = 256;
__global__ void __launch_bounds__(kOrderTile) k_order(IParams P)
{
    __shared__ int tileB[kOrderTile];
    const int s = blockIdx.x * kOrderTile + threadIdx.x;
    const int Bs = s < P.n_snakes ? P.Bn[s] : 0;
    int rank = 0;
    for (int base = 0; base < P.n_snakes; base += kOrderTile) {
        const int t = base + threadIdx.x;
        tileB[threadIdx.x] = t < P.n_snakes ? P.Bn[t] : -1;
        __syncthreads();
        const int lim = min(kOrderTile, P.n_snakes - base);
        for (int u = 0; u < lim; ++u) {
            const int Bt = tileB[u];
            rank += (Bt > Bs || (Bt == Bs && base + u < s)) ? 1 : 0;
        }
        __syncthreads();
    }
    if (s < P.n_snakes) {
        P.order[rank] = s;
        P.bucket[s] = Bs <= 1 ? 0 : 32 - __builtin_clz((unsigned)(Bs - 1));
    }
}

}  // namespace

hipError_t launch_index(const IParams& P, hipStream_t stream)
{
    hipLaunchKernelGGL(k_offsets, dim3(1), dim3(kScanThreads), 0, stream, P);
    if (P.n_blocks > 0)
        hipLaunchKernelGGL(k_blocks, dim3((P.n_blocks + 255) / 256), dim3(256), 0, stream, P);
    hipLaunchKernelGGL(k_degree, dim3((P.N + 255) / 256), dim3(256), 0, stream, P);
    hipLaunchKernelGGL(k_color, dim3((P.n_snakes + 63) / 64), dim3(64), 0, stream, P);
    hipLaunchKernelGGL(k_order, dim3((P.n_snakes + kOrderTile - 1) / kOrderTile), dim3(kOrderTile), 0,
                       stream, P);
    return hipGetLastError();
}

}  // namespace snake
