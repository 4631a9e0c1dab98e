// Top-k bitstring extraction (paper Sec. 3.3.2, Selective Distribution
// Exploration): per subgraph, the k bitstrings with the largest probability
// pi(z) = |psi(z)|^2, ordered by (pi descending, z ascending).
//
// Each candidate becomes one unique 64-bit key, (bits of pi as float) << 32 |
// (0xFFFFFFFF - z): pi >= 0, so the float bit pattern orders like the value,
// and a larger low word means a smaller z. Stage 1 sorts the candidates of
// one 4096-amplitude tile in LDS (bitonic) and keeps the best k; stage 2
// folds the per-tile lists of a subgraph 2048 keys at a time into a running
// best-k. Canonical mode takes only z with bit 0 clear (pi(z) = pi(~z)).
#include "common.h"

namespace pq {

constexpr int SORT_N = 4096;

// descending bitonic sort of s[0..n) (n a power of two, n <= SORT_N)
__device__ void bitonic_desc(uint64_t* s, int n)
{
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < (n >> 1); i += blockDim.x) {
                const int lo = 2 * stride * (i / stride) + (i % stride);
                const int hi = lo + stride;
                const uint64_t a = s[lo], b = s[hi];
                const bool desc = (lo & size) == 0;
                if (desc ? (a < b) : (a > b)) {
                    s[lo] = b;
                    s[hi] = a;
                }
            }
            __syncthreads();
        }
    }
}

__device__ inline uint64_t make_key(float2 a, uint32_t z)
{
    const float pr = a.x * a.x + a.y * a.y;
    return ((uint64_t)__float_as_uint(pr) << 32) | (uint64_t)(0xFFFFFFFFu - z);
}

// stage 1: one tile of one subgraph -> best k keys of that tile
__global__ __launch_bounds__(THREADS) void k_topk_tile(const uint8_t* ws, const SubDesc* subs, const int2* work,
                                                      int k, int canonical, uint64_t* out)
{
    __shared__ uint64_t s[SORT_N];
    const int2 wk = work[blockIdx.x];
    const SubDesc d = subs[wk.x];
    const uint32_t t = (uint32_t)wk.y;
    const float2* st = (const float2*)(ws + d.psi);
    const uint32_t dim = 1u << d.n;
    const uint32_t span = dim < (uint32_t)TILE ? dim : (uint32_t)TILE;
    const uint32_t step = canonical ? 2u : 1u;
    const uint32_t cnt = span / step;  // candidates in this tile
    int n2 = 1;
    while (n2 < (int)cnt) n2 <<= 1;
    for (int i = threadIdx.x; i < n2; i += THREADS) {
        uint64_t key = 0;
        if ((uint32_t)i < cnt) {
            const uint32_t z = t * TILE + (uint32_t)i * step;
            key = make_key(st[z], z);
        }
        s[i] = key;
    }
    __syncthreads();
    bitonic_desc(s, n2);
    uint64_t* o = out + ((size_t)d.tile_base + t) * k;
    for (int i = threadIdx.x; i < k; i += THREADS) o[i] = (i < n2) ? s[i] : 0ull;
}

// stage 2: fold the ntiles*k keys of a subgraph into its best k; write results
__global__ __launch_bounds__(THREADS) void k_topk_merge(const SubDesc* subs, int k, int canonical, const uint64_t* in,
                                                       uint32_t* idx, float* prob)
{
    __shared__ uint64_t s[SORT_N];
    const int b = blockIdx.x;
    const SubDesc d = subs[b];
    if (d.skip) {
        // edgeless subgraph: |psi|^2 = 2^-n everywhere, ties broken by index
        const uint32_t step = canonical ? 2u : 1u;
        const uint64_t cnt = (1ull << d.n) / step;
        for (int i = threadIdx.x; i < k; i += THREADS) {
            const bool ok = (uint64_t)i < cnt;
            idx[(size_t)b * k + i] = ok ? (uint32_t)i * step : 0xFFFFFFFFu;
            prob[(size_t)b * k + i] = ok ? ldexpf(1.0f, -d.n) : -1.0f;
        }
        return;
    }
    const size_t total = (size_t)d.ntiles * k;
    const uint64_t* src = in + (size_t)d.tile_base * k;
    const int chunk = SORT_N / 2;
    for (int i = threadIdx.x; i < SORT_N; i += THREADS) s[i] = 0ull;
    __syncthreads();
    for (size_t off = 0; off < total; off += chunk) {
        // slots [0, k) hold the running best; [k, k + chunk) the next keys
        for (int i = threadIdx.x; i < SORT_N - k; i += THREADS) {
            const size_t j = off + (size_t)i;
            s[k + i] = (i < chunk && j < total) ? src[j] : 0ull;
        }
        __syncthreads();
        bitonic_desc(s, SORT_N);
    }
    for (int i = threadIdx.x; i < k; i += THREADS) {
        const uint64_t key = s[i];
        if (key == 0ull) {
            idx[(size_t)b * k + i] = 0xFFFFFFFFu;
            prob[(size_t)b * k + i] = -1.0f;
        } else {
            idx[(size_t)b * k + i] = 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull);
            prob[(size_t)b * k + i] = __uint_as_float((uint32_t)(key >> 32));
        }
    }
}

hipError_t launch_topk(uint8_t* ws, const SubDesc* subs, const int2* work, int nwork, int B, int k,
                       int canonical, uint64_t* keys_a, uint64_t* keys_b, uint32_t* idx, float* prob,
                       hipStream_t s)
{
    (void)keys_b;
    if (nwork > 0) {
        hipLaunchKernelGGL(k_topk_tile, dim3(nwork), dim3(THREADS), 0, s, ws, subs, work, k, canonical, keys_a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_topk_merge, dim3(B), dim3(THREADS), 0, s, subs, k, canonical, keys_a, idx, prob);
    return hipGetLastError();
}

}  // namespace pq
