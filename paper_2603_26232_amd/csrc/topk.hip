// Top-k bitstring extraction (paper Sec. 3.3.2, Selective Distribution
// Exploration): per subgraph, the k bitstrings with the largest probability
// pi(z) = |psi(z)|^2, ordered by (pi descending, z ascending).
//
// Each candidate becomes one unique 64-bit key, (bits of pi as float) << 32 |
// (0xFFFFFFFF - z): pi >= 0, so the float bit pattern orders like the value,
// and a larger low word means a smaller z. Every valid key is nonzero (z <
// 2^30), so 0 serves as padding below all of them.
//
// Both stages find the k largest keys of a set by a most-significant-digit
// radix select in LDS (8-bit digits, one histogram per digit, stopping as
// soon as every key that shares the current prefix is needed), instead of
// sorting: stage 1 takes one 4096-amplitude tile of the reduced state per
// block, with its candidates in registers, and writes the tile's best k
// unsorted; stage 2 selects a subgraph's best k from its per-tile lists and
// sorts only those.
// Canonical mode takes only z with bit 0 clear (pi(z) = pi(~z)).
#include "common.h"

namespace pq {

struct SelState {
    int hist[256];
    int wsum[16];
    int digit, qrem, done, count;
    uint64_t out[MAX_K];
};

// the digit (from the top) that holds the q-th largest counted key; sets
// done when exactly q keys were counted (then all of them are taken)
__device__ void pick_digit(SelState& S, int q)
{
    const int t = threadIdx.x;
    int h = 0, incl = 0;
    if (t < 256) {
        h = S.hist[255 - t];
        incl = h;
        const int lane = t & 63;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        if (lane == 63) S.wsum[t >> 6] = incl;
    }
    __syncthreads();
    if (t < 256) {
        int base = 0;
        for (int w = 0; w < (t >> 6); ++w) base += S.wsum[w];
        incl += base;
        const int excl = incl - h;
        if (t == 255) S.done = (incl == q);
        if (h > 0 && excl < q && q <= incl) {
            S.digit = 255 - t;
            S.qrem = q - excl;
        }
    }
    __syncthreads();
}

// Radix select of the q largest keys produced by src(i), i < n_local per
// thread. Returns (prefix, digits) such that a key is among the q largest iff
// digits == 0 or key >> (64 - 8 digits) >= prefix. With unique keys this
// selects exactly q; with repeated keys (padding) it may select more.
template <typename Src>
__device__ void radix_select(SelState& S, const Src& src, int n_local, int q, uint64_t& prefix, int& digits)
{
    const int t = threadIdx.x;
    prefix = 0;
    digits = 0;
    for (int r = 0; r < 8; ++r) {
        if (t < 256) S.hist[t] = 0;
        __syncthreads();
        const int shift = 56 - 8 * r;
        for (int i = 0; i < n_local; ++i) {
            const uint64_t key = src(i);
            if (r == 0 || (key >> (shift + 8)) == prefix) atomicAdd(&S.hist[(int)((key >> shift) & 255)], 1);
        }
        __syncthreads();
        pick_digit(S, q);
        if (S.done) return;
        prefix = (prefix << 8) | (uint64_t)S.digit;
        q = S.qrem;
        digits = r + 1;
        __syncthreads();  // everyone has read digit/qrem before the next round
    }
}

__device__ inline bool selected(uint64_t key, uint64_t prefix, int digits)
{
    return digits == 0 || (key >> (64 - 8 * digits)) >= prefix;
}

__device__ inline uint64_t make_key(float pr, uint32_t z)
{
    return ((uint64_t)__float_as_uint(pr) << 32) | (uint64_t)(0xFFFFFFFFu - z);
}

// stage 1: one tile of one subgraph -> its best k keys (unsorted, 0-padded)
template <bool CANON>
__global__ __launch_bounds__(THREADS) void k_topk_tile(const uint8_t* ws, const SubDesc* subs, const int2* work,
                                                      int k, uint64_t* out)
{
    // The stored state is reduced: amplitude z' (top bit clear, scaled by
    // sqrt(2)) stands for z' and its complement z' ^ (2^n - 1), each with
    // probability |phi(z')|^2 / 2. The canonical one of the pair is the one
    // with bit 0 clear; raw mode takes both.
    constexpr int AMPS = TILE / THREADS;          // 16 amplitudes per thread
    constexpr int PER = CANON ? AMPS : 2 * AMPS;  // candidates per thread
    __shared__ SelState S;
    const int2 wk = work[blockIdx.x];
    const SubDesc* d = subs + wk.x;
    const int n = d->n;
    const uint32_t base = (uint32_t)wk.y * TILE;
    const float2* st = (const float2*)(ws + d->psi) + base;
    const uint32_t span = n - 1 < TILE_BITS ? (1u << (n - 1)) : (uint32_t)TILE;
    const uint32_t full = (uint32_t)((1ull << n) - 1ull);
    const int t = threadIdx.x;
    uint64_t key[PER];
#pragma unroll
    for (int j = 0; j < AMPS; ++j) {
        const uint32_t c = (uint32_t)t + (uint32_t)j * THREADS;
        const bool ok = c < span;
        float2 a = make_float2(0.f, 0.f);
        if (ok) a = st[c];
        const float pr = 0.5f * (a.x * a.x + a.y * a.y);
        const uint32_t z = base + c;
        if (CANON) {
            key[j] = ok ? make_key(pr, (z & 1u) ? z ^ full : z) : 0ull;
        } else {
            key[2 * j] = ok ? make_key(pr, z) : 0ull;
            key[2 * j + 1] = ok ? make_key(pr, z ^ full) : 0ull;
        }
    }
    const int cnt = (int)(CANON ? span : 2 * span);
    const int q = k < cnt ? k : cnt;
    uint64_t prefix;
    int digits;
    if (t == 0) S.count = 0;
    radix_select(S, [&](int i) { return key[i]; }, PER, q, prefix, digits);
    uint64_t* o = out + ((size_t)d->tile_base + wk.y) * k;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        if (key[i] != 0ull && selected(key[i], prefix, digits)) {
            const int slot = atomicAdd(&S.count, 1);
            if (slot < k) o[slot] = key[i];
        }
    }
    __syncthreads();
    for (int i = S.count + t; i < k; i += THREADS) o[i] = 0ull;
}

// stage 2: a subgraph's ntiles * k keys -> its best k, sorted; results
constexpr int MERGE_THREADS = 1024;

__global__ __launch_bounds__(MERGE_THREADS) void k_topk_merge(const SubDesc* subs, int k, int canonical,
                                                             const uint64_t* in, uint32_t* idx, float* prob)
{
    __shared__ SelState S;
    const int b = blockIdx.x;
    const SubDesc* d = subs + b;
    const int t = threadIdx.x;
    if (d->skip) {
        // edgeless subgraph: |psi|^2 = 2^-n everywhere, ties broken by index
        const uint32_t step = canonical ? 2u : 1u;
        const uint64_t cnt = (1ull << d->n) / step;
        for (int i = t; i < k; i += MERGE_THREADS) {
            const bool ok = (uint64_t)i < cnt;
            idx[(size_t)b * k + i] = ok ? (uint32_t)i * step : 0xFFFFFFFFu;
            prob[(size_t)b * k + i] = ok ? ldexpf(1.0f, -d->n) : -1.0f;
        }
        return;
    }
    const int total = d->ntiles * k;
    const uint64_t* src = in + (size_t)d->tile_base * k;
    const int nloc = (total - t + MERGE_THREADS - 1) / MERGE_THREADS;  // keys t, t + 1024, ...
    uint64_t prefix;
    int digits;
    if (t == 0) S.count = 0;
    if (t < MAX_K) S.out[t] = 0ull;
    radix_select(S, [&](int i) { return src[t + (size_t)i * MERGE_THREADS]; }, nloc, k, prefix, digits);
    for (int i = 0; i < nloc; ++i) {
        const uint64_t key = src[t + (size_t)i * MERGE_THREADS];
        if (key != 0ull && selected(key, prefix, digits)) {
            const int slot = atomicAdd(&S.count, 1);
            if (slot < k) S.out[slot] = key;
        }
    }
    __syncthreads();
    // sort the (at most 64) winners descending: bitonic over 64 slots
    for (int size = 2; size <= MAX_K; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (t < MAX_K / 2) {
                const int lo = 2 * stride * (t / stride) + (t % stride);
                const int hi = lo + stride;
                const uint64_t a = S.out[lo], c = S.out[hi];
                const bool desc = (lo & size) == 0;
                if (desc ? (a < c) : (a > c)) {
                    S.out[lo] = c;
                    S.out[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int i = t; i < k; i += MERGE_THREADS) {
        const uint64_t key = S.out[i];
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
                       int canonical, uint64_t* keys, uint32_t* idx, float* prob, hipStream_t s)
{
    if (nwork > 0) {
        if (canonical)
            hipLaunchKernelGGL(k_topk_tile<true>, dim3(nwork), dim3(THREADS), 0, s, ws, subs, work, k, keys);
        else
            hipLaunchKernelGGL(k_topk_tile<false>, dim3(nwork), dim3(THREADS), 0, s, ws, subs, work, k, keys);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_topk_merge, dim3(B), dim3(MERGE_THREADS), 0, s, subs, k, canonical, keys, idx, prob);
    return hipGetLastError();
}

}  // namespace pq
