// Top-k bitstring extraction (paper Sec. 3.3.2, Selective Distribution
// Exploration): per subgraph, the k bitstrings with the largest probability
// pi(z) = |psi(z)|^2.
//
// Ties. pi(z) is exactly invariant under flipping the bit of a free vertex
// (one without an edge of positive weight in the subgraph: its qubit stays
// in |+>) and under the complement. The candidates these moves connect form
// a tie group: with Fm = the free vertices (other than vertex 0 in canonical
// mode), a group is {r0 ^ S} or, when the complement move stays inside the
// candidates (raw mode, or canonical mode with vertex 0 free) and the
// subgraph has a vertex that is not free, {r0 ^ S} u {r1 ^ S}, S over the
// subsets of Fm; r0 < r1 have no bit in Fm and are each other's complement
// (with bit 0 flipped back in canonical mode) restricted to the other bits.
// The order is the group's probability descending, then r0 ascending, then
// a fixed bijective rank of the string inside the group; in FP32, members of
// one group would otherwise be ordered by rounding noise. So stage 1 keeps
// only the representatives r0, and stage 2 expands each selected group into
// its members in rank order: member j of a group of 2^m is the index
// x = rank^-1(j) (half in the low bit when there are two halves, the bits of
// S at Fm above it), rank(x) = g(A g(x) mod 2^m), g(x) = x ^ (x >> ceil(m/2))
// (a xorshift step, its own inverse on m bits) and A = 2654435761 (Knuth's
// multiplicative hashing); rank^-1(j) = g(A^-1 g(j) mod 2^m).
//
// Each representative becomes one unique 64-bit key, (bits of pi as float)
// << 32 | (0xFFFFFFFF - z): pi >= 0, so the float bit pattern orders like
// the value, and a larger low word means a smaller z. Every valid key is
// nonzero (z < 2^30), so 0 serves as padding below all of them.
//
// Both stages find the k largest keys of a set by a most-significant-digit
// radix select in LDS (8-bit digits, one histogram per digit, stopping as
// soon as every key that shares the current prefix is needed), instead of
// sorting: stage 1 takes one 4096-amplitude tile of the reduced state per
// block, with its candidates in registers, and writes the tile's best k
// unsorted; stage 2 selects a subgraph's best k from its per-tile lists,
// sorts only those and expands them.
// Canonical mode takes only z with bit 0 clear (pi(z) = pi(~z)).
#include "common.h"

namespace pq {

// tie groups of one subgraph (see the file comment)
struct TieGroups {
    uint32_t fm;    // free vertices that a group's strings may differ in
    uint32_t full;  // all n bits
    int halves;     // 2: a group also holds the complement-side half
    int m;          // a group has 2^m strings
    int canonical;
};

__device__ inline TieGroups tie_groups(const SubDesc* d, int canonical)
{
    TieGroups t;
    t.full = (uint32_t)((1ull << d->n) - 1ull);
    t.fm = canonical ? (d->freem & ~1u) : d->freem;
    const bool part_ok = canonical ? (d->freem & 1u) != 0u : true;
    t.halves = (part_ok && d->freem != t.full) ? 2 : 1;
    t.m = __popc(t.fm) + (t.halves == 2 ? 1 : 0);
    t.canonical = canonical;
    return t;
}

// the complement move restricted to the bits outside Fm
__device__ inline uint32_t partner_base(const TieGroups& t, uint32_t z)
{
    const uint32_t c = (~z & t.full) ^ (t.canonical ? 1u : 0u);
    return c & ~t.fm;
}

// is z the representative (smallest base) of its tie group?
__device__ inline bool is_representative(const TieGroups& t, uint32_t z)
{
    if (z & t.fm) return false;
    return t.halves == 1 || z <= partner_base(t, z);
}

constexpr uint32_t TIE_MUL_INV = 0x0E8B2F51u;  // 2654435761^-1 mod 2^32
static_assert(2654435761u * TIE_MUL_INV == 1u, "multiplicative inverse");

__device__ inline uint32_t tie_unrank(uint32_t j, int m)
{
    if (m <= 0) return 0u;
    const uint32_t mask = m >= 32 ? 0xFFFFFFFFu : ((1u << m) - 1u);
    const int s = (m + 1) / 2;
    uint32_t x = j ^ (j >> s);
    x = (x * TIE_MUL_INV) & mask;  // mod 2^32 then mod 2^m
    return x ^ (x >> s);
}

// deposit the low bits of v at the set positions of mask
__device__ inline uint32_t deposit_bits(uint32_t v, uint32_t mask)
{
    uint32_t out = 0;
    for (int j = 0; j < 32 && mask; ++j) {
        const uint32_t low = mask & (0u - mask);
        if (v & 1u) out |= low;
        v >>= 1;
        mask ^= low;
    }
    return out;
}

// string j (in rank order) of the group with representative r0
__device__ inline uint32_t tie_member(const TieGroups& t, uint32_t r0, uint32_t j)
{
    const uint32_t x = tie_unrank(j, t.m);
    const uint32_t half = t.halves == 2 ? (x & 1u) : 0u;
    const uint32_t sp = t.halves == 2 ? (x >> 1) : x;
    const uint32_t base = half ? partner_base(t, r0) : r0;
    return base ^ deposit_bits(sp, t.fm);
}

struct SelState {
    int hist[256];
    int wsum[16];
    int digit, qrem, done, count, nonzero;
    uint64_t out[MAX_K];
};

// number of nonzero keys over the block (each thread passes its own count)
__device__ inline int count_nonzero(SelState& S, int mine)
{
    if (threadIdx.x == 0) S.nonzero = 0;
    __syncthreads();
    for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
    if ((threadIdx.x & 63u) == 0 && mine) atomicAdd(&S.nonzero, mine);
    __syncthreads();
    return S.nonzero;
}

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
// thread. Returns (prefix, digits) such that a nonzero key is among the q
// largest iff digits == 0 or key >> (64 - 8 digits) >= prefix. Zero keys
// (padding) are not counted, so q must not exceed the number of nonzero
// keys (otherwise no digit is found); with unique keys this selects exactly q.
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
            if (key != 0ull && (r == 0 || (key >> (shift + 8)) == prefix))
                atomicAdd(&S.hist[(int)((key >> shift) & 255)], 1);
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
    const TieGroups tg = tie_groups(d, CANON ? 1 : 0);
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
        // only the representatives of tie groups are ranked
        if (CANON) {
            const uint32_t zc = (z & 1u) ? z ^ full : z;
            key[j] = (ok && is_representative(tg, zc)) ? make_key(pr, zc) : 0ull;
        } else {
            key[2 * j] = (ok && is_representative(tg, z)) ? make_key(pr, z) : 0ull;
            key[2 * j + 1] = (ok && is_representative(tg, z ^ full)) ? make_key(pr, z ^ full) : 0ull;
        }
    }
    int mine = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) mine += key[i] != 0ull;
    const int cnt = count_nonzero(S, mine);  // the tile's representatives
    const int q = k < cnt ? k : cnt;
    uint64_t prefix = 0;
    int digits = 0;
    if (t == 0) S.count = 0;
    if (q > 0) radix_select(S, [&](int i) { return key[i]; }, PER, q, prefix, digits);
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
    const TieGroups tg = tie_groups(d, canonical);
    if (d->skip) {
        // edgeless subgraph: |psi|^2 = 2^-n everywhere, so all candidates form
        // one tie group (every vertex free) with representative 0
        if (t == 0) {
            const uint64_t group = 1ull << tg.m;
            for (int i = 0; i < k; ++i) {
                const bool ok = (uint64_t)i < group;
                idx[(size_t)b * k + i] = ok ? tie_member(tg, 0u, (uint32_t)i) : 0xFFFFFFFFu;
                prob[(size_t)b * k + i] = ok ? ldexpf(1.0f, -d->n) : -1.0f;
            }
        }
        return;
    }
    const int total = d->ntiles * k;
    const uint64_t* src = in + (size_t)d->tile_base * k;
    const int nloc = (total - t + MERGE_THREADS - 1) / MERGE_THREADS;  // keys t, t + 1024, ...
    uint64_t prefix = 0;
    int digits = 0;
    int mine = 0;
    for (int i = 0; i < nloc; ++i) mine += src[t + (size_t)i * MERGE_THREADS] != 0ull;
    const int cnt = count_nonzero(S, mine);
    const int q = k < cnt ? k : cnt;
    if (t == 0) S.count = 0;
    if (t < MAX_K) S.out[t] = 0ull;
    if (q > 0) radix_select(S, [&](int i) { return src[t + (size_t)i * MERGE_THREADS]; }, nloc, q, prefix, digits);
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
    // expand the selected groups, in order, into their strings in rank order
    if (t == 0) {
        const uint64_t group = 1ull << tg.m;
        int out = 0;
        for (int i = 0; i < k && out < k; ++i) {
            const uint64_t key = S.out[i];
            if (key == 0ull) break;
            const uint32_t r0 = 0xFFFFFFFFu - (uint32_t)(key & 0xFFFFFFFFull);
            const float pr = __uint_as_float((uint32_t)(key >> 32));
            for (uint64_t j = 0; j < group && out < k; ++j, ++out) {
                idx[(size_t)b * k + out] = tie_member(tg, r0, (uint32_t)j);
                prob[(size_t)b * k + out] = pr;
            }
        }
        for (; out < k; ++out) {
            idx[(size_t)b * k + out] = 0xFFFFFFFFu;
            prob[(size_t)b * k + out] = -1.0f;
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
