// Merge of the per-subgraph candidate sets (paper Sec. 3.4, Alg. 2) as a
// level-wise beam on the GPU.
//
// Level i holds the chain subgraph V_i = [start_i, start_i + size_i); V_i
// shares its first vertex with V_{i-1}. Candidate set B_i = {b_j, ~b_j}; a
// path takes one member of B_1, then at every later level the member of each
// pair whose bit for the shared vertex agrees with the path (so a path has
// 2K choices at level 1 and K at each later level: 2 K^M leaves). Path order
// is the depth-first order of Alg. 2 (digits 2j+o at level 1, j later).
//
// Score of a partial path = cut of the edges whose endpoints are both
// assigned. By the cut decomposition of Sec. 3.4.1 a child's score is its
// parent's plus C_i(b_j) (the intra-subgraph cut, orientation free) plus the
// back edges (u assigned earlier, v new in V_i): sum_k (y_k ? W_k - A_k : A_k)
// with y_k the child's bit for local vertex k, W_k the back-edge weight into
// k and A_k the weight of those back edges whose earlier endpoint is 1 in the
// parent. After each level the W best paths by (score desc, path order asc)
// survive; with W >= 2 K^(M-1) this is the exhaustive merge.
//
// Keys: 32-bit, score + 1 (zero marks an invalid candidate); a key's index
// in the level's key array is its path order, parent_rank * K + j (level 1:
// 2j + o). Survivors are kept in path order, so a survivor's rank is its
// position.
#include "common.h"

namespace pq {

__device__ inline int level_k(const uint32_t* cand, int K, int i)
{
    int k = 0;
    while (k < K && cand[(size_t)i * K + k] != 0xFFFFFFFFu) ++k;
    return k;
}

// C_i(b_j) for every level and candidate
__global__ void k_merge_intra(const MergeLevel* lv, const int32_t* intra, const uint32_t* cand, int K,
                              int64_t* ccut)
{
    const int i = blockIdx.x;
    const MergeLevel L = lv[i];
    for (int j = threadIdx.x; j < K; j += blockDim.x) {
        const uint32_t b = cand[(size_t)i * K + j];
        int64_t c = 0;
        if (b != 0xFFFFFFFFu) {
            for (int e = 0; e < L.intra_cnt; ++e) {
                const int32_t* E = intra + 3 * (size_t)(L.intra_off + e);
                if (((b >> E[0]) ^ (b >> E[1])) & 1u) c += E[2];
            }
        }
        ccut[(size_t)i * K + j] = c;
    }
}

// level 1: the 2 K_1 paths (j, o) in order b_1, ~b_1, b_2, ~b_2, ...
__global__ void k_merge_first(const uint32_t* cand, int K, const int64_t* ccut, uint32_t* keys, int32_t* npaths)
{
    const int Kv = level_k(cand, K, 0);
    for (int d = threadIdx.x; d < 2 * K; d += blockDim.x) {
        const int j = d >> 1;
        keys[d] = j < Kv ? (uint32_t)(ccut[j] + 1) : 0u;
    }
    if (threadIdx.x == 0) npaths[0] = 1;
}

__device__ inline uint32_t row_bit(const uint32_t* row, int v) { return (row[v >> 5] >> (v & 31)) & 1u; }

// level i >= 1: one block per parent path, one thread per candidate j
__global__ void k_merge_expand(const MergeLevel* lv, int i, const int32_t* back, const uint32_t* cand, int K,
                               const int64_t* ccut, const uint32_t* rows, int nw, const int64_t* scores,
                               const int32_t* npaths, uint32_t* keys)
{
    __shared__ int32_t A[32];
    const int p = blockIdx.x;
    if (p >= npaths[i]) return;
    const MergeLevel& L = lv[i];  // read in place (uniform loads), not copied
    const uint32_t* row = rows + (size_t)p * nw;
    if (threadIdx.x < 32) A[threadIdx.x] = 0;
    __syncthreads();
    // the level's back edges spread over the lanes (independent loads); the
    // sums are integers (total weight < 2^31), so their order does not matter
    const int nb = L.kbeg[32];
    for (int e = threadIdx.x; e < nb; e += blockDim.x) {
        const int32_t* E = back + 3 * (size_t)(L.back_off + e);
        if (row_bit(row, E[0])) atomicAdd(&A[E[1]], E[2]);
    }
    __syncthreads();
    const int Kv = level_k(cand, K, i);
    const uint32_t xs = row_bit(row, L.start);
    const int64_t ps = scores[p];
    const int size = L.size;
    for (int j = threadIdx.x; j < K; j += blockDim.x) {
        uint32_t key = 0;
        if (j < Kv) {
            const uint32_t b = cand[(size_t)i * K + j];
            const uint32_t o = (b & 1u) ^ xs;
            int64_t s = ps + ccut[(size_t)i * K + j];
            for (int k = 1; k < size; ++k) {
                const uint32_t y = ((b >> k) & 1u) ^ o;
                s += y ? (L.wk[k] - (int64_t)A[k]) : (int64_t)A[k];
            }
            key = (uint32_t)(s + 1);
        }
        keys[(size_t)p * K + j] = key;
    }
}

constexpr int SEL_THREADS = 1024;
constexpr int SEL_WAVES = SEL_THREADS / 64;
constexpr int SEL_BINS = 4096;
static_assert(SEL_THREADS * 64 == MERGE_KEY_PAD, "key buffer padding covers one resident round");

__device__ inline int32_t wave_sum(int32_t x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}
__device__ inline uint32_t wave_max(uint32_t x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t y = __shfl_xor(x, o, 64);
        x = y > x ? y : x;
    }
    return x;
}
__device__ inline uint32_t wave_min(uint32_t x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t y = __shfl_xor(x, o, 64);
        x = y < x ? y : x;
    }
    return x;
}
// exclusive prefix of the per-wave values slots[0..SEL_WAVES) at wave wv,
// and their total (lanes 0..SEL_WAVES-1 read one slot each)
__device__ inline void wave_slots_prefix(const int32_t* slots, int wv, int32_t& before, int32_t& total)
{
    const int lane = threadIdx.x & 63;
    const int32_t v = lane < SEL_WAVES ? slots[lane] : 0;
    int32_t incl = v;
#pragma unroll
    for (int o = 1; o < SEL_WAVES; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    before = __shfl(incl - v, wv, 64);
    total = __shfl(incl, SEL_WAVES - 1, 64);
}
// the value of x unknown to the optimiser (keeps it from holding values
// derived from x live across the kernel instead of recomputing them)
__device__ inline int32_t opaque(int32_t x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Keep the Wsel best keys among keys[0..N) (N = paths * Kmul, key index =
// path order) by (key desc, index asc) and write them as survivors in index
// order; the survivor count is the next level's path count. One workgroup;
// the keys are visited in rounds of SEL_THREADS * PER, wave w of a round
// holding keys [w * 64 PER, (w + 1) * 64 PER) of it in registers (64
// consecutive keys per register). RESIDENT: N <= SEL_THREADS * PER (the
// caller guarantees it), one round, the keys are read from memory once;
// otherwise every step below re-reads them round by round. The key buffer
// is padded to a multiple of MERGE_KEY_PAD entries, so every round reads in
// bounds; entries at N and beyond are masked. (1) count, largest and
// smallest valid key; (2) threshold key k* and the number R of keys equal to
// k* that survive (every key above k* does), from histograms of
// (hi - key) >> shift over [lo, hi] with 4096 bins, refined to the bin
// holding the Wsel-th key until shift = 0 (at most three histograms for
// 31-bit keys); (3) compaction in index order by wave ballots.
template <int PER, bool RESIDENT>
__global__ __launch_bounds__(SEL_THREADS) void k_merge_select(const uint32_t* keys, const int32_t* npaths, int Kmul,
                                                              int Wsel, int first, Surv* surv, int32_t* nsurv)
{
    __shared__ int32_t hist[SEL_BINS];
    __shared__ int32_t wa[SEL_WAVES], wb[SEL_WAVES];
    __shared__ uint32_t s_hi, s_lo;
    __shared__ int32_t s_above;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int32_t N = *npaths * Kmul;  // <= QAOA_MAX_BEAM * 2 QAOA_MAX_K
    constexpr int32_t RW = SEL_THREADS * PER;
    const int rounds = RESIDENT ? 1 : (N + RW - 1) / RW;
    uint32_t sc[PER];
    auto load = [&](int r) {
        const int32_t b = opaque(r * RW + wv * 64 * PER + lane);
        const uint32_t* kp = keys + b;
        const int32_t lim = N - b;  // register j holds a key iff 64 j < lim
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t v = kp[64 * j];
            sc[j] = 64 * j < lim ? v : 0u;
        }
    };
    // (1)
    int32_t valid = 0;
    uint32_t mx = 0, mn = 0xFFFFFFFFu;  // mn: smallest valid key - 1
    for (int r = 0; r < rounds; ++r) {
        load(r);
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t k = sc[j];
            valid += k != 0u;
            mx = k > mx ? k : mx;
            mn = k - 1u < mn ? k - 1u : mn;  // invalid (0) wraps to the maximum
        }
    }
    valid = wave_sum(valid);
    mx = wave_max(mx);
    mn = wave_min(mn);
    if (lane == 0) {
        wa[wv] = valid;
        wb[wv] = (int32_t)mx;
        hist[wv] = (int32_t)mn;
    }
    __syncthreads();
    int32_t nvalid, unused;
    wave_slots_prefix(wa, 0, unused, nvalid);
    uint32_t hi = wave_max(lane < SEL_WAVES ? (uint32_t)wb[lane] : 0u);
    uint32_t lo = wave_min(lane < SEL_WAVES ? (uint32_t)hist[lane] : 0xFFFFFFFFu) + 1u;  // >= 1 if any valid
    // (2)
    uint32_t kstar = 0;  // nvalid <= Wsel: every valid key (> 0) survives
    int32_t R = 0;
    if (nvalid > Wsel) {
        int32_t above = 0;  // keys above the current range [lo, hi]
        for (;;) {
            int shift = 0;
            while (((hi - lo) >> shift) >= (uint32_t)SEL_BINS) ++shift;
            __syncthreads();  // the previous reads of hist / wa are done
            for (int c = tid; c < SEL_BINS; c += SEL_THREADS) hist[c] = 0;
            __syncthreads();
            for (int r = 0; r < rounds; ++r) {
                if (!RESIDENT) load(r);
#pragma unroll
                for (int j = 0; j < PER; ++j) {
                    const uint32_t k = sc[j];
                    if (k >= lo && k <= hi) atomicAdd(&hist[(hi - k) >> shift], 1);  // lo >= 1: valid keys only
                }
            }
            __syncthreads();
            // thread t owns bins 4t .. 4t + 3; block exclusive scan of their sums
            int32_t h4[4], part = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                h4[c] = hist[4 * tid + c];
                part += h4[c];
            }
            int32_t incl = part;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int32_t y = __shfl_up(incl, o, 64);
                if (lane >= o) incl += y;
            }
            if (lane == 63) wa[wv] = incl;
            __syncthreads();
            int32_t wbefore, wtotal;
            wave_slots_prefix(wa, wv, wbefore, wtotal);
            int32_t run = above + wbefore + incl - part;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                if (run < Wsel && run + h4[c] >= Wsel) {  // exactly one bin of one thread
                    const uint32_t bin = (uint32_t)(4 * tid + c);
                    s_above = run;
                    s_hi = hi - (bin << shift);
                    const uint32_t w = (bin << shift) + ((1u << shift) - 1u);  // hi - (the bin's lowest key)
                    s_lo = (hi - lo > w) ? hi - w : lo;
                }
                run += h4[c];
            }
            __syncthreads();
            above = s_above;
            hi = s_hi;
            lo = s_lo;
            if (shift == 0) {  // the bin is the single key value k*
                kstar = hi;
                R = Wsel - above;
                break;
            }
        }
    }
    // (3)
    const uint64_t below = (1ull << lane) - 1ull;
    int32_t carry_gt = 0, carry_eq = 0;
    for (int r = 0; r < rounds; ++r) {
        if (!RESIDENT) load(r);
        int32_t gt = 0, eq = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t k = sc[j];
            gt += k > kstar;
            eq += k == kstar;  // kstar = 0 only if R = 0, where eq does not matter
        }
        gt = wave_sum(gt);
        eq = wave_sum(eq);
        __syncthreads();  // wa / wb free
        if (lane == 0) {
            wa[wv] = gt;
            wb[wv] = eq;
        }
        __syncthreads();
        int32_t gt_before, eq_before, gt_tot, eq_tot;
        wave_slots_prefix(wa, wv, gt_before, gt_tot);
        wave_slots_prefix(wb, wv, eq_before, eq_tot);
        gt_before += carry_gt;
        eq_before += carry_eq;
        carry_gt += gt_tot;
        carry_eq += eq_tot;
        const int32_t b = opaque(r * RW + wv * 64 * PER + lane);
        const uint32_t ks = (uint32_t)opaque((int32_t)kstar);  // recompute the ballots, do not keep them
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t k = sc[j];
            const bool g = k > ks, e = k == ks;
            const uint64_t bg = __ballot(g), be = __ballot(e);
            const int32_t my_gt = gt_before + __popcll(bg & below), my_eq = eq_before + __popcll(be & below);
            if (g || (e && my_eq < R)) {
                const int32_t q = b + 64 * j;
                const int pos = my_gt + (my_eq < R ? my_eq : R);
                Surv sv;
                sv.parent = first ? 0 : q / Kmul;
                sv.digit = first ? q : q % Kmul;
                sv.score = opaque((int32_t)k) - 1;  // computed here, not hoisted for every register
                surv[pos] = sv;
            }
            gt_before += __popcll(bg);
            eq_before += __popcll(be);
        }
    }
    if (tid == 0) *nsurv = nvalid < Wsel ? nvalid : Wsel;
}

// rows of the surviving paths: parent row prefix plus the bits of V_i
__global__ void k_merge_build(const MergeLevel* lv, int i, const uint32_t* cand, int K, const Surv* surv,
                              const int32_t* nsurv, const uint32_t* prow, uint32_t* nrow, int nw, int64_t* scores,
                              int final_out, int nV)
{
    const int r = blockIdx.x;
    if (r >= *nsurv) return;
    const MergeLevel& L = lv[i];
    const Surv s = surv[r];
    const int end = L.start + L.size;
    const int nwp = final_out ? nw : (end + 31) >> 5;
    uint32_t* dst = nrow + (size_t)r * nw;
    const bool first = (i == 0);
    const uint32_t* src = first ? nullptr : prow + (size_t)s.parent * nw;
    for (int q = threadIdx.x; q < nwp; q += blockDim.x) dst[q] = first ? 0u : src[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int j = first ? (s.digit >> 1) : s.digit;
        const uint32_t b = cand[(size_t)i * K + j];
        uint32_t o;
        if (first) o = (uint32_t)(s.digit & 1);
        else o = (b & 1u) ^ ((src[L.start >> 5] >> (L.start & 31)) & 1u);
        const uint32_t bits = (b ^ (o ? 0xFFFFFFFFu : 0u)) & (L.size == 32 ? 0xFFFFFFFFu : ((1u << L.size) - 1u));
        // place bits [start, end) : spans at most two words
        const int w0 = L.start >> 5, sh = L.start & 31;
        const uint64_t lm = (L.size == 32 ? 0xFFFFFFFFull : ((1ull << L.size) - 1ull)) << sh;
        const uint64_t val = (uint64_t)bits << sh;
        uint64_t cur = (uint64_t)dst[w0];
        if (w0 + 1 < nw) cur |= (uint64_t)dst[w0 + 1] << 32;
        cur = (cur & ~lm) | val;
        dst[w0] = (uint32_t)cur;
        if (w0 + 1 < nw && (sh + L.size) > 32) dst[w0 + 1] = (uint32_t)(cur >> 32);
        if (final_out) {
            // clear the bits past the last vertex
            if (nV & 31) dst[nw - 1] &= (1u << (nV & 31)) - 1u;
        }
        scores[r] = s.score;
    }
}

__global__ void k_merge_fail(uint32_t* out, int nw, int64_t* cut, const int32_t* nsurv)
{
    if (*nsurv > 0) return;
    for (int q = threadIdx.x; q < nw; q += blockDim.x) out[q] = 0u;
    if (threadIdx.x == 0) *cut = -1;
}

hipError_t launch_merge(const MergeBufs& m, int M, int K, int W, int nw, int nV, const uint32_t* cand,
                        uint32_t* best, int64_t* best_cut, hipStream_t s)
{
    hipLaunchKernelGGL(k_merge_intra, dim3(M), dim3(64), 0, s, m.lv, m.intra, cand, K, m.ccut);
    hipLaunchKernelGGL(k_merge_first, dim3(1), dim3(128), 0, s, cand, K, m.ccut, m.keys, m.counts);
    int cur = 0;
    for (int i = 0; i < M; ++i) {
        const bool last = i == M - 1;
        const int wsel = last ? 1 : W;
        const int kmul = i == 0 ? 2 * K : K;
        const int64_t nmax = i == 0 ? 2 * K : (int64_t)W * K;  // keys at this level, at most
        if (i > 0)
            hipLaunchKernelGGL(k_merge_expand, dim3(W), dim3(64), 0, s, m.lv, i, m.back, cand, K, m.ccut,
                               m.rows[cur], nw, m.scores, m.counts, m.keys);
        // counts[i] = paths at level i, counts[i + 1] = its survivors
        const int first = i == 0 ? 1 : 0;
        if (nmax <= (int64_t)SEL_THREADS * 16)
            hipLaunchKernelGGL((k_merge_select<16, true>), dim3(1), dim3(SEL_THREADS), 0, s, m.keys, m.counts + i,
                               kmul, wsel, first, m.surv, m.counts + i + 1);
        else if (nmax <= (int64_t)SEL_THREADS * 64)
            hipLaunchKernelGGL((k_merge_select<64, true>), dim3(1), dim3(SEL_THREADS), 0, s, m.keys, m.counts + i,
                               kmul, wsel, first, m.surv, m.counts + i + 1);
        else
            hipLaunchKernelGGL((k_merge_select<16, false>), dim3(1), dim3(SEL_THREADS), 0, s, m.keys, m.counts + i,
                               kmul, wsel, first, m.surv, m.counts + i + 1);
        uint32_t* dst = last ? best : m.rows[cur ^ 1];
        hipLaunchKernelGGL(k_merge_build, dim3(last ? 1 : W), dim3(64), 0, s, m.lv, i, cand, K, m.surv,
                           m.counts + i + 1, m.rows[cur], dst, nw, last ? best_cut : m.scores, last ? 1 : 0, nV);
        if (last) hipLaunchKernelGGL(k_merge_fail, dim3(1), dim3(64), 0, s, best, nw, best_cut, m.counts + M);
        cur ^= 1;
    }
    return hipGetLastError();
}

}  // namespace pq
