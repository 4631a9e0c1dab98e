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
//
// Level 1 (2K keys) runs in one workgroup (k_merge_select + k_merge_build).
// Every later level runs in three launches over all surviving parents:
//   expand  - the children's keys, and a histogram of (H - key): 65536 fine
//             bins of one key value and 4096 coarse bins of 16, H an upper
//             bound of the level's keys (previous best key + the level's
//             largest possible increment); each block aggregates its keys in
//             LDS and adds only its nonzero bins to the global histogram;
//   count   - every block finds the threshold key k* (keys above it survive,
//             plus the first R keys equal to it in path order) from the
//             coarse bins and 16 fine bins, then counts its parents'
//             survivors; if the W-th key lies below the histogram's window
//             (scores spread over more than 65536 values) each block
//             computes k* from the keys themselves instead;
//   scatter - the prefix of the per-parent counts gives each survivor its
//             position; the survivors' rows are built; the histogram is
//             cleared for the next level.
#include "common.h"

namespace pq {

__device__ inline uint32_t row_bit(const uint32_t* row, int v) { return (row[v >> 5] >> (v & 31)) & 1u; }

constexpr int FINE_BINS = 65536;
constexpr int COARSE_SHIFT = 4;
constexpr int COARSE_BINS = FINE_BINS >> COARSE_SHIFT;  // 4096
static_assert(FINE_BINS + COARSE_BINS == MERGE_HIST_INTS, "histogram layout");
constexpr int MX_THREADS = 256;  // expand / count / scatter blocks
constexpr int LOCAL_BINS = 1024;

// C_i(b_j) for every level and candidate; the number of valid candidates
// (those before the first 0xFFFFFFFF of the row); the level's largest
// possible score increment (max_j C_i(b_j) + its total back-edge weight); the
// histogram cleared for level 2. One wave per level (K <= 64).
__global__ void k_merge_intra(const MergeLevel* lv, const int32_t* intra, const uint32_t* cand, int K, int64_t* ccut,
                              int32_t* lvk, uint32_t* maxinc, int32_t* hist, int32_t* below)
{
    const int i = blockIdx.x;
    const MergeLevel& L = lv[i];
    {
        const int lane = threadIdx.x;
        const uint64_t bad = __ballot(lane < K && cand[(size_t)i * K + lane] == 0xFFFFFFFFu);
        if (lane == 0) lvk[i] = bad ? __ffsll((unsigned long long)bad) - 1 : K;
    }
    int32_t best = 0;  // total weight < 2^31
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
        best = (int32_t)c > best ? (int32_t)c : best;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int32_t y = __shfl_xor(best, o, 64);
        best = y > best ? y : best;
    }
    if (threadIdx.x == 0) {
        int64_t wb = 0;
        for (int k = 0; k < 32; ++k) wb += L.wk[k];
        maxinc[i] = (uint32_t)(best + wb);
    }
    for (int x = blockIdx.x * blockDim.x + threadIdx.x; x < MERGE_HIST_INTS; x += gridDim.x * blockDim.x) hist[x] = 0;
    if (i == 0 && threadIdx.x == 0) *below = 0;
}

// level 1: the 2 K_1 paths (j, o) in order b_1, ~b_1, b_2, ~b_2, ...
__global__ void k_merge_first(const int32_t* lvk, int K, const int64_t* ccut, uint32_t* keys, int32_t* npaths)
{
    const int Kv = lvk[0];
    for (int d = threadIdx.x; d < 2 * K; d += blockDim.x) {
        const int j = d >> 1;
        keys[d] = j < Kv ? (uint32_t)(ccut[j] + 1) : 0u;
    }
    if (threadIdx.x == 0) npaths[0] = 1;
}

// ---------------------------------------------------------------------------
// Threshold selection inside one workgroup (level 1, and the fallback of the
// count kernel)
// ---------------------------------------------------------------------------
constexpr int SEL_BINS = 4096;

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
// exclusive prefix of the per-wave values slots[0..NW) at wave wv, and their
// total (lanes 0..NW-1 read one slot each)
template <int NW>
__device__ inline void wave_slots_prefix(const int32_t* slots, int wv, int32_t& before, int32_t& total)
{
    const int lane = threadIdx.x & 63;
    const int32_t v = lane < NW ? slots[lane] : 0;
    int32_t incl = v;
#pragma unroll
    for (int o = 1; o < NW; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    before = __shfl(incl - v, wv, 64);
    total = __shfl(incl, NW - 1, 64);
}
// the value of x unknown to the optimiser (keeps it from holding values
// derived from x live across the kernel instead of recomputing them)
__device__ inline int32_t opaque(int32_t x)
{
    asm volatile("" : "+v"(x));
    return x;
}
// lanes of the wave that hold the children of this lane's parent (2^lgKp
// consecutive lanes)
__device__ inline uint64_t parent_lanes(int lane, int lgKp)
{
    if (lgKp >= 6) return ~0ull;
    return ((1ull << (1 << lgKp)) - 1ull) << ((lane >> lgKp) << lgKp);
}

template <int THREADS>
struct SelShared {
    int32_t hist[SEL_BINS];
    int32_t wa[THREADS / 64], wb[THREADS / 64];
    uint32_t s_hi, s_lo;
    int32_t s_above;
};

struct SelResult {
    int32_t nvalid;
    uint32_t best;   // largest key (0 if none)
    uint32_t kstar;  // keys > kstar survive (0: every valid key)
    int32_t R;       // and the first R keys == kstar in index order
};

// The Wsel best keys among keys[0..N) by (key desc, index asc), as a
// threshold. The keys are visited in rounds of THREADS * PER, wave w of a
// round holding keys [w * 64 PER, (w + 1) * 64 PER) of it in registers (64
// consecutive keys per register). RESIDENT: N <= THREADS * PER (the caller
// guarantees it), one round, the keys are read from memory once; otherwise
// every step re-reads them round by round. The key buffer is padded to a
// multiple of MERGE_KEY_PAD entries, so every round reads in bounds; entries
// at N and beyond are masked. (1) count, largest and smallest valid key;
// (2) threshold key k* and the number R of keys equal to k* that survive,
// from histograms of (hi - key) >> shift over [lo, hi] with 4096 bins,
// refined to the bin holding the Wsel-th key until shift = 0 (at most three
// histograms for 31-bit keys). On return sc[] holds the last round.
template <int THREADS, int PER, bool RESIDENT>
__device__ SelResult select_threshold(const uint32_t* keys, int32_t N, int Wsel, uint32_t (&sc)[PER],
                                      SelShared<THREADS>& S)
{
    constexpr int NW = THREADS / 64;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int32_t RW = THREADS * PER;
    const int rounds = RESIDENT ? 1 : (N + RW - 1) / RW;
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
    __syncthreads();  // S is free (an earlier use has been read)
    if (lane == 0) {
        S.wa[wv] = valid;
        S.wb[wv] = (int32_t)mx;
        S.hist[wv] = (int32_t)mn;
    }
    __syncthreads();
    SelResult res;
    int32_t unused;
    wave_slots_prefix<NW>(S.wa, 0, unused, res.nvalid);
    uint32_t hi = wave_max(lane < NW ? (uint32_t)S.wb[lane] : 0u);
    uint32_t lo = wave_min(lane < NW ? (uint32_t)S.hist[lane] : 0xFFFFFFFFu) + 1u;  // >= 1 if any valid
    res.best = hi;
    res.kstar = 0;
    res.R = 0;
    // (2)
    if (res.nvalid > Wsel) {
        int32_t above = 0;  // keys above the current range [lo, hi]
        for (;;) {
            int shift = 0;
            while (((hi - lo) >> shift) >= (uint32_t)SEL_BINS) ++shift;
            __syncthreads();  // the previous reads of hist / wa are done
            for (int c = tid; c < SEL_BINS; c += THREADS) S.hist[c] = 0;
            __syncthreads();
            for (int r = 0; r < rounds; ++r) {
                if (!RESIDENT) load(r);
#pragma unroll
                for (int j = 0; j < PER; ++j) {
                    const uint32_t k = sc[j];
                    if (k >= lo && k <= hi) atomicAdd(&S.hist[(hi - k) >> shift], 1);  // lo >= 1: valid keys only
                }
            }
            __syncthreads();
            // thread t owns bins t * BPT .. (t + 1) * BPT - 1; block exclusive scan of their sums
            constexpr int BPT = SEL_BINS / THREADS;
            int32_t hb[BPT], part = 0;
#pragma unroll
            for (int c = 0; c < BPT; ++c) {
                hb[c] = S.hist[BPT * tid + c];
                part += hb[c];
            }
            int32_t incl = part;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int32_t y = __shfl_up(incl, o, 64);
                if (lane >= o) incl += y;
            }
            if (lane == 63) S.wa[wv] = incl;
            __syncthreads();
            int32_t wbefore, wtotal;
            wave_slots_prefix<NW>(S.wa, wv, wbefore, wtotal);
            int32_t run = above + wbefore + incl - part;
#pragma unroll
            for (int c = 0; c < BPT; ++c) {
                if (run < Wsel && run + hb[c] >= Wsel) {  // exactly one bin of one thread
                    const uint32_t bin = (uint32_t)(BPT * tid + c);
                    S.s_above = run;
                    S.s_hi = hi - (bin << shift);
                    const uint32_t w = (bin << shift) + ((1u << shift) - 1u);  // hi - (the bin's lowest key)
                    S.s_lo = (hi - lo > w) ? hi - w : lo;
                }
                run += hb[c];
            }
            __syncthreads();
            above = S.s_above;
            hi = S.s_hi;
            lo = S.s_lo;
            if (shift == 0) {  // the bin is the single key value k*
                res.kstar = hi;
                res.R = Wsel - above;
                break;
            }
        }
    }
    return res;
}

// Level 1: keep the Wsel best of the 2K keys and write them as survivors in
// index order (one workgroup); st receives the level's threshold and best key.
constexpr int SEL_THREADS = 1024;
constexpr int SEL_PER = 16;
static_assert(SEL_THREADS * SEL_PER <= MERGE_KEY_PAD, "key buffer padding covers one round");

__global__ __launch_bounds__(SEL_THREADS) void k_merge_select(const uint32_t* keys, const int32_t* npaths, int Kmul,
                                                              int Wsel, Surv* surv, int32_t* nsurv,
                                                              MergeLvState* st)
{
    __shared__ SelShared<SEL_THREADS> S;
    constexpr int NW = SEL_THREADS / 64;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int32_t N = *npaths * Kmul;  // <= 2 QAOA_MAX_K
    uint32_t sc[SEL_PER];
    const SelResult res = select_threshold<SEL_THREADS, SEL_PER, true>(keys, N, Wsel, sc, S);
    const uint32_t kstar = res.kstar;
    const int32_t R = res.R;
    // compaction in index order by wave ballots
    int32_t gt = 0, eq = 0;
#pragma unroll
    for (int j = 0; j < SEL_PER; ++j) {
        gt += sc[j] > kstar;
        eq += sc[j] == kstar;  // kstar = 0 only if R = 0, where eq does not matter
    }
    gt = wave_sum(gt);
    eq = wave_sum(eq);
    __syncthreads();
    if (lane == 0) {
        S.wa[wv] = gt;
        S.wb[wv] = eq;
    }
    __syncthreads();
    int32_t gt_before, eq_before, tot;
    wave_slots_prefix<NW>(S.wa, wv, gt_before, tot);
    wave_slots_prefix<NW>(S.wb, wv, eq_before, tot);
    const uint64_t below = (1ull << lane) - 1ull;
    const int32_t b = opaque(wv * 64 * SEL_PER + lane);
#pragma unroll
    for (int j = 0; j < SEL_PER; ++j) {
        const uint32_t k = sc[j];
        const bool g = k > kstar, e = k == kstar;
        const uint64_t bg = __ballot(g), be = __ballot(e);
        const int32_t my_gt = gt_before + __popcll(bg & below), my_eq = eq_before + __popcll(be & below);
        if (g || (e && my_eq < R)) {
            Surv sv;
            sv.parent = 0;
            sv.digit = b + 64 * j;
            sv.score = opaque((int32_t)k) - 1;
            surv[my_gt + (my_eq < R ? my_eq : R)] = sv;
        }
        gt_before += __popcll(bg);
        eq_before += __popcll(be);
    }
    if (tid == 0) {
        const int32_t count = res.nvalid < Wsel ? res.nvalid : Wsel;
        *nsurv = count;
        st->best = res.best;
        st->kstar = kstar;
        st->R = R;
        st->count = count;
    }
}

// place the level's bits [start, start + size) into word q of a row (the
// bits span at most two words)
__device__ inline uint32_t place_bits(uint32_t word, int q, int start, int size, uint32_t bits)
{
    const int w0 = start >> 5, sh = start & 31;
    const uint64_t lm = (size == 32 ? 0xFFFFFFFFull : ((1ull << size) - 1ull)) << sh;
    const uint64_t val = (uint64_t)bits << sh;
    if (q == w0) return (word & ~(uint32_t)lm) | (uint32_t)val;
    if (q == w0 + 1) return (word & ~(uint32_t)(lm >> 32)) | (uint32_t)(val >> 32);
    return word;
}

__device__ inline uint32_t level_bits(uint32_t b, uint32_t o, int size)
{
    return (b ^ (o ? 0xFFFFFFFFu : 0u)) & (size == 32 ? 0xFFFFFFFFu : ((1u << size) - 1u));
}

// rows of level 1's survivors: the level's bits only
__global__ void k_merge_build(const MergeLevel* lv, const uint32_t* cand, const Surv* surv, const int32_t* nsurv,
                              uint32_t* nrow, int nw, int64_t* scores, int final_out, int nV)
{
    const int r = blockIdx.x;
    if (r >= *nsurv) return;
    const MergeLevel& L = lv[0];
    const Surv s = surv[r];
    const int nwp = final_out ? nw : (L.start + L.size + 31) >> 5;
    const uint32_t bits = level_bits(cand[s.digit >> 1], (uint32_t)(s.digit & 1), L.size);
    uint32_t* dst = nrow + (size_t)r * nw;
    for (int q = threadIdx.x; q < nwp; q += blockDim.x) {
        uint32_t w = place_bits(0u, q, L.start, L.size, bits);
        if (final_out && q == nw - 1 && (nV & 31)) w &= (1u << (nV & 31)) - 1u;
        dst[q] = w;
    }
    if (threadIdx.x == 0) scores[r] = s.score;
}

// ---------------------------------------------------------------------------
// Levels 2..M: expand / count / scatter
// ---------------------------------------------------------------------------
// A block covers PPB = MX_THREADS / Kp parents, Kp = K rounded up to a power
// of two; thread t is child j = t % Kp of local parent t / Kp (j >= K idle),
// so a parent's children are consecutive lanes of one wave.

constexpr int EDGE_STAGE = 2048;  // back edges staged in LDS per round
constexpr int ROW_STAGE = 4096;   // row words staged in LDS (else read from memory)

__global__ __launch_bounds__(MX_THREADS) void k_merge_expand(const MergeLevel* lv, int i, const int32_t* back,
                                                             const uint32_t* cand, int K, int lgKp,
                                                             const int64_t* ccut, const int32_t* lvk,
                                                             const uint32_t* rows, int nw, const int64_t* scores,
                                                             const int32_t* npaths, const MergeLvState* lvs,
                                                             const uint32_t* maxinc, uint32_t* keys, int32_t* hist,
                                                             int32_t* below)
{
    __shared__ int32_t A[MX_THREADS][32];
    __shared__ int32_t lh[LOCAL_BINS];
    __shared__ int32_t se_u[EDGE_STAGE], se_w[EDGE_STAGE];
    __shared__ uint32_t srow[ROW_STAGE];
    __shared__ int32_t s_kbeg[33];
    __shared__ uint32_t s_dmin;
    const int t = threadIdx.x;
    const int PPB = MX_THREADS >> lgKp;
    const int pl = t >> lgKp, j = t & ((1 << lgKp) - 1);
    const int p0 = blockIdx.x * PPB;
    const int np = npaths[i];
    if (p0 >= np) return;  // uniform
    const int nact = np - p0 < PPB ? np - p0 : PPB;
    const MergeLevel& L = lv[i];
    const int p = p0 + pl;
    const bool mine = pl < nact && j < K;
    // this child's inputs, loaded ahead of the staging
    const uint32_t b = mine ? cand[(size_t)i * K + j] : 0u;
    const int64_t base_score = mine ? scores[p] + ccut[(size_t)i * K + j] : 0;
    const bool act = mine && j < lvk[i];
    const uint32_t H = lvs[i - 1].best + maxinc[i];  // >= every key of the level
    // rows of the block's parents up to the word of the shared vertex
    const int wl = (L.start >> 5) + 1;
    const bool rows_lds = nact * wl <= ROW_STAGE;
    if (rows_lds)
        for (int q = 0; q < nact; ++q)
            for (int w = t; w < wl; w += MX_THREADS) srow[q * wl + w] = rows[(size_t)(p0 + q) * nw + w];
    for (int x = t; x < LOCAL_BINS; x += MX_THREADS) lh[x] = 0;
    for (int x = t; x < nact * 32; x += MX_THREADS) A[x >> 5][x & 31] = 0;
    if (t < 33) s_kbeg[t] = L.kbeg[t];
    if (t == 0) s_dmin = 0xFFFFFFFFu;
    auto bit_of = [&](int q, int v) -> uint32_t {
        return rows_lds ? (srow[q * wl + (v >> 5)] >> (v & 31)) & 1u : row_bit(rows + (size_t)(p0 + q) * nw, v);
    };
    // back-edge weights A_k of every parent: the thread that owns (q, k) sums
    // the edges into local vertex k (sorted by k) whose earlier endpoint is 1
    // in parent q
    const int nb = L.kbeg[32];
    for (int e0 = 0; e0 < nb || e0 == 0; e0 += EDGE_STAGE) {
        const int ne = nb - e0 < EDGE_STAGE ? nb - e0 : EDGE_STAGE;
        __syncthreads();  // the previous round's readers are done (first round: staging above is visible)
        for (int x = t; x < ne; x += MX_THREADS) {
            const int32_t* E = back + 3 * (size_t)(L.back_off + e0 + x);
            se_u[x] = E[0];
            se_w[x] = E[2];
        }
        __syncthreads();
        for (int x = t; x < nact * 32; x += MX_THREADS) {
            const int q = x >> 5, k = x & 31;
            const int lo = (s_kbeg[k] > e0 ? s_kbeg[k] : e0) - e0;
            const int hi = (s_kbeg[k + 1] < e0 + ne ? s_kbeg[k + 1] : e0 + ne) - e0;
            int32_t sum = 0;
            int e = lo;
            for (; e + 4 <= hi; e += 4) {  // four independent LDS chains in flight
                const int u0 = se_u[e], u1 = se_u[e + 1], u2 = se_u[e + 2], u3 = se_u[e + 3];
                const int32_t w0 = se_w[e], w1 = se_w[e + 1], w2 = se_w[e + 2], w3 = se_w[e + 3];
                sum += (bit_of(q, u0) ? w0 : 0) + (bit_of(q, u1) ? w1 : 0) + (bit_of(q, u2) ? w2 : 0) +
                       (bit_of(q, u3) ? w3 : 0);
            }
            for (; e < hi; ++e) sum += bit_of(q, se_u[e]) ? se_w[e] : 0;
            A[q][k] += sum;  // (q, k) has one owner
        }
        if (nb == 0) break;
    }
    __syncthreads();
    uint32_t key = 0;
    if (act) {
        const uint32_t o = (b & 1u) ^ bit_of(pl, L.start);
        int64_t s = base_score;
        const int size = L.size;
        for (int k = 1; k < size; ++k) {
            const uint32_t y = ((b >> k) & 1u) ^ o;
            s += y ? (L.wk[k] - (int64_t)A[pl][k]) : (int64_t)A[pl][k];
        }
        key = (uint32_t)(s + 1);
    }
    if (mine) keys[(size_t)p * K + j] = key;
    // histogram of d = H - key
    const uint32_t d = H - key;
    const bool inwin = key != 0u && d < (uint32_t)FINE_BINS;
    const int32_t nbelow = wave_sum(key != 0u && !inwin);
    if ((t & 63) == 0 && nbelow) atomicAdd(below, nbelow);
    const uint32_t wmin = wave_min(inwin ? d : 0xFFFFFFFFu);
    if ((t & 63) == 0 && wmin != 0xFFFFFFFFu) atomicMin(&s_dmin, wmin);
    __syncthreads();
    const uint32_t dmin = s_dmin;
    if (dmin == 0xFFFFFFFFu) return;  // no key of the block in the window (uniform)
    const uint32_t base = dmin & ~(uint32_t)((1 << COARSE_SHIFT) - 1);  // local bins align with coarse bins
    if (inwin) {
        const uint32_t lb = d - base;
        if (lb < (uint32_t)LOCAL_BINS) {
            atomicAdd(&lh[lb], 1);
        } else {  // the block's keys spread wider than the local window
            atomicAdd(&hist[d], 1);
            atomicAdd(&hist[FINE_BINS + (d >> COARSE_SHIFT)], 1);
        }
    }
    __syncthreads();
    // flush: thread t owns local bins 4t .. 4t + 3; four threads make one coarse bin
    int32_t c4 = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int32_t n = lh[4 * t + c];
        if (n) atomicAdd(&hist[base + 4 * t + c], n);
        c4 += n;
    }
    c4 += __shfl_xor(c4, 1, 64);
    c4 += __shfl_xor(c4, 2, 64);
    if ((t & 3) == 0 && c4) atomicAdd(&hist[FINE_BINS + (base >> COARSE_SHIFT) + (t >> 2)], c4);
}

// Threshold of the level from the histogram (every block identically), then
// each parent's number of children above and at the threshold (gt in the
// low, eq in the high 32 bits of pcnt[parent]).
__global__ __launch_bounds__(MX_THREADS) void k_merge_count(int i, int K, int lgKp, const int32_t* npaths_in,
                                                            int Wsel, const MergeLvState* lvs_prev,
                                                            const uint32_t* maxinc, const uint32_t* keys,
                                                            const int32_t* hist, const int32_t* below,
                                                            int64_t* pcnt, MergeLvState* st, int32_t* npaths_out)
{
    __shared__ SelShared<MX_THREADS> S;
    __shared__ int32_t s_first, s_cross;
    constexpr int NW = MX_THREADS / 64;
    constexpr int CPT = COARSE_BINS / MX_THREADS;  // 16 coarse bins per thread
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int np = *npaths_in;
    const int32_t N = np * K;
    const uint32_t H = lvs_prev->best + maxinc[i];
    const int32_t* coarse = hist + FINE_BINS;
    int32_t cb[CPT], part = 0;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        cb[c] = coarse[CPT * t + c];
        part += cb[c];
    }
    int32_t incl = part;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) S.wa[wv] = incl;
    if (t == 0) {
        s_first = COARSE_BINS;
        s_cross = -1;
    }
    __syncthreads();
    int32_t wbefore, inwin;
    wave_slots_prefix<NW>(S.wa, wv, wbefore, inwin);
    const int32_t nvalid = inwin + *below;
    const int32_t need = nvalid < Wsel ? nvalid : Wsel;  // survivors
    int32_t run = wbefore + incl - part;
    int first = -1;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        if (cb[c] && first < 0) first = CPT * t + c;
        if (run < need && run + cb[c] >= need) {  // exactly one bin of one thread, if any
            S.s_above = run;
            s_cross = CPT * t + c;
        }
        run += cb[c];
    }
    if (first >= 0) atomicMin(&s_first, first);
    __syncthreads();
    SelResult res;
    res.nvalid = nvalid;
    res.best = 0;
    res.kstar = 0;
    res.R = 0;
    if (need > 0 && s_cross >= 0) {
        // fine bins of the first nonzero coarse bin (the best key) and of the crossing one
        const int fb = s_first << COARSE_SHIFT;
        int dtop = fb;
        for (int c = 0; c < (1 << COARSE_SHIFT); ++c)
            if (hist[fb + c]) {
                dtop = fb + c;
                break;
            }
        res.best = H - (uint32_t)dtop;
        if (nvalid > Wsel) {
            const int xb = s_cross << COARSE_SHIFT;
            int32_t r2 = S.s_above;
            for (int c = 0; c < (1 << COARSE_SHIFT); ++c) {
                const int32_t n = hist[xb + c];
                if (r2 < Wsel && r2 + n >= Wsel) {
                    res.kstar = H - (uint32_t)(xb + c);
                    res.R = Wsel - r2;
                    break;
                }
                r2 += n;
            }
        }
    } else if (need > 0) {
        // the Wsel-th key (or the best one) lies below the window: select from the keys
        uint32_t sc[4];
        res = select_threshold<MX_THREADS, 4, false>(keys, N, Wsel, sc, S);
    }
    if (blockIdx.x == 0 && t == 0) {
        st->best = res.best;
        st->kstar = res.kstar;
        st->R = res.R;
        st->count = need;
        *npaths_out = need;
    }
    // per-parent counts
    const int PPB = MX_THREADS >> lgKp;
    const int pl = t >> lgKp, j = t & ((1 << lgKp) - 1);
    const int p = blockIdx.x * PPB + pl;
    if (blockIdx.x * PPB >= np) return;  // uniform
    const uint32_t key = (p < np && j < K) ? keys[(size_t)p * K + j] : 0u;
    const bool g = key > res.kstar, e = key != 0u && key == res.kstar;
    const uint64_t seg = parent_lanes(lane, lgKp);
    const int32_t ng = __popcll(__ballot(g) & seg), ne = __popcll(__ballot(e) & seg);
    if (j == 0 && p < np) pcnt[p] = (int64_t)ng | ((int64_t)ne << 32);
}

// Survivors' positions (path order) and rows; clears the histogram.
__global__ __launch_bounds__(MX_THREADS) void k_merge_scatter(const MergeLevel* lv, int i, const uint32_t* cand,
                                                              int K, int lgKp, const int32_t* npaths,
                                                              const MergeLvState* st, const uint32_t* keys,
                                                              const int64_t* pcnt, const uint32_t* prow,
                                                              uint32_t* nrow, int nw, int64_t* scores, int final_out,
                                                              int nV, int32_t* hist, int32_t* below)
{
    __shared__ int64_t s_red[MX_THREADS / 64];
    __shared__ int64_t s_pc[MX_THREADS];
    __shared__ int32_t s_n;
    __shared__ int32_t s_pos[MX_THREADS], s_src[MX_THREADS];
    __shared__ uint32_t s_bits[MX_THREADS];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    {  // the next level's histogram starts from zero (every block clears its share)
        const int per = (MERGE_HIST_INTS + (int)gridDim.x - 1) / (int)gridDim.x;
        const int lo = blockIdx.x * per, hi = lo + per < MERGE_HIST_INTS ? lo + per : MERGE_HIST_INTS;
        for (int x = lo + t; x < hi; x += MX_THREADS) hist[x] = 0;
        if (blockIdx.x == 0 && t == 0) *below = 0;
    }
    const int PPB = MX_THREADS >> lgKp;
    const int p0 = blockIdx.x * PPB;
    const int np = npaths[i];
    if (p0 >= np) return;  // uniform
    const int pl = t >> lgKp, j = t & ((1 << lgKp) - 1);
    const int p = p0 + pl;
    const MergeLevel& L = lv[i];
    // independent loads first: this child's key, candidate and the parent's
    // bit of the shared vertex, the threshold, the block's parent counts
    const bool mine = p < np && j < K;
    const uint32_t key = mine ? keys[(size_t)p * K + j] : 0u;
    const uint32_t b = mine ? cand[(size_t)i * K + j] : 0u;
    const uint32_t xs = mine ? row_bit(prow + (size_t)p * nw, L.start) : 0u;
    const uint32_t kstar = st->kstar;
    const int32_t R = st->R;
    s_pc[t] = (t < PPB && p0 + t < np) ? pcnt[p0 + t] : 0;
    if (t == 0) s_n = 0;
    // (gt, eq) counts of the parents before this block
    int64_t acc = 0;
    for (int x = t; x < p0; x += MX_THREADS) acc += pcnt[x];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) s_red[wv] = acc;
    __syncthreads();
    int64_t before = 0;
    for (int w = 0; w < MX_THREADS / 64; ++w) before += s_red[w];
    for (int q = 0; q < pl; ++q) before += s_pc[q];  // the block's earlier parents
    const bool g = key > kstar, e = key != 0u && key == kstar;
    const uint64_t earlier = ((1ull << lane) - 1ull) & parent_lanes(lane, lgKp);
    const int32_t my_gt = (int32_t)(before & 0xFFFFFFFFll) + __popcll(__ballot(g) & earlier);
    const int32_t my_eq = (int32_t)(before >> 32) + __popcll(__ballot(e) & earlier);
    if (g || (e && my_eq < R)) {
        const int32_t pos = my_gt + (my_eq < R ? my_eq : R);
        const uint32_t o = (b & 1u) ^ xs;
        const int slot = atomicAdd(&s_n, 1);
        s_pos[slot] = pos;
        s_src[slot] = p;
        s_bits[slot] = level_bits(b, o, L.size);
        scores[final_out ? 0 : pos] = (int64_t)key - 1;  // final: the best cut
    }
    __syncthreads();
    // rows: wave w builds survivors w, w + 4, ...; lanes over the words
    const int nwp = final_out ? nw : (L.start + L.size + 31) >> 5;
    const int n = s_n;
    for (int s = wv; s < n; s += MX_THREADS / 64) {
        const uint32_t* src = prow + (size_t)s_src[s] * nw;
        uint32_t* dst = nrow + (size_t)(final_out ? 0 : s_pos[s]) * nw;
        const uint32_t bits = s_bits[s];
        for (int q = lane; q < nwp; q += 64) {
            uint32_t w = place_bits(src[q], q, L.start, L.size, bits);
            if (final_out && q == nw - 1 && (nV & 31)) w &= (1u << (nV & 31)) - 1u;
            dst[q] = w;
        }
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
    hipLaunchKernelGGL(k_merge_intra, dim3(M), dim3(64), 0, s, m.lv, m.intra, cand, K, m.ccut, m.lvk, m.maxinc,
                       m.hist, m.below);
    hipLaunchKernelGGL(k_merge_first, dim3(1), dim3(128), 0, s, m.lvk, K, m.ccut, m.keys, m.counts);
    // level 1: counts[0] = 1 path, counts[1] = its survivors
    const bool last0 = M == 1;
    hipLaunchKernelGGL(k_merge_select, dim3(1), dim3(SEL_THREADS), 0, s, m.keys, m.counts, 2 * K, last0 ? 1 : W,
                       m.surv, m.counts + 1, m.lvs);
    hipLaunchKernelGGL(k_merge_build, dim3(last0 ? 1 : W), dim3(64), 0, s, m.lv, cand, m.surv, m.counts + 1,
                       last0 ? best : m.rows[0], nw, last0 ? best_cut : m.scores, last0 ? 1 : 0, nV);
    int lgKp = 0;
    while ((1 << lgKp) < K) ++lgKp;
    const int PPB = MX_THREADS >> lgKp;
    const int nblk = (W + PPB - 1) / PPB;
    int cur = 0;
    for (int i = 1; i < M; ++i) {
        const bool last = i == M - 1;
        hipLaunchKernelGGL(k_merge_expand, dim3(nblk), dim3(MX_THREADS), 0, s, m.lv, i, m.back, cand, K, lgKp,
                           m.ccut, m.lvk, m.rows[cur], nw, m.scores, m.counts, m.lvs, m.maxinc, m.keys, m.hist,
                           m.below);
        hipLaunchKernelGGL(k_merge_count, dim3(nblk), dim3(MX_THREADS), 0, s, i, K, lgKp, m.counts + i,
                           last ? 1 : W, m.lvs + (i - 1), m.maxinc, m.keys, m.hist, m.below, m.pcnt, m.lvs + i,
                           m.counts + i + 1);
        hipLaunchKernelGGL(k_merge_scatter, dim3(nblk), dim3(MX_THREADS), 0, s, m.lv, i, cand, K, lgKp, m.counts,
                           m.lvs + i, m.keys, m.pcnt, m.rows[cur], last ? best : m.rows[cur ^ 1], nw,
                           last ? best_cut : m.scores, last ? 1 : 0, nV, m.hist, m.below);
        cur ^= 1;
    }
    hipLaunchKernelGGL(k_merge_fail, dim3(1), dim3(64), 0, s, best, nw, best_cut, m.counts + M);
    return hipGetLastError();
}

}  // namespace pq
