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
// Keys: (score + 1) << 32 | (0xFFFFFFFF - order), order = parent_rank * K + j
// (level 1: 2j + o); zero marks an invalid candidate. Survivors are kept in
// path order, so a survivor's rank is its position.
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
__global__ void k_merge_first(const uint32_t* cand, int K, const int64_t* ccut, uint64_t* keys)
{
    const int Kv = level_k(cand, K, 0);
    for (int d = threadIdx.x; d < 2 * K; d += blockDim.x) {
        const int j = d >> 1;
        uint64_t key = 0;
        if (j < Kv) key = ((uint64_t)(ccut[j] + 1) << 32) | (uint64_t)(0xFFFFFFFFu - (uint32_t)d);
        keys[d] = key;
    }
}

__device__ inline uint32_t row_bit(const uint32_t* row, int v) { return (row[v >> 5] >> (v & 31)) & 1u; }

// level i >= 1: one block per parent path, one thread per candidate j
__global__ void k_merge_expand(const MergeLevel* lv, int i, const int32_t* back, const uint32_t* cand, int K,
                               const int64_t* ccut, const uint32_t* rows, int nw, const int64_t* scores,
                               const int32_t* npaths, uint64_t* keys)
{
    __shared__ int32_t A[32];
    const int p = blockIdx.x;
    if (p >= *npaths) return;
    const MergeLevel L = lv[i];
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
    for (int j = threadIdx.x; j < K; j += blockDim.x) {
        uint64_t key = 0;
        if (j < Kv) {
            const uint32_t b = cand[(size_t)i * K + j];
            const uint32_t o = (b & 1u) ^ xs;
            int64_t s = ps + ccut[(size_t)i * K + j];
            for (int k = 1; k < L.size; ++k) {
                const uint32_t y = ((b >> k) & 1u) ^ o;
                s += y ? (L.wk[k] - (int64_t)A[k]) : (int64_t)A[k];
            }
            const uint32_t order = (uint32_t)p * (uint32_t)K + (uint32_t)j;
            key = ((uint64_t)(s + 1) << 32) | (uint64_t)(0xFFFFFFFFu - order);
        }
        keys[(size_t)p * K + j] = key;
    }
}

constexpr int SEL_THREADS = 1024;
constexpr int SEL_BATCH = 8;
constexpr int SEL_BINS = 4096;

__device__ inline int64_t key_score(uint64_t k) { return (int64_t)(k >> 32) - 1; }

// block-wide exclusive scan of one int per thread (fixed order)
__device__ inline int32_t block_exscan(int32_t x, int32_t* buf, int32_t* total)
{
    const int tid = threadIdx.x;
    buf[tid] = x;
    __syncthreads();
    for (int off = 1; off < SEL_THREADS; off <<= 1) {
        const int32_t y = tid >= off ? buf[tid - off] : 0;
        __syncthreads();
        buf[tid] += y;
        __syncthreads();
    }
    const int32_t incl = buf[tid];
    *total = buf[SEL_THREADS - 1];
    __syncthreads();
    return incl - x;
}

// Keep the Wsel best keys among keys[0..N) (N = paths * Kmul, key index =
// path order) by (score desc, index asc) and write them as survivors in
// index order. One workgroup: (1) best score and number of valid keys;
// (2) histogram of (hi - score) over a window of 4096 scores to find the
// threshold score s* at which the count reaches Wsel (the window slides down
// if needed); (3) compaction in index order keeping every key above s* and
// the first R keys equal to s*.
__global__ __launch_bounds__(SEL_THREADS) void k_merge_select(const uint64_t* keys, const int32_t* Nptr, int Kmul,
                                                              int Wsel, int first, Surv* surv, int32_t* nsurv)
{
    __shared__ int32_t hist[SEL_BINS];
    __shared__ int32_t buf[SEL_THREADS];
    __shared__ int64_t s_best;
    __shared__ int32_t s_valid, s_found;
    __shared__ int64_t s_star;
    __shared__ int32_t s_R;
    const int tid = threadIdx.x;
    const int64_t N = (int64_t)(*Nptr) * Kmul;
    if (tid == 0) {
        s_best = 0;
        s_valid = 0;
    }
    __syncthreads();
    int64_t best = INT64_MIN;
    int32_t valid = 0;
    // loads in batches of SEL_BATCH independent keys per thread (latency, not
    // bandwidth, bounds a single workgroup)
    for (int64_t q0 = tid; q0 < N; q0 += (int64_t)SEL_THREADS * SEL_BATCH) {
        uint64_t kb[SEL_BATCH];
#pragma unroll
        for (int j = 0; j < SEL_BATCH; ++j) {
            const int64_t q = q0 + (int64_t)j * SEL_THREADS;
            kb[j] = q < N ? keys[q] : 0ull;
        }
#pragma unroll
        for (int j = 0; j < SEL_BATCH; ++j) {
            if (kb[j]) {
                ++valid;
                const int64_t sc = key_score(kb[j]);
                best = sc > best ? sc : best;
            }
        }
    }
    atomicAdd(&s_valid, valid);
    if (valid) atomicMax((unsigned long long*)&s_best, (unsigned long long)best);  // scores are >= 0
    __syncthreads();
    const int32_t nvalid = s_valid;
    const int64_t hi0 = s_best;
    const int count = nvalid < Wsel ? nvalid : Wsel;
    if (nvalid <= Wsel) {
        if (tid == 0) {
            s_star = INT64_MIN;  // every valid key is above the threshold
            s_R = 0;
        }
    } else {
        int64_t hi = hi0;
        int32_t above = 0;  // keys with score > hi
        for (;;) {
            for (int b = tid; b < SEL_BINS; b += SEL_THREADS) hist[b] = 0;
            if (tid == 0) s_found = 0;
            __syncthreads();
            for (int64_t q0 = tid; q0 < N; q0 += (int64_t)SEL_THREADS * SEL_BATCH) {
                uint64_t kb[SEL_BATCH];
#pragma unroll
                for (int j = 0; j < SEL_BATCH; ++j) {
                    const int64_t q = q0 + (int64_t)j * SEL_THREADS;
                    kb[j] = q < N ? keys[q] : 0ull;
                }
#pragma unroll
                for (int j = 0; j < SEL_BATCH; ++j) {
                    if (!kb[j]) continue;
                    const int64_t d = hi - key_score(kb[j]);
                    if (d >= 0 && d < SEL_BINS) atomicAdd(&hist[d], 1);
                }
            }
            __syncthreads();
            // each thread owns 4 consecutive bins
            int32_t h4[4], part = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                h4[i] = hist[4 * tid + i];
                part += h4[i];
            }
            int32_t win_total;
            const int32_t before = above + block_exscan(part, buf, &win_total);
            int32_t run = before;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (run < Wsel && run + h4[i] >= Wsel) {
                    s_star = hi - (4 * tid + i);
                    s_R = Wsel - run;
                    s_found = 1;
                }
                run += h4[i];
            }
            __syncthreads();
            if (s_found) break;
            above += win_total;
            hi -= SEL_BINS;
            __syncthreads();
        }
    }
    __syncthreads();
    const int64_t star = s_star;
    const int32_t R = s_R;
    // compaction in index order: wave w owns keys [w*S, (w+1)*S), read 64
    // consecutive keys at a time; ballots give each lane its rank among the
    // wave's keys above / at the threshold, one barrier gives the wave bases
    __shared__ int32_t wgt[SEL_THREADS / 64], weq[SEL_THREADS / 64];
    const int lane = tid & 63, wv = tid >> 6;
    constexpr int NWV = SEL_THREADS / 64;
    const int64_t S = (N + NWV - 1) / NWV;
    const int64_t lo = (int64_t)wv * S, up = lo + S < N ? lo + S : N;
    const uint64_t below = (1ull << lane) - 1ull;
    int32_t gt = 0, eq = 0;
    for (int64_t b0 = lo; b0 < up; b0 += 64 * SEL_BATCH) {
        uint64_t kb[SEL_BATCH];
#pragma unroll
        for (int j = 0; j < SEL_BATCH; ++j) {
            const int64_t q = b0 + 64 * j + lane;
            kb[j] = q < up ? keys[q] : 0ull;
        }
#pragma unroll
        for (int j = 0; j < SEL_BATCH; ++j) {
            const uint64_t k = kb[j];
            const int64_t sc = k ? key_score(k) : 0;
            gt += __popcll(__ballot(k && sc > star));
            eq += __popcll(__ballot(k && sc == star));
        }
    }
    if (lane == 0) {
        wgt[wv] = gt;
        weq[wv] = eq;
    }
    __syncthreads();
    int32_t gt_before = 0, eq_before = 0;
    for (int w = 0; w < wv; ++w) {
        gt_before += wgt[w];
        eq_before += weq[w];
    }
    for (int64_t b0 = lo; b0 < up; b0 += 64 * SEL_BATCH) {
        uint64_t kb[SEL_BATCH];
#pragma unroll
        for (int j = 0; j < SEL_BATCH; ++j) {
            const int64_t q = b0 + 64 * j + lane;
            kb[j] = q < up ? keys[q] : 0ull;
        }
#pragma unroll
        for (int j = 0; j < SEL_BATCH; ++j) {
            const int64_t q = b0 + 64 * j + lane;
            const uint64_t k = kb[j];
            const int64_t sc = k ? key_score(k) : 0;
            const bool g = k && sc > star, e = k && sc == star;
            const uint64_t bg = __ballot(g), be = __ballot(e);
            const int32_t my_gt = gt_before + __popcll(bg & below), my_eq = eq_before + __popcll(be & below);
            if (g || (e && my_eq < R)) {
                const int pos = my_gt + (my_eq < R ? my_eq : R);
                Surv sv;
                sv.parent = first ? 0 : (int32_t)(q / Kmul);
                sv.digit = first ? (int32_t)q : (int32_t)(q % Kmul);
                sv.score = sc;
                surv[pos] = sv;
            }
            gt_before += __popcll(bg);
            eq_before += __popcll(be);
        }
    }
    if (tid == 0) *nsurv = count;
}

// rows of the surviving paths: parent row prefix plus the bits of V_i
__global__ void k_merge_build(const MergeLevel* lv, int i, const uint32_t* cand, int K, const Surv* surv,
                              const int32_t* nsurv, const uint32_t* prow, uint32_t* nrow, int nw, int64_t* scores,
                              int final_out, int nV)
{
    const int r = blockIdx.x;
    if (r >= *nsurv) return;
    const MergeLevel L = lv[i];
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

__global__ void k_set_count(int32_t* c, int v)
{
    if (threadIdx.x == 0) *c = v;
}

__global__ void k_copy_count(int32_t* c)
{
    if (threadIdx.x == 0) c[0] = c[1];
}

hipError_t launch_merge(const MergeBufs& m, int M, int K, int W, int nw, int nV, const uint32_t* cand,
                        uint32_t* best, int64_t* best_cut, hipStream_t s)
{
    hipLaunchKernelGGL(k_merge_intra, dim3(M), dim3(64), 0, s, m.lv, m.intra, cand, K, m.ccut);
    hipLaunchKernelGGL(k_merge_first, dim3(1), dim3(128), 0, s, cand, K, m.ccut, m.keys);
    hipLaunchKernelGGL(k_set_count, dim3(1), dim3(64), 0, s, m.counts, 1);
    int cur = 0;
    for (int i = 0; i < M; ++i) {
        const bool last = i == M - 1;
        const int wsel = last ? 1 : W;
        if (i > 0)
            hipLaunchKernelGGL(k_merge_expand, dim3(W), dim3(64), 0, s, m.lv, i, m.back, cand, K, m.ccut,
                               m.rows[cur], nw, m.scores, m.counts, m.keys);
        hipLaunchKernelGGL(k_merge_select, dim3(1), dim3(SEL_THREADS), 0, s, m.keys, m.counts,
                           i == 0 ? 2 * K : K, wsel, i == 0 ? 1 : 0, m.surv, m.counts + 1);
        uint32_t* dst = last ? best : m.rows[cur ^ 1];
        hipLaunchKernelGGL(k_merge_build, dim3(last ? 1 : W), dim3(64), 0, s, m.lv, i, cand, K, m.surv,
                           m.counts + 1, m.rows[cur], dst, nw, last ? best_cut : m.scores, last ? 1 : 0, nV);
        if (last) {
            hipLaunchKernelGGL(k_merge_fail, dim3(1), dim3(64), 0, s, best, nw, best_cut, m.counts + 1);
        } else {
            // survivors become the current paths
            hipLaunchKernelGGL(k_copy_count, dim3(1), dim3(64), 0, s, m.counts);
        }
        cur ^= 1;
    }
    return hipGetLastError();
}

}  // namespace pq
