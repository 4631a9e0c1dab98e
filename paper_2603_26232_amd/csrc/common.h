// Internal declarations shared by the HIP translation units of libparaqaoa.
// Nothing here is part of the public C ABI (include/paraqaoa.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/paraqaoa.h"

namespace pq {

// One tile = 2^12 amplitudes of one subgraph's state; a workgroup of 256
// threads holds it in registers (16 amplitudes per thread) and exchanges
// register layouts through LDS.
constexpr int TILE_BITS = 12;
constexpr int TILE = 1 << TILE_BITS;
constexpr int THREADS = 256;
constexpr int REGS = TILE / THREADS;  // 16
constexpr int LDS_TILE = TILE + TILE / 16;  // one pad slot per 16 amplitudes
constexpr int MAX_GROUPS = 4;  // qubit groups per subgraph (n <= 30)
constexpr int MAX_P = 32;      // QAOA depth limit
constexpr int MAX_K = 64;      // top-k limit
constexpr int LUT_MAX = 2048;  // phase table entries per layer (sum of weights + 1)
// Stored states are symmetry-reduced: the ansatz state is invariant under
// flipping every bit (psi(~z) = psi(z)), so only the 2^(n-1) amplitudes with
// the top bit clear are stored, scaled by sqrt(2) to unit norm.
constexpr int HALF_BITS = TILE_BITS - 1;  // qubits 0..10 in group 0; tile bit 11 = the complement
constexpr int SMALL_MAX_N = 13;  // n <= 13: the reduced state (<= 4096 amplitudes) is one workgroup's tile
// the tile passes address a stored state with 32-bit byte offsets
static_assert((8ull << (QAOA_MAX_QUBITS - 1)) <= (1ull << 32), "a stored state must fit 32-bit byte offsets");
constexpr int B_GROUP_MAX = 8;   // active qubits of a strided (high) group

// Per-subgraph descriptor, resident in the workspace.
struct SubDesc {
    int32_t n;        // qubits
    int32_t ngroups;  // 1 for n <= 13 (whole-state kernel), else 1 + ceil((n-12)/8)
    int32_t gstart[MAX_GROUPS];  // first qubit of group g (group 0 starts at 0)
    int32_t gsize[MAX_GROUPS];   // qubits in group g (group 0: n when n <= 13, else 12)
    int32_t lut_len;  // sum of weights + 1 (phase table length per layer)
    int32_t ntiles;   // max(1, 2^(n-12))
    int32_t tile_base;  // first global tile index
    int32_t nedges;
    int32_t skip;  // edgeless and not simulated (closed form)
    int32_t tabw;  // bytes per cut-table entry: 1 (weight sum <= 255) or 2
    uint32_t freem;  // vertices without an edge of positive weight (bit j = local vertex j)
    int32_t pad_;
    uint64_t psi, lam, tab, tabB, lut, coef, edges;  // byte offsets into the workspace
};

// Which part of the circuit one tile pass applies (layers are 0-based,
// -1 = absent). Forward: RX(pre), phase(ph), RX(post). Backward: unmix(pre)
// with the beta-gradient, gamma-gradient + unphase(ph), unmix(post).
struct PassOps {
    int32_t group;
    int32_t pre, ph, post;
    int32_t init;      // forward: synthesise |+> instead of loading
    int32_t epi_e;     // forward: write the <C> partial of each tile
    int32_t fused;     // backward: forward RX(pre) + <C> + lambda = C psi first
    int32_t last;      // backward: the inverse of the first forward pass; nothing stored
    int32_t nopsi;     // backward: psi is not needed after this pass (not stored)
    // psi slots: a forward pass reads slot psi_in and writes slot psi_out; a
    // backward pass reads psi from slot psi_in (with gradient checkpoints
    // every forward pass writes its own slot, which the backward pass that
    // undoes it reads; otherwise everything stays in slot 0)
    int32_t psi_in, psi_out;
};

// Bytes of one stored (symmetry-reduced) state of an n-qubit subgraph: one
// psi slot.
__host__ __device__ inline uint64_t state_bytes(int n) { return 8ull << (n - 1); }

// Rotation parameters of one layer of one subgraph: e^{-i beta X} =
// f (I - i t X) X^flip with (f, t) = (c, tan beta) (mode 0, |cos| >= |sin|,
// no flip) or (-i s, -cot beta) (mode 1, flip). Ff[g] / Fi[g] are the
// per-qubit factors raised to the size of group g, forward (c or -i s) and
// inverse (c or +i s).
struct RxCoef {
    float2 cs;  // (cos beta, sin beta)
    float t;
    int32_t mode;
    float fsq;  // |per-qubit factor|^2
    float pad;
    float2 Ff[MAX_GROUPS];
    float2 Fi[MAX_GROUPS];
};

struct Partials {
    double* e;   // [total_tiles]
    double* gb;  // [(l*MAX_GROUPS + g) * total_tiles + tile]
    double* gg;  // [l * total_tiles + tile]
    int32_t total_tiles;
};

// ---- merge (merge.hip) ----
struct MergeLevel {
    int32_t start, size;
    int32_t intra_off, intra_cnt;  // intra edges (local a, local b, w)
    int32_t back_off;              // back edges (global u, local k, w), sorted by k
    int32_t pad;
    int32_t kbeg[33];              // back edges into local k: [back_off + kbeg[k], back_off + kbeg[k+1])
    int32_t pad2[3];
    int64_t wk[32];                // total back weight into local k
};

struct Surv {
    int32_t parent;  // rank of the parent path (level 1: 0)
    int32_t digit;   // j (level 1: 2j + o)
    int64_t score;
};

// per level: the selection's outcome
struct MergeLvState {
    uint32_t best;   // largest key (score + 1) of the level
    uint32_t kstar;  // keys above kstar survive ...
    int32_t R;       // ... and the first R keys equal to it
    int32_t count;   // survivors
};

constexpr int MERGE_HIST_INTS = 65536 + 4096;  // fine + coarse bins

struct MergeBufs {
    const MergeLevel* lv;
    const int32_t* intra;
    const int32_t* back;
    int64_t* ccut;
    uint32_t* keys;   // score + 1 per candidate (0 = none), index = path order
    Surv* surv;       // level 1's survivors
    int32_t* counts;  // [i] = paths at level i (M + 1 entries)
    uint32_t* rows[2];
    int64_t* scores;
    MergeLvState* lvs;  // [M]
    uint32_t* maxinc;   // [M] largest possible score increment of level i
    int32_t* lvk;       // [M] valid candidates of level i
    int32_t* hist;      // [MERGE_HIST_INTS]
    int32_t* below;     // keys below the histogram's window
    int64_t* pcnt;      // [W] per parent: survivors above (low) / at (high) the threshold
};

hipError_t launch_merge(const MergeBufs& m, int M, int K, int W, int nw, int nV, const uint32_t* cand,
                        uint32_t* best, int64_t* best_cut, hipStream_t s);
constexpr int MERGE_MAX_SIZE = 32;  // vertices per level (one uint32 bitstring)
constexpr int MERGE_KEY_PAD = 65536;  // the key buffer holds a multiple of this many entries

// ---- angle predictor (mlp.hip) ----
constexpr int MLP_MAX_IN = 64, MLP_MAX_H = 256, MLP_MAX_OUT = 64;
struct MlpDims {
    int in, H, out;
};
int64_t mlp_num_params(const MlpDims& d);
// scratch for the backward pass: floats [B * (2H + out)] then doubles [B]
inline size_t mlp_scratch_bytes(int B, const MlpDims& d)
{
    return sizeof(float) * ((size_t)B * (2 * d.H + d.out) + 2) + sizeof(double) * (size_t)B + 8;
}
hipError_t launch_mlp_forward(int B, MlpDims d, const double* P, const float* X, float* Y, float* act, hipStream_t s);
// the backward pass's device scratch for callers that cannot allocate (bytes)
constexpr size_t MLP_STATIC_SCRATCH_BYTES = 8u << 20;
// device address of that scratch on the current device (looked up once per device)
hipError_t mlp_static_scratch(void** out);
hipError_t launch_warm_angles(int B, int p, const float* Y, const float* mu, const float* sd, double* theta,
                              hipStream_t s);
hipError_t launch_keep_better(int B, int p, const double* E_alt, const double* theta_alt, double* E, double* theta,
                              hipStream_t s);
hipError_t launch_mlp_backward(int B, MlpDims d, const double* P, const float* X, const float* Y, const float* act,
                               const float* T, float* scratch, double* G, double* loss, hipStream_t s);

// ---- launchers (sim.hip) ----
hipError_t launch_cut_tables(uint8_t* ws, const SubDesc* subs, const int2* work, int nwork,
                             hipStream_t s);
// chain: layout-chain code of the pass's group (3: group 0; 2 / 4: a high
// group of 8 / 5..7 qubits; 1 / 5: a high group of 4 / 1..3 qubits)
hipError_t launch_fwd_pass(uint8_t* ws, const SubDesc* subs, const int2* work, int nwork, int chain,
                           PassOps ops, Partials part, int lut_max, int prec, hipStream_t s);
hipError_t launch_bwd_pass(uint8_t* ws, const SubDesc* subs, const int2* work, int nwork, int chain,
                           PassOps ops, Partials part, int lut_max, hipStream_t s);
hipError_t launch_small(uint8_t* ws, const SubDesc* subs, const int32_t* list, int nlist, int p,
                        int grad, Partials part, int lut_max, hipStream_t s);
// ---- launchers (optim.hip) ----
hipError_t launch_angle_prep(uint8_t* ws, const SubDesc* subs, int B, int p, const double* gamma,
                             const double* beta, hipStream_t s);
hipError_t launch_reduce(const SubDesc* subs, int B, int p, int grad, Partials part, double* E,
                         double* dgamma, double* dbeta, hipStream_t s);
// ---- launchers (topk.hip) ----
hipError_t launch_topk(uint8_t* ws, const SubDesc* subs, const int2* work, int nwork, int B, int k,
                       int canonical, uint64_t* keys, uint32_t* idx, float* prob, hipStream_t s);
// ---- launchers (cut.hip) ----
hipError_t launch_maxcut_eval(int32_t nV, int64_t nE, const int32_t* u, const int32_t* v,
                              const int32_t* w, int64_t A, const uint32_t* assign, int64_t* cut,
                              hipStream_t s);
// deterministic block sum of one double per thread: wave tree, then the
// waves in order (thread 0 holds the result; blockDim a multiple of 64)
__device__ inline double block_sum(double x, double* red)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    const uint32_t tid = threadIdx.x;
    if ((tid & 63u) == 0) red[tid >> 6] = x;
    __syncthreads();
    double s = 0.0;
    if (tid == 0) {
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    }
    __syncthreads();
    return s;
}

// Adam (Kingma and Ba 2015) update of one parameter in FP64 with the bias
// corrections c1 = 1 - b1^t, c2 = 1 - b2^t; sign +1 ascends. The standalone
// step and the fused optimiser kernel share it; floating-point contraction is
// off in its body, so every product and sum is rounded on its own (no FMAs,
// which the compiler could choose differently in the two kernels) and both
// give the same bits.
__device__ __noinline__ inline void adam_update(double& th, double& m, double& v, double g, double c1, double c2, double lr,
                                   double b1, double b2, double eps, double sign)
{
#pragma clang fp contract(off)
    const double mi = __dadd_rn(__dmul_rn(b1, m), __dmul_rn(__dsub_rn(1.0, b1), g));
    const double vi = __dadd_rn(__dmul_rn(b2, v), __dmul_rn(__dmul_rn(__dsub_rn(1.0, b2), g), g));
    m = mi;
    v = vi;
    const double step = __ddiv_rn(__dmul_rn(__dmul_rn(sign, lr), __ddiv_rn(mi, c1)),
                                  __dadd_rn(__dsqrt_rn(__ddiv_rn(vi, c2)), eps));
    th = __dadd_rn(th, step);
}
// reduction of the gradient, Adam ascent step and the next step's tables,
// one block per (subgraph, layer) (optim.hip)
hipError_t launch_reduce_adam(uint8_t* ws, const SubDesc* subs, int B, int p, Partials part, double* theta,
                              double* m, double* v, const int32_t* step, int32_t it, double lr, double b1,
                              double b2, double eps, double* E, hipStream_t s);
hipError_t launch_step_advance(int32_t* step, int32_t n, hipStream_t s);
hipError_t launch_adam(int32_t count, double* theta, const double* grad, double* m, double* v,
                       int32_t* step, double lr, double b1, double b2, double eps, double sign,
                       hipStream_t s);

}  // namespace pq
