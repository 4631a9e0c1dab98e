// C ABI of libparaqaoa (declared in include/paraqaoa.h): argument checks,
// workspace layout, host-side pass programs and kernel launches.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/paraqaoa.h"
#include "common.h"

using namespace pq;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local char g_err[512] = "";

static qaoa_status_t fail(qaoa_status_t s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static qaoa_status_t fail(qaoa_status_t s, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

static qaoa_status_t ok()
{
    g_err[0] = 0;
    return QAOA_OK;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(QAOA_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// host-to-device uploads of metadata images: a ring of pinned staging
// buffers, each grown as needed and reused once the copy from it has
// completed (an event recorded after the copy). An upload enqueues without
// waiting for the stream's earlier work; it waits only if the slot's
// previous upload (STAGE_SLOTS uploads ago) has not left it yet.
// ---------------------------------------------------------------------------
namespace {
constexpr int STAGE_SLOTS = 4;
struct StageSlot {
    void* buf = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    int dev = -1;
    bool pending = false;
};
struct Staging {
    std::mutex mu;
    StageSlot slot[STAGE_SLOTS];
    int next = 0;
};
Staging g_stage;
}  // namespace

static qaoa_status_t upload_async(void* d_dst, const void* src, size_t bytes, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(g_stage.mu);
    StageSlot& S = g_stage.slot[g_stage.next];
    g_stage.next = (g_stage.next + 1) % STAGE_SLOTS;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (S.pending) {
        HIP_TRY(hipEventSynchronize(S.ev));  // the slot's buffer is free again
        S.pending = false;
    }
    if (S.ev && S.dev != dev) {
        HIP_TRY(hipEventDestroy(S.ev));
        S.ev = nullptr;
    }
    if (!S.ev) {
        HIP_TRY(hipEventCreateWithFlags(&S.ev, hipEventDisableTiming));
        S.dev = dev;
    }
    if (bytes > S.cap) {
        if (S.buf) HIP_TRY(hipHostFree(S.buf));
        S.buf = nullptr;
        S.cap = 0;
        HIP_TRY(hipHostMalloc(&S.buf, bytes, hipHostMallocPortable));
        S.cap = bytes;
    }
    memcpy(S.buf, src, bytes);
    HIP_TRY(hipMemcpyAsync(d_dst, S.buf, bytes, hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(S.ev, st));
    S.pending = true;
    return QAOA_OK;
}

// ---------------------------------------------------------------------------
// kernel timing (measurement hook)
// ---------------------------------------------------------------------------
namespace {
struct ProfRec {
    hipEvent_t a, b;
};
struct Profiler {
    bool on = false;
    std::string only;  // empty: every kernel; else only this name is timed
    std::map<std::string, std::vector<ProfRec>> recs;
    std::map<std::string, double> bytes;  // algorithmic bytes of the recorded launches
    std::vector<ProfRec> pool;
};
Profiler g_prof;

struct ProfScope {
    const char* name;
    hipStream_t s;
    ProfRec r{};
    bool active;
    ProfScope(const char* n, hipStream_t st, double algo_bytes = 0.0)
        : name(n), s(st), active(g_prof.on && (g_prof.only.empty() || g_prof.only == n))
    {
        if (!active) return;
        g_prof.bytes[name] += algo_bytes;
        if (!g_prof.pool.empty()) {
            r = g_prof.pool.back();
            g_prof.pool.pop_back();
        } else {
            // timing only: no system-scope fence (no cache writeback between kernels)
            (void)hipEventCreateWithFlags(&r.a, hipEventDisableSystemFence);
            (void)hipEventCreateWithFlags(&r.b, hipEventDisableSystemFence);
        }
        (void)hipEventRecord(r.a, s);
    }
    ~ProfScope()
    {
        if (!active) return;
        (void)hipEventRecord(r.b, s);
        g_prof.recs[name].push_back(r);
    }
};
}  // namespace

extern "C" qaoa_status_t qaoa_profile_enable(int32_t on)
{
    for (auto& kv : g_prof.recs)
        for (auto& r : kv.second) {
            (void)hipEventSynchronize(r.b);
            g_prof.pool.push_back(r);
        }
    g_prof.recs.clear();
    g_prof.bytes.clear();
    g_prof.on = on != 0;
    return ok();
}

extern "C" qaoa_status_t qaoa_profile_select(const char* kernel)
{
    g_prof.only = kernel ? kernel : "";
    return ok();
}

extern "C" qaoa_status_t qaoa_profile_read(const char* kernel, int64_t* launches, double* total_ms,
                                           double* algo_bytes)
{
    if (!kernel || !launches || !total_ms || !algo_bytes) return fail(QAOA_ERR_INVALID_ARG, "NULL argument");
    *launches = 0;
    *total_ms = 0.0;
    *algo_bytes = g_prof.bytes.count(kernel) ? g_prof.bytes[kernel] : 0.0;
    auto it = g_prof.recs.find(kernel);
    if (it == g_prof.recs.end()) return ok();
    for (auto& r : it->second) {
        HIP_TRY(hipEventSynchronize(r.b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        *total_ms += ms;
        *launches += 1;
    }
    return ok();
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
namespace {

struct Plan {
    int32_t B = 0, max_p = 0, max_k = 0;
    uint32_t flags = 0;
    int prec = 0;  // mixer block: 0 vector units, 1 FP32 MFMA, 2 / 3 BF16 split MFMA
    bool ckpt = false;  // gradient checkpoints: one psi slot per forward pass
    std::vector<SubDesc> subs;
    int32_t total_tiles = 0;
    int64_t total_edges = 0;
    int lut_max = 1;
    // region offsets
    uint64_t o_subs = 0, o_work_all = 0, o_small = 0, o_edges = 0, o_coef = 0, o_lut = 0, o_pe = 0,
             o_pgb = 0,
             o_pgg = 0, o_keys = 0, total = 0;
    int nsmall = 0;
    // host images of the metadata regions
    std::vector<int2> work_all;
    std::vector<int32_t> small;
    // subgraphs with the same group count and group shapes share one pass
    // program and one launch per pass
    struct Class {
        int G;
        int chain[MAX_GROUPS];
        std::vector<int2> work;
        uint64_t o_work;
        double tab_bytes;  // cut-table bytes of one pass over the class's tiles
    };
    std::vector<Class> classes;
};

// MI355X's Infinity Cache (the memory-side last-level cache) and the share
// of it a batch's live states may take to count as cache-resident
constexpr uint64_t CACHE_BYTES = 256ull << 20;
constexpr uint64_t CACHE_FIT_BYTES = 224ull << 20;

// layout-chain code of group g (see launch_fwd_pass): 3 for group 0; for a
// high group 2 (8 qubits), 4 (5..7), 1 (4), 5 (1..3)
int chain_of(const SubDesc& d, int g)
{
    if (g == 0) return 3;
    const int nb = d.gsize[g];
    return nb == 8 ? 2 : (nb >= 5 ? 4 : (nb == 4 ? 1 : 5));
}

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

int groups_for(int n)
{
    if (n <= SMALL_MAX_N) return 1;
    const int rest = n - TILE_BITS;
    return 1 + (rest + B_GROUP_MAX - 1) / B_GROUP_MAX;
}

// Tuned sizes of the strided qubit groups per qubit count (empty = even
// split into the fewest groups); read when a batch is planned.
std::mutex g_split_mu;
std::vector<int> g_split[QAOA_MAX_QUBITS + 1];

std::vector<int> group_split(int n)
{
    {
        std::lock_guard<std::mutex> lk(g_split_mu);
        if (!g_split[n].empty()) return g_split[n];
    }
    std::vector<int> v;
    const int G1 = groups_for(n) - 1, rest = n - TILE_BITS;
    for (int g = 1; g <= G1; ++g) v.push_back(rest / G1 + (g <= rest % G1 ? 1 : 0));
    return v;
}

qaoa_status_t make_plan(int32_t B, const int32_t* nq, const int64_t* eoff, const int32_t* ew, int32_t max_p,
                        int32_t max_k, uint32_t flags, Plan& P)
{
    if (B < 1) return fail(QAOA_ERR_INVALID_ARG, "B = %d must be >= 1", B);
    if (!nq || !eoff) return fail(QAOA_ERR_INVALID_ARG, "num_qubits and edge_offsets are required");
    if (max_p < 1 || max_p > MAX_P) return fail(QAOA_ERR_OUT_OF_RANGE, "max_p = %d outside 1..%d", max_p, MAX_P);
    if (max_k < 1 || max_k > MAX_K) return fail(QAOA_ERR_OUT_OF_RANGE, "max_k = %d outside 1..%d", max_k, MAX_K);
    const uint32_t mixer =
        flags & (QAOA_FLAG_MIXER_MFMA_F32 | QAOA_FLAG_MIXER_MFMA_BF16X3 | QAOA_FLAG_MIXER_MFMA_BF16X4);
    if (flags & ~(QAOA_FLAG_GRADIENT | QAOA_FLAG_TOPK_RAW | QAOA_FLAG_SKIP_EDGELESS | QAOA_FLAG_GRADIENT_INPLACE |
                  QAOA_FLAG_GRADIENT_CHECKPOINTS | QAOA_FLAG_CONCURRENT_CLASSES | mixer))
        return fail(QAOA_ERR_INVALID_ARG, "unknown flag bits 0x%x", flags);
    if ((flags & QAOA_FLAG_GRADIENT_INPLACE) && (flags & QAOA_FLAG_GRADIENT_CHECKPOINTS))
        return fail(QAOA_ERR_INVALID_ARG, "QAOA_FLAG_GRADIENT_INPLACE and QAOA_FLAG_GRADIENT_CHECKPOINTS together");
    if (mixer & (mixer - 1)) return fail(QAOA_ERR_INVALID_ARG, "at most one mixer precision mode may be set");
    if (mixer && (flags & QAOA_FLAG_GRADIENT))
        return fail(QAOA_ERR_NOT_SUPPORTED, "the matrix-core mixer modes have no gradient path");
    if (eoff[0] != 0) return fail(QAOA_ERR_INVALID_ARG, "edge_offsets[0] = %lld must be 0", (long long)eoff[0]);
    P.B = B;
    P.max_p = max_p;
    P.max_k = max_k;
    P.flags = flags;
    P.prec = mixer == QAOA_FLAG_MIXER_MFMA_F32 ? 1 : mixer == QAOA_FLAG_MIXER_MFMA_BF16X3 ? 2
           : mixer == QAOA_FLAG_MIXER_MFMA_BF16X4 ? 3 : 0;
    P.subs.assign(B, SubDesc{});
    const bool grad = flags & QAOA_FLAG_GRADIENT;
    P.ckpt = false;  // decided once the subgraphs are known
    int64_t tiles = 0;
    for (int b = 0; b < B; ++b) {
        const int n = nq[b];
        if (n < 1 || n > QAOA_MAX_QUBITS)
            return fail(QAOA_ERR_OUT_OF_RANGE, "subgraph %d has %d qubits (1..%d)", b, n, QAOA_MAX_QUBITS);
        if (eoff[b + 1] < eoff[b])
            return fail(QAOA_ERR_INVALID_ARG, "edge_offsets not monotone at %d", b);
        int64_t wsum = 0;
        for (int64_t e = eoff[b]; e < eoff[b + 1]; ++e) {
            const int64_t w = ew ? ew[e] : 1;
            if (w < 0) return fail(QAOA_ERR_INVALID_ARG, "edge %lld has negative weight", (long long)e);
            wsum += w;
        }
        if (wsum > QAOA_MAX_WEIGHT_SUM)
            return fail(QAOA_ERR_NOT_SUPPORTED, "subgraph %d weight sum %lld exceeds %d", b, (long long)wsum,
                        QAOA_MAX_WEIGHT_SUM);
        SubDesc& d = P.subs[b];
        d.n = n;
        // group 0: qubits 0..10 and the top qubit (the complement of a reduced
        // index, tile bit 11); strided groups: qubits 11..n-2 of the reduced index
        d.gstart[0] = 0;
        d.gsize[0] = n <= SMALL_MAX_N ? n : TILE_BITS;
        d.ngroups = 1;
        if (n > SMALL_MAX_N) {
            int q = HALF_BITS;
            for (int sz : group_split(n)) {
                d.gstart[d.ngroups] = q;
                d.gsize[d.ngroups] = sz;
                q += sz;
                ++d.ngroups;
            }
        }
        d.lut_len = (int32_t)wsum + 1;
        d.tabw = wsum <= 255 ? 1 : 2;
        d.skip = (flags & QAOA_FLAG_SKIP_EDGELESS) && eoff[b + 1] == eoff[b];
        d.ntiles = d.skip ? 0 : (n > SMALL_MAX_N ? (1 << (n - 1 - TILE_BITS)) : 1);
        d.tile_base = (int32_t)tiles;
        d.nedges = (int32_t)(eoff[b + 1] - eoff[b]);
        tiles += d.ntiles;
        if (d.lut_len > P.lut_max) P.lut_max = d.lut_len;
    }
    if (tiles > (1ll << 30)) return fail(QAOA_ERR_OUT_OF_RANGE, "batch too large (%lld tiles)", (long long)tiles);
    P.total_tiles = (int32_t)tiles;
    P.total_edges = eoff[B];
    if (grad) {
        // Gradient memory: checkpoints unless asked otherwise, except when the
        // single-slot states and tables fit the 256 MB Infinity Cache and the
        // checkpoints would not (there the cache serves the adjoint sweep's
        // re-reads of psi faster than HBM serves the checkpoints)
        uint64_t inplace = 0, ckpt = 0;
        for (const SubDesc& d : P.subs) {
            if (d.skip) continue;
            const uint64_t st = state_bytes(d.n), tb = (1ull << (d.n - 1)) * d.tabw * (d.ngroups >= 2 ? 2 : 1);
            const uint64_t slots = d.ngroups >= 2 ? (uint64_t)max_p * (d.ngroups - 1) : 1;
            inplace += 2 * st + tb;
            ckpt += (slots + 1) * st + tb;
        }
        if (flags & QAOA_FLAG_GRADIENT_INPLACE) P.ckpt = false;
        else if (flags & QAOA_FLAG_GRADIENT_CHECKPOINTS) P.ckpt = true;
        else P.ckpt = !(inplace <= CACHE_FIT_BYTES && ckpt > CACHE_BYTES);
    }

    // work lists: every tile (tables, top-k); per group-count class (passes)
    P.work_all.reserve(tiles);
    for (int b = 0; b < B; ++b)
        for (int t = 0; t < P.subs[b].ntiles; ++t) P.work_all.push_back(make_int2(b, t));
    {
        // larger subgraphs first within each class
        std::vector<int> order;
        for (int b = 0; b < B; ++b)
            if (P.subs[b].ngroups >= 2) order.push_back(b);
        std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return P.subs[a].n > P.subs[c].n; });
        for (int b : order) {
            const SubDesc& d = P.subs[b];
            if (d.skip) continue;
            int ci = -1;
            for (size_t k = 0; k < P.classes.size(); ++k) {
                bool same = P.classes[k].G == d.ngroups;
                for (int g = 0; same && g < d.ngroups; ++g) same = P.classes[k].chain[g] == chain_of(d, g);
                if (same) ci = (int)k;
            }
            if (ci < 0) {
                Plan::Class c{};
                c.G = d.ngroups;
                for (int g = 0; g < d.ngroups; ++g) c.chain[g] = chain_of(d, g);
                P.classes.push_back(c);
                ci = (int)P.classes.size() - 1;
            }
            for (int t = 0; t < d.ntiles; ++t) P.classes[ci].work.push_back(make_int2(b, t));
            P.classes[ci].tab_bytes += (double)d.ntiles * TILE * d.tabw;
        }
    }
    for (int b = 0; b < B; ++b)
        if (P.subs[b].ngroups == 1 && !P.subs[b].skip) P.small.push_back(b);
    P.nsmall = (int)P.small.size();

    // regions
    uint64_t o = 0;
    auto region = [&](uint64_t bytes, uint64_t align) {
        o = align_up(o, align);
        const uint64_t r = o;
        o += bytes;
        return r;
    };
    P.o_subs = region(sizeof(SubDesc) * B, 256);
    P.o_work_all = region(sizeof(int2) * tiles, 256);
    for (auto& c : P.classes) c.o_work = region(sizeof(int2) * c.work.size(), 256);
    P.o_small = region(sizeof(int32_t) * (P.nsmall + 1), 256);
    P.o_edges = region(sizeof(int32_t) * 3 * (P.total_edges + 1), 256);
    P.o_coef = region(sizeof(RxCoef) * B * max_p, 256);
    uint64_t lut_total = 0;
    for (int b = 0; b < B; ++b) lut_total += (uint64_t)max_p * P.subs[b].lut_len;
    P.o_lut = region(sizeof(float2) * lut_total, 256);
    P.o_pe = region(sizeof(double) * tiles, 256);
    P.o_pgb = region(grad ? sizeof(double) * tiles * max_p * MAX_GROUPS : 0, 256);
    P.o_pgg = region(grad ? sizeof(double) * tiles * max_p : 0, 256);
    P.o_keys = region(sizeof(uint64_t) * tiles * max_k, 256);
    uint64_t lut_o = P.o_lut, eo = P.o_edges;
    for (int b = 0; b < B; ++b) {
        SubDesc& d = P.subs[b];
        const uint64_t dim = 1ull << (d.n - 1);  // reduced state
        d.coef = P.o_coef + sizeof(RxCoef) * (uint64_t)b * max_p;
        d.lut = lut_o;
        lut_o += sizeof(float2) * (uint64_t)max_p * d.lut_len;
        d.edges = eo + sizeof(int32_t) * 3 * (uint64_t)eoff[b];
        if (d.skip) continue;  // closed form, nothing stored
        // with checkpoints, one psi slot per forward pass of the gradient
        // sweep that precedes the fused turn: p (G - 1) at the largest depth
        const uint64_t slots = (P.ckpt && d.ngroups >= 2) ? (uint64_t)max_p * (d.ngroups - 1) : 1;
        d.psi = region(slots * dim * sizeof(float2), 4096);
        d.lam = grad ? region(dim * sizeof(float2), 4096) : 0;
        d.tab = region(dim * (uint64_t)d.tabw, 4096);
        d.tabB = d.ngroups >= 2 ? region(dim * (uint64_t)d.tabw, 4096) : 0;
    }
    P.total = align_up(o, 4096);
    return ok();
}

// Serpentine pass program for a subgraph class with G >= 2 qubit groups.
struct Op {
    bool phase;
    int g, l;
};

std::vector<Op> forward_ops(int G, int p)
{
    std::vector<Op> ops;
    for (int l = 0; l < p; ++l) {
        ops.push_back({true, -1, l});
        for (int i = 0; i < G; ++i) ops.push_back({false, (l % 2 == 0) ? i : G - 1 - i, l});
    }
    return ops;
}

std::vector<PassOps> group_passes(const std::vector<Op>& ops)
{
    std::vector<PassOps> out;
    PassOps cur{};
    bool have = false;
    int pending = -1;
    for (const Op& op : ops) {
        if (op.phase) {
            pending = op.l;
            continue;
        }
        if (have && cur.group == op.g && cur.ph < 0 && cur.post < 0) {
            cur.ph = pending;
            cur.post = op.l;
            pending = -1;
            continue;
        }
        if (have) out.push_back(cur);
        cur = PassOps{};
        cur.group = op.g;
        cur.pre = pending < 0 ? op.l : -1;
        cur.ph = pending;
        cur.post = pending < 0 ? -1 : op.l;
        pending = -1;
        have = true;
    }
    if (have) {
        if (pending >= 0) cur.ph = pending;  // trailing phase of a reversed program
        out.push_back(cur);
    }
    return out;
}

// Profiling name of a pass kernel: direction, kind and qubit group (each is
// its own kernel instantiation), e.g. "bwd_mid_g0".
const char* pass_name(const PassOps& o, bool backward)
{
    static const char* const fk[] = {"first", "single", "mid", "last"};
    static const char* const bk[] = {"fused", "single", "mid", "last", "single_nopsi", "mid_nopsi"};
    static std::string names[2][6][MAX_GROUPS];
    static std::once_flag once;
    std::call_once(once, [] {
        for (int g = 0; g < MAX_GROUPS; ++g) {
            for (int k = 0; k < 4; ++k) names[0][k][g] = std::string("fwd_") + fk[k] + "_g" + std::to_string(g);
            for (int k = 0; k < 6; ++k) names[1][k][g] = std::string("bwd_") + bk[k] + "_g" + std::to_string(g);
        }
    });
    int k;
    if (!backward) k = o.init ? 0 : o.epi_e ? 3 : o.ph >= 0 ? 2 : 1;
    else if (o.fused) k = 0;
    else if (o.last) k = 3;
    else k = (o.ph >= 0 ? 2 : 1) + (o.nopsi ? 3 : 0);
    return names[backward ? 1 : 0][k][o.group].c_str();
}

// algorithmic HBM bytes of one pass over a class: states read and written
// once, the cut table (1 or 2 B per amplitude) where the pass needs C(z)
double pass_bytes(const PassOps& o, bool backward, int nwork, double tab_bytes)
{
    const double amps = (double)nwork * TILE;
    double per;
    bool tab;
    if (!backward) {
        per = o.init ? 8.0 : 16.0;
        tab = o.ph >= 0 || o.epi_e;
    } else if (o.fused) {
        per = 8.0 + 8.0;  // read psi, write lambda
        tab = true;
    } else if (o.last) {
        per = 8.0;  // read lambda (psi is synthesised)
        tab = true;
    } else {
        per = 16.0 + (o.nopsi ? 8.0 : 16.0);
        tab = o.ph >= 0;
    }
    return per * amps + (tab ? tab_bytes : 0.0);
}

double angle_bytes(const Plan& P, int p)
{
    double b = 0.0;
    for (const SubDesc& d : P.subs) b += (double)p * (d.lut_len * 8.0 + 8.0 + 16.0);
    return b;
}

// whole-state-in-LDS kernel: cut table once per layer (and per adjoint layer),
// the state written once (forward)
double small_bytes(const Plan& P, int p, bool grad)
{
    double b = 0.0;
    for (const SubDesc& d : P.subs)
        if (d.ngroups == 1 && !d.skip)
            b += (double)(1ull << (d.n - 1)) * (grad ? d.tabw * (2.0 * p + 2) : (d.tabw * (p + 1.0) + 8.0));
    return b;
}

}  // namespace

extern "C" qaoa_status_t qaoa_tune_group_split(int32_t n, int32_t count, const int32_t* sizes)
{
    if (n <= SMALL_MAX_N || n > QAOA_MAX_QUBITS)
        return fail(QAOA_ERR_OUT_OF_RANGE, "n = %d outside %d..%d", n, SMALL_MAX_N + 1, QAOA_MAX_QUBITS);
    if (count < 0 || count > MAX_GROUPS - 1)
        return fail(QAOA_ERR_OUT_OF_RANGE, "count = %d outside 0..%d", count, MAX_GROUPS - 1);
    std::vector<int> v;
    int sum = 0;
    for (int i = 0; i < count; ++i) {
        if (!sizes) return fail(QAOA_ERR_INVALID_ARG, "sizes is NULL");
        if (sizes[i] < 1 || sizes[i] > B_GROUP_MAX)
            return fail(QAOA_ERR_OUT_OF_RANGE, "group size %d outside 1..%d", sizes[i], B_GROUP_MAX);
        v.push_back(sizes[i]);
        sum += sizes[i];
    }
    if (count > 0 && sum != n - TILE_BITS)
        return fail(QAOA_ERR_INVALID_ARG, "group sizes add up to %d, not n - %d = %d", sum, TILE_BITS, n - TILE_BITS);
    std::lock_guard<std::mutex> lk(g_split_mu);
    g_split[n] = v;
    return ok();
}

// ---------------------------------------------------------------------------
// side streams of the concurrent-classes mode: per device, created once
// (default priority) and kept until the process ends; one lock serialises the
// fork/join sequences of all batches, so the shared events are never
// re-recorded before the waits that read them are enqueued
// ---------------------------------------------------------------------------
constexpr int NSIDE = 3;
constexpr int SIDE_MAX_DEVICES = 64;
struct SideStreams {
    hipStream_t s[NSIDE];
    hipEvent_t fork;
    hipEvent_t join[NSIDE];
};
std::mutex g_side_mu;
SideStreams* g_side[SIDE_MAX_DEVICES] = {};

static qaoa_status_t side_streams(SideStreams** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= SIDE_MAX_DEVICES) return fail(QAOA_ERR_NOT_SUPPORTED, "device %d", dev);
    std::lock_guard<std::mutex> lk(g_side_mu);
    if (!g_side[dev]) {
        SideStreams* ss = new SideStreams();
        for (int j = 0; j < NSIDE; ++j) {
            HIP_TRY(hipStreamCreateWithFlags(&ss->s[j], hipStreamNonBlocking));
            HIP_TRY(hipEventCreateWithFlags(&ss->join[j], hipEventDisableTiming));
        }
        HIP_TRY(hipEventCreateWithFlags(&ss->fork, hipEventDisableTiming));
        g_side[dev] = ss;
    }
    *out = g_side[dev];
    return QAOA_OK;
}

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct qaoa_batch_s {
    Plan P;
    uint8_t* ws = nullptr;
    SubDesc* d_subs = nullptr;
    Partials part{};
    SideStreams* side = nullptr;  // set with QAOA_FLAG_CONCURRENT_CLASSES
    bool state_valid = false;     // psi holds the ansatz state of the last apply
    bool e_valid = false;         // <C> partials are fresh
};

// Runs body(class index or -1 for the small-subgraph kernel, stream) for the
// small-subgraph kernel (if any) and every class. Default: all on st, in
// order. Concurrent classes: class 0 (the largest subgraphs) on st, the rest
// each on the side stream with the least work so far (tiles x passes),
// forked from st and joined back into it.
template <typename F>
static qaoa_status_t for_each_class(qaoa_batch_t h, int32_t p, hipStream_t st, F body)
{
    const Plan& P = h->P;
    const int nc = (int)P.classes.size();
    if (!h->side || nc + (P.nsmall ? 1 : 0) < 2) {
        qaoa_status_t s;
        if (P.nsmall && (s = body(-1, st)) != QAOA_OK) return s;
        for (int k = 0; k < nc; ++k)
            if ((s = body(k, st)) != QAOA_OK) return s;
        return QAOA_OK;
    }
    SideStreams& ss = *h->side;
    std::lock_guard<std::mutex> lk(g_side_mu);
    HIP_TRY(hipEventRecord(ss.fork, st));
    double load[NSIDE] = {};
    bool used[NSIDE] = {};
    hipError_t ferr = hipSuccess;  // first failure of a fork or join call
    auto note = [&](hipError_t e) {
        if (e != hipSuccess && ferr == hipSuccess) ferr = e;
    };
    auto pick = [&](double w) -> hipStream_t {
        int j = 0;
        for (int i = 1; i < NSIDE; ++i)
            if (load[i] < load[j]) j = i;
        load[j] += w;
        if (!used[j]) {
            used[j] = true;
            note(hipStreamWaitEvent(ss.s[j], ss.fork, 0));
        }
        return ss.s[j];
    };
    qaoa_status_t s = QAOA_OK;
    if (nc > 0) s = body(0, st);
    for (int k = 1; k < nc && s == QAOA_OK && ferr == hipSuccess; ++k)
        s = body(k, pick((double)P.classes[k].work.size() * (double)(p * (P.classes[k].G - 1) + 1)));
    if (P.nsmall && s == QAOA_OK && ferr == hipSuccess) s = body(-1, pick((double)P.nsmall * p));
    // join every side stream that was forked, also after an error
    for (int j = 0; j < NSIDE; ++j) {
        if (!used[j]) continue;
        note(hipEventRecord(ss.join[j], ss.s[j]));
        note(hipStreamWaitEvent(st, ss.join[j], 0));
    }
    if (s == QAOA_OK && ferr != hipSuccess)
        return fail(QAOA_ERR_HIP, "fork/join of the concurrent classes: %s", hipGetErrorString(ferr));
    return s;
}

extern "C" const char* qaoa_status_string(qaoa_status_t s)
{
    switch (s) {
    case QAOA_OK: return "ok";
    case QAOA_ERR_INVALID_ARG: return "invalid argument";
    case QAOA_ERR_OUT_OF_RANGE: return "argument out of range";
    case QAOA_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case QAOA_ERR_HIP: return "HIP runtime error";
    case QAOA_ERR_STATE: return "call order violated";
    case QAOA_ERR_NOT_SUPPORTED: return "not supported";
    }
    return "unknown status";
}

extern "C" const char* qaoa_last_error(void) { return g_err; }

extern "C" qaoa_status_t qaoa_workspace_bytes(int32_t B, const int32_t* num_qubits, const int64_t* edge_offsets,
                                              const int32_t* edge_w, int32_t max_p, int32_t max_k,
                                              uint32_t flags, size_t* out_bytes)
{
    if (!out_bytes) return fail(QAOA_ERR_INVALID_ARG, "out_bytes is NULL");
    Plan P;
    qaoa_status_t s = make_plan(B, num_qubits, edge_offsets, edge_w, max_p, max_k, flags, P);
    if (s != QAOA_OK) return s;
    *out_bytes = (size_t)P.total;
    return ok();
}

extern "C" qaoa_status_t qaoa_batch_create(int32_t B, const int32_t* num_qubits, const int64_t* edge_offsets,
                                           const int32_t* edge_u, const int32_t* edge_v, const int32_t* edge_w,
                                           int32_t max_p, int32_t max_k, uint32_t flags, void* d_workspace,
                                           size_t workspace_bytes, qaoa_stream_t stream, qaoa_batch_t* out)
{
    if (!out) return fail(QAOA_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    Plan P;
    qaoa_status_t s = make_plan(B, num_qubits, edge_offsets, edge_w, max_p, max_k, flags, P);
    if (s != QAOA_OK) return s;
    if (P.total_edges > 0 && (!edge_u || !edge_v)) return fail(QAOA_ERR_INVALID_ARG, "edge_u/edge_v are NULL");
    for (int b = 0; b < B; ++b) {
        const int n = P.subs[b].n;
        for (int64_t e = edge_offsets[b]; e < edge_offsets[b + 1]; ++e) {
            const int32_t u = edge_u[e], v = edge_v[e];
            if (u < 0 || v < 0 || u >= n || v >= n || u == v)
                return fail(QAOA_ERR_INVALID_ARG, "subgraph %d edge %lld = (%d, %d) invalid for n = %d", b,
                            (long long)e, u, v, n);
        }
    }
    // free vertices: no edge of positive weight inside the subgraph; the
    // state is exactly invariant under flipping their bits (top-k ties)
    for (int b = 0; b < B; ++b) {
        SubDesc& d = P.subs[b];
        uint32_t busy = 0;
        for (int64_t e = edge_offsets[b]; e < edge_offsets[b + 1]; ++e)
            if (!edge_w || edge_w[e] > 0) busy |= (1u << edge_u[e]) | (1u << edge_v[e]);
        d.freem = (uint32_t)((1ull << d.n) - 1ull) & ~busy;
    }
    if (!d_workspace) return fail(QAOA_ERR_INVALID_ARG, "d_workspace is NULL");
    if (((uintptr_t)d_workspace) % 256) return fail(QAOA_ERR_INVALID_ARG, "d_workspace not 256-byte aligned");
    if (workspace_bytes < P.total)
        return fail(QAOA_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %llu", workspace_bytes,
                    (unsigned long long)P.total);

    // metadata image: [subs | work_all | work classes | small | edges]
    const uint64_t meta_end = P.o_coef;
    std::vector<uint8_t> img(meta_end, 0);
    memcpy(img.data() + P.o_subs, P.subs.data(), sizeof(SubDesc) * B);
    memcpy(img.data() + P.o_work_all, P.work_all.data(), sizeof(int2) * P.work_all.size());
    for (const auto& c : P.classes)
        memcpy(img.data() + c.o_work, c.work.data(), sizeof(int2) * c.work.size());
    if (P.nsmall) memcpy(img.data() + P.o_small, P.small.data(), sizeof(int32_t) * P.nsmall);
    int32_t* E = (int32_t*)(img.data() + P.o_edges);
    for (int64_t e = 0; e < P.total_edges; ++e) {
        E[3 * e] = edge_u[e];
        E[3 * e + 1] = edge_v[e];
        E[3 * e + 2] = edge_w ? edge_w[e] : 1;
    }
    hipStream_t st = (hipStream_t)stream;
    uint8_t* ws = (uint8_t*)d_workspace;
    s = upload_async(ws, img.data(), meta_end, st);
    if (s != QAOA_OK) return s;

    SideStreams* side = nullptr;
    if (flags & QAOA_FLAG_CONCURRENT_CLASSES) {
        s = side_streams(&side);
        if (s != QAOA_OK) return s;
    }
    qaoa_batch_s* h = new qaoa_batch_s();
    h->side = side;
    h->P = std::move(P);
    h->ws = ws;
    h->d_subs = (SubDesc*)(ws + h->P.o_subs);
    h->part.e = (double*)(ws + h->P.o_pe);
    h->part.gb = (double*)(ws + h->P.o_pgb);
    h->part.gg = (double*)(ws + h->P.o_pgg);
    h->part.total_tiles = h->P.total_tiles;
    {
        double tb = 0.0;
        for (const SubDesc& d : h->P.subs)
            if (!d.skip) tb += (double)(1ull << (d.n - 1)) * d.tabw * (d.ngroups >= 2 ? 2.0 : 1.0);
        ProfScope ps("cut_tables", st, tb);
        hipError_t e = launch_cut_tables(ws, h->d_subs, (const int2*)(ws + h->P.o_work_all), h->P.total_tiles, st);
        if (e != hipSuccess) {
            delete h;
            return fail(QAOA_ERR_HIP, "cut table kernel: %s", hipGetErrorString(e));
        }
    }
    *out = h;
    return ok();
}

extern "C" qaoa_status_t qaoa_batch_destroy(qaoa_batch_t h)
{
    delete h;
    return ok();
}

static qaoa_status_t check_angles(qaoa_batch_t h, int32_t p, const double* g, const double* b)
{
    if (!h) return fail(QAOA_ERR_INVALID_ARG, "handle is NULL");
    if (p < 1 || p > h->P.max_p) return fail(QAOA_ERR_OUT_OF_RANGE, "p = %d outside 1..%d", p, h->P.max_p);
    if (!g || !b) return fail(QAOA_ERR_INVALID_ARG, "d_gamma/d_beta are NULL");
    return QAOA_OK;
}

extern "C" qaoa_status_t qaoa_apply_layers(qaoa_batch_t h, int32_t p, const double* d_gamma, const double* d_beta,
                                           qaoa_stream_t stream)
{
    qaoa_status_t s = check_angles(h, p, d_gamma, d_beta);
    if (s != QAOA_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    Plan& P = h->P;
    {
        ProfScope ps("angle_prep", st, angle_bytes(P, p));
        HIP_TRY(launch_angle_prep(h->ws, h->d_subs, P.B, p, d_gamma, d_beta, st));
    }
    s = for_each_class(h, p, st, [&](int k, hipStream_t cs) -> qaoa_status_t {
        if (k < 0) {
            ProfScope ps("small", cs, small_bytes(P, p, false));
            HIP_TRY(launch_small(h->ws, h->d_subs, (const int32_t*)(h->ws + P.o_small), P.nsmall, p, 0, h->part,
                                 P.lut_max, cs));
            return QAOA_OK;
        }
        const auto& c = P.classes[k];
        const int2* work = (const int2*)(h->ws + c.o_work);
        const int nw = (int)c.work.size();
        std::vector<PassOps> passes = group_passes(forward_ops(c.G, p));
        for (size_t i = 0; i < passes.size(); ++i) {
            PassOps o = passes[i];
            o.init = i == 0;
            o.epi_e = i + 1 == passes.size();
            ProfScope ps(pass_name(o, false), cs, pass_bytes(o, false, nw, c.tab_bytes));
            HIP_TRY(launch_fwd_pass(h->ws, h->d_subs, work, nw, c.chain[o.group], o, h->part, P.lut_max, P.prec,
                                    cs));
        }
        return QAOA_OK;
    });
    if (s != QAOA_OK) return s;
    h->state_valid = true;
    h->e_valid = true;
    return ok();
}

extern "C" qaoa_status_t qaoa_expectation(qaoa_batch_t h, double* d_out, qaoa_stream_t stream)
{
    if (!h) return fail(QAOA_ERR_INVALID_ARG, "handle is NULL");
    if (!d_out) return fail(QAOA_ERR_INVALID_ARG, "d_out is NULL");
    if (!h->e_valid) return fail(QAOA_ERR_STATE, "no state: call qaoa_apply_layers first");
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps("reduce", st, 8.0 * h->P.total_tiles);
    HIP_TRY(launch_reduce(h->d_subs, h->P.B, 1, 0, h->part, d_out, nullptr, nullptr, st));
    return ok();
}

extern "C" qaoa_status_t qaoa_topk(qaoa_batch_t h, int32_t k, uint32_t* d_idx, float* d_prob, qaoa_stream_t stream)
{
    if (!h) return fail(QAOA_ERR_INVALID_ARG, "handle is NULL");
    if (k < 1 || k > h->P.max_k) return fail(QAOA_ERR_OUT_OF_RANGE, "k = %d outside 1..%d", k, h->P.max_k);
    if (!d_idx || !d_prob) return fail(QAOA_ERR_INVALID_ARG, "d_idx/d_prob are NULL");
    if (!h->state_valid) return fail(QAOA_ERR_STATE, "no ansatz state: call qaoa_apply_layers first");
    hipStream_t st = (hipStream_t)stream;
    const Plan& P = h->P;
    double tk = 0.0;
    for (const SubDesc& d : P.subs)
        if (!d.skip) tk += (double)(1ull << (d.n - 1)) * 8.0;
    ProfScope ps("topk", st, tk + 16.0 * P.total_tiles * k);
    HIP_TRY(launch_topk(h->ws, h->d_subs, (const int2*)(h->ws + P.o_work_all), P.total_tiles, P.B, k,
                        (P.flags & QAOA_FLAG_TOPK_RAW) ? 0 : 1, (uint64_t*)(h->ws + P.o_keys), d_idx, d_prob,
                        st));
    return ok();
}

// one class's tile passes of a gradient evaluation (forward sweep, fused
// turn, adjoint sweep), or the small-subgraph kernel (k < 0)
static qaoa_status_t enqueue_class_grad(qaoa_batch_t h, int k, int32_t p, hipStream_t st)
{
    Plan& P = h->P;
    if (k < 0) {
        ProfScope ps("small", st, small_bytes(P, p, true));
        HIP_TRY(launch_small(h->ws, h->d_subs, (const int32_t*)(h->ws + P.o_small), P.nsmall, p, 1, h->part,
                             P.lut_max, st));
        return QAOA_OK;
    }
    {
        const auto& c = P.classes[k];
        const int2* work = (const int2*)(h->ws + c.o_work);
        const int nw = (int)c.work.size();
        std::vector<Op> ops = forward_ops(c.G, p);
        std::vector<PassOps> fwd = group_passes(ops);
        const int F = (int)fwd.size();
        // with checkpoints, forward pass i writes psi slot i (reading slot
        // i - 1), and the backward pass that undoes it reads slot i and
        // stores only lambda; otherwise every pass works in slot 0 and the
        // backward passes rebuild psi as they go
        const bool ck = P.ckpt;
        for (int i = 0; i + 1 < F; ++i) {
            PassOps o = fwd[i];
            o.init = i == 0;
            o.psi_in = ck && i > 0 ? i - 1 : 0;
            o.psi_out = ck ? i : 0;
            ProfScope ps(pass_name(o, false), st, pass_bytes(o, false, nw, c.tab_bytes));
            HIP_TRY(launch_fwd_pass(h->ws, h->d_subs, work, nw, c.chain[o.group], o, h->part, P.lut_max, 0, st));
        }
        std::vector<Op> rev(ops.rbegin(), ops.rend());
        std::vector<PassOps> bwd = group_passes(rev);
        // the last forward pass (RX of the last group, layer p-1) and the
        // first backward pass (its inverse) share one kernel
        PassOps f = fwd.back();
        f.fused = 1;
        f.psi_in = ck ? F - 2 : 0;
        {
            ProfScope ps(pass_name(f, true), st, pass_bytes(f, true, nw, c.tab_bytes));
            HIP_TRY(launch_bwd_pass(h->ws, h->d_subs, work, nw, c.chain[f.group], f, h->part, P.lut_max, st));
        }
        for (int i = 1; i < (int)bwd.size(); ++i) {
            PassOps o = bwd[i];
            o.last = i + 1 == (int)bwd.size();
            o.nopsi = ck || i + 2 == (int)bwd.size();  // the last pass synthesises psi
            o.psi_in = ck ? F - 1 - i : 0;
            ProfScope ps(pass_name(o, true), st, pass_bytes(o, true, nw, c.tab_bytes));
            HIP_TRY(launch_bwd_pass(h->ws, h->d_subs, work, nw, c.chain[o.group], o, h->part, P.lut_max, st));
        }
    }
    return QAOA_OK;
}

// the small-subgraph kernel and every tile pass of one gradient evaluation
// (forward sweep, fused turn, adjoint sweep), after the angle tables are set
static qaoa_status_t enqueue_grad_passes(qaoa_batch_t h, int32_t p, hipStream_t st)
{
    return for_each_class(h, p, st, [&](int k, hipStream_t cs) { return enqueue_class_grad(h, k, p, cs); });
}

extern "C" qaoa_status_t qaoa_expectation_grad(qaoa_batch_t h, int32_t p, const double* d_gamma,
                                               const double* d_beta, double* d_E, double* d_dgamma,
                                               double* d_dbeta, qaoa_stream_t stream)
{
    qaoa_status_t s = check_angles(h, p, d_gamma, d_beta);
    if (s != QAOA_OK) return s;
    if (!(h->P.flags & QAOA_FLAG_GRADIENT))
        return fail(QAOA_ERR_STATE, "batch was created without QAOA_FLAG_GRADIENT");
    if (!d_E || !d_dgamma || !d_dbeta) return fail(QAOA_ERR_INVALID_ARG, "output pointers are NULL");
    hipStream_t st = (hipStream_t)stream;
    Plan& P = h->P;
    {
        ProfScope ps("angle_prep", st, angle_bytes(P, p));
        HIP_TRY(launch_angle_prep(h->ws, h->d_subs, P.B, p, d_gamma, d_beta, st));
    }
    s = enqueue_grad_passes(h, p, st);
    if (s != QAOA_OK) return s;
    {
        ProfScope ps("reduce", st, 8.0 * P.total_tiles * (1.0 + p * (MAX_GROUPS + 1.0)));
        HIP_TRY(launch_reduce(h->d_subs, P.B, p, 1, h->part, d_E, d_dgamma, d_dbeta, st));
    }
    h->state_valid = false;
    h->e_valid = true;
    return ok();
}

static bool adam_constants_ok(double lr, double beta1, double beta2, double eps)
{
    return beta1 >= 0.0 && beta1 < 1.0 && beta2 >= 0.0 && beta2 < 1.0 && eps > 0.0 && lr >= 0.0;
}

extern "C" qaoa_status_t qaoa_optimize(qaoa_batch_t h, int32_t p, int32_t iters, double* d_theta, double* d_m,
                                       double* d_v, int32_t* d_step, double lr, double beta1, double beta2,
                                       double eps, double* d_E, qaoa_stream_t stream)
{
    if (!d_theta) return fail(QAOA_ERR_INVALID_ARG, "d_theta is NULL");
    qaoa_status_t s = check_angles(h, p, d_theta, d_theta + (size_t)(h ? h->P.B : 0) * p);
    if (s != QAOA_OK) return s;
    if (!(h->P.flags & QAOA_FLAG_GRADIENT))
        return fail(QAOA_ERR_STATE, "batch was created without QAOA_FLAG_GRADIENT");
    if (iters < 0) return fail(QAOA_ERR_INVALID_ARG, "iters = %d must be >= 0", iters);
    if (!d_m || !d_v || !d_step) return fail(QAOA_ERR_INVALID_ARG, "d_m/d_v/d_step are NULL");
    if (!adam_constants_ok(lr, beta1, beta2, eps)) return fail(QAOA_ERR_OUT_OF_RANGE, "Adam constants out of range");
    if (iters == 0) return ok();
    hipStream_t st = (hipStream_t)stream;
    Plan& P = h->P;
    const size_t BP = (size_t)P.B * p;
    {
        ProfScope ps("angle_prep", st, angle_bytes(P, p));
        HIP_TRY(launch_angle_prep(h->ws, h->d_subs, P.B, p, d_theta, d_theta + BP, st));
    }
    for (int it = 0; it < iters; ++it) {
        s = enqueue_grad_passes(h, p, st);
        if (s != QAOA_OK) return s;
        ProfScope ps("reduce_adam", st,
                     8.0 * P.total_tiles * (1.0 + p * (MAX_GROUPS + 1.0)) + 7.0 * 8.0 * 2.0 * BP + angle_bytes(P, p));
        HIP_TRY(launch_reduce_adam(h->ws, h->d_subs, P.B, p, h->part, d_theta, d_m, d_v, d_step, it, lr, beta1,
                                   beta2, eps, d_E, st));
    }
    HIP_TRY(launch_step_advance(d_step, iters, st));
    h->state_valid = false;
    h->e_valid = true;
    return ok();
}

extern "C" qaoa_status_t qaoa_adam_step(int32_t count, double* d_theta, const double* d_grad, double* d_m,
                                        double* d_v, int32_t* d_step, double lr, double beta1, double beta2,
                                        double eps, int32_t maximise, qaoa_stream_t stream)
{
    if (count < 1) return fail(QAOA_ERR_INVALID_ARG, "count = %d must be >= 1", count);
    if (!d_theta || !d_grad || !d_m || !d_v || !d_step) return fail(QAOA_ERR_INVALID_ARG, "NULL pointer");
    if (!adam_constants_ok(lr, beta1, beta2, eps)) return fail(QAOA_ERR_OUT_OF_RANGE, "Adam constants out of range");
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps("adam", st, 7.0 * 8.0 * count);
    HIP_TRY(launch_adam(count, d_theta, d_grad, d_m, d_v, d_step, lr, beta1, beta2, eps, maximise ? 1.0 : -1.0, st));
    return ok();
}

extern "C" qaoa_status_t maxcut_eval(int32_t num_vertices, int64_t num_edges, const int32_t* d_u,
                                     const int32_t* d_v, const int32_t* d_w, int64_t num_assign,
                                     const uint32_t* d_assign, int64_t* d_cut, qaoa_stream_t stream)
{
    if (num_vertices < 1) return fail(QAOA_ERR_INVALID_ARG, "num_vertices = %d", num_vertices);
    if (num_edges < 0 || num_assign < 0) return fail(QAOA_ERR_INVALID_ARG, "negative count");
    if (num_edges > 0 && (!d_u || !d_v)) return fail(QAOA_ERR_INVALID_ARG, "d_u/d_v are NULL");
    if (num_assign > 0 && (!d_assign || !d_cut)) return fail(QAOA_ERR_INVALID_ARG, "d_assign/d_cut are NULL");
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps("maxcut", st, (double)num_edges * (d_w ? 12.0 : 8.0) * (num_assign > 0 ? 1.0 : 0.0) +
                                   4.0 * num_assign * ((num_vertices + 31) / 32) + 8.0 * num_assign);
    HIP_TRY(launch_maxcut_eval(num_vertices, num_edges, d_u, d_v, d_w, num_assign, d_assign, d_cut, st));
    return ok();
}

extern "C" qaoa_status_t qaoa_gradient_checkpoints(qaoa_batch_t h, int32_t* out)
{
    if (!h || !out) return fail(QAOA_ERR_INVALID_ARG, "NULL argument");
    *out = h->P.ckpt ? 1 : 0;
    return ok();
}

extern "C" qaoa_status_t qaoa_state_offset(qaoa_batch_t h, int32_t b, size_t* out_offset)
{
    if (!h || !out_offset) return fail(QAOA_ERR_INVALID_ARG, "NULL argument");
    if (b < 0 || b >= h->P.B) return fail(QAOA_ERR_OUT_OF_RANGE, "b = %d outside 0..%d", b, h->P.B - 1);
    if (h->P.subs[b].skip) return fail(QAOA_ERR_STATE, "subgraph %d is edgeless and was not simulated", b);
    *out_offset = (size_t)h->P.subs[b].psi;
    return ok();
}

// ---------------------------------------------------------------------------
// merge (Sec. 3.4, Alg. 2): host preparation of the level structure
// ---------------------------------------------------------------------------
namespace {
struct MergePlan {
    uint64_t o_lv, o_intra, o_back, o_ccut, o_keys, o_surv, o_counts, o_rows0, o_rows1, o_scores, o_lvs, o_maxinc,
        o_hist, o_below, o_pcnt, o_lvk, total;
    int nw;
};

MergePlan merge_plan(int32_t nV, int32_t M, int64_t nE, int32_t K, int32_t W)
{
    MergePlan P{};
    P.nw = (nV + 31) / 32;
    uint64_t o = 0;
    auto region = [&](uint64_t bytes) {
        o = align_up(o, 256);
        const uint64_t r = o;
        o += bytes;
        return r;
    };
    const uint64_t nkeys = align_up(std::max<uint64_t>((uint64_t)W * K, 2ull * K), MERGE_KEY_PAD);
    P.o_lv = region(sizeof(MergeLevel) * M);
    P.o_intra = region(sizeof(int32_t) * 3 * (nE + 1));
    P.o_back = region(sizeof(int32_t) * 3 * (nE + 1));
    P.o_ccut = region(sizeof(int64_t) * M * K);
    P.o_keys = region(sizeof(uint32_t) * nkeys);
    P.o_surv = region(sizeof(Surv) * W);
    P.o_counts = region(sizeof(int32_t) * (M + 1));
    P.o_rows0 = region(sizeof(uint32_t) * (uint64_t)W * P.nw);
    P.o_rows1 = region(sizeof(uint32_t) * (uint64_t)W * P.nw);
    P.o_scores = region(sizeof(int64_t) * W);
    P.o_lvs = region(sizeof(MergeLvState) * (M + 1));
    P.o_maxinc = region(sizeof(uint32_t) * M);
    P.o_hist = region(sizeof(int32_t) * MERGE_HIST_INTS);
    P.o_below = region(sizeof(int32_t));
    P.o_pcnt = region(sizeof(int64_t) * W);
    P.o_lvk = region(sizeof(int32_t) * M);
    P.total = align_up(o, 4096);
    return P;
}

qaoa_status_t merge_check(int32_t nV, int32_t M, int64_t nE, int32_t K, int32_t W)
{
    if (nV < 1 || M < 1) return fail(QAOA_ERR_INVALID_ARG, "num_vertices = %d, M = %d", nV, M);
    if (nE < 0) return fail(QAOA_ERR_INVALID_ARG, "num_edges < 0");
    if (K < 1 || K > MAX_K) return fail(QAOA_ERR_OUT_OF_RANGE, "K = %d outside 1..%d", K, MAX_K);
    if (W < 1 || W > QAOA_MAX_BEAM) return fail(QAOA_ERR_OUT_OF_RANGE, "W = %d outside 1..%d", W, QAOA_MAX_BEAM);
    return QAOA_OK;
}
}  // namespace

extern "C" qaoa_status_t qaoa_merge_workspace_bytes(int32_t num_vertices, int32_t M, int64_t num_edges, int32_t K,
                                                    int32_t W, size_t* out_bytes)
{
    if (!out_bytes) return fail(QAOA_ERR_INVALID_ARG, "out_bytes is NULL");
    qaoa_status_t s = merge_check(num_vertices, M, num_edges, K, W);
    if (s != QAOA_OK) return s;
    *out_bytes = (size_t)merge_plan(num_vertices, M, num_edges, K, W).total;
    return ok();
}

extern "C" qaoa_status_t qaoa_merge_beam(int32_t num_vertices, int32_t M, const int32_t* h_start,
                                         const int32_t* h_size, int64_t num_edges, const int32_t* h_u,
                                         const int32_t* h_v, const int32_t* h_w, int32_t K, const uint32_t* d_cand,
                                         int32_t W, void* d_workspace, size_t workspace_bytes,
                                         uint32_t* d_best_assign, int64_t* d_best_cut, qaoa_stream_t stream)
{
    qaoa_status_t s = merge_check(num_vertices, M, num_edges, K, W);
    if (s != QAOA_OK) return s;
    if (!h_start || !h_size) return fail(QAOA_ERR_INVALID_ARG, "h_start/h_size are NULL");
    if (num_edges > 0 && (!h_u || !h_v)) return fail(QAOA_ERR_INVALID_ARG, "h_u/h_v are NULL");
    if (!d_cand || !d_best_assign || !d_best_cut) return fail(QAOA_ERR_INVALID_ARG, "device pointer is NULL");
    if (!d_workspace || ((uintptr_t)d_workspace) % 256)
        return fail(QAOA_ERR_INVALID_ARG, "d_workspace NULL or not 256-byte aligned");
    const MergePlan P = merge_plan(num_vertices, M, num_edges, K, W);
    if (workspace_bytes < P.total)
        return fail(QAOA_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes, need %llu", workspace_bytes,
                    (unsigned long long)P.total);
    // chain: contiguous ranges sharing one vertex, covering [0, nV)
    if (h_start[0] != 0 || h_start[M - 1] + h_size[M - 1] != num_vertices)
        return fail(QAOA_ERR_INVALID_ARG, "ranges do not cover [0, %d)", num_vertices);
    for (int i = 0; i < M; ++i) {
        if (h_size[i] < (M > 1 ? 2 : 1) || h_size[i] > MERGE_MAX_SIZE)
            return fail(QAOA_ERR_OUT_OF_RANGE, "subgraph %d has %d vertices (2..%d)", i, h_size[i], MERGE_MAX_SIZE);
        if (i > 0 && h_start[i] != h_start[i - 1] + h_size[i - 1] - 1)
            return fail(QAOA_ERR_INVALID_ARG, "subgraph %d does not start at the last vertex of %d", i, i - 1);
    }
    // level at which each vertex is first assigned
    std::vector<int32_t> first(num_vertices);
    for (int i = 0; i < M; ++i)
        for (int v = h_start[i] + (i > 0 ? 1 : 0); v < h_start[i] + h_size[i]; ++v) first[v] = i;
    std::vector<MergeLevel> lv(M);
    std::vector<std::vector<int32_t>> intra(M), backk(M);
    int64_t wsum = 0;
    for (int64_t e = 0; e < num_edges; ++e) {
        const int32_t a = h_u[e], b = h_v[e], w = h_w ? h_w[e] : 1;
        if (a < 0 || b < 0 || a >= num_vertices || b >= num_vertices || a == b)
            return fail(QAOA_ERR_INVALID_ARG, "edge %lld = (%d, %d) invalid", (long long)e, a, b);
        if (w < 0) return fail(QAOA_ERR_INVALID_ARG, "edge %lld has negative weight", (long long)e);
        wsum += w;
        const int32_t lo = std::min(a, b), hi = std::max(a, b);
        const int L = first[hi];
        const int32_t st = h_start[L];
        if (lo >= st) {
            intra[L].push_back(lo - st);
            intra[L].push_back(hi - st);
            intra[L].push_back(w);
        } else {
            backk[L].push_back(lo);
            backk[L].push_back(hi - st);
            backk[L].push_back(w);
        }
    }
    if (wsum > 0x7FFFFFF0ll) return fail(QAOA_ERR_NOT_SUPPORTED, "total weight %lld too large", (long long)wsum);
    const uint64_t meta_end = P.o_ccut;
    std::vector<uint8_t> img(meta_end, 0);
    int32_t* I = (int32_t*)(img.data() + P.o_intra);
    int32_t* Bk = (int32_t*)(img.data() + P.o_back);
    int32_t io = 0, bo = 0;
    for (int i = 0; i < M; ++i) {
        MergeLevel& L = lv[i];
        memset(&L, 0, sizeof(L));
        L.start = h_start[i];
        L.size = h_size[i];
        L.intra_off = io;
        L.intra_cnt = (int32_t)(intra[i].size() / 3);
        memcpy(I + 3 * (size_t)io, intra[i].data(), intra[i].size() * sizeof(int32_t));
        io += L.intra_cnt;
        // back edges sorted by local endpoint k (counting sort, stable)
        const int nb = (int)(backk[i].size() / 3);
        int cnt[33] = {0};
        for (int e = 0; e < nb; ++e) cnt[backk[i][3 * e + 1] + 1]++;
        for (int k = 0; k < 32; ++k) cnt[k + 1] += cnt[k];
        for (int k = 0; k <= 32; ++k) L.kbeg[k] = cnt[k];
        L.back_off = bo;
        int fill[33];
        memcpy(fill, cnt, sizeof(fill));
        for (int e = 0; e < nb; ++e) {
            const int k = backk[i][3 * e + 1];
            const int slot = bo + fill[k]++;
            Bk[3 * (size_t)slot] = backk[i][3 * e];
            Bk[3 * (size_t)slot + 1] = k;
            Bk[3 * (size_t)slot + 2] = backk[i][3 * e + 2];
            L.wk[k] += backk[i][3 * e + 2];
        }
        bo += nb;
    }
    memcpy(img.data() + P.o_lv, lv.data(), sizeof(MergeLevel) * M);
    hipStream_t st = (hipStream_t)stream;
    uint8_t* ws = (uint8_t*)d_workspace;
    s = upload_async(ws, img.data(), meta_end, st);
    if (s != QAOA_OK) return s;
    MergeBufs m;
    m.lv = (const MergeLevel*)(ws + P.o_lv);
    m.intra = (const int32_t*)(ws + P.o_intra);
    m.back = (const int32_t*)(ws + P.o_back);
    m.ccut = (int64_t*)(ws + P.o_ccut);
    m.keys = (uint32_t*)(ws + P.o_keys);
    m.surv = (Surv*)(ws + P.o_surv);
    m.counts = (int32_t*)(ws + P.o_counts);
    m.rows[0] = (uint32_t*)(ws + P.o_rows0);
    m.rows[1] = (uint32_t*)(ws + P.o_rows1);
    m.scores = (int64_t*)(ws + P.o_scores);
    m.lvs = (MergeLvState*)(ws + P.o_lvs);
    m.maxinc = (uint32_t*)(ws + P.o_maxinc);
    m.hist = (int32_t*)(ws + P.o_hist);
    m.below = (int32_t*)(ws + P.o_below);
    m.pcnt = (int64_t*)(ws + P.o_pcnt);
    m.lvk = (int32_t*)(ws + P.o_lvk);
    ProfScope ps("merge", st, 0.0);
    HIP_TRY(launch_merge(m, M, K, W, P.nw, num_vertices, d_cand, d_best_assign, d_best_cut, st));
    return ok();
}

// ---------------------------------------------------------------------------
// angle predictor
// ---------------------------------------------------------------------------
static qaoa_status_t mlp_check(int32_t batch, int32_t in_dim, int32_t hidden, int32_t out_dim)
{
    if (batch < 1) return fail(QAOA_ERR_INVALID_ARG, "batch = %d", batch);
    if (in_dim < 1 || in_dim > MLP_MAX_IN || hidden < 1 || hidden > MLP_MAX_H || out_dim < 1 || out_dim > MLP_MAX_OUT)
        return fail(QAOA_ERR_OUT_OF_RANGE, "dims (%d, %d, %d) outside (1..%d, 1..%d, 1..%d)", in_dim, hidden, out_dim,
                    MLP_MAX_IN, MLP_MAX_H, MLP_MAX_OUT);
    return QAOA_OK;
}

extern "C" qaoa_status_t qaoa_mlp_num_params(int32_t in_dim, int32_t hidden, int32_t out_dim, int64_t* out)
{
    qaoa_status_t s = mlp_check(1, in_dim, hidden, out_dim);
    if (s != QAOA_OK) return s;
    if (!out) return fail(QAOA_ERR_INVALID_ARG, "out is NULL");
    *out = mlp_num_params(MlpDims{in_dim, hidden, out_dim});
    return ok();
}

extern "C" qaoa_status_t qaoa_mlp_forward(int32_t batch, int32_t in_dim, int32_t hidden, int32_t out_dim,
                                          const double* d_params, const float* d_x, float* d_y, float* d_act,
                                          qaoa_stream_t stream)
{
    qaoa_status_t s = mlp_check(batch, in_dim, hidden, out_dim);
    if (s != QAOA_OK) return s;
    if (!d_params || !d_x || !d_y || !d_act) return fail(QAOA_ERR_INVALID_ARG, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps("mlp_forward", st, 0.0);
    HIP_TRY(launch_mlp_forward(batch, MlpDims{in_dim, hidden, out_dim}, d_params, d_x, d_y, d_act, st));
    return ok();
}

extern "C" qaoa_status_t qaoa_mlp_scratch_bytes(int32_t batch, int32_t in_dim, int32_t hidden, int32_t out_dim,
                                                size_t* out)
{
    qaoa_status_t s = mlp_check(batch, in_dim, hidden, out_dim);
    if (s != QAOA_OK) return s;
    if (!out) return fail(QAOA_ERR_INVALID_ARG, "out is NULL");
    *out = mlp_scratch_bytes(batch, MlpDims{in_dim, hidden, out_dim});
    return ok();
}

extern "C" qaoa_status_t qaoa_mlp_backward(int32_t batch, int32_t in_dim, int32_t hidden, int32_t out_dim,
                                           const double* d_params, const float* d_x, const float* d_y,
                                           const float* d_act, const float* d_target, void* d_scratch,
                                           size_t scratch_bytes, double* d_grad, double* d_loss, qaoa_stream_t stream)
{
    qaoa_status_t s = mlp_check(batch, in_dim, hidden, out_dim);
    if (s != QAOA_OK) return s;
    if (!d_params || !d_x || !d_y || !d_act || !d_target || !d_scratch || !d_grad || !d_loss)
        return fail(QAOA_ERR_INVALID_ARG, "NULL pointer");
    const MlpDims d{in_dim, hidden, out_dim};
    if (scratch_bytes < mlp_scratch_bytes(batch, d))
        return fail(QAOA_ERR_WORKSPACE_TOO_SMALL, "scratch %zu bytes, need %zu", scratch_bytes,
                    mlp_scratch_bytes(batch, d));
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps("mlp_backward", st, 0.0);
    HIP_TRY(launch_mlp_backward(batch, d, d_params, d_x, d_y, d_act, d_target, (float*)d_scratch, d_grad, d_loss, st));
    return ok();
}

extern "C" qaoa_status_t qaoa_mlp_backward_noalloc(int32_t batch, int32_t in_dim, int32_t hidden, int32_t out_dim,
                                                   const double* d_params, const float* d_x, const float* d_y,
                                                   const float* d_act, const float* d_target, double* d_grad,
                                                   double* d_loss, qaoa_stream_t stream)
{
    qaoa_status_t s = mlp_check(batch, in_dim, hidden, out_dim);
    if (s != QAOA_OK) return s;
    if (!d_params || !d_x || !d_y || !d_act || !d_target || !d_grad || !d_loss)
        return fail(QAOA_ERR_INVALID_ARG, "NULL pointer");
    const MlpDims d{in_dim, hidden, out_dim};
    const size_t need = mlp_scratch_bytes(batch, d);
    if (need > MLP_STATIC_SCRATCH_BYTES)
        return fail(QAOA_ERR_OUT_OF_RANGE, "batch %d needs %zu bytes of scratch, more than the %zu the library holds",
                    batch, need, (size_t)MLP_STATIC_SCRATCH_BYTES);
    void* scr = nullptr;
    HIP_TRY(mlp_static_scratch(&scr));
    // (no timing scope: it may create events)
    HIP_TRY(launch_mlp_backward(batch, d, d_params, d_x, d_y, d_act, d_target, (float*)scr, d_grad, d_loss,
                                (hipStream_t)stream));
    return ok();
}

extern "C" qaoa_status_t qaoa_warm_angles(int32_t B, int32_t p, const float* d_y, const float* d_mu,
                                          const float* d_sd, double* d_theta, qaoa_stream_t stream)
{
    if (B < 1) return fail(QAOA_ERR_INVALID_ARG, "B = %d", B);
    if (p < 1 || p > MAX_P) return fail(QAOA_ERR_OUT_OF_RANGE, "p = %d outside 1..%d", p, MAX_P);
    if ((int64_t)2 * B * p > INT32_MAX) return fail(QAOA_ERR_OUT_OF_RANGE, "2 B p too large");
    if (!d_y || !d_mu || !d_sd || !d_theta) return fail(QAOA_ERR_INVALID_ARG, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps("warm_angles", st, (4.0 + 8.0) * 2.0 * B * p);
    HIP_TRY(launch_warm_angles(B, p, d_y, d_mu, d_sd, d_theta, st));
    return ok();
}

extern "C" qaoa_status_t qaoa_keep_better(int32_t B, int32_t p, const double* d_E_alt, const double* d_theta_alt,
                                          double* d_E, double* d_theta, qaoa_stream_t stream)
{
    if (B < 1) return fail(QAOA_ERR_INVALID_ARG, "B = %d", B);
    if (p < 1 || p > MAX_P) return fail(QAOA_ERR_OUT_OF_RANGE, "p = %d outside 1..%d", p, MAX_P);
    if ((int64_t)2 * B * p > INT32_MAX) return fail(QAOA_ERR_OUT_OF_RANGE, "2 B p too large");
    if (!d_E_alt || !d_theta_alt || !d_E || !d_theta) return fail(QAOA_ERR_INVALID_ARG, "NULL pointer");
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps("keep_better", st, 8.0 * 3.0 * B);
    HIP_TRY(launch_keep_better(B, p, d_E_alt, d_theta_alt, d_E, d_theta, st));
    return ok();
}
