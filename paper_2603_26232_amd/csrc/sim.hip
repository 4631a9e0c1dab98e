// Batched QAOA state-vector simulation for gfx950 (CDNA4, wave64).
//
// What is computed (paper Sec. 2.2 and 3.3): for every subgraph b of the
// partition, |psi_b> = U_M(beta_p) U_C(gamma_p) ... U_M(beta_1) U_C(gamma_1)
// |+>^n with U_C = e^{-i gamma H_C}, H_C = diag(C_b(z)) the subgraph's cut
// function, and U_M = prod_j (cos beta I - i sin beta X_j); then
// <C>_b = sum_z |psi_b(z)|^2 C_b(z) and, for the angle optimiser, the exact
// gradient by the adjoint sweep.
//
// How (MI355X design): the state of one subgraph (complex64, 2^n amplitudes)
// is processed in tiles of 2^12 amplitudes. Qubits are split into groups:
// group 0 = qubits 0..11 (a tile is 4096 contiguous amplitudes), groups 1..
// = up to 8 higher qubits each (a tile is 2^(12-nb) contiguous amplitudes
// times 2^nb strided rows). A workgroup keeps its tile in registers (16
// amplitudes per lane) and applies the RX rotations of 4 register-resident
// qubits at a time; between rounds the tile changes register layout through
// LDS. Consecutive layers visit the groups in alternating (serpentine) order,
// so the last group of layer l and the first group of layer l+1 share one
// HBM pass, with the diagonal phase of layer l+1 applied in registers from
// a precomputed integer cut table C(z) (uint16) and an FP64-built phase
// table e^{-i gamma c} rounded to complex64. <C> and the gradient inner
// products are accumulated in FP64 per tile and reduced per subgraph in a
// fixed order, so every result is bit-reproducible.
#include "common.h"

namespace pq {

// ---------------------------------------------------------------------------
// tile geometry
// ---------------------------------------------------------------------------
struct Geo {
    uint32_t zb;  // fixed z bits of this tile
    int c;        // passive low tile bits (contiguous amplitudes)
    int g0;       // first qubit of the group
    int nb;       // qubits in the group (active tile bits = [c, 12))
};

__device__ inline Geo group_geo(const SubDesc& d, int g, uint32_t t)
{
    Geo r;
    if (g == 0) {
        r.c = 0;
        r.g0 = 0;
        r.nb = TILE_BITS;
        r.zb = t << TILE_BITS;
    } else {
        r.nb = d.gsize[g];
        r.g0 = d.gstart[g];
        r.c = TILE_BITS - r.nb;
        const int L = r.g0 - r.c;  // fixed bits between the passive block and the group
        const uint32_t tlo = t & ((1u << L) - 1u), thi = t >> L;
        r.zb = (tlo << r.c) | (thi << (r.g0 + r.nb));
    }
    return r;
}

// tile position q -> z offset (bit deposit; zb supplies the fixed bits)
__device__ inline uint32_t gmap(const Geo& g, uint32_t q)
{
    return (q & ((1u << g.c) - 1u)) | ((q >> g.c) << g.g0);
}

// Register layouts of a 4096-amplitude tile over 256 lanes x 16 registers.
// LLIN: lanes = tile bits 0..7, registers = bits 8..11 (coalesced rows)
// LL0 : lanes = bits 4..11,    registers = bits 0..3
// LL1 : lanes = bits 0..3 and 8..11, registers = bits 4..7
enum { LLIN = 0, LL0 = 1, LL1 = 2 };

__device__ inline uint32_t thread_part(int L, uint32_t tid)
{
    return L == LLIN ? tid : (L == LL0 ? (tid << 4) : ((tid & 15u) | ((tid >> 4) << 8)));
}
__device__ inline uint32_t reg_part(int L, uint32_t r)
{
    return L == LLIN ? (r << 8) : (L == LL0 ? r : (r << 4));
}
__device__ inline int layout_bit0(int L) { return L == LLIN ? 8 : (L == LL0 ? 0 : 4); }
__device__ inline uint32_t lds_idx(uint32_t q) { return q + (q >> 4); }

// register bits whose tile bit is an active qubit of the group
__device__ inline unsigned active_mask(int L, int c)
{
    unsigned m = 0;
    const int b0 = layout_bit0(L);
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (b0 + k >= c) m |= 1u << k;
    return m;
}

struct Chain {
    int len;
    int l[3];
};

// layouts visited to bring every active tile bit into registers once
__device__ inline Chain group_chain(int g, int nb)
{
    Chain c;
    if (g == 0) {
        c.len = 3;
        c.l[0] = LLIN;
        c.l[1] = LL0;
        c.l[2] = LL1;
    } else if (nb >= 5) {
        c.len = 2;
        c.l[0] = LLIN;
        c.l[1] = LL1;
        c.l[2] = LL1;
    } else {
        c.len = 1;
        c.l[0] = c.l[1] = c.l[2] = LLIN;
    }
    return c;
}

__device__ inline void lds_write(float2* lds, int L, uint32_t tid, const float2 (&v)[REGS])
{
    const uint32_t tp = thread_part(L, tid);
#pragma unroll
    for (int r = 0; r < REGS; ++r) lds[lds_idx(tp | reg_part(L, r))] = v[r];
}

__device__ inline void lds_read(const float2* lds, int L, uint32_t tid, float2 (&v)[REGS])
{
    const uint32_t tp = thread_part(L, tid);
#pragma unroll
    for (int r = 0; r < REGS; ++r) v[r] = lds[lds_idx(tp | reg_part(L, r))];
}

__device__ inline void xchg(float2* lds, int from, int to, uint32_t tid, float2 (&v)[REGS])
{
    lds_write(lds, from, tid, v);
    __syncthreads();
    lds_read(lds, to, tid, v);
    __syncthreads();
}

// (a, b) <- (c a - i s b, -i s a + c b): e^{-i beta X} on one amplitude pair
// with c = cos beta, s = sin beta (s -> -s gives the inverse).
__device__ inline void rx_pair(float2& a, float2& b, float c, float s)
{
    const float2 na = make_float2(c * a.x + s * b.y, c * a.y - s * b.x);
    const float2 nb = make_float2(c * b.x + s * a.y, c * b.y - s * a.x);
    a = na;
    b = nb;
}

__device__ inline void rx_regs(float2 (&v)[REGS], unsigned mask, float c, float s)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (mask & (1u << k)) {
#pragma unroll
            for (int r = 0; r < REGS; ++r)
                if (!(r & (1 << k))) rx_pair(v[r], v[r | (1 << k)], c, s);
        }
    }
}

// sum over active register bits of Im conj(lam(z)) psi(z ^ bit), both ways
__device__ inline float xb_regs(const float2 (&ps)[REGS], const float2 (&la)[REGS], unsigned mask)
{
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (mask & (1u << k)) {
#pragma unroll
            for (int r = 0; r < REGS; ++r) {
                if (r & (1 << k)) continue;
                const int r1 = r | (1 << k);
                acc += la[r].x * ps[r1].y - la[r].y * ps[r1].x;
                acc += la[r1].x * ps[r].y - la[r1].y * ps[r].x;
            }
        }
    }
    return acc;
}

__device__ inline int cur_layout(const Chain& ch, bool at_start) { return at_start ? ch.l[0] : ch.l[ch.len - 1]; }

// RX of one layer on every qubit of the group, walking the layout chain from
// the current end to the other one.
__device__ inline void seg_fwd(float2 (&v)[REGS], float2* lds, const Chain& ch, bool& at_start, int c,
                               float cs, float sn, uint32_t tid)
{
    if (at_start) {
        for (int i = 0; i < ch.len; ++i) {
            if (i > 0) xchg(lds, ch.l[i - 1], ch.l[i], tid, v);
            rx_regs(v, active_mask(ch.l[i], c), cs, sn);
        }
    } else {
        for (int i = ch.len - 1; i >= 0; --i) {
            if (i < ch.len - 1) xchg(lds, ch.l[i + 1], ch.l[i], tid, v);
            rx_regs(v, active_mask(ch.l[i], c), cs, sn);
        }
    }
    at_start = !at_start;
}

// inverse RX on psi and lambda, accumulating the beta-gradient inner product
__device__ inline void seg_bwd(float2 (&ps)[REGS], float2 (&la)[REGS], float2* lds, const Chain& ch,
                               bool& at_start, int c, float cs, float sn, uint32_t tid, double& xacc)
{
    if (at_start) {
        for (int i = 0; i < ch.len; ++i) {
            if (i > 0) {
                xchg(lds, ch.l[i - 1], ch.l[i], tid, ps);
                xchg(lds, ch.l[i - 1], ch.l[i], tid, la);
            }
            const unsigned m = active_mask(ch.l[i], c);
            xacc += (double)xb_regs(ps, la, m);
            rx_regs(ps, m, cs, -sn);
            rx_regs(la, m, cs, -sn);
        }
    } else {
        for (int i = ch.len - 1; i >= 0; --i) {
            if (i < ch.len - 1) {
                xchg(lds, ch.l[i + 1], ch.l[i], tid, ps);
                xchg(lds, ch.l[i + 1], ch.l[i], tid, la);
            }
            const unsigned m = active_mask(ch.l[i], c);
            xacc += (double)xb_regs(ps, la, m);
            rx_regs(ps, m, cs, -sn);
            rx_regs(la, m, cs, -sn);
        }
    }
    at_start = !at_start;
}

__device__ inline float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// C(z) for the 16 amplitudes a lane holds in layout L. Group 0 reads the
// natural-order table, the last group its tile-order copy.
__device__ inline void load_cut(uint16_t (&cr)[REGS], const uint8_t* ws, const SubDesc& d, int g,
                                const Geo& geo, uint32_t t, int L, uint32_t tid)
{
    const uint32_t tp = thread_part(L, tid);
    const uint16_t* tab = (g == 0) ? (const uint16_t*)(ws + d.tab) + geo.zb
                                   : (const uint16_t*)(ws + d.tabB) + (size_t)t * TILE;
#pragma unroll
    for (int r = 0; r < REGS; ++r) cr[r] = tab[tp | reg_part(L, r)];
}

// deterministic block sum (wave64 butterfly, then the 4 wave totals in order)
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

__device__ inline uint32_t cut_of(uint32_t z, const int32_t* E, int ne)
{
    uint32_t c = 0;
    for (int e = 0; e < ne; ++e) {
        const int32_t u = E[3 * e], v = E[3 * e + 1], w = E[3 * e + 2];
        c += (((z >> u) ^ (z >> v)) & 1u) ? (uint32_t)w : 0u;
    }
    return c;
}

// ---------------------------------------------------------------------------
// K1: integer cut tables (natural order + tile order of the last group)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(THREADS) void k_cut_tables(uint8_t* ws, const SubDesc* subs, const int2* work)
{
    const int2 wk = work[blockIdx.x];
    const SubDesc d = subs[wk.x];
    const uint32_t t = (uint32_t)wk.y;
    const int32_t* E = (const int32_t*)(ws + d.edges);
    uint16_t* tab = (uint16_t*)(ws + d.tab);
    const uint32_t dim = 1u << d.n;
    const uint32_t span = dim < (uint32_t)TILE ? dim : (uint32_t)TILE;
    for (uint32_t q = threadIdx.x; q < span; q += THREADS) {
        const uint32_t z = t * TILE + q;
        tab[z] = (uint16_t)cut_of(z, E, d.nedges);
        if (d.ngroups >= 2) {
            const Geo geo = group_geo(d, d.ngroups - 1, t);
            uint16_t* tabB = (uint16_t*)(ws + d.tabB);
            tabB[(size_t)t * TILE + q] = (uint16_t)cut_of(geo.zb | gmap(geo, q), E, d.nedges);
        }
    }
}

// ---------------------------------------------------------------------------
// K2: angle preparation. LUT[c] = e^{-i gamma c} from an FP64 product and
// FP64 sine/cosine, rounded to complex64; (cos beta, sin beta) as float.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(THREADS) void k_angle_prep(uint8_t* ws, const SubDesc* subs, int p,
                                                        const double* gamma, const double* beta)
{
    const int b = blockIdx.x / p, l = blockIdx.x % p;
    const SubDesc d = subs[b];
    const double gm = gamma[(size_t)b * p + l];
    float2* lut = (float2*)(ws + d.lut) + (size_t)l * d.lut_len;
    for (int c = threadIdx.x; c < d.lut_len; c += THREADS) {
        double sv, cv;
        sincos(gm * (double)c, &sv, &cv);
        lut[c] = make_float2((float)cv, (float)(-sv));
    }
    if (threadIdx.x == 0) {
        const double bt = beta[(size_t)b * p + l];
        ((float2*)(ws + d.coef))[l] = make_float2((float)cos(bt), (float)sin(bt));
    }
}

// ---------------------------------------------------------------------------
// Forward tile pass: [init | load] RX(pre) phase(ph) RX(post) [<C> partial] store
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(THREADS) void k_fwd_pass(uint8_t* ws, const SubDesc* subs, const int2* work,
                                                      PassOps ops, Partials part)
{
    extern __shared__ float2 smem[];
    float2* lds = smem;
    float2* lut = smem + LDS_TILE;
    __shared__ double red[THREADS / 64];
    const uint32_t tid = threadIdx.x;
    const int2 wk = work[blockIdx.x];
    const SubDesc d = subs[wk.x];
    const uint32_t t = (uint32_t)wk.y;
    const int g = ops.group;
    const Geo geo = group_geo(d, g, t);
    const Chain ch = group_chain(g, geo.nb);
    float2* st = (float2*)(ws + d.psi);
    const float2* coef = (const float2*)(ws + d.coef);

    if (ops.ph >= 0) {
        const float2* L = (const float2*)(ws + d.lut) + (size_t)ops.ph * d.lut_len;
        for (int i = tid; i < d.lut_len; i += THREADS) lut[i] = L[i];
    }
    const int nseg = (ops.pre >= 0) + (ops.post >= 0);
    uint16_t cr[REGS];
    if (ops.ph >= 0 || ops.epi_e) {
        // the phase comes after RX(pre); <C> after all segments
        const bool at_end = (ops.ph >= 0) ? (ops.pre >= 0) : (nseg & 1);
        load_cut(cr, ws, d, g, geo, t, at_end ? ch.l[ch.len - 1] : ch.l[0], tid);
    }
    float2 v[REGS];
    {
        const uint32_t base = geo.zb | gmap(geo, thread_part(LLIN, tid));
        if (ops.init) {
            const float a = (float)(1.0 / sqrt((double)(1ull << d.n)));
#pragma unroll
            for (int r = 0; r < REGS; ++r) v[r] = make_float2(a, 0.f);
        } else {
#pragma unroll
            for (int r = 0; r < REGS; ++r) v[r] = st[base | gmap(geo, reg_part(LLIN, r))];
        }
    }
    __syncthreads();  // phase table staged
    bool at_start = true;
    if (ops.pre >= 0) {
        const float2 cf = coef[ops.pre];
        seg_fwd(v, lds, ch, at_start, geo.c, cf.x, cf.y, tid);
    }
    if (ops.ph >= 0) {
#pragma unroll
        for (int r = 0; r < REGS; ++r) v[r] = cmul(v[r], lut[cr[r]]);
    }
    if (ops.post >= 0) {
        const float2 cf = coef[ops.post];
        seg_fwd(v, lds, ch, at_start, geo.c, cf.x, cf.y, tid);
    }
    if (ops.epi_e) {
        double acc = 0.0;
#pragma unroll
        for (int r = 0; r < REGS; ++r)
            acc += ((double)v[r].x * v[r].x + (double)v[r].y * v[r].y) * (double)cr[r];
        acc = block_sum(acc, red);
        if (tid == 0) part.e[d.tile_base + t] = acc;
    }
    const int L = cur_layout(ch, at_start);
    const uint32_t base = geo.zb | gmap(geo, thread_part(L, tid));
#pragma unroll
    for (int r = 0; r < REGS; ++r) st[base | gmap(geo, reg_part(L, r))] = v[r];
}

// ---------------------------------------------------------------------------
// Backward tile pass (adjoint sweep) on psi and lambda = C psi_p.
// fused: RX(pre) on psi, <C> partial, lambda = C psi, then the inverse of
//        RX(pre) on both with the beta-gradient; only lambda is stored
//        (psi in memory already is the state before RX(pre)).
// else : unmix(pre) + beta-grad, gamma-grad + unphase(ph), unmix(post) +
//        beta-grad; store both unless this is the last pass.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(THREADS) void k_bwd_pass(uint8_t* ws, const SubDesc* subs, const int2* work,
                                                      PassOps ops, Partials part)
{
    extern __shared__ float2 smem[];
    float2* lds = smem;
    float2* lut = smem + LDS_TILE;
    __shared__ double red[THREADS / 64];
    const uint32_t tid = threadIdx.x;
    const int2 wk = work[blockIdx.x];
    const SubDesc d = subs[wk.x];
    const uint32_t t = (uint32_t)wk.y;
    const int g = ops.group;
    const Geo geo = group_geo(d, g, t);
    const Chain ch = group_chain(g, geo.nb);
    float2* sp = (float2*)(ws + d.psi);
    float2* sl = (float2*)(ws + d.lam);
    const float2* coef = (const float2*)(ws + d.coef);
    const int T = part.total_tiles;
    const int tile = d.tile_base + (int)t;

    if (ops.ph >= 0 && !ops.last) {
        const float2* L = (const float2*)(ws + d.lut) + (size_t)ops.ph * d.lut_len;
        for (int i = tid; i < d.lut_len; i += THREADS) lut[i] = L[i];
    }
    uint16_t cr[REGS];
    if (ops.fused || ops.ph >= 0) load_cut(cr, ws, d, g, geo, t, ch.l[ch.len - 1], tid);

    float2 ps[REGS], la[REGS];
    {
        const uint32_t base = geo.zb | gmap(geo, thread_part(LLIN, tid));
#pragma unroll
        for (int r = 0; r < REGS; ++r) ps[r] = sp[base | gmap(geo, reg_part(LLIN, r))];
        if (!ops.fused) {
#pragma unroll
            for (int r = 0; r < REGS; ++r) la[r] = sl[base | gmap(geo, reg_part(LLIN, r))];
        }
    }
    __syncthreads();
    bool at_start = true;
    double acc_pre = 0.0, acc_ph = 0.0, acc_post = 0.0, acc_e = 0.0;
    if (ops.fused) {
        const float2 cf = coef[ops.pre];
        seg_fwd(ps, lds, ch, at_start, geo.c, cf.x, cf.y, tid);
#pragma unroll
        for (int r = 0; r < REGS; ++r) {
            const float c = (float)cr[r];
            acc_e += ((double)ps[r].x * ps[r].x + (double)ps[r].y * ps[r].y) * (double)cr[r];
            la[r] = make_float2(c * ps[r].x, c * ps[r].y);
        }
        seg_bwd(ps, la, lds, ch, at_start, geo.c, cf.x, cf.y, tid, acc_pre);
    } else {
        if (ops.pre >= 0) {
            const float2 cf = coef[ops.pre];
            seg_bwd(ps, la, lds, ch, at_start, geo.c, cf.x, cf.y, tid, acc_pre);
        }
        if (ops.ph >= 0) {
            float a = 0.f;
#pragma unroll
            for (int r = 0; r < REGS; ++r)
                a += (float)cr[r] * (la[r].x * ps[r].y - la[r].y * ps[r].x);
            acc_ph = (double)a;
            if (!ops.last) {
#pragma unroll
                for (int r = 0; r < REGS; ++r) {
                    float2 f = lut[cr[r]];
                    f.y = -f.y;
                    ps[r] = cmul(ps[r], f);
                    la[r] = cmul(la[r], f);
                }
            }
        }
        if (ops.post >= 0) {
            const float2 cf = coef[ops.post];
            seg_bwd(ps, la, lds, ch, at_start, geo.c, cf.x, cf.y, tid, acc_post);
        }
    }
    // partial sums (every thread takes part in each block_sum)
    if (ops.fused) {
        const double e = block_sum(acc_e, red);
        const double x = block_sum(acc_pre, red);
        if (tid == 0) {
            part.e[tile] = e;
            part.gb[((size_t)ops.pre * MAX_GROUPS + g) * T + tile] = x;
        }
    } else {
        if (ops.pre >= 0) {
            const double x = block_sum(acc_pre, red);
            if (tid == 0) part.gb[((size_t)ops.pre * MAX_GROUPS + g) * T + tile] = x;
        }
        if (ops.ph >= 0) {
            const double x = block_sum(acc_ph, red);
            if (tid == 0) part.gg[(size_t)ops.ph * T + tile] = x;
        }
        if (ops.post >= 0) {
            const double x = block_sum(acc_post, red);
            if (tid == 0) part.gb[((size_t)ops.post * MAX_GROUPS + g) * T + tile] = x;
        }
    }
    if (ops.last) return;
    const int L = cur_layout(ch, at_start);
    const uint32_t base = geo.zb | gmap(geo, thread_part(L, tid));
    if (!ops.fused) {
#pragma unroll
        for (int r = 0; r < REGS; ++r) sp[base | gmap(geo, reg_part(L, r))] = ps[r];
    }
#pragma unroll
    for (int r = 0; r < REGS; ++r) sl[base | gmap(geo, reg_part(L, r))] = la[r];
}

// ---------------------------------------------------------------------------
// Subgraphs with n <= 12: one workgroup runs the whole circuit (and, with
// grad, the whole adjoint sweep) in LDS, one qubit at a time.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(THREADS) void k_small(uint8_t* ws, const SubDesc* subs, const int32_t* list,
                                                   int p, int grad, Partials part)
{
    extern __shared__ float2 smem[];
    __shared__ double red[THREADS / 64];
    const uint32_t tid = threadIdx.x;
    const SubDesc d = subs[list[blockIdx.x]];
    const int n = d.n;
    const uint32_t dim = 1u << n, half = dim >> 1;
    float2* ps = smem;
    float2* la = smem + TILE;
    float2* lut = smem + (grad ? 2 * TILE : TILE);
    const uint16_t* tab = (const uint16_t*)(ws + d.tab);
    const float2* coef = (const float2*)(ws + d.coef);
    const float2* luts = (const float2*)(ws + d.lut);
    const int T = part.total_tiles;
    const int tile = d.tile_base;

    const float a0 = (float)(1.0 / sqrt((double)dim));
    for (uint32_t z = tid; z < dim; z += THREADS) ps[z] = make_float2(a0, 0.f);
    for (int l = 0; l < p; ++l) {
        __syncthreads();
        for (int i = tid; i < d.lut_len; i += THREADS) lut[i] = luts[(size_t)l * d.lut_len + i];
        __syncthreads();
        for (uint32_t z = tid; z < dim; z += THREADS) ps[z] = cmul(ps[z], lut[tab[z]]);
        const float2 cf = coef[l];
        for (int j = 0; j < n; ++j) {
            __syncthreads();
            for (uint32_t i = tid; i < half; i += THREADS) {
                const uint32_t z = ((i >> j) << (j + 1)) | (i & ((1u << j) - 1u));
                rx_pair(ps[z], ps[z | (1u << j)], cf.x, cf.y);
            }
        }
    }
    __syncthreads();
    double acc = 0.0;
    for (uint32_t z = tid; z < dim; z += THREADS)
        acc += ((double)ps[z].x * ps[z].x + (double)ps[z].y * ps[z].y) * (double)tab[z];
    acc = block_sum(acc, red);
    if (tid == 0) part.e[tile] = acc;
    if (!grad) {
        float2* st = (float2*)(ws + d.psi);
        for (uint32_t z = tid; z < dim; z += THREADS) st[z] = ps[z];
        return;
    }
    for (uint32_t z = tid; z < dim; z += THREADS) {
        const float c = (float)tab[z];
        la[z] = make_float2(c * ps[z].x, c * ps[z].y);
    }
    for (int l = p - 1; l >= 0; --l) {
        const float2 cf = coef[l];
        double xb = 0.0;
        for (int j = 0; j < n; ++j) {
            __syncthreads();
            float a = 0.f;
            for (uint32_t i = tid; i < half; i += THREADS) {
                const uint32_t z = ((i >> j) << (j + 1)) | (i & ((1u << j) - 1u));
                const uint32_t z1 = z | (1u << j);
                a += la[z].x * ps[z1].y - la[z].y * ps[z1].x;
                a += la[z1].x * ps[z].y - la[z1].y * ps[z].x;
                rx_pair(ps[z], ps[z1], cf.x, -cf.y);
                rx_pair(la[z], la[z1], cf.x, -cf.y);
            }
            xb += (double)a;
        }
        __syncthreads();
        xb = block_sum(xb, red);
        if (tid == 0) part.gb[((size_t)l * MAX_GROUPS + 0) * T + tile] = xb;
        double gg = 0.0;
        for (uint32_t z = tid; z < dim; z += THREADS)
            gg += (double)((float)tab[z] * (la[z].x * ps[z].y - la[z].y * ps[z].x));
        gg = block_sum(gg, red);
        if (tid == 0) part.gg[(size_t)l * T + tile] = gg;
        if (l > 0) {
            for (int i = tid; i < d.lut_len; i += THREADS) lut[i] = luts[(size_t)l * d.lut_len + i];
            __syncthreads();
            for (uint32_t z = tid; z < dim; z += THREADS) {
                float2 f = lut[tab[z]];
                f.y = -f.y;
                ps[z] = cmul(ps[z], f);
                la[z] = cmul(la[z], f);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// K5: per-subgraph fixed-order reduction of the tile partials.
// dE/dgamma = 2 sum gg, dE/dbeta = 2 sum gb (the factor 2 of 2 Im <.|.|.>).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(THREADS) void k_reduce(const SubDesc* subs, int p, int grad, Partials part,
                                                    double* E, double* dgamma, double* dbeta)
{
    __shared__ double red[THREADS / 64];
    const int b = blockIdx.x;
    const SubDesc d = subs[b];
    const int T = part.total_tiles, tb = d.tile_base, nt = d.ntiles;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nt; i += THREADS) acc += part.e[tb + i];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0 && E) E[b] = acc;
    if (!grad) return;
    for (int l = 0; l < p; ++l) {
        double xb = 0.0;
        for (int g = 0; g < d.ngroups; ++g)
            for (int i = threadIdx.x; i < nt; i += THREADS)
                xb += part.gb[((size_t)l * MAX_GROUPS + g) * T + tb + i];
        xb = block_sum(xb, red);
        double gg = 0.0;
        for (int i = threadIdx.x; i < nt; i += THREADS) gg += part.gg[(size_t)l * T + tb + i];
        gg = block_sum(gg, red);
        if (threadIdx.x == 0) {
            dbeta[(size_t)b * p + l] = 2.0 * xb;
            dgamma[(size_t)b * p + l] = 2.0 * gg;
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_cut_tables(uint8_t* ws, const SubDesc* subs, const int2* work, int nwork, hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cut_tables, dim3(nwork), dim3(THREADS), 0, s, ws, subs, work);
    return hipGetLastError();
}

hipError_t launch_angle_prep(uint8_t* ws, const SubDesc* subs, int B, int p, const double* gamma,
                             const double* beta, hipStream_t s)
{
    hipLaunchKernelGGL(k_angle_prep, dim3(B * p), dim3(THREADS), 0, s, ws, subs, p, gamma, beta);
    return hipGetLastError();
}

static size_t pass_lds(int lut_max) { return (size_t)(LDS_TILE + lut_max) * sizeof(float2); }

hipError_t launch_fwd_pass(uint8_t* ws, const SubDesc* subs, const int2* work, int nwork, PassOps ops,
                           Partials part, int lut_max, hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fwd_pass, dim3(nwork), dim3(THREADS), pass_lds(lut_max), s, ws, subs, work, ops,
                       part);
    return hipGetLastError();
}

hipError_t launch_bwd_pass(uint8_t* ws, const SubDesc* subs, const int2* work, int nwork, PassOps ops,
                           Partials part, int lut_max, hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bwd_pass, dim3(nwork), dim3(THREADS), pass_lds(lut_max), s, ws, subs, work, ops,
                       part);
    return hipGetLastError();
}

hipError_t launch_small(uint8_t* ws, const SubDesc* subs, const int32_t* list, int nlist, int p, int grad,
                        Partials part, int lut_max, hipStream_t s)
{
    if (nlist <= 0) return hipSuccess;
    const size_t lds = (size_t)((grad ? 2 : 1) * TILE + lut_max) * sizeof(float2);
    hipLaunchKernelGGL(k_small, dim3(nlist), dim3(THREADS), lds, s, ws, subs, list, p, grad, part);
    return hipGetLastError();
}

hipError_t launch_reduce(const SubDesc* subs, int B, int p, int grad, Partials part, double* E,
                         double* dgamma, double* dbeta, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce, dim3(B), dim3(THREADS), 0, s, subs, p, grad, part, E, dgamma, dbeta);
    return hipGetLastError();
}

}  // namespace pq
