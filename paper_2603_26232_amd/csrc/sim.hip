// Batched QAOA state-vector simulation for gfx950 (CDNA4, wave64).
//
// What is computed (paper Sec. 2.2 and 3.3): for every subgraph b of the
// partition, |psi_b> = U_M(beta_p) U_C(gamma_p) ... U_M(beta_1) U_C(gamma_1)
// |+>^n with U_C = e^{-i gamma H_C}, H_C = diag(C_b(z)) the subgraph's cut
// function, and U_M = prod_j (cos beta I - i sin beta X_j); then
// <C>_b = sum_z |psi_b(z)|^2 C_b(z) and, for the angle optimiser, the exact
// gradient by the adjoint sweep.
//
// How (MI355X design): the state is invariant under flipping every bit
// (C(~z) = C(z); X on every qubit commutes with both operators and fixes
// |+>), so only the 2^(n-1) amplitudes with the top bit clear are stored,
// scaled by sqrt(2); on them the top qubit's X maps an index to its
// complement. The stored state is processed in tiles of 2^12 amplitudes.
// Qubits are split into groups: group 0 = qubits 0..10 plus the top qubit (a
// tile is a block of 2048 contiguous amplitudes and its mirror block, tile
// bit 11 choosing between them), groups 1.. = up to 8 of the qubits 11..n-2
// each (a tile is 2^(12-nb) contiguous amplitudes times 2^nb strided rows). A workgroup keeps its tile in registers (16
// amplitudes per lane) and applies the rotations of 4 register-resident
// qubits at a time; between rounds the tile changes register layout through
// LDS. Consecutive layers visit the groups in alternating (serpentine) order,
// so the last group of layer l and the first group of layer l+1 share one
// HBM pass, with the diagonal phase of layer l+1 applied in registers from
// a precomputed integer cut table C(z) (1 byte per entry when the weight sum
// is at most 255, else 2) and an FP64-built phase table e^{-i gamma c}
// rounded to complex64. <C> and the gradient inner products are accumulated
// in FP64 per tile and reduced per subgraph in a fixed order, so every result
// is bit-reproducible.
//
// Rotation arithmetic: e^{-i beta X} = f (I - i t X) X^flip with (f, t, flip)
// = (cos beta, tan beta, 0) when |cos| >= |sin|, else (-i sin beta,
// -cot beta, 1), so |t| <= 1. The bracketed operator costs two FMAs per real
// component; the per-qubit factor f of a whole group is applied once per
// segment, folded into the next phase multiply when there is one; the X^flip
// permutation is never executed but carried as an XOR mask on tile positions
// into cut-table reads and store addresses. Gradient inner products taken on
// scaled states are rescaled by the known |f|^2 powers.
#include "common.h"

// Occupancy targets of the tile passes (waves per SIMD): the register budget
// the compiler may use is 512 / target VGPRs per lane.
#ifndef PQ_FWD_WAVES
#define PQ_FWD_WAVES 4
#endif
#ifndef PQ_BWD_WAVES
#define PQ_BWD_WAVES 2
#endif
#ifndef PQ_MF_WAVES
#define PQ_MF_WAVES 3
#endif

namespace pq {

// ---------------------------------------------------------------------------
// tile geometry
// ---------------------------------------------------------------------------
struct Geo {
    uint32_t zb;   // fixed index bits of this tile
    int c;         // passive low tile bits (contiguous amplitudes)
    int g0;        // first qubit of the group
    int nb;        // qubits in the group (active tile bits = [c, 12))
    uint32_t mir;  // group 0: 2^(n-1) - 1 (the complement of a reduced index)
};

// tile position q -> z offset (bit deposit; zb supplies the fixed bits)
__device__ inline uint32_t gmap(const Geo& g, uint32_t q)
{
    return (q & ((1u << g.c) - 1u)) | ((q >> g.c) << g.g0);
}

// Group 0 tiles pair a block of 2048 reduced indices with its mirror block:
// tile bits 0..10 are qubits 0..10 and tile bit 11 selects the block or its
// complement (index XOR 2^(n-1) - 1). In the reduced state the top qubit's
// X maps an index to its complement, so it acts on tile bit 11 like any other
// qubit on its bit. The map is XOR-linear, as the deposit of the other groups.
__device__ inline uint32_t gmap0(const Geo& g, uint32_t q)
{
    return (q & ((1u << HALF_BITS) - 1u)) ^ ((q >> HALF_BITS) & 1u ? g.mir : 0u);
}

template <bool G0>
__device__ inline uint32_t gmapT(const Geo& g, uint32_t q)
{
    if constexpr (G0) return gmap0(g, q);
    else return gmap(g, q);
}

// Register layouts of a 4096-amplitude tile over 256 lanes x 16 registers.
// LLIN: lanes = tile bits 0..7, registers = bits 8..11 (coalesced rows)
// LL0 : lanes = bits 4..11,    registers = bits 0..3
// LL1 : lanes = bits 0..3 and 8..11, registers = bits 4..7
enum { LLIN = 0, LL0 = 1, LL1 = 2 };

template <int L>
__device__ inline uint32_t thread_part(uint32_t tid)
{
    return L == LLIN ? tid : (L == LL0 ? (tid << 4) : ((tid & 15u) | ((tid >> 4) << 8)));
}
template <int L>
__host__ __device__ constexpr uint32_t reg_part(uint32_t r)
{
    return L == LLIN ? (r << 8) : (L == LL0 ? r : (r << 4));
}
template <int L>
__host__ __device__ constexpr int layout_bit0()
{
    return L == LLIN ? 8 : (L == LL0 ? 0 : 4);
}
// padded LDS slot; lds_idx(a | b) = lds_idx(a) + lds_idx(b) for disjoint bits
__host__ __device__ constexpr uint32_t lds_idx(uint32_t q) { return q + (q >> 4); }

// register bits whose tile bit is an active qubit of the group
template <int L>
__device__ inline unsigned active_mask(int c)
{
    unsigned m = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (layout_bit0<L>() + k >= c) m |= 1u << k;
    return m;
}

// Layout chains per group shape: CH = 3 (group 0: every tile bit active),
// 2 (a high group of 5..8 qubits), 1 (a high group of at most 4 qubits).
template <int CH, int I>
struct ChainAt {
    static constexpr int L = (CH == 3) ? (I == 0 ? LLIN : (I == 1 ? LL0 : LL1)) : (CH == 2 ? (I == 0 ? LLIN : LL1) : LLIN);
};

template <int L>
__device__ inline void lds_write(float2* lds, uint32_t tid, const float2 (&v)[REGS])
{
    float2* p = lds + lds_idx(thread_part<L>(tid));
#pragma unroll
    for (int r = 0; r < REGS; ++r) p[lds_idx(reg_part<L>(r))] = v[r];
}

template <int L>
__device__ inline void lds_read(const float2* lds, uint32_t tid, float2 (&v)[REGS])
{
    const float2* p = lds + lds_idx(thread_part<L>(tid));
#pragma unroll
    for (int r = 0; r < REGS; ++r) v[r] = p[lds_idx(reg_part<L>(r))];
}

// LL0 and LL1 place the same 1024 amplitudes in each wave (thread bits 6, 7
// are tile bits 10, 11 in both), so an exchange between them stays inside the
// wave and needs no workgroup barrier: the LDS performs one wave's operations
// in the order the wave issues them, so it is enough that the compiler keeps
// the reads after the writes and the next writes after the reads. Every other
// exchange moves data between waves.
template <int LF, int LT>
__host__ __device__ constexpr bool wave_local()
{
    return (LF == LL0 && LT == LL1) || (LF == LL1 && LT == LL0);
}

__device__ inline void wave_lds_order() { asm volatile("" ::: "memory"); }

// LEAD: a barrier before the writes, for a workgroup exchange that follows a
// wave-local one (other waves may still read their slots). The chains only
// leave LL0 for LLIN after arriving from LL1, hence the default.
template <int LF, int LT, bool LEAD = (LF == LL0 && LT == LLIN)>
__device__ inline void xchg(float2* lds, uint32_t tid, float2 (&v)[REGS])
{
    if constexpr (wave_local<LF, LT>()) {
        lds_write<LF>(lds, tid, v);
        wave_lds_order();
        lds_read<LT>(lds, tid, v);
        wave_lds_order();
    } else {
        if constexpr (LEAD) __syncthreads();
        lds_write<LF>(lds, tid, v);
        __syncthreads();
        lds_read<LT>(lds, tid, v);
        __syncthreads();
    }
    __builtin_amdgcn_sched_barrier(0);
}

// Reduced pair rotation (I - i t X) on (a, b) = (psi(z), psi(z ^ bit)):
// (a, b) -> (a - i t b, b - i t a). t = 0 is exactly the identity.
__device__ inline void rx_tan(float2& a, float2& b, float t)
{
    const float2 na = make_float2(a.x + t * b.y, a.y - t * b.x);
    const float2 nb = make_float2(b.x + t * a.y, b.y - t * a.x);
    a = na;
    b = nb;
}

template <int K>
__device__ inline void rx_bit(float2 (&v)[REGS], float t)
{
#pragma unroll
    for (int r = 0; r < REGS; ++r)
        if (!(r & (1 << K))) rx_tan(v[r], v[r | (1 << K)], t);
}

// one round: the four register bits with their own coefficients (0 for a
// register bit that is not an active qubit of the group)
__device__ inline void rx_round(float2 (&v)[REGS], const float (&tk)[4])
{
    rx_bit<0>(v, tk[0]);
    rx_bit<1>(v, tk[1]);
    rx_bit<2>(v, tk[2]);
    rx_bit<3>(v, tk[3]);
}

// sum over one register bit of Im conj(lam(z)) psi(z ^ bit), both directions,
// as FMA chains into two accumulators
template <int K>
__device__ inline float xb_bit(const float2 (&ps)[REGS], const float2 (&la)[REGS])
{
    float a0 = 0.f, a1 = 0.f;
#pragma unroll
    for (int r = 0; r < REGS; ++r) {
        if (r & (1 << K)) continue;
        const int r1 = r | (1 << K);
        a0 = fmaf(la[r].x, ps[r1].y, a0);
        a0 = fmaf(-la[r].y, ps[r1].x, a0);
        a1 = fmaf(la[r1].x, ps[r].y, a1);
        a1 = fmaf(-la[r1].y, ps[r].x, a1);
    }
    return a0 + a1;
}

__device__ inline float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ inline void scale_regs(float2 (&v)[REGS], float2 f)
{
#pragma unroll
    for (int r = 0; r < REGS; ++r) v[r] = cmul(v[r], f);
}

// Per-layer rotation parameters (built in FP64 by the angle-prep kernel):
// e^{-i beta X} = f (I - i t X) X^flip per qubit.
struct RxC {
    float t;
    int flip;
    float fsq;      // |f|^2
    float2 Ff, Fi;  // f^(group size), forward and inverse
};

__device__ inline RxC load_rx(const RxCoef* cf, int l, int g)
{
    RxC r;
    r.t = cf[l].t;
    r.flip = cf[l].mode;
    r.fsq = cf[l].fsq;
    r.Ff = cf[l].Ff[g];
    r.Fi = cf[l].Fi[g];
    return r;
}

// FULL: every register bit of every layout in the chain is an active qubit
// (group 0, and high groups of exactly 4 or 8 qubits); then no per-bit
// selection is needed.
template <int L, bool FULL>
__device__ inline void round_coef(float (&tk)[4], float t, int c)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) tk[k] = (FULL || layout_bit0<L>() + k >= c) ? t : 0.f;
}

// Tile bits of the group's qubits (the ones a flip permutes).
__device__ inline uint32_t group_bits(int c) { return ((uint32_t)TILE - 1u) & ~((1u << c) - 1u); }

// ---------------------------------------------------------------------------
// Mixer block on the matrix cores (precision modes). In layout LL0 a wave
// holds 32 blocks of 32 amplitudes: registers = tile bits 0..3, lane bit 5 =
// tile bit 9, lane bits 0..4 = the block index (tile bits 4..8). The reduced
// rotation of those five qubits, U = prod_j (I - i t X_j), is one dense 32 x 32
// complex matrix with U[a'][a] = (-i t)^popcount(a' ^ a); as a real 64 x 64
// matrix [[Re U, -Im U], [Im U, Re U]] it multiplies the 64 x 32 real block
// matrix of the wave. The output rows are numbered so that the accumulator
// layout of a 32 x 32 MFMA tile (lane L, register r holds row
// 8 (r / 4) + 4 (L / 32) + r % 4 of column L % 32) is again layout LL0.
// PREC 1: FP32 MFMA (32x32x2). PREC 2: BF16 MFMA (32x32x16) on hi/lo splits,
// x = hi + lo, of both operands, keeping the hi*hi, hi*lo and lo*hi products.
// PREC 3: as 2, but the block matrix is split in three BF16 terms (hi + mid +
// lo, exact to FP32 rounding) and the products are hi*hi, hi*lo, mid*hi and
// lo*hi: the rounding of the constant block then no longer makes it
// measurably non-unitary (the two-term split changes the norm by ~1e-6 per
// application, the same sign every time).
// ---------------------------------------------------------------------------
enum { PREC_VALU = 0, PREC_MFMA_F32 = 1, PREC_MFMA_BF16X3 = 2, PREC_MFMA_BF16X4 = 3 };

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ inline uint16_t bf16_bits(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
    return (uint16_t)(u >> 16);
}
__device__ inline float bf16_value(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ inline void split_bf16(float x, __bf16& hi, __bf16& lo)
{
    const uint16_t h = bf16_bits(x);
    hi = __builtin_bit_cast(__bf16, h);
    lo = __builtin_bit_cast(__bf16, bf16_bits(x - bf16_value(h)));
}

template <int PREC>
__device__ inline void mfma_block(float2 (&v)[REGS], float t, uint32_t tid)
{
    const uint32_t lane = tid & 63u;
    const uint32_t i = lane & 31u, h = lane >> 5;
    // output amplitude of A row i: a' = (4 (i / 8) + i % 4) | ((i / 4) % 2) << 4
    const uint32_t arow = (4u * (i >> 3) + (i & 3u)) | (((i >> 2) & 1u) << 4);
    const float t2 = t * t, t3 = t2 * t, t4 = t2 * t2, t5 = t4 * t;
    // Re U and Im U of row arow, column a = s | h << 4, s = 0..15
    float ure[16], uim[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int d = __popc(arow ^ ((uint32_t)s | (h << 4)));
        // (-i t)^d = 1, -i t, -t^2, i t^3, t^4, -i t^5
        const float w = d == 0 ? 1.f : d == 1 ? -t : d == 2 ? -t2 : d == 3 ? t3 : d == 4 ? t4 : -t5;
        ure[s] = (d & 1) ? 0.f : w;
        uim[s] = (d & 1) ? w : 0.f;
    }
    floatx16 re = {0.f}, im = {0.f};
    if constexpr (PREC == PREC_MFMA_F32) {
        // K row (2 s + h) of step s < 16 is Re psi(a), of step s + 16 Im psi(a)
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            re = __builtin_amdgcn_mfma_f32_32x32x2f32(ure[s], v[s].x, re, 0, 0, 0);
            im = __builtin_amdgcn_mfma_f32_32x32x2f32(uim[s], v[s].x, im, 0, 0, 0);
        }
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            re = __builtin_amdgcn_mfma_f32_32x32x2f32(-uim[s], v[s].y, re, 0, 0, 0);
            im = __builtin_amdgcn_mfma_f32_32x32x2f32(ure[s], v[s].y, im, 0, 0, 0);
        }
    } else {
        // step q (0..3): K rows 16 q + 8 h + e, e = 0..7, hold component q / 2
        // of psi(a), a = 8 (q % 2) + e | h << 4
        constexpr bool X4 = PREC == PREC_MFMA_BF16X4;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = q >> 1, o = 8 * (q & 1);
            bf16x8 bh, bl, rh, rm, rl, ih, im_, il;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                __bf16 x, y;
                split_bf16(c ? v[o + e].y : v[o + e].x, x, y);
                bh[e] = x;
                bl[e] = y;
                const float ar = c ? -uim[o + e] : ure[o + e];
                const float ai = c ? ure[o + e] : uim[o + e];
                split_bf16(ar, x, y);
                rh[e] = x;
                rm[e] = y;
                if constexpr (X4) {
                    const float rest = (ar - bf16_value(__builtin_bit_cast(uint16_t, x))) -
                                       bf16_value(__builtin_bit_cast(uint16_t, y));
                    rl[e] = __builtin_bit_cast(__bf16, bf16_bits(rest));
                }
                split_bf16(ai, x, y);
                ih[e] = x;
                im_[e] = y;
                if constexpr (X4) {
                    const float rest = (ai - bf16_value(__builtin_bit_cast(uint16_t, x))) -
                                       bf16_value(__builtin_bit_cast(uint16_t, y));
                    il[e] = __builtin_bit_cast(__bf16, bf16_bits(rest));
                }
            }
            // smallest terms first
            if constexpr (X4) re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rl, bh, re, 0, 0, 0);
            re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rm, bh, re, 0, 0, 0);
            re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rh, bl, re, 0, 0, 0);
            re = __builtin_amdgcn_mfma_f32_32x32x16_bf16(rh, bh, re, 0, 0, 0);
            if constexpr (X4) im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(il, bh, im, 0, 0, 0);
            im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(im_, bh, im, 0, 0, 0);
            im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ih, bl, im, 0, 0, 0);
            im = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ih, bh, im, 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < REGS; ++r) v[r] = make_float2(re[r], im[r]);
}

// One rotation round in layout L. With a matrix-core mode, group 0 (CH 3)
// rotates tile bits 0..3 and 9 by mfma_block in LL0 and leaves bit 9
// (register bit 1 of LLIN) out of the LLIN round.
template <int CH, int L, bool FULL, int PREC>
__device__ inline void rot_round(float2 (&v)[REGS], int c, float t, uint32_t tid)
{
    if constexpr (PREC != PREC_VALU && CH == 3 && L == LL0) {
        mfma_block<PREC>(v, t, tid);
    } else {
        float tk[4];
        round_coef<L, FULL>(tk, t, c);
        if constexpr (PREC != PREC_VALU && CH == 3 && L == LLIN) tk[1] = 0.f;
        rx_round(v, tk);
    }
}

// One RX segment (all qubits of the group, one layer) walking the layout
// chain in direction DIR (true: start -> end), coefficient t.
template <int CH, bool FULL, bool DIR, int PREC = PREC_VALU>
__device__ inline void seg_rot(float2 (&v)[REGS], float2* lds, int c, float t, uint32_t tid)
{
    constexpr int L0 = ChainAt<CH, DIR ? 0 : CH - 1>::L;
    rot_round<CH, L0, FULL, PREC>(v, c, t, tid);
    if constexpr (CH >= 2) {
        constexpr int L1 = ChainAt<CH, DIR ? 1 : CH - 2>::L;
        xchg<L0, L1>(lds, tid, v);
        rot_round<CH, L1, FULL, PREC>(v, c, t, tid);
        if constexpr (CH >= 3) {
            constexpr int L2 = ChainAt<CH, DIR ? 2 : 0>::L;
            xchg<L1, L2>(lds, tid, v);
            rot_round<CH, L2, FULL, PREC>(v, c, t, tid);
        }
    }
}

// Inverse rotation on psi and lambda with the beta-gradient terms. A round's
// inner products are all taken before its rotations, on states scaled by
// |f|^(-done) (done = qubits already rotated in earlier rounds of this
// segment), so they are multiplied back by fsq^done.
template <int L, bool FULL>
__device__ inline void bwd_round(float2 (&ps)[REGS], float2 (&la)[REGS], int c, float t, float fsq, float& wdone,
                                 double& xacc)
{
    float tk[4], wk[4];
    float w = wdone;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool act = FULL || layout_bit0<L>() + k >= c;
        tk[k] = act ? -t : 0.f;
        wk[k] = act ? wdone : 0.f;
        w = act ? w * fsq : w;
    }
    const float a = wk[0] * xb_bit<0>(ps, la) + wk[1] * xb_bit<1>(ps, la) + wk[2] * xb_bit<2>(ps, la) +
                    wk[3] * xb_bit<3>(ps, la);
    xacc += (double)a;
    rx_round(ps, tk);
    rx_round(la, tk);
    wdone = w;
}

template <int CH, bool FULL, bool DIR>
__device__ inline void seg_bwd(float2 (&ps)[REGS], float2 (&la)[REGS], float2* lds, int c, const RxC& rc,
                               uint32_t tid, double& xacc)
{
    float wdone = 1.f;
    constexpr int L0 = ChainAt<CH, DIR ? 0 : CH - 1>::L;
    bwd_round<L0, FULL>(ps, la, c, rc.t, rc.fsq, wdone, xacc);
    if constexpr (CH >= 2) {
        constexpr int L1 = ChainAt<CH, DIR ? 1 : CH - 2>::L;
        xchg<L0, L1>(lds, tid, ps);
        xchg<L0, L1>(lds, tid, la);
        bwd_round<L1, FULL>(ps, la, c, rc.t, rc.fsq, wdone, xacc);
        if constexpr (CH >= 3) {
            constexpr int L2 = ChainAt<CH, DIR ? 2 : 0>::L;
            xchg<L1, L2>(lds, tid, ps);
            xchg<L1, L2, false>(lds, tid, la);
            bwd_round<L2, FULL>(ps, la, c, rc.t, rc.fsq, wdone, xacc);
        }
    }
}

// The beta-gradient terms of a whole segment on states that are not rotated:
// both states walk the layout chain and every register bit that is a qubit
// of the group contributes its inner products.
template <int L, bool FULL>
__device__ inline float xb_round(const float2 (&ps)[REGS], const float2 (&la)[REGS], int c)
{
    float a = 0.f;
    if (FULL || layout_bit0<L>() + 0 >= c) a += xb_bit<0>(ps, la);
    if (FULL || layout_bit0<L>() + 1 >= c) a += xb_bit<1>(ps, la);
    if (FULL || layout_bit0<L>() + 2 >= c) a += xb_bit<2>(ps, la);
    if (FULL || layout_bit0<L>() + 3 >= c) a += xb_bit<3>(ps, la);
    return a;
}

template <int CH, bool FULL, bool DIR>
__device__ inline void seg_xb(float2 (&ps)[REGS], float2 (&la)[REGS], float2* lds, int c, uint32_t tid,
                              double& xacc)
{
    constexpr int L0 = ChainAt<CH, DIR ? 0 : CH - 1>::L;
    xacc += (double)xb_round<L0, FULL>(ps, la, c);
    if constexpr (CH >= 2) {
        constexpr int L1 = ChainAt<CH, DIR ? 1 : CH - 2>::L;
        xchg<L0, L1>(lds, tid, ps);
        xchg<L0, L1>(lds, tid, la);
        xacc += (double)xb_round<L1, FULL>(ps, la, c);
        if constexpr (CH >= 3) {
            constexpr int L2 = ChainAt<CH, DIR ? 2 : 0>::L;
            xchg<L1, L2>(lds, tid, ps);
            xchg<L1, L2, false>(lds, tid, la);
            xacc += (double)xb_round<L2, FULL>(ps, la, c);
        }
    }
}

// C(z) for the 16 amplitudes a lane holds in layout L, for data permuted by
// the flip mask m (slot q holds amplitude q ^ m). Group 0 reads the natural
// table, the last group its tile-order copy (contiguous per tile).
// A subgraph's cut table: 1 byte per entry when its weight sum is at most
// 255, else 2 (the width is uniform per workgroup).
struct CutTab {
    const uint8_t* p;
    int w;
    __device__ uint32_t at(uint32_t i) const { return w == 1 ? (uint32_t)p[i] : (uint32_t)((const uint16_t*)p)[i]; }
};

template <int L, bool G0 = false, typename T = uint16_t>
__device__ inline void load_cut_L(T (&cr)[REGS], const CutTab& tab, uint32_t tid, uint32_t m)
{
    if constexpr (G0) {
        // group 0 flips all twelve tile bits or none, so the register bits
        // of m are all set or all clear: the per-register offsets are then
        // constants, in one of two orders chosen by a uniform branch
        constexpr uint32_t R = reg_part<L>(REGS - 1);
        const uint32_t base = (thread_part<L>(tid) ^ m) & ~R;
        const bool rev = (m & R) != 0u;
        if (tab.w == 1) {
            const uint8_t* p = tab.p + base;
            if (rev) {
#pragma unroll
                for (int r = 0; r < REGS; ++r) cr[r] = p[reg_part<L>(REGS - 1 - r)];
            } else {
#pragma unroll
                for (int r = 0; r < REGS; ++r) cr[r] = p[reg_part<L>(r)];
            }
        } else {
            const uint16_t* p = (const uint16_t*)tab.p + base;
            if (rev) {
#pragma unroll
                for (int r = 0; r < REGS; ++r) cr[r] = p[reg_part<L>(REGS - 1 - r)];
            } else {
#pragma unroll
                for (int r = 0; r < REGS; ++r) cr[r] = p[reg_part<L>(r)];
            }
        }
        return;
    }
    const uint32_t tp = thread_part<L>(tid) ^ m;
    if (tab.w == 1) {
#pragma unroll
        for (int r = 0; r < REGS; ++r) cr[r] = tab.p[tp ^ reg_part<L>(r)];
    } else {
        const uint16_t* t16 = (const uint16_t*)tab.p;
#pragma unroll
        for (int r = 0; r < REGS; ++r) cr[r] = t16[tp ^ reg_part<L>(r)];
    }
}

// the tile's slice of the table: both tables are stored in tile order (group
// 0's mirror-paired tiles and the last group's strided tiles)
__device__ inline CutTab tile_tab(const uint8_t* ws, const SubDesc* sd, int g, uint32_t t)
{
    const int w = sd->tabw;
    return CutTab{(g == 0 ? ws + sd->tab : ws + sd->tabB) + (size_t)t * TILE * w, w};
}

// OFF32: addresses as 32-bit byte offsets from the state's (uniform) base
// (a stored state of n <= 30 qubits spans at most 2^29 amplitudes = 4 GiB).
// The map is XOR-linear, so a register's offset is the lane's offset XOR a
// per-register value that is uniform across the workgroup: one vector XOR
// per access instead of an XOR and a 64-bit address add.
__device__ inline const float2& at_off(const float2* st, uint32_t off)
{
    return *(const float2*)((const uint8_t*)st + off);
}
__device__ inline float2& at_off(float2* st, uint32_t off) { return *(float2*)((uint8_t*)st + off); }

template <int L, bool G0, bool OFF32 = false>
__device__ inline void load_state(float2 (&v)[REGS], const float2* st, const Geo& geo, uint32_t tid)
{
    if constexpr (OFF32) {
        uint32_t base = (geo.zb ^ gmapT<G0>(geo, thread_part<L>(tid))) << 3;
        asm volatile("" : "+v"(base));  // keeps the shift out of the per-register XOR
#pragma unroll
        for (int r = 0; r < REGS; ++r) v[r] = at_off(st, base ^ (gmapT<G0>(geo, reg_part<L>(r)) << 3));
    } else {
        const uint32_t base = geo.zb ^ gmapT<G0>(geo, thread_part<L>(tid));
#pragma unroll
        for (int r = 0; r < REGS; ++r) v[r] = st[base ^ gmapT<G0>(geo, reg_part<L>(r))];
    }
    __builtin_amdgcn_sched_barrier(0);
}

// store slot q to amplitude q ^ m (gmap is a bit deposit, so it commutes with xor)
template <int L, bool G0, bool OFF32 = false>
__device__ inline void store_state(const float2 (&v)[REGS], float2* st, const Geo& geo, uint32_t tid, uint32_t m)
{
    // address arithmetic stays here (hoisting it holds 2 VGPRs per register)
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (OFF32) {
        uint32_t base = (geo.zb ^ gmapT<G0>(geo, thread_part<L>(tid)) ^ gmapT<G0>(geo, m)) << 3;
        asm volatile("" : "+v"(base));
#pragma unroll
        for (int r = 0; r < REGS; ++r)
            at_off(st, base ^ (gmapT<G0>(geo, reg_part<L>(r)) << 3)) = v[r];
    } else {
        const uint32_t base = geo.zb ^ gmapT<G0>(geo, thread_part<L>(tid)) ^ gmapT<G0>(geo, m);
#pragma unroll
        for (int r = 0; r < REGS; ++r) st[base ^ gmapT<G0>(geo, reg_part<L>(r))] = v[r];
    }
}

// deterministic block sum (wave64 butterfly, then the 4 wave totals in order)
// three deterministic block sums with one barrier pair
__device__ inline void block_sum3(double& a, double& b, double& c, double* red)
{
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
        c += __shfl_xor(c, off);
    }
    const uint32_t tid = threadIdx.x;
    const int nw = (int)(blockDim.x >> 6);
    if ((tid & 63u) == 0) {
        red[tid >> 6] = a;
        red[nw + (tid >> 6)] = b;
        red[2 * nw + (tid >> 6)] = c;
    }
    __syncthreads();
    if (tid == 0) {
        double x = 0.0, y = 0.0, z = 0.0;
        for (int i = 0; i < nw; ++i) {
            x += red[i];
            y += red[nw + i];
            z += red[2 * nw + i];
        }
        a = x;
        b = y;
        c = z;
    }
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

__device__ inline Geo make_geo(const SubDesc* sd, int g, uint32_t t)
{
    Geo r;
    r.mir = 0;
    if (g == 0) {
        r.c = 0;
        r.g0 = 0;
        r.nb = TILE_BITS;
        r.zb = t << HALF_BITS;
        r.mir = (1u << (sd->n - 1)) - 1u;
    } else {
        r.nb = sd->gsize[g];
        r.g0 = sd->gstart[g];
        r.c = TILE_BITS - r.nb;
        const int L = r.g0 - r.c;  // fixed bits between the passive block and the group
        const uint32_t tlo = t & ((1u << L) - 1u), thi = t >> L;
        r.zb = (tlo << r.c) | (thi << (r.g0 + r.nb));
    }
    return r;
}

// ---------------------------------------------------------------------------
// K1: integer cut tables (natural order + tile order of the last group)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(THREADS) void k_cut_tables(uint8_t* ws, const SubDesc* subs, const int2* work)
{
    // C(z) of the reduced indices (top bit clear: C of the full index is the
    // same). Whole-state subgraphs: natural order; tiled ones: group 0's
    // mirror-paired tile order in tab, the last group's tile order in tabB.
    const int2 wk = work[blockIdx.x];
    const SubDesc* sd = subs + wk.x;
    const uint32_t t = (uint32_t)wk.y;
    const int n = sd->n, ne = sd->nedges, G = sd->ngroups;
    const int32_t* E = (const int32_t*)(ws + sd->edges);
    uint8_t* tab = ws + sd->tab;
    const uint32_t dim = 1u << (n - 1);
    const uint32_t span = dim < (uint32_t)TILE ? dim : (uint32_t)TILE;
    const Geo geoA = make_geo(sd, 0, t);
    const Geo geoB = make_geo(sd, G >= 2 ? G - 1 : 0, t);
    uint8_t* tabB = ws + sd->tabB;
    const bool w1 = sd->tabw == 1;
    // four consecutive entries per thread, written as whole 32-bit words
    // (span is 2^(n-1) or 4096; below 4 only for n <= 2, entry by entry)
    if (span >= 4) {
        for (uint32_t q0 = 4 * threadIdx.x; q0 < span; q0 += 4 * THREADS) {
            // one pass over the edges for all eight entries of the thread
            uint32_t z[4], zB[4], c[4] = {0, 0, 0, 0}, cb[4] = {0, 0, 0, 0};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                z[i] = G >= 2 ? geoA.zb ^ gmap0(geoA, q0 + i) : q0 + i;
                zB[i] = geoB.zb | gmap(geoB, q0 + i);
            }
            for (int e = 0; e < ne; ++e) {
                const int32_t u = E[3 * e], v = E[3 * e + 1];
                const uint32_t w = (uint32_t)E[3 * e + 2];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    c[i] += (((z[i] >> u) ^ (z[i] >> v)) & 1u) ? w : 0u;
                    cb[i] += (((zB[i] >> u) ^ (zB[i] >> v)) & 1u) ? w : 0u;
                }
            }
            const size_t z0 = (size_t)t * TILE + q0;
            if (w1) {
                *(uint32_t*)(tab + z0) = c[0] | (c[1] << 8) | (c[2] << 16) | (c[3] << 24);
                if (G >= 2) *(uint32_t*)(tabB + z0) = cb[0] | (cb[1] << 8) | (cb[2] << 16) | (cb[3] << 24);
            } else {
                uint32_t* o = (uint32_t*)(tab + 2 * z0);
                o[0] = c[0] | (c[1] << 16);
                o[1] = c[2] | (c[3] << 16);
                if (G >= 2) {
                    uint32_t* ob = (uint32_t*)(tabB + 2 * z0);
                    ob[0] = cb[0] | (cb[1] << 16);
                    ob[1] = cb[2] | (cb[3] << 16);
                }
            }
        }
    } else {
        for (uint32_t q = threadIdx.x; q < span; q += THREADS) {
            const uint32_t c = cut_of(q, E, ne);
            if (w1) tab[q] = (uint8_t)c;
            else ((uint16_t*)tab)[q] = (uint16_t)c;
        }
    }
}

// ---------------------------------------------------------------------------
// Forward tile pass. Pass kinds (fixed at compile time so the state has one
// straight-line life): FIRST = synthesise |+>, phase, RX; SINGLE = RX;
// MID = RX, phase, RX; LAST = RX and the <C> partial of the tile.
// ---------------------------------------------------------------------------
enum { F_FIRST = 0, F_SINGLE = 1, F_MID = 2, F_LAST = 3 };

template <int CH, bool FULL, int KIND, int PREC>
__device__ __forceinline__ void fwd_pass_body(uint8_t* ws, const SubDesc* subs, const int2* work, PassOps ops,
                                              Partials part)
{
    extern __shared__ float2 smem[];
    float2* lds = smem;
    float2* lut = smem + LDS_TILE;
    __shared__ double red[THREADS / 64];
    constexpr int LS = ChainAt<CH, 0>::L, LE = ChainAt<CH, CH - 1>::L;
    constexpr bool HAS_PRE = KIND != F_FIRST, HAS_PH = KIND == F_FIRST || KIND == F_MID;
    constexpr bool HAS_POST = HAS_PH;
    const uint32_t tid = threadIdx.x;
    const int2 wk = work[blockIdx.x];
    const SubDesc* sd = subs + wk.x;
    const uint32_t t = (uint32_t)wk.y;
    const int g = ops.group;
    const Geo geo = make_geo(sd, g, t);
    const float2* src = (const float2*)(ws + sd->psi + (uint64_t)ops.psi_in * state_bytes(sd->n));
    float2* st = (float2*)(ws + sd->psi + (uint64_t)ops.psi_out * state_bytes(sd->n));
    const RxCoef* cf = (const RxCoef*)(ws + sd->coef);
    const int lut_len = sd->lut_len;
    const CutTab tab = tile_tab(ws, sd, g, t);
    const uint32_t gb = group_bits(geo.c);
    RxC pre{}, post{};
    if constexpr (HAS_PRE) pre = load_rx(cf, ops.pre, g);
    if constexpr (HAS_POST) post = load_rx(cf, ops.post, g);
    const uint32_t m_pre = (HAS_PRE && pre.flip) ? gb : 0u;                   // after RX(pre)
    const uint32_t m_end = m_pre ^ ((HAS_POST && post.flip) ? gb : 0u);      // after RX(post)
    uint16_t cr[REGS];
    if constexpr (HAS_PH) {
        // phase table, with the factors of the segments before and after it
        // folded in (the rotations are linear, so the factor of the one after
        // may be applied before it)
        const float2* L = (const float2*)(ws + sd->lut) + (size_t)ops.ph * lut_len;
        // (the first pass also folds in the amplitude 2^(-(n-1)/2) of |+>)
        const float amp = (float)(1.0 / sqrt((double)(1ull << (sd->n - 1))));
        const float2 F = HAS_PRE ? cmul(pre.Ff, post.Ff) : make_float2(amp * post.Ff.x, amp * post.Ff.y);
        for (int i = tid; i < lut_len; i += THREADS) lut[i] = cmul(L[i], F);
        if constexpr (HAS_PRE) load_cut_L<LE>(cr, tab, tid, m_pre);
        else load_cut_L<LS>(cr, tab, tid, 0u);
    }
    if constexpr (KIND == F_LAST) load_cut_L<LE>(cr, tab, tid, m_end);
    float2 v[REGS];
    if constexpr (KIND != F_FIRST) load_state<LS, CH == 3>(v, src, geo, tid);
    __syncthreads();  // phase table staged
    if constexpr (HAS_PRE) {
        seg_rot<CH, FULL, true, PREC>(v, lds, geo.c, pre.t, tid);
        if constexpr (!HAS_PH) scale_regs(v, pre.Ff);
    }
    if constexpr (HAS_PH) {
        if constexpr (KIND == F_FIRST) {
#pragma unroll
            for (int r = 0; r < REGS; ++r) v[r] = lut[cr[r]];  // |+> after the phase separator
        } else {
#pragma unroll
            for (int r = 0; r < REGS; ++r) v[r] = cmul(v[r], lut[cr[r]]);
        }
        // FIRST walks start -> end, MID walks back end -> start
        seg_rot<CH, FULL, KIND == F_FIRST, PREC>(v, lds, geo.c, post.t, tid);
    }
    double acc = 0.0;
    if constexpr (KIND == F_LAST) {
#pragma unroll
        for (int r = 0; r < REGS; ++r)
            acc += ((double)v[r].x * v[r].x + (double)v[r].y * v[r].y) * (double)cr[r];
    }
    // after one segment the layout is the chain end; after two it is back at
    // the start (stores first: they drain while the partial sum is reduced)
    if constexpr (KIND == F_MID) store_state<LS, CH == 3>(v, st, geo, tid, m_end);
    else store_state<LE, CH == 3>(v, st, geo, tid, m_end);
    if constexpr (KIND == F_LAST) {
        acc = block_sum(acc, red);
        if (tid == 0) part.e[sd->tile_base + t] = acc;
    }
}

template <int CH, bool FULL, int KIND>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(PQ_FWD_WAVES))) void k_fwd_pass(
    uint8_t* ws, const SubDesc* subs, const int2* work, PassOps ops, Partials part)
{
    fwd_pass_body<CH, FULL, KIND, PREC_VALU>(ws, subs, work, ops, part);
}

// group 0 with the mixer block on the matrix cores (more registers per lane)
template <int KIND, int PREC>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(PQ_MF_WAVES))) void k_fwd_pass_mf(
    uint8_t* ws, const SubDesc* subs, const int2* work, PassOps ops, Partials part)
{
    fwd_pass_body<3, true, KIND, PREC>(ws, subs, work, ops, part);
}

// ---------------------------------------------------------------------------
// Backward tile pass (adjoint sweep) on psi and lambda = C psi_p. Kinds:
// FUSED : RX(pre) on psi, <C> partial, lambda = C psi, then the inverse of
//         RX(pre) on both with the beta-gradient; only lambda is stored (psi
//         in memory already is the state before RX(pre)).
// SINGLE: unmix(pre) with the beta-gradient; store both.
// MID   : unmix(pre), gamma-gradient + unphase(ph), unmix(post); store both.
// LAST  : the inverse of the first forward pass (group 0 of layer 1): lambda
//         is rotated back alone; psi at that point is the phased uniform
//         state (stored half: 2^(-(n-1)/2) e^{-i gamma_1 C(z)}), so it is
//         synthesised from the cut
//         table instead of read, and the beta terms of the segment are taken
//         there (X_j commutes with every rotation of the layer, so the inner
//         product <lambda|X_j|psi> is the same at any point of the layer);
//         nothing stored.
// STORE_PSI = false drops the psi store of the pass before LAST (LAST does
// not read psi).
// ---------------------------------------------------------------------------
enum { B_FUSED = 0, B_SINGLE = 1, B_MID = 2, B_LAST = 3 };

// The fused kind on group 0 is held to four waves per SIMD (the most that
// its LDS tile allows); left free, it takes 130 registers and runs three.
template <int CH, bool FULL, int KIND, bool STORE_PSI = true>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu((KIND == B_FUSED || KIND == B_LAST) && CH == 3 ? 4 : PQ_BWD_WAVES))) void k_bwd_pass(
    uint8_t* ws, const SubDesc* subs, const int2* work, PassOps ops, Partials part)
{
    extern __shared__ float2 smem[];
    float2* lds = smem;
    float2* lut = smem + LDS_TILE;
    __shared__ double red[3 * THREADS / 64];
    constexpr int LS = ChainAt<CH, 0>::L, LE = ChainAt<CH, CH - 1>::L;
    const uint32_t tid = threadIdx.x;
    const int2 wk = work[blockIdx.x];
    const SubDesc* sd = subs + wk.x;
    const uint32_t t = (uint32_t)wk.y;
    const int g = ops.group;
    const Geo geo = make_geo(sd, g, t);
    float2* sp = (float2*)(ws + sd->psi + (uint64_t)ops.psi_in * state_bytes(sd->n));
    float2* sl = (float2*)(ws + sd->lam);
    const RxCoef* cf = (const RxCoef*)(ws + sd->coef);
    const int lut_len = sd->lut_len;
    const int T = part.total_tiles;
    const int tile = sd->tile_base + (int)t;
    const CutTab tab = tile_tab(ws, sd, g, t);
    const uint32_t gb = group_bits(geo.c);
    const RxC pre = load_rx(cf, ops.pre, g);
    RxC post{};
    if constexpr (KIND == B_MID) post = load_rx(cf, ops.post, g);
    const uint32_t m_pre = pre.flip ? gb : 0u;
    const uint32_t m_end = m_pre ^ ((KIND == B_MID && post.flip) ? gb : 0u);
    if constexpr (KIND == B_MID) {
        // conjugate phase table with the inverse factors of the segments
        // before and after it (the one after scales the states it rotates,
        // so its beta terms are divided by |F|^2 at the end)
        const float2* L = (const float2*)(ws + sd->lut) + (size_t)ops.ph * lut_len;
        const float2 F = cmul(pre.Fi, post.Fi);
        for (int i = tid; i < lut_len; i += THREADS) {
            const float2 e = L[i];
            lut[i] = cmul(make_float2(e.x, -e.y), F);
        }
    } else if constexpr (KIND == B_LAST) {
        // the phase table of layer 1 as the forward pass used it, times the
        // amplitude 2^(-(n-1)/2) of the stored |+> and the conjugate of the
        // inverse factor of RX(pre): every sum of this pass is bilinear in
        // conj(lambda) and psi, so scaling psi by conj(Fi) stands for scaling
        // lambda by Fi
        const float2* L = (const float2*)(ws + sd->lut) + (size_t)ops.ph * lut_len;
        const float amp = (float)(1.0 / sqrt((double)(1ull << (sd->n - 1))));
        const float2 F = make_float2(amp * pre.Fi.x, -amp * pre.Fi.y);
        for (int i = tid; i < lut_len; i += THREADS) lut[i] = cmul(L[i], F);
    }
    // the last kind synthesises psi in every layout of the chain from the
    // cut values of that layout (group 0 only: its chain is LLIN, LL0, LL1),
    // instead of moving psi through LDS with lambda
    constexpr bool SYNTH = KIND == B_LAST && CH == 3;
    // the cut values (used after the first segment) are loaded with the
    // states, so their latency is hidden behind that segment
    uint16_t cr[REGS];
    if constexpr (KIND != B_SINGLE) load_cut_L<LE, SYNTH>(cr, tab, tid, m_pre);
    uint32_t cr0[SYNTH ? REGS : 1], crI[SYNTH ? REGS : 1];
    if constexpr (SYNTH) {
        load_cut_L<LL0, true>(cr0, tab, tid, m_pre);
        load_cut_L<LLIN, true>(crI, tab, tid, m_pre);
    }
    float2 ps[REGS], la[REGS];
    // the kinds with the busiest vector units use the one-XOR offsets
    constexpr bool O32 = KIND == B_MID || KIND == B_LAST;
    if constexpr (KIND != B_LAST) load_state<LS, CH == 3, O32>(ps, sp, geo, tid);
    if constexpr (KIND != B_FUSED) load_state<LS, CH == 3, O32>(la, sl, geo, tid);
    __syncthreads();
    double acc_pre = 0.0, acc_ph = 0.0, acc_post = 0.0, acc_e = 0.0;
    if constexpr (KIND == B_LAST) {
        // lambda back through RX(pre) (its factor Fi is in the table); slot q
        // then holds amplitude q ^ m_pre
        seg_rot<CH, FULL, true>(la, lds, geo.c, -pre.t, tid);
        float a = 0.f;
#pragma unroll
        for (int r = 0; r < REGS; ++r) {
            ps[r] = lut[cr[r]];
            // C(z) Im(conj(lambda) psi)
            a = fmaf((float)cr[r], fmaf(la[r].x, ps[r].y, -la[r].y * ps[r].x), a);
        }
        acc_ph = (double)a;
        if constexpr (SYNTH) {
            // the beta terms in the three layouts, lambda walking back LL1 ->
            // LL0 -> LLIN and psi synthesised afresh in each
            acc_pre += (double)xb_round<LL1, FULL>(ps, la, geo.c);
            xchg<LL1, LL0>(lds, tid, la);
#pragma unroll
            for (int r = 0; r < REGS; ++r) ps[r] = lut[cr0[r]];
            acc_pre += (double)xb_round<LL0, FULL>(ps, la, geo.c);
            xchg<LL0, LLIN>(lds, tid, la);
#pragma unroll
            for (int r = 0; r < REGS; ++r) ps[r] = lut[crI[r]];
            acc_pre += (double)xb_round<LLIN, FULL>(ps, la, geo.c);
        } else {
            seg_xb<CH, FULL, false>(ps, la, lds, geo.c, tid, acc_pre);
        }
    } else if constexpr (KIND == B_FUSED) {
        // psi_p = RX(pre) psi (slot q then holds amplitude q ^ m_pre)
        seg_rot<CH, FULL, true>(ps, lds, geo.c, pre.t, tid);
        scale_regs(ps, pre.Ff);
#pragma unroll
        for (int r = 0; r < REGS; ++r) {
            const float c = (float)cr[r];
            acc_e += ((double)ps[r].x * ps[r].x + (double)ps[r].y * ps[r].y) * (double)cr[r];
            la[r] = make_float2(c * ps[r].x, c * ps[r].y);
        }
        // the inverse rotation flips back: the stored lambda is unpermuted
        seg_bwd<CH, FULL, false>(ps, la, lds, geo.c, pre, tid, acc_pre);
        scale_regs(la, pre.Fi);
    } else {
        seg_bwd<CH, FULL, true>(ps, la, lds, geo.c, pre, tid, acc_pre);
        if constexpr (KIND == B_SINGLE) {
            scale_regs(ps, pre.Fi);
            scale_regs(la, pre.Fi);
        } else {
            // on the rotated-but-unscaled states; rescale by |F|^2
            float a = 0.f;
#pragma unroll
            for (int r = 0; r < REGS; ++r) {
                // C(z) Im(conj(lambda) psi)
                a = fmaf((float)cr[r], fmaf(la[r].x, ps[r].y, -la[r].y * ps[r].x), a);
            }
            acc_ph = (double)a * (double)(pre.Fi.x * pre.Fi.x + pre.Fi.y * pre.Fi.y);
            if constexpr (KIND == B_MID) {
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int r = 0; r < REGS; ++r) {
                    const float2 f = lut[cr[r]];
                    ps[r] = cmul(ps[r], f);
                    la[r] = cmul(la[r], f);
                }
                __builtin_amdgcn_sched_barrier(0);
                seg_bwd<CH, FULL, false>(ps, la, lds, geo.c, post, tid, acc_post);
                acc_post /= (double)post.Fi.x * post.Fi.x + (double)post.Fi.y * post.Fi.y;
            }
        }
    }
    // results first (the stores drain while the partial sums are reduced)
    if constexpr (KIND == B_FUSED) {
        store_state<LS, CH == 3>(la, sl, geo, tid, 0u);
    } else if constexpr (KIND == B_SINGLE) {
        if constexpr (STORE_PSI) store_state<LE, CH == 3>(ps, sp, geo, tid, m_end);
        store_state<LE, CH == 3>(la, sl, geo, tid, m_end);
    } else if constexpr (KIND == B_MID) {
        if constexpr (STORE_PSI) store_state<LS, CH == 3, true>(ps, sp, geo, tid, m_end);
        store_state<LS, CH == 3, true>(la, sl, geo, tid, m_end);
    }
    // partial sums: (<C> or gamma, beta of pre, beta of post)
    double s0 = KIND == B_FUSED ? acc_e : acc_ph, s1 = acc_pre, s2 = acc_post;
    block_sum3(s0, s1, s2, red);
    if (tid == 0) {
        if constexpr (KIND == B_FUSED) part.e[tile] = s0;
        if constexpr (KIND == B_MID || KIND == B_LAST) part.gg[(size_t)ops.ph * T + tile] = s0;
        part.gb[((size_t)ops.pre * MAX_GROUPS + g) * T + tile] = s1;
        if constexpr (KIND == B_MID) part.gb[((size_t)ops.post * MAX_GROUPS + g) * T + tile] = s2;
    }
}

// ---------------------------------------------------------------------------
// Subgraphs with n <= 13: one workgroup runs the whole circuit (and, with
// grad, the whole adjoint sweep) in LDS, one qubit at a time, with the
// plain (cos, sin) form of each rotation.
// ---------------------------------------------------------------------------
__device__ inline void rx_pair(float2& a, float2& b, float c, float s)
{
    const float2 na = make_float2(c * a.x + s * b.y, c * a.y - s * b.x);
    const float2 nb = make_float2(c * b.x + s * a.y, c * b.y - s * a.x);
    a = na;
    b = nb;
}

__global__ __launch_bounds__(THREADS) void k_small(uint8_t* ws, const SubDesc* subs, const int32_t* list,
                                                   int p, int grad, Partials part)
{
    extern __shared__ float2 smem[];
    __shared__ double red[THREADS / 64];
    const uint32_t tid = threadIdx.x;
    const SubDesc* sd = subs + list[blockIdx.x];
    const int n = sd->n;
    // the reduced state: qubits 0..n-2 act on the index bits, the top qubit's
    // X on an index pairs it with its complement (dim - 1 - index); for n = 1
    // that pair is the single amplitude itself
    const uint32_t dim = 1u << (n - 1), half = dim >> 1, comp = dim - 1;
    float2* ps = smem;
    float2* la = smem + TILE;
    float2* lut = smem + (grad ? 2 * TILE : TILE);
    const CutTab tab{ws + sd->tab, sd->tabw};
    const RxCoef* cf = (const RxCoef*)(ws + sd->coef);
    const float2* luts = (const float2*)(ws + sd->lut);
    const int lut_len = sd->lut_len;
    const int T = part.total_tiles;
    const int tile = sd->tile_base;

    const float a0 = (float)(1.0 / sqrt((double)dim));
    for (uint32_t z = tid; z < dim; z += THREADS) ps[z] = make_float2(a0, 0.f);
    for (int l = 0; l < p; ++l) {
        __syncthreads();
        for (int i = tid; i < lut_len; i += THREADS) lut[i] = luts[(size_t)l * lut_len + i];
        __syncthreads();
        for (uint32_t z = tid; z < dim; z += THREADS) ps[z] = cmul(ps[z], lut[tab.at(z)]);
        const float2 cs = cf[l].cs;
        for (int j = 0; j < n - 1; ++j) {
            __syncthreads();
            for (uint32_t i = tid; i < half; i += THREADS) {
                const uint32_t z = ((i >> j) << (j + 1)) | (i & ((1u << j) - 1u));
                rx_pair(ps[z], ps[z | (1u << j)], cs.x, cs.y);
            }
        }
        __syncthreads();
        for (uint32_t i = tid; i < half; i += THREADS) rx_pair(ps[i], ps[i ^ comp], cs.x, cs.y);
        if (dim == 1 && tid == 0) ps[0] = cmul(ps[0], make_float2(cs.x, -cs.y));
    }
    __syncthreads();
    double acc = 0.0;
    for (uint32_t z = tid; z < dim; z += THREADS)
        acc += ((double)ps[z].x * ps[z].x + (double)ps[z].y * ps[z].y) * (double)tab.at(z);
    acc = block_sum(acc, red);
    if (tid == 0) part.e[tile] = acc;
    if (!grad) {
        float2* st = (float2*)(ws + sd->psi);
        for (uint32_t z = tid; z < dim; z += THREADS) st[z] = ps[z];
        return;
    }
    for (uint32_t z = tid; z < dim; z += THREADS) {
        const float c = (float)tab.at(z);
        la[z] = make_float2(c * ps[z].x, c * ps[z].y);
    }
    for (int l = p - 1; l >= 0; --l) {
        const float2 cs = cf[l].cs;
        double xb = 0.0;
        // the top qubit (complement pairs) first, then qubits n-2..0
        for (int j = n - 1; j >= 0; --j) {
            __syncthreads();
            float a = 0.f;
            if (j == n - 1 && dim == 1) {
                if (tid == 0) {
                    a += la[0].x * ps[0].y - la[0].y * ps[0].x;
                    ps[0] = cmul(ps[0], make_float2(cs.x, cs.y));
                    la[0] = cmul(la[0], make_float2(cs.x, cs.y));
                }
            } else {
                for (uint32_t i = tid; i < half; i += THREADS) {
                    const uint32_t z = j == n - 1 ? i : ((i >> j) << (j + 1)) | (i & ((1u << j) - 1u));
                    const uint32_t z1 = j == n - 1 ? i ^ comp : z | (1u << j);
                    a += la[z].x * ps[z1].y - la[z].y * ps[z1].x;
                    a += la[z1].x * ps[z].y - la[z1].y * ps[z].x;
                    rx_pair(ps[z], ps[z1], cs.x, -cs.y);
                    rx_pair(la[z], la[z1], cs.x, -cs.y);
                }
            }
            xb += (double)a;
        }
        __syncthreads();
        xb = block_sum(xb, red);
        if (tid == 0) part.gb[((size_t)l * MAX_GROUPS + 0) * T + tile] = xb;
        double gg = 0.0;
        for (uint32_t z = tid; z < dim; z += THREADS)
            gg += (double)((float)tab.at(z) * (la[z].x * ps[z].y - la[z].y * ps[z].x));
        gg = block_sum(gg, red);
        if (tid == 0) part.gg[(size_t)l * T + tile] = gg;
        if (l > 0) {
            for (int i = tid; i < lut_len; i += THREADS) lut[i] = luts[(size_t)l * lut_len + i];
            __syncthreads();
            for (uint32_t z = tid; z < dim; z += THREADS) {
                float2 f = lut[tab.at(z)];
                f.y = -f.y;
                ps[z] = cmul(ps[z], f);
                la[z] = cmul(la[z], f);
            }
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

static size_t pass_lds(int lut_max) { return (size_t)(LDS_TILE + lut_max) * sizeof(float2); }

// chain codes: 3 = group 0; 2 / 4 = a high group of 8 / 5..7 qubits;
// 1 / 5 = a high group of 4 / 1..3 qubits (the second of each pair has
// register bits that are not active qubits)
#define PQ_LAUNCH_CH(KERNEL, KIND)                                                                              \
    do {                                                                                                        \
        switch (chain) {                                                                                        \
        case 3: hipLaunchKernelGGL((KERNEL<3, true, KIND>), g, b, lds, s, ws, subs, work, ops, part); break;    \
        case 2: hipLaunchKernelGGL((KERNEL<2, true, KIND>), g, b, lds, s, ws, subs, work, ops, part); break;    \
        case 4: hipLaunchKernelGGL((KERNEL<2, false, KIND>), g, b, lds, s, ws, subs, work, ops, part); break;   \
        case 1: hipLaunchKernelGGL((KERNEL<1, true, KIND>), g, b, lds, s, ws, subs, work, ops, part); break;    \
        default: hipLaunchKernelGGL((KERNEL<1, false, KIND>), g, b, lds, s, ws, subs, work, ops, part); break;  \
        }                                                                                                       \
    } while (0)

// group 0 with a matrix-core mixer block (PREC 1 or 2)
#define PQ_LAUNCH_MF(KIND)                                                                                      \
    do {                                                                                                        \
        if (prec == PREC_MFMA_F32)                                                                              \
            hipLaunchKernelGGL((k_fwd_pass_mf<KIND, PREC_MFMA_F32>), g, b, lds, s, ws, subs, work, ops, part);  \
        else if (prec == PREC_MFMA_BF16X3)                                                                      \
            hipLaunchKernelGGL((k_fwd_pass_mf<KIND, PREC_MFMA_BF16X3>), g, b, lds, s, ws, subs, work, ops,      \
                               part);                                                                           \
        else                                                                                                    \
            hipLaunchKernelGGL((k_fwd_pass_mf<KIND, PREC_MFMA_BF16X4>), g, b, lds, s, ws, subs, work, ops,      \
                               part);                                                                           \
    } while (0)

#define PQ_LAUNCH_CH2(KERNEL, KIND, X)                                                                          \
    do {                                                                                                        \
        switch (chain) {                                                                                        \
        case 3: hipLaunchKernelGGL((KERNEL<3, true, KIND, X>), g, b, lds, s, ws, subs, work, ops, part); break; \
        case 2: hipLaunchKernelGGL((KERNEL<2, true, KIND, X>), g, b, lds, s, ws, subs, work, ops, part); break; \
        case 4: hipLaunchKernelGGL((KERNEL<2, false, KIND, X>), g, b, lds, s, ws, subs, work, ops, part); break;\
        case 1: hipLaunchKernelGGL((KERNEL<1, true, KIND, X>), g, b, lds, s, ws, subs, work, ops, part); break; \
        default: hipLaunchKernelGGL((KERNEL<1, false, KIND, X>), g, b, lds, s, ws, subs, work, ops, part);      \
        }                                                                                                       \
    } while (0)

hipError_t launch_fwd_pass(uint8_t* ws, const SubDesc* subs, const int2* work, int nwork, int chain, PassOps ops,
                           Partials part, int lut_max, int prec, hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    const size_t lds = pass_lds(lut_max);
    const dim3 g(nwork), b(THREADS);
    if (prec != PREC_VALU && chain == 3) {
        if (ops.init) PQ_LAUNCH_MF(F_FIRST);
        else if (ops.epi_e) PQ_LAUNCH_MF(F_LAST);
        else if (ops.ph >= 0) PQ_LAUNCH_MF(F_MID);
        else PQ_LAUNCH_MF(F_SINGLE);
        return hipGetLastError();
    }
    if (ops.init) PQ_LAUNCH_CH(k_fwd_pass, F_FIRST);
    else if (ops.epi_e) PQ_LAUNCH_CH(k_fwd_pass, F_LAST);
    else if (ops.ph >= 0) PQ_LAUNCH_CH(k_fwd_pass, F_MID);
    else PQ_LAUNCH_CH(k_fwd_pass, F_SINGLE);
    return hipGetLastError();
}

hipError_t launch_bwd_pass(uint8_t* ws, const SubDesc* subs, const int2* work, int nwork, int chain, PassOps ops,
                           Partials part, int lut_max, hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    const size_t lds = pass_lds(lut_max);
    const dim3 g(nwork), b(THREADS);
    // the last pass mirrors the first forward pass (group 0 of layer 1)
    if (ops.last && (ops.group != 0 || chain != 3)) return hipErrorInvalidValue;
    if (ops.fused) PQ_LAUNCH_CH(k_bwd_pass, B_FUSED);
    else if (ops.last) PQ_LAUNCH_CH(k_bwd_pass, B_LAST);
    else if (ops.ph >= 0 && ops.nopsi) PQ_LAUNCH_CH2(k_bwd_pass, B_MID, false);
    else if (ops.ph >= 0) PQ_LAUNCH_CH(k_bwd_pass, B_MID);
    else if (ops.nopsi) PQ_LAUNCH_CH2(k_bwd_pass, B_SINGLE, false);
    else PQ_LAUNCH_CH(k_bwd_pass, B_SINGLE);
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

}  // namespace pq
