// Angle optimisation kernels of the batch (paper Sec. 2.2: the classical
// outer loop that tunes gamma and beta): the rotation and phase tables of a
// set of angles, the fixed-order reduction of the per-tile gradient and <C>
// partials that the tile passes write, and the fused optimiser step
// (reduction + Adam + the next step's tables).
#include "common.h"

namespace pq {

// ---------------------------------------------------------------------------
// Angle preparation. LUT[c] = e^{-i gamma c} from an FP64 product and
// FP64 sine/cosine, rounded to complex64; the rotation parameters of the
// layer in FP64, rounded to float.
// ---------------------------------------------------------------------------
__device__ inline void cpow_d(double re, double im, int e, double& ore, double& oim)
{
    double r = 1.0, i = 0.0;
    for (int k = 0; k < e; ++k) {
        const double nr = r * re - i * im, ni = r * im + i * re;
        r = nr;
        i = ni;
    }
    ore = r;
    oim = i;
}

// entry c of layer l's phase table: e^{-i gamma c} (c = 0 .. weight sum).
// This and prep_coef are compiled once (not inlined), so the standalone table
// kernel and the fused optimiser kernel produce the same bits.
__device__ __noinline__ void prep_lut_entry(uint8_t* ws, const SubDesc* sd, int l, int c, double gm)
{
    double sv, cv;
    sincos(gm * (double)c, &sv, &cv);
    ((float2*)(ws + sd->lut))[(size_t)l * sd->lut_len + c] = make_float2((float)cv, (float)(-sv));
}

// rotation parameters of layer l (one thread)
__device__ __noinline__ void prep_coef(uint8_t* ws, const SubDesc* sd, int l, double bt)
{
    double s, c;
    sincos(bt, &s, &c);
    RxCoef rc;
    rc.cs = make_float2((float)c, (float)s);
    // e^{-i beta X} = c (I - i tan(beta) X)            when |cos| >= |sin|
    //               = -i s X (I + i cot(beta) X)       otherwise
    // i.e. f (I - i t X) X^flip with (f, t) = (c, tan) or (-i s, -cot)
    const bool tanm = fabs(c) >= fabs(s);
    rc.mode = tanm ? 0 : 1;
    rc.t = (float)(tanm ? s / c : -c / s);
    rc.fsq = (float)(tanm ? c * c : s * s);
    // per-qubit factors: forward c or -i s, inverse c or +i s
    const double fr = tanm ? c : 0.0, fi_f = tanm ? 0.0 : -s, fi_i = tanm ? 0.0 : s;
    for (int g = 0; g < MAX_GROUPS; ++g) {
        const int nq = g < sd->ngroups ? sd->gsize[g] : 0;
        double r, i;
        cpow_d(fr, fi_f, nq, r, i);
        rc.Ff[g] = make_float2((float)r, (float)i);
        cpow_d(fr, fi_i, nq, r, i);
        rc.Fi[g] = make_float2((float)r, (float)i);
    }
    ((RxCoef*)(ws + sd->coef))[l] = rc;
}

__global__ __launch_bounds__(THREADS) void k_angle_prep(uint8_t* ws, const SubDesc* subs, int p,
                                                        const double* gamma, const double* beta)
{
    const int b = blockIdx.x / p, l = blockIdx.x % p;
    const SubDesc* sd = subs + b;
    const double gm = gamma[(size_t)b * p + l];
    for (int c = threadIdx.x; c < sd->lut_len; c += THREADS) prep_lut_entry(ws, sd, l, c, gm);
    if (threadIdx.x == 0) prep_coef(ws, sd, l, beta[(size_t)b * p + l]);
}

// ---------------------------------------------------------------------------
// Per-subgraph fixed-order reduction of the tile partials.
// dE/dgamma = 2 sum gg, dE/dbeta = 2 sum gb (the factor 2 of 2 Im <.|.|.>).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(THREADS) void k_reduce(const SubDesc* subs, int p, int grad, Partials part,
                                                    double* E, double* dgamma, double* dbeta)
{
    // block (b, q): q = 0 sums <C>, q = 1..p the gamma term of layer q - 1,
    // q = p + 1..2p the beta terms of layer q - p - 1 (over every group)
    __shared__ double red[THREADS / 64];
    const int b = blockIdx.x, q = blockIdx.y;
    const SubDesc* sd = subs + b;
    const int T = part.total_tiles, tb = sd->tile_base, nt = sd->ntiles, G = sd->ngroups;
    double acc = 0.0;
    if (q == 0) {
        for (int i = threadIdx.x; i < nt; i += THREADS) acc += part.e[tb + i];
    } else if (q <= p) {
        for (int i = threadIdx.x; i < nt; i += THREADS) acc += part.gg[(size_t)(q - 1) * T + tb + i];
    } else {
        const int l = q - p - 1;
        for (int i = threadIdx.x; i < nt; i += THREADS)
            for (int g = 0; g < G; ++g) acc += part.gb[((size_t)l * MAX_GROUPS + g) * T + tb + i];
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) {
        if (q == 0) {
            if (E) E[b] = acc;
        } else if (q <= p) {
            dgamma[(size_t)b * p + q - 1] = 2.0 * acc;
        } else {
            dbeta[(size_t)b * p + q - p - 1] = 2.0 * acc;
        }
    }
}

// ---------------------------------------------------------------------------
// One step of the angle optimisation after its gradient passes. Block
// (b, l) owns layer l of subgraph b: it sums the tile partials of dE/dgamma_l
// and dE/dbeta_l (and of <C> for l = 0) exactly as k_reduce does, takes the
// Adam ascent step on gamma_l and beta_l (theta = [gamma of every subgraph |
// beta of every subgraph]) as k_adam does, and prepares the phase table and
// rotation parameters of the new angles as k_angle_prep does. Step `it` of
// a run reads the step count the run started from and takes step
// count + it + 1; the count itself advances once, after the run's last step
// (k_step_advance), so no block waits for or signals another.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(THREADS) void k_reduce_adam(uint8_t* ws, const SubDesc* subs, int B, int p,
                                                         Partials part, double* theta, double* m, double* v,
                                                         const int32_t* step, int32_t it, double lr, double b1,
                                                         double b2, double eps, double* E)
{
    constexpr int NW = THREADS / 64;
    __shared__ double red[3][NW];
    __shared__ double s_gamma, s_beta;
    const int b = blockIdx.x / p, l = blockIdx.x % p;
    const SubDesc* sd = subs + b;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int32_t t = *step + it + 1;
    const int T = part.total_tiles, tb = sd->tile_base, nt = sd->ntiles, G = sd->ngroups;
    // sums (k_reduce's terms and order: per thread in tile order, groups
    // inner; the wave tree; the waves in order): 0 = dE/dgamma_l,
    // 1 = dE/dbeta_l, 2 = <C>
    double x0 = 0.0, x1 = 0.0, x2 = 0.0;
    for (int i = threadIdx.x; i < nt; i += THREADS) {
        x0 += part.gg[(size_t)l * T + tb + i];
        for (int g = 0; g < G; ++g) x1 += part.gb[((size_t)l * MAX_GROUPS + g) * T + tb + i];
        if (l == 0) x2 += part.e[tb + i];
    }
    for (int off = 32; off > 0; off >>= 1) {
        x0 += __shfl_xor(x0, off);
        x1 += __shfl_xor(x1, off);
        x2 += __shfl_xor(x2, off);
    }
    if (lane == 0) {
        red[0][wv] = x0;
        red[1][wv] = x1;
        red[2][wv] = x2;
    }
    // bias corrections while the sums complete
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    __syncthreads();
    if (threadIdx.x < 2) {
        const int q = threadIdx.x;  // 0: gamma_l, 1: beta_l
        double acc = 0.0;
        for (int w = 0; w < NW; ++w) acc += red[q][w];
        const size_t idx = (q == 0 ? 0 : (size_t)B * p) + (size_t)b * p + l;
        double th = theta[idx], mi = m[idx], vi = v[idx];
        adam_update(th, mi, vi, 2.0 * acc, c1, c2, lr, b1, b2, eps, 1.0);
        m[idx] = mi;
        v[idx] = vi;
        theta[idx] = th;
        if (q == 0) s_gamma = th;
        else s_beta = th;
    } else if (threadIdx.x == 64 && l == 0 && E) {
        double e = 0.0;
        for (int w = 0; w < NW; ++w) e += red[2][w];
        E[b] = e;
    }
    __syncthreads();
    // the new angles' tables: the rotation parameters on the last thread,
    // beside the phase-table entries of the others
    if (threadIdx.x == THREADS - 1) prep_coef(ws, sd, l, s_beta);
    const double gm = s_gamma;
    for (int c = threadIdx.x; c < sd->lut_len; c += THREADS) prep_lut_entry(ws, sd, l, c, gm);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_reduce_adam(uint8_t* ws, const SubDesc* subs, int B, int p, Partials part, double* theta,
                              double* m, double* v, const int32_t* step, int32_t it, double lr, double b1,
                              double b2, double eps, double* E, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_adam, dim3(B * p), dim3(THREADS), 0, s, ws, subs, B, p, part, theta, m, v, step,
                       it, lr, b1, b2, eps, E);
    return hipGetLastError();
}

__global__ void k_step_advance(int32_t* step, int32_t n)
{
    if (threadIdx.x == 0) *step += n;
}

hipError_t launch_step_advance(int32_t* step, int32_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(64), 0, s, step, n);
    return hipGetLastError();
}

hipError_t launch_angle_prep(uint8_t* ws, const SubDesc* subs, int B, int p, const double* gamma,
                             const double* beta, hipStream_t s)
{
    hipLaunchKernelGGL(k_angle_prep, dim3(B * p), dim3(THREADS), 0, s, ws, subs, p, gamma, beta);
    return hipGetLastError();
}

hipError_t launch_reduce(const SubDesc* subs, int B, int p, int grad, Partials part, double* E,
                         double* dgamma, double* dbeta, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce, dim3(B, grad ? 1 + 2 * p : 1), dim3(THREADS), 0, s, subs, p, grad, part, E, dgamma,
                       dbeta);
    return hipGetLastError();
}

}  // namespace pq
