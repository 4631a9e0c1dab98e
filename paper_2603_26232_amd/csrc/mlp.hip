// Angle predictor for the learned warm start: a multilayer perceptron
// in -> H -> H -> out (ReLU hidden layers, linear output) over per-subgraph
// features, trained with a mean-squared error on optimised angles. The
// paper motivates it only indirectly (Sec. 2.2: initialisation affects the
// quality and the iteration count of the angle optimisation).
//
// Parameters are FP64 master weights (updated by the FP64 Adam kernel);
// forward and backward arithmetic is FP32 with FP64 gradient accumulation.
// Flat layout, row-major: W1[H][in], b1[H], W2[H][H], b2[H], W3[out][H],
// b3[out]. Every reduction runs in a fixed order (bit-reproducible).
#include <mutex>

#include "common.h"

namespace pq {

__host__ __device__ inline int64_t mlp_off_b1(const MlpDims& d) { return (int64_t)d.H * d.in; }
__host__ __device__ inline int64_t mlp_off_W2(const MlpDims& d) { return mlp_off_b1(d) + d.H; }
__host__ __device__ inline int64_t mlp_off_b2(const MlpDims& d) { return mlp_off_W2(d) + (int64_t)d.H * d.H; }
__host__ __device__ inline int64_t mlp_off_W3(const MlpDims& d) { return mlp_off_b2(d) + d.H; }
__host__ __device__ inline int64_t mlp_off_b3(const MlpDims& d) { return mlp_off_W3(d) + (int64_t)d.out * d.H; }
__host__ __device__ int64_t mlp_nparams(const MlpDims& d) { return mlp_off_b3(d) + d.out; }
int64_t mlp_num_params(const MlpDims& d) { return mlp_nparams(d); }

// one workgroup per sample; act[s] = (h1[H], h2[H])
__global__ __launch_bounds__(MLP_MAX_H) void k_mlp_fwd(int B, MlpDims d, const double* P, const float* X, float* Y,
                                                      float* act)
{
    __shared__ float xs[MLP_MAX_IN], h1s[MLP_MAX_H], h2s[MLP_MAX_H];
    const int s = blockIdx.x, i = threadIdx.x;
    const double* W1 = P;
    const double* b1 = P + mlp_off_b1(d);
    const double* W2 = P + mlp_off_W2(d);
    const double* b2 = P + mlp_off_b2(d);
    const double* W3 = P + mlp_off_W3(d);
    const double* b3 = P + mlp_off_b3(d);
    if (i < d.in) xs[i] = X[(size_t)s * d.in + i];
    __syncthreads();
    if (i < d.H) {
        float a = (float)b1[i];
        for (int f = 0; f < d.in; ++f) a += (float)W1[(size_t)i * d.in + f] * xs[f];
        a = a > 0.f ? a : 0.f;
        h1s[i] = a;
        act[(size_t)s * 2 * d.H + i] = a;
    }
    __syncthreads();
    if (i < d.H) {
        float a = (float)b2[i];
        for (int j = 0; j < d.H; ++j) a += (float)W2[(size_t)i * d.H + j] * h1s[j];
        a = a > 0.f ? a : 0.f;
        h2s[i] = a;
        act[(size_t)s * 2 * d.H + d.H + i] = a;
    }
    __syncthreads();
    if (i < d.out) {
        float a = (float)b3[i];
        for (int j = 0; j < d.H; ++j) a += (float)W3[(size_t)i * d.H + j] * h2s[j];
        Y[(size_t)s * d.out + i] = a;
    }
}

// per-sample back-propagated errors: delta[s] = (d1[H], d2[H], d3[out]); the
// squared error of the sample goes to sq[s]
__global__ __launch_bounds__(MLP_MAX_H) void k_mlp_delta(int B, MlpDims d, const double* P, const float* Y,
                                                        const float* act, const float* T, float* delta, double* sq)
{
    __shared__ float d3s[MLP_MAX_OUT], d2s[MLP_MAX_H];
    __shared__ double sqs[MLP_MAX_OUT];
    const int s = blockIdx.x, i = threadIdx.x;
    const double* W2 = P + mlp_off_W2(d);
    const double* W3 = P + mlp_off_W3(d);
    const float scale = 1.0f / ((float)B * (float)d.out);
    const float* h1 = act + (size_t)s * 2 * d.H;
    const float* h2 = h1 + d.H;
    float* dl = delta + (size_t)s * (2 * d.H + d.out);
    if (i < d.out) {
        const float r = Y[(size_t)s * d.out + i] - T[(size_t)s * d.out + i];
        d3s[i] = 2.f * r * scale;
        sqs[i] = (double)r * (double)r;
        dl[2 * d.H + i] = d3s[i];
    }
    __syncthreads();
    if (i == 0) {
        double a = 0.0;
        for (int o = 0; o < d.out; ++o) a += sqs[o];
        sq[s] = a;
    }
    if (i < d.H) {
        float a = 0.f;
        for (int o = 0; o < d.out; ++o) a += (float)W3[(size_t)o * d.H + i] * d3s[o];
        a = h2[i] > 0.f ? a : 0.f;
        d2s[i] = a;
        dl[d.H + i] = a;
    }
    __syncthreads();
    if (i < d.H) {
        float a = 0.f;
        for (int k = 0; k < d.H; ++k) a += (float)W2[(size_t)k * d.H + i] * d2s[k];
        dl[i] = h1[i] > 0.f ? a : 0.f;
    }
}

// one thread per parameter: sum over samples in order (FP32 products, FP64 sum)
__global__ void k_mlp_wgrad(int B, MlpDims d, const float* X, const float* act, const float* delta, double* G)
{
    const int64_t np = mlp_nparams(d);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    const int DS = 2 * d.H + d.out;
    int dsel, drow, isel, icol;  // delta slot / input slot (-1: bias)
    // isel: 0 = x, 1 = h1, 2 = h2; dsel: 0 = d1, 1 = d2, 2 = d3
    if (p < mlp_off_b1(d)) {
        dsel = 0; drow = (int)(p / d.in); isel = 0; icol = (int)(p % d.in);
    } else if (p < mlp_off_W2(d)) {
        dsel = 0; drow = (int)(p - mlp_off_b1(d)); isel = -1; icol = 0;
    } else if (p < mlp_off_b2(d)) {
        const int64_t q = p - mlp_off_W2(d);
        dsel = 1; drow = (int)(q / d.H); isel = 1; icol = (int)(q % d.H);
    } else if (p < mlp_off_W3(d)) {
        dsel = 1; drow = (int)(p - mlp_off_b2(d)); isel = -1; icol = 0;
    } else if (p < mlp_off_b3(d)) {
        const int64_t q = p - mlp_off_W3(d);
        dsel = 2; drow = (int)(q / d.H); isel = 2; icol = (int)(q % d.H);
    } else {
        dsel = 2; drow = (int)(p - mlp_off_b3(d)); isel = -1; icol = 0;
    }
    const int doff = dsel == 0 ? 0 : (dsel == 1 ? d.H : 2 * d.H);
    double acc = 0.0;
    for (int s = 0; s < B; ++s) {
        const float dv = delta[(size_t)s * DS + doff + drow];
        float in = 1.f;
        if (isel == 0) in = X[(size_t)s * d.in + icol];
        else if (isel == 1) in = act[(size_t)s * 2 * d.H + icol];
        else if (isel == 2) in = act[(size_t)s * 2 * d.H + d.H + icol];
        acc += (double)(dv * in);
    }
    G[p] = acc;
}

__global__ void k_mlp_loss(int B, int out, const double* sq, double* loss)
{
    __shared__ double red[256];
    double a = 0.0;
    for (int s = threadIdx.x; s < B; s += blockDim.x) a += sq[s];
    red[threadIdx.x] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += red[i];
        *loss = t / ((double)B * (double)out);
    }
}

// Warm-start angles from the predictor's standardised outputs: output o of
// subgraph b becomes y * sd[o] + mu[o] (FP32, rounded as written), then FP64;
// outputs 0..p-1 are gamma_1..p, outputs p..2p-1 are beta_1..p, and theta is
// laid out [gamma (B p) | beta (B p)], row b = subgraph b.
__global__ void k_warm_angles(int B, int p, const float* Y, const float* mu, const float* sd, double* theta)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * B * p) return;
    const int b = i / (2 * p), o = i % (2 * p);
    const float a = Y[i] * sd[o] + mu[o];  // two roundings, never one fused multiply-add
    const size_t dst = o < p ? (size_t)b * p + o : (size_t)B * p + (size_t)b * p + (o - p);
    theta[dst] = (double)a;
}

// Per subgraph, keep the start with the larger <C>: if E_alt[b] > E[b], row b
// of theta (its gamma and beta) and E[b] take the alternative's values. One
// thread per subgraph, so the comparison and the copy see the same E[b].
__global__ void k_keep_better(int B, int p, const double* E_alt, const double* theta_alt, double* E, double* theta)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double ea = E_alt[b];
    if (!(ea > E[b])) return;
    for (int l = 0; l < p; ++l) {
        const size_t g = (size_t)b * p + l, t = (size_t)B * p + g;
        theta[g] = theta_alt[g];
        theta[t] = theta_alt[t];
    }
    E[b] = ea;
}

hipError_t launch_warm_angles(int B, int p, const float* Y, const float* mu, const float* sd, double* theta,
                              hipStream_t s)
{
    const int n = 2 * B * p;
    hipLaunchKernelGGL(k_warm_angles, dim3((n + 255) / 256), dim3(256), 0, s, B, p, Y, mu, sd, theta);
    return hipGetLastError();
}

hipError_t launch_keep_better(int B, int p, const double* E_alt, const double* theta_alt, double* E, double* theta,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_keep_better, dim3((B + 255) / 256), dim3(256), 0, s, B, p, E_alt, theta_alt, E, theta);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(int B, MlpDims d, const double* P, const float* X, float* Y, float* act, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_fwd, dim3(B), dim3(MLP_MAX_H), 0, s, B, d, P, X, Y, act);
    return hipGetLastError();
}

hipError_t launch_mlp_backward(int B, MlpDims d, const double* P, const float* X, const float* Y, const float* act,
                               const float* T, float* scratch, double* G, double* loss, hipStream_t s)
{
    float* delta = scratch;
    double* sq = (double*)(scratch + (size_t)B * (2 * d.H + d.out) + 1);  // 8-byte aligned below
    sq = (double*)(((uintptr_t)sq + 7) & ~(uintptr_t)7);
    hipLaunchKernelGGL(k_mlp_delta, dim3(B), dim3(MLP_MAX_H), 0, s, B, d, P, Y, act, T, delta, sq);
    const int64_t np = mlp_num_params(d);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, B, d, X, act, delta, G);
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, s, B, d.out, sq, loss);
    return hipGetLastError();
}

// Scratch of the backward pass for callers that cannot allocate: a
// file-scope device array (each device holds its own copy until the process
// ends). Host code never passes the array's name to a kernel: its device
// address is looked up once per device with hipGetSymbolAddress and kept.
static __device__ __align__(256) uint8_t scratch[MLP_STATIC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t mlp_static_scratch(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace pq
