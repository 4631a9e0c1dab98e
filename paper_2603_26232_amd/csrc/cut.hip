// Integer cut evaluation (paper Sec. 2.1 CutVal, used on merged full-graph
// assignments in Alg. 2) and the FP64 Adam step of the angle optimiser.
#include "common.h"

namespace pq {

__device__ inline int64_t block_sum_i64(int64_t x, int64_t* red)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    const uint32_t tid = threadIdx.x;
    if ((tid & 63u) == 0) red[tid >> 6] = x;
    __syncthreads();
    int64_t s = 0;
    if (tid == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    __syncthreads();
    return s;
}

// cut[a] = sum_e w_e [x_a(u_e) != x_a(v_e)], x_a bit-packed (vertex t = word
// t/32, bit t%32). An edge id outside [0, nV) makes the result -1.
__global__ __launch_bounds__(THREADS) void k_maxcut(int32_t nV, int64_t nE, const int32_t* u, const int32_t* v,
                                                   const int32_t* w, int64_t A, const uint32_t* assign,
                                                   int64_t* cut)
{
    __shared__ int64_t red[THREADS / 64];
    const int64_t nw = (nV + 31) / 32;
    for (int64_t a = blockIdx.x; a < A; a += gridDim.x) {
        const uint32_t* x = assign + a * nw;
        int64_t acc = 0, bad = 0;
        for (int64_t e = threadIdx.x; e < nE; e += THREADS) {
            const int32_t p = u[e], q = v[e];
            if ((uint32_t)p >= (uint32_t)nV || (uint32_t)q >= (uint32_t)nV) {
                bad = 1;
                continue;
            }
            const uint32_t xp = (x[p >> 5] >> (p & 31)) & 1u;
            const uint32_t xq = (x[q >> 5] >> (q & 31)) & 1u;
            if (xp != xq) acc += w ? (int64_t)w[e] : 1;
        }
        acc = block_sum_i64(acc, red);
        bad = block_sum_i64(bad, red);
        if (threadIdx.x == 0) cut[a] = bad ? -1 : acc;
    }
}

hipError_t launch_maxcut_eval(int32_t nV, int64_t nE, const int32_t* u, const int32_t* v, const int32_t* w,
                              int64_t A, const uint32_t* assign, int64_t* cut, hipStream_t s)
{
    if (A <= 0) return hipSuccess;
    const int64_t grid = A < 65536 ? A : 65536;
    hipLaunchKernelGGL(k_maxcut, dim3((unsigned)grid), dim3(THREADS), 0, s, nV, nE, u, v, w, A, assign, cut);
    return hipGetLastError();
}

// Adam (Kingma and Ba 2015) in FP64; sign = +1 ascends (the QAOA objective
// is maximised), -1 descends. The step counter lives in device memory so a
// captured graph can replay the step.
__global__ __launch_bounds__(1024) void k_adam(int32_t count, double* theta, const double* grad, double* m,
                                              double* v, int32_t* step, double lr, double b1, double b2,
                                              double eps, double sign)
{
    const int32_t t = *step + 1;
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int32_t i = threadIdx.x; i < count; i += blockDim.x) {
        double th = theta[i], mi = m[i], vi = v[i];
        adam_update(th, mi, vi, grad[i], c1, c2, lr, b1, b2, eps, sign);
        m[i] = mi;
        v[i] = vi;
        theta[i] = th;
    }
    __syncthreads();
    if (threadIdx.x == 0) *step = t;
}

hipError_t launch_adam(int32_t count, double* theta, const double* grad, double* m, double* v, int32_t* step,
                       double lr, double b1, double b2, double eps, double sign, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3(1), dim3(1024), 0, s, count, theta, grad, m, v, step, lr, b1, b2, eps, sign);
    return hipGetLastError();
}

}  // namespace pq
