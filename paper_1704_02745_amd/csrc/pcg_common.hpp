// Pieces of the host-driven preconditioned CG loops (the DIA form and the
// multigrid form): fixed-order block reductions, the device-side scalars and
// stopping flag in SyncState, and the vector kernels of the section 2.2
// listing. Every kernel after the start returns at once when the flag is
// set, so the host only polls it every few iterations.
#pragma once

#include "pb_internal.hpp"
#include "solver.hpp"

#include <algorithm>

namespace pb {
namespace {

constexpr int kBS = 256;
constexpr int kPoll = 8;   // host checks the stopping flag every kPoll iterations

struct Ranges {
    int nblk;
    int64_t per;
};

// Block ranges of the kernels that also store per-block sums: about 1024
// positions per block, at most 4096 blocks (the single-workgroup scalar
// kernels sum every block's partials; at 16384 blocks that alone took about
// 15 us per reduction). The block length is a multiple of 4 (the four-wide
// kernels' groups).
Ranges ranges_for(int64_t npad) {
    Ranges r;
    const int64_t nb = std::min<int64_t>(4096, std::max<int64_t>(1, (npad + 1023) / 1024));
    r.per = ((npad + nb - 1) / nb + 3) / 4 * 4;
    r.nblk = (int)((npad + r.per - 1) / r.per);
    return r;
}

__device__ __forceinline__ bool stop(const SyncState* S) { return *(volatile const int*)&S->done != 0; }

template <int NP>
__device__ void block_sum_store(double (&acc)[NP], double* dst) {
    __shared__ double s[NP][kBS];
#pragma unroll
    for (int i = 0; i < NP; ++i) s[i][threadIdx.x] = acc[i];
    __syncthreads();
    for (int w = kBS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int i = 0; i < NP; ++i) s[i][threadIdx.x] += s[i][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < NP; ++i) dst[i] = s[i][0];
}

template <int NP>
__device__ void sum_blocks(const double* partials, int nblk, double (&out)[NP]) {
    __shared__ double s[NP][kBS];
    double acc[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) acc[i] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kBS)
#pragma unroll
        for (int i = 0; i < NP; ++i) acc[i] += partials[(size_t)b * kMaxPartials + i];
#pragma unroll
    for (int i = 0; i < NP; ++i) s[i][threadIdx.x] = acc[i];
    __syncthreads();
    for (int w = kBS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int i = 0; i < NP; ++i) s[i][threadIdx.x] += s[i][threadIdx.x + w];
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) out[i] = s[i][0];
}

// Diagonals in the padded layout at offsets {0, -1, +1, -nx, +nx, -sp, +sp}.
__global__ __launch_bounds__(kBS) void k_scalar_init(SyncState* S, const double* partials, int nblk,
                                                     double tol, int maxiter) {
    double s[3];
    sum_blocks<3>(partials, nblk, s);
    if (threadIdx.x == 0) {
        S->rho = s[0];
        S->rr = s[1];
        S->bb = s[2];
        S->iters = 0;
        S->alpha = 0.0;
        int done = 0, status = PB_OK;
        if (!(s[2] - s[2] == 0.0) || !(s[1] - s[1] == 0.0)) { done = 1; status = PB_ERR_NONFINITE; }
        else if (s[2] == 0.0) { done = 1; S->zero_rhs = 1; }
        else if (sqrt(s[1]) / sqrt(s[2]) < tol) done = 1;
        else if (maxiter <= 0) { done = 1; status = PB_NOT_CONVERGED; }
        S->status = status;
        S->done = done;
    }
}

template <typename T>
__global__ __launch_bounds__(kBS) void k_dot(const T* __restrict__ a, const T* __restrict__ b, int64_t npad,
                                             int64_t per, double* __restrict__ partials, const SyncState* S) {
    if (stop(S)) return;
    double acc[1] = {0.0};
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(lo + per, npad);
    for (int64_t t = lo + threadIdx.x; t < hi; t += kBS) acc[0] += (double)a[t] * (double)b[t];
    block_sum_store<1>(acc, partials + (size_t)blockIdx.x * kMaxPartials);
}

__global__ __launch_bounds__(kBS) void k_scalar_alpha(SyncState* S, const double* partials, int nblk) {
    if (stop(S)) return;
    double s[1];
    sum_blocks<1>(partials, nblk, s);
    if (threadIdx.x == 0) {
        const double pq = s[0];
        S->pq = pq;
        if (!(pq > 0.0) || !(pq - pq == 0.0)) {
            S->status = PB_ERR_BREAKDOWN;
            S->alpha = 0.0;
            S->done = 2;   // 2: stop before the x update of this iteration
        } else {
            S->alpha = S->rho / pq;
        }
    }
}

template <typename T>
__global__ void k_axpy2(T* __restrict__ x, const T* __restrict__ p, T* __restrict__ r, const T* __restrict__ q,
                        int64_t npad, const SyncState* S) {
    if (stop(S)) return;
    const T alpha = (T)S->alpha;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x) {
        x[t] = x[t] + alpha * p[t];
        r[t] = r[t] - alpha * q[t];
    }
}

__global__ __launch_bounds__(kBS) void k_scalar_beta(SyncState* S, const double* partials, int nblk,
                                                     double tol, int maxiter) {
    if (stop(S)) return;
    double s[2];
    sum_blocks<2>(partials, nblk, s);
    if (threadIdx.x == 0) {
        const int iters = S->iters + 1;
        S->iters = iters;
        S->beta = s[0] / S->rho;
        S->rho = s[0];
        S->rr = s[1];
        const double rel = sqrt(s[1]) / sqrt(S->bb);
        if (!(rel - rel == 0.0)) { S->done = 1; S->status = PB_ERR_BREAKDOWN; }
        else if (rel < tol) { S->done = 1; S->status = PB_OK; }
        else if (iters >= maxiter) { S->done = 1; S->status = PB_NOT_CONVERGED; }
    }
}

template <typename T>
__global__ void k_xpay(const T* __restrict__ z, T* __restrict__ p, int64_t npad, const SyncState* S) {
    if (stop(S)) return;
    const T beta = (T)S->beta;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x)
        p[t] = z[t] + beta * p[t];
}

template <typename T>
__global__ void k_zero_if_zero_rhs(T* __restrict__ x, int64_t npad, const SyncState* S) {
    if (!S->zero_rhs) return;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x)
        x[t] = T(0);
}

unsigned stream_grid(int64_t n) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kBS - 1) / kBS, 16384));
}

}  // namespace
}  // namespace pb
