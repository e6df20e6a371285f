// DIA-format Jacobi PCG: the plain GPU form.
//
// The paper's fastest GPU solver stored the 7-band matrix in the diagonal
// (DIA) format and ran Jacobi-preconditioned CG (the algorithm of section
// 2.2) as a host-driven loop of library calls (section 2.6, Table 1, Fig. 5).
// This file keeps that structure, an explicit 7-diagonal SpMV plus vector
// kernels, with the vector work grouped into three kernels per iteration:
// the SpMV also sums p.q per block; one kernel updates x and r and sums
// r.(r/d) and r.r (z = r/d is never stored); one forms the new direction
// p = r/d + beta p. Alpha, beta and the stopping flag stay on the device,
// so the host only polls the flag every few iterations.
#include "pcg_common.hpp"
#include "solver.hpp"

#include <algorithm>

namespace pb {

namespace {

template <typename T>
__global__ void k_dia_build(Op<T> op, int nx, int64_t sp, int64_t npad, T* __restrict__ val) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x) {
        val[t] = op.d[t];
        val[npad + t] = t >= 1 ? -op.cx[t - 1] : T(0);
        val[2 * npad + t] = -op.cx[t];
        val[3 * npad + t] = t >= nx ? -op.cy[t - nx] : T(0);
        val[4 * npad + t] = -op.cy[t];
        val[5 * npad + t] = t >= sp ? -op.cz[t - sp] : T(0);
        val[6 * npad + t] = -op.cz[t];
    }
}

// y = A v by the 7 stored diagonals (one row per thread).
template <typename T>
__global__ __launch_bounds__(kBS) void k_dia_spmv(const T* __restrict__ val, const T* __restrict__ v,
                                                  int nx, int64_t sp, int64_t npad, T* __restrict__ y,
                                                  const SyncState* S) {
    if (S && stop(S)) return;
    const int64_t off[7] = {0, -1, 1, -(int64_t)nx, (int64_t)nx, -sp, sp};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x) {
        T acc = T(0);
#pragma unroll
        for (int dgl = 0; dgl < 7; ++dgl) {
            const int64_t c = t + off[dgl];
            if (c >= 0 && c < npad) acc += val[dgl * npad + t] * v[c];
        }
        y[t] = acc;
    }
}

// The SpMV q = A p of one block's range of rows, and the block's p.q.
template <typename T>
__global__ __launch_bounds__(kBS) void k_dia_spmv_dot(const T* __restrict__ val, const T* __restrict__ p, int nx,
                                                      int64_t sp, int64_t npad, int64_t per, T* __restrict__ q,
                                                      double* __restrict__ partials, const SyncState* S) {
    if (stop(S)) return;
    const int64_t off[7] = {0, -1, 1, -(int64_t)nx, (int64_t)nx, -sp, sp};
    double acc[1] = {0.0};
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(lo + per, npad);
    for (int64_t t = lo + threadIdx.x; t < hi; t += kBS) {
        T y = T(0);
#pragma unroll
        for (int dgl = 0; dgl < 7; ++dgl) {
            const int64_t c = t + off[dgl];
            if (c >= 0 && c < npad) y += val[dgl * npad + t] * p[c];
        }
        q[t] = y;
        acc[0] += (double)p[t] * (double)y;
    }
    block_sum_store<1>(acc, partials + (size_t)blockIdx.x * kMaxPartials);
}

// x += alpha p, r -= alpha q over a block's range, and the block's r.(r/d)
// and r.r for beta and the stopping test.
template <typename T>
__global__ __launch_bounds__(kBS) void k_dia_update(T* __restrict__ x, const T* __restrict__ p, T* __restrict__ r,
                                                    const T* __restrict__ q, const T* __restrict__ d, int64_t npad,
                                                    int64_t per, double* __restrict__ partials, const SyncState* S) {
    if (stop(S)) return;
    const T alpha = (T)S->alpha;
    double acc[2] = {0.0, 0.0};
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(lo + per, npad);
    for (int64_t t = lo + threadIdx.x; t < hi; t += kBS) {
        x[t] = x[t] + alpha * p[t];
        const T rv = r[t] - alpha * q[t];
        r[t] = rv;
        const T zv = rv / d[t];
        acc[0] += (double)rv * (double)zv;
        acc[1] += (double)rv * (double)rv;
    }
    block_sum_store<2>(acc, partials + (size_t)blockIdx.x * kMaxPartials);
}

// p = r/d + beta p.
template <typename T>
__global__ void k_dia_direction(const T* __restrict__ r, const T* __restrict__ d, T* __restrict__ p, int64_t npad,
                                const SyncState* S) {
    if (stop(S)) return;
    const T beta = (T)S->beta;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x)
        p[t] = r[t] / d[t] + beta * p[t];
}

// Initial state: r = b - A x (q holds A x), p = r/d; partials r.(r/d), r.r, b.b.
template <typename T>
__global__ __launch_bounds__(kBS) void k_init(const T* __restrict__ b, const T* __restrict__ q,
                                              const T* __restrict__ d, T* __restrict__ r, T* __restrict__ p,
                                              int64_t npad, int64_t per, double* __restrict__ partials) {
    double acc[3] = {0.0, 0.0, 0.0};
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(lo + per, npad);
    for (int64_t t = lo + threadIdx.x; t < hi; t += kBS) {
        const T rv = b[t] - q[t];
        const T zv = rv / d[t];
        r[t] = rv;
        p[t] = zv;
        acc[0] += (double)rv * (double)zv;
        acc[1] += (double)rv * (double)rv;
        acc[2] += (double)b[t] * (double)b[t];
    }
    block_sum_store<3>(acc, partials + (size_t)blockIdx.x * kMaxPartials);
}

}  // namespace

// Host loop of the DIA form; S holds the device-side scalars and the stopping flag.
template <typename T>
pb_status dia_jpcg_impl(const Layout& L, const SolveBufs<T>& s, SyncState* S, double* partials, double tol,
                        int maxiter, hipStream_t st, SolveResult* res) {
    const int64_t npad = L.npad;
    const Ranges R = ranges_for(npad);
    const unsigned g = stream_grid(npad);
    if (launch_fill<int>((int*)S, (int64_t)(sizeof(SyncState) / sizeof(int)), 0, st) != PB_OK) return PB_ERR_HIP;
    hipEvent_t ev[2] = {nullptr, nullptr};
    const bool timed = !(res && res->untimed);
    if (timed) {
        PB_HIP(hipEventCreate(&ev[0]));
        PB_HIP(hipEventCreate(&ev[1]));
    }
    hipLaunchKernelGGL(k_dia_build<T>, dim3(g), dim3(kBS), 0, st, s.op, L.nx, L.sp, npad, s.dia);
    // r = b - A x0 (x0 = 0 gives r = b exactly)
    hipLaunchKernelGGL(k_dia_spmv<T>, dim3(g), dim3(kBS), 0, st, s.dia, (const T*)s.x, L.nx, L.sp, npad, s.q,
                       (const SyncState*)nullptr);
    hipLaunchKernelGGL(k_init<T>, dim3(R.nblk), dim3(kBS), 0, st, s.b, (const T*)s.q, s.op.d, s.r, s.p0, npad,
                       R.per, partials);
    hipLaunchKernelGGL(k_scalar_init, dim3(1), dim3(kBS), 0, st, S, (const double*)partials, R.nblk, tol, maxiter);
    PB_HIP(hipGetLastError());
    if (timed) PB_HIP(hipEventRecord(ev[0], st));
    int it = 0;
    SyncState h{};
    for (;;) {
        for (int u = 0; u < kPoll && it < maxiter; ++u, ++it) {
            hipLaunchKernelGGL(k_dia_spmv_dot<T>, dim3(R.nblk), dim3(kBS), 0, st, s.dia, (const T*)s.p0, L.nx,
                               L.sp, npad, R.per, s.q, partials, (const SyncState*)S);
            hipLaunchKernelGGL(k_scalar_alpha, dim3(1), dim3(kBS), 0, st, S, (const double*)partials, R.nblk);
            hipLaunchKernelGGL(k_dia_update<T>, dim3(R.nblk), dim3(kBS), 0, st, s.x, (const T*)s.p0, s.r,
                               (const T*)s.q, s.op.d, npad, R.per, partials, (const SyncState*)S);
            hipLaunchKernelGGL(k_scalar_beta, dim3(1), dim3(kBS), 0, st, S, (const double*)partials, R.nblk, tol,
                               maxiter);
            hipLaunchKernelGGL(k_dia_direction<T>, dim3(g), dim3(kBS), 0, st, (const T*)s.r, s.op.d, s.p0, npad,
                               (const SyncState*)S);
        }
        PB_HIP(hipGetLastError());
        PB_HIP(hipMemcpyAsync(&h, S, sizeof(SyncState), hipMemcpyDeviceToHost, st));
        PB_HIP(hipStreamSynchronize(st));
        if (h.done || it >= maxiter) break;
    }
    if (timed) PB_HIP(hipEventRecord(ev[1], st));
    hipLaunchKernelGGL(k_zero_if_zero_rhs<T>, dim3(g), dim3(kBS), 0, st, s.x, npad, (const SyncState*)S);
    PB_HIP(hipGetLastError());
    PB_HIP(hipMemcpyAsync(&h, S, sizeof(SyncState), hipMemcpyDeviceToHost, st));
    PB_HIP(hipStreamSynchronize(st));
    float ms = 0.0f;
    if (timed) {
        PB_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
    }
    if (res) {
        res->kernel_seconds = 1e-3 * ms;
        res->status = h.done ? h.status : (int)PB_NOT_CONVERGED;
        res->iters = h.iters;
        res->rr = h.rr;
        res->bb = h.bb;
    }
    return PB_OK;
}

template pb_status dia_jpcg_impl<float>(const Layout&, const SolveBufs<float>&, SyncState*, double*, double, int,
                                        hipStream_t, SolveResult*);
template pb_status dia_jpcg_impl<double>(const Layout&, const SolveBufs<double>&, SyncState*, double*, double,
                                         int, hipStream_t, SolveResult*);

}  // namespace pb
