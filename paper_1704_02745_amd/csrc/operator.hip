// Operator preparation, FP64 residual and small vector kernels.
//
// The caller's arrays (staggered edge dielectrics, kbar^2, right-hand side,
// potential) are converted once per solve into the padded internal layout
// (see Layout in pb_internal.hpp): coupling arrays cx, cy, cz with the 1/h^2
// factor applied, and the full diagonal of Eq. 3, d = (sum of the six edge
// dielectrics)/h^2 + kbar^2. With the free-space boundary the couplings are
// zero across the box faces; with the periodic boundary the last node of a
// row, column or z-line holds the wrap coupling to the first.
#include "pb_internal.hpp"
#include "solver.hpp"

namespace pb {

__device__ __forceinline__ bool finite_d(double v) { return v - v == 0.0; }

// Unpadded node index -> (i, j, k); plane stride sp in the padded layout.
__global__ void k_prepare64(const double* __restrict__ ex, const double* __restrict__ ey,
                            const double* __restrict__ ez, const double* __restrict__ k2,
                            const double* __restrict__ rhs, const double* __restrict__ xin,
                            int warm, int per, int nx, int ny, int nz, int64_t sp, double hh,
                            double* __restrict__ cx, double* __restrict__ cy, double* __restrict__ cz,
                            double* __restrict__ d, double* __restrict__ b, double* __restrict__ x,
                            int* __restrict__ flags) {
    const int64_t plane = (int64_t)nx * ny;
    const int64_t npad = sp * nz;
    int bad = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = t / sp;
        const int64_t pp = t - k * sp;
        if (pp >= plane) {   // pad slot
            cx[t] = 0.0; cy[t] = 0.0; cz[t] = 0.0; d[t] = 1.0; b[t] = 0.0; x[t] = 0.0;
            continue;
        }
        const int64_t j = pp / nx, i = pp - j * nx;
        const int64_t n = pp + plane * k;
        const double exm = ex[i + (int64_t)(nx + 1) * (j + (int64_t)ny * k)];
        const double exp_ = ex[i + 1 + (int64_t)(nx + 1) * (j + (int64_t)ny * k)];
        const double eym = ey[i + (int64_t)nx * (j + (int64_t)(ny + 1) * k)];
        const double eyp = ey[i + (int64_t)nx * (j + 1 + (int64_t)(ny + 1) * k)];
        const double ezm = ez[i + (int64_t)nx * (j + (int64_t)ny * k)];
        const double ezp = ez[i + (int64_t)nx * (j + (int64_t)ny * (k + 1))];
        const double kk = k2[n];
        const double dd = (((((exm + exp_) + eym) + eyp) + ezm) + ezp) / hh + kk;
        if (!(exm >= 0.0 && exp_ >= 0.0 && eym >= 0.0 && eyp >= 0.0 && ezm >= 0.0 && ezp >= 0.0 &&
              kk >= 0.0 && finite_d(dd) && dd > 0.0))
            bad |= FLAG_BAD_COEF;
        cx[t] = (per || i < nx - 1) ? exp_ / hh : 0.0;
        cy[t] = (per || j < ny - 1) ? eyp / hh : 0.0;
        cz[t] = (per || k < nz - 1) ? ezp / hh : 0.0;
        if (kk > 0.0) bad |= FLAG_HAS_SALT;
        d[t] = dd;
        const double bv = rhs[n];
        if (!finite_d(bv)) bad |= FLAG_BAD_RHS;
        b[t] = bv;
        double xv = 0.0;
        if (warm) {
            xv = xin[n];
            if (!finite_d(xv)) bad |= FLAG_BAD_GUESS;
        }
        x[t] = xv;
    }
    if (bad) atomicOr(flags, bad);
}

// FP32 rounding of the FP64 operator (the inner matrix of refinement is the
// FP32 rounding of the FP64 coefficients).
__global__ void k_round32(const double* __restrict__ cx, const double* __restrict__ cy,
                          const double* __restrict__ cz, const double* __restrict__ d,
                          const double* __restrict__ b, const double* __restrict__ x, int64_t npad,
                          float* __restrict__ cx32, float* __restrict__ cy32, float* __restrict__ cz32,
                          float* __restrict__ d32, float* __restrict__ b32, float* __restrict__ x32) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x) {
        cx32[t] = (float)cx[t];
        cy32[t] = (float)cy[t];
        cz32[t] = (float)cz[t];
        d32[t] = (float)d[t];
        if (b32) b32[t] = (float)b[t];
        if (x32) x32[t] = (float)x[t];
    }
}

// r = b - A x in FP64 over the padded layout, with per-block partial sums of
// r.r and b.b (each block handles a contiguous range; the block order is fixed).
// Optionally writes r (FP64) and its FP32 rounding.
// Periodic boundary (PER): neighbours wrap within each row, column and
// z-line; the wrap coupling sits at the last node of the line.
template <int BS, bool PER>
__global__ __launch_bounds__(BS) void k_residual64(
        const double* __restrict__ cx, const double* __restrict__ cy, const double* __restrict__ cz,
        const double* __restrict__ d, const double* __restrict__ b, const double* __restrict__ x,
        int nx, int ny, int nz, int64_t sp, int64_t npad, int64_t per_block, double* __restrict__ r64,
        float* __restrict__ r32, double* __restrict__ partials) {
    const int64_t lo = (int64_t)blockIdx.x * per_block;
    const int64_t hi = min(lo + per_block, npad);
    const int64_t plane = (int64_t)nx * ny;
    double rr = 0.0, bb = 0.0;
    for (int64_t t = lo + threadIdx.x; t < hi; t += BS) {
        double nb;
        if constexpr (PER) {
            const int64_t k = t / sp, pp = t - k * sp;
            if (pp >= plane) {
                nb = 0.0;
            } else {
                const int64_t j = pp / nx, i = pp - j * nx;
                const int64_t xr = (i == nx - 1) ? t - (nx - 1) : t + 1;
                const int64_t xl = (i == 0) ? t + (nx - 1) : t - 1;
                const int64_t yu = (j == ny - 1) ? t - (int64_t)(ny - 1) * nx : t + nx;
                const int64_t yd = (j == 0) ? t + (int64_t)(ny - 1) * nx : t - nx;
                const int64_t zu = (k == nz - 1) ? t - (int64_t)(nz - 1) * sp : t + sp;
                const int64_t zd = (k == 0) ? t + (int64_t)(nz - 1) * sp : t - sp;
                nb = cx[t] * x[xr];
                nb += cx[xl] * x[xl];
                nb += cy[t] * x[yu];
                nb += cy[yd] * x[yd];
                nb += cz[t] * x[zu];
                nb += cz[zd] * x[zd];
            }
        } else {
            nb = cx[t] * (t + 1 < npad ? x[t + 1] : 0.0);
            nb += (t >= 1 ? cx[t - 1] * x[t - 1] : 0.0);
            nb += cy[t] * (t + nx < npad ? x[t + nx] : 0.0);
            nb += (t >= nx ? cy[t - nx] * x[t - nx] : 0.0);
            nb += cz[t] * (t + sp < npad ? x[t + sp] : 0.0);
            nb += (t >= sp ? cz[t - sp] * x[t - sp] : 0.0);
        }
        const double bv = b[t];
        const double rv = bv - (d[t] * x[t] - nb);
        if (r64) r64[t] = rv;
        if (r32) r32[t] = (float)rv;
        rr += rv * rv;
        bb += bv * bv;
    }
    __shared__ double s[2][BS];
    s[0][threadIdx.x] = rr;
    s[1][threadIdx.x] = bb;
    __syncthreads();
    for (int w = BS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] += s[0][threadIdx.x + w];
            s[1][threadIdx.x] += s[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s[0][0];
        partials[2 * blockIdx.x + 1] = s[1][0];
    }
}

// Fixed-order reduction of `nblk` pairs of partials into out[0..1].
__global__ __launch_bounds__(256) void k_reduce_pairs(const double* __restrict__ partials, int nblk,
                                                      double* __restrict__ out) {
    __shared__ double s[2][256];
    double a = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < nblk; i += 256) {
        a += partials[2 * i];
        c += partials[2 * i + 1];
    }
    s[0][threadIdx.x] = a;
    s[1][threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] += s[0][threadIdx.x + w];
            s[1][threadIdx.x] += s[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s[0][0];
        out[1] = s[1][0];
    }
}

// Per-block partial sums of v over the real nodes of the padded layout
// (fixed block ranges), as (sum, 0) pairs for k_reduce_pairs.
template <int BS>
__global__ __launch_bounds__(BS) void k_real_sum(const double* __restrict__ v, int64_t plane, int64_t sp,
                                                 int64_t npad, int64_t per_block, double* __restrict__ partials) {
    const int64_t lo = (int64_t)blockIdx.x * per_block;
    const int64_t hi = min(lo + per_block, npad);
    double acc = 0.0;
    for (int64_t t = lo + threadIdx.x; t < hi; t += BS)
        if (t % sp < plane) acc += v[t];
    __shared__ double s[BS];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = BS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s[0];
        partials[2 * blockIdx.x + 1] = 0.0;
    }
}

// v -= sum[0] / n on the real nodes (pads stay zero).
__global__ void k_sub_mean(double* __restrict__ v, const double* __restrict__ sum, double n, int64_t plane,
                           int64_t sp, int64_t npad) {
    const double m = sum[0] / n;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x)
        if (t % sp < plane) v[t] = v[t] - m;
}

// x64 += (double) dx (padded layout).
__global__ void k_add_correction(double* __restrict__ x, const float* __restrict__ dx, int64_t npad) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x)
        x[t] = x[t] + (double)dx[t];
}

// Padded (T) -> caller's unpadded FP64 array.
template <typename T>
__global__ void k_unpad(const T* __restrict__ xp, int nx, int ny, int nz, int64_t sp,
                        double* __restrict__ out) {
    const int64_t plane = (int64_t)nx * ny;
    const int64_t n = plane * nz;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = t / plane;
        out[t] = (double)xp[t - k * plane + k * sp];
    }
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T v) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        p[t] = v;
}

__global__ void k_f32_to_f64(const float* __restrict__ a, double* __restrict__ b, int64_t n) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        b[t] = (double)a[t];
}

// The free-space k_residual64 with two consecutive positions per thread
// (16-byte loads of the node's own values and of the planes above and below;
// per_block even, so every pair is aligned): each r is formed with the same
// operations in the same order, so r64 and r32 are bit for bit those of
// k_residual64; the partial sums add the pair's two terms in turn.
__device__ __forceinline__ double2 ld2(const double* p) { return *reinterpret_cast<const double2*>(p); }
template <int BS>
__global__ __launch_bounds__(BS) void k_residual64_pairs(
        const double* __restrict__ cx, const double* __restrict__ cy, const double* __restrict__ cz,
        const double* __restrict__ d, const double* __restrict__ b, const double* __restrict__ x, int nx,
        int64_t sp, int64_t npad, int64_t per_block, double* __restrict__ r64, float* __restrict__ r32,
        double* __restrict__ partials) {
    const int64_t lo = (int64_t)blockIdx.x * per_block;
    const int64_t hi = min(lo + per_block, npad);
    double rr = 0.0, bb = 0.0;
    for (int64_t t = lo + 2 * (int64_t)threadIdx.x; t < hi; t += 2 * BS) {
        const double2 cxv = ld2(cx + t), cyv = ld2(cy + t), czv = ld2(cz + t), dv = ld2(d + t), bv2 = ld2(b + t),
                      xv = ld2(x + t);
        const double2 xzu = t + sp < npad ? ld2(x + t + sp) : make_double2(0.0, 0.0);
        const double2 xzd = t >= sp ? ld2(x + t - sp) : make_double2(0.0, 0.0);
        const double2 czd = t >= sp ? ld2(cz + t - sp) : make_double2(0.0, 0.0);
        const double xl = t >= 1 ? x[t - 1] : 0.0, cxl = t >= 1 ? cx[t - 1] : 0.0;
        const double xr = t + 2 < npad ? x[t + 2] : 0.0;
        double r2[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int64_t q = t + u;
            const double cxq = u ? cxv.y : cxv.x, cyq = u ? cyv.y : cyv.x, czq = u ? czv.y : czv.x;
            const double xq = u ? xv.y : xv.x;
            const double xnext = u ? xr : xv.y;                 // x[q + 1]
            const double xprev = u ? xv.x : xl, cprev = u ? cxv.x : cxl;   // x[q - 1], cx[q - 1]
            double nb = cxq * (q + 1 < npad ? xnext : 0.0);
            nb += (q >= 1 ? cprev * xprev : 0.0);
            nb += cyq * (q + nx < npad ? x[q + nx] : 0.0);
            nb += (q >= nx ? cy[q - nx] * x[q - nx] : 0.0);
            nb += czq * (q + sp < npad ? (u ? xzu.y : xzu.x) : 0.0);
            nb += (q >= sp ? (u ? czd.y : czd.x) * (u ? xzd.y : xzd.x) : 0.0);
            const double bq = u ? bv2.y : bv2.x;
            const double rv = bq - ((u ? dv.y : dv.x) * xq - nb);
            r2[u] = rv;
            rr += rv * rv;
            bb += bq * bq;
        }
        if (r64) *reinterpret_cast<double2*>(r64 + t) = make_double2(r2[0], r2[1]);
        if (r32) *reinterpret_cast<float2*>(r32 + t) = make_float2((float)r2[0], (float)r2[1]);
    }
    __shared__ double s[2][BS];
    s[0][threadIdx.x] = rr;
    s[1][threadIdx.x] = bb;
    __syncthreads();
    for (int w = BS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] += s[0][threadIdx.x + w];
            s[1][threadIdx.x] += s[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s[0][0];
        partials[2 * blockIdx.x + 1] = s[1][0];
    }
}

// ---------------------------------------------------------------- host wrappers

static unsigned grid_for(int64_t n, int bs = 256, int64_t cap = 8192) {
    int64_t b = (n + bs - 1) / bs;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

pb_status launch_prepare64(const double* ex, const double* ey, const double* ez, const double* k2,
                           const double* rhs, const double* xin, int warm, int periodic, const Layout& L,
                           double h, Op<double> op, double* b, double* x, int* flags, hipStream_t st) {
    hipLaunchKernelGGL(k_prepare64, dim3(grid_for(L.npad)), dim3(256), 0, st, ex, ey, ez, k2, rhs, xin,
                       warm, periodic, L.nx, L.ny, L.nz, L.sp, h * h, (double*)op.cx, (double*)op.cy,
                       (double*)op.cz, (double*)op.d, b, x, flags);
    PB_HIP(hipGetLastError());
    return PB_OK;
}

pb_status launch_round32(Op<double> op64, const double* b, const double* x, int64_t npad, Op<float> op32,
                         float* b32, float* x32, hipStream_t st) {
    hipLaunchKernelGGL(k_round32, dim3(grid_for(npad)), dim3(256), 0, st, op64.cx, op64.cy, op64.cz,
                       op64.d, b, x, npad, (float*)op32.cx, (float*)op32.cy, (float*)op32.cz,
                       (float*)op32.d, b32, x32);
    PB_HIP(hipGetLastError());
    return PB_OK;
}

int residual_blocks(const Layout& L) {
    return (int)std::min<int64_t>(4096, std::max<int64_t>(1, (L.npad + 4095) / 4096));
}

pb_status launch_residual64(Op<double> op, const double* b, const double* x, const Layout& L, int periodic,
                            double* r64, float* r32, double* partials, double* out2, hipStream_t st) {
    int nblk = residual_blocks(L);
    int64_t per = (L.npad + nblk - 1) / nblk;
    if (periodic) {
        hipLaunchKernelGGL((k_residual64<256, true>), dim3(nblk), dim3(256), 0, st, op.cx, op.cy, op.cz, op.d, b,
                           x, L.nx, L.ny, L.nz, L.sp, L.npad, per, r64, r32, partials);
    } else {
        per = (per + 1) & ~(int64_t)1;   // pairs: even ranges (npad is a multiple of 64)
        nblk = (int)((L.npad + per - 1) / per);
        hipLaunchKernelGGL(k_residual64_pairs<256>, dim3(nblk), dim3(256), 0, st, op.cx, op.cy, op.cz, op.d, b, x,
                           L.nx, L.sp, L.npad, per, r64, r32, partials);
    }
    hipLaunchKernelGGL(k_reduce_pairs, dim3(1), dim3(256), 0, st, partials, nblk, out2);
    PB_HIP(hipGetLastError());
    return PB_OK;
}

pb_status launch_remove_mean(double* v, const Layout& L, double* partials, double* out2, hipStream_t st) {
    const int nblk = residual_blocks(L);
    const int64_t per = (L.npad + nblk - 1) / nblk;
    hipLaunchKernelGGL(k_real_sum<256>, dim3(nblk), dim3(256), 0, st, v, L.plane, L.sp, L.npad, per, partials);
    hipLaunchKernelGGL(k_reduce_pairs, dim3(1), dim3(256), 0, st, partials, nblk, out2);
    hipLaunchKernelGGL(k_sub_mean, dim3(grid_for(L.npad)), dim3(256), 0, st, v, (const double*)out2,
                       (double)L.n, L.plane, L.sp, L.npad);
    PB_HIP(hipGetLastError());
    return PB_OK;
}

pb_status launch_add_correction(double* x, const float* dx, int64_t npad, hipStream_t st) {
    hipLaunchKernelGGL(k_add_correction, dim3(grid_for(npad)), dim3(256), 0, st, x, dx, npad);
    PB_HIP(hipGetLastError());
    return PB_OK;
}

pb_status launch_f32_to_f64(const float* a, double* b, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_f32_to_f64, dim3(grid_for(n)), dim3(256), 0, st, a, b, n);
    PB_HIP(hipGetLastError());
    return PB_OK;
}

template <typename T>
pb_status launch_unpad(const T* xp, const Layout& L, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_unpad<T>, dim3(grid_for(L.n)), dim3(256), 0, st, xp, L.nx, L.ny, L.nz, L.sp, out);
    PB_HIP(hipGetLastError());
    return PB_OK;
}
template pb_status launch_unpad<float>(const float*, const Layout&, double*, hipStream_t);
template pb_status launch_unpad<double>(const double*, const Layout&, double*, hipStream_t);

template <typename T>
pb_status launch_fill(T* p, int64_t n, T v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
    PB_HIP(hipGetLastError());
    return PB_OK;
}
template pb_status launch_fill<float>(float*, int64_t, float, hipStream_t);
template pb_status launch_fill<double>(double*, int64_t, double, hipStream_t);
template pb_status launch_fill<int>(int*, int64_t, int, hipStream_t);

}  // namespace pb
