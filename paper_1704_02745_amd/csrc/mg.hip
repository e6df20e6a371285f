// Geometric-multigrid-preconditioned CG on the stencil of Eq. 3.
//
// The paper points to geometric multigrid as the next step for these systems
// (sections 3.2 and 4) without fixing a scheme. This one:
//   levels    vertex coarsening by two per axis: coarse node I sits at fine
//             node 2I+1 (floor(n/2) nodes, spacing 2h); coarsening stops when
//             an axis would drop below 3 nodes or a level has <= 512 nodes;
//   operator  every level is Eq. 3 at its spacing, with edge dielectrics from
//             the finer level: the series (harmonic) combination of the two
//             fine edges an edge spans, averaged over the nine fine lines
//             around it with weights (1,2,1)x(1,2,1)/16, and kbar^2 averaged
//             with full weighting; so each level is a 7-point stencil and
//             the fine-level kernels apply to all of them;
//   transfer  trilinear prolongation P (coarse ghosts zero), R = P^T/8;
//   cycle     the preconditioner z = M r is one V-cycle from z = 0 with two
//             damped-Jacobi sweeps (omega 0.8) before and after the coarse
//             correction and 40 sweeps on the coarsest level: a fixed
//             symmetric positive definite operator, as CG requires;
//   outer     the section 2.2 listing with that M, host-driven like the DIA
//             form (device-side scalars, the host polls the stopping flag).
#include "pcg_common.hpp"
#include "solver.hpp"

#include <type_traits>
#include <vector>

namespace pb {
namespace {

constexpr int kMgNu = 2;            // Jacobi sweeps before and after the coarse correction
constexpr int kMgCoarseSweeps = 40;  // sweeps on the coarsest level
constexpr int64_t kMgMinNodes = 512;
constexpr double kMgOmega = 0.8;

__device__ __forceinline__ double w3(int a) { return a == 0 ? 0.5 : 0.25; }   // a in -1..1
// a / d in the smoothers: exact division in FP64; in FP32 a times the
// hardware reciprocal of d (within 1 ulp), which keeps the sweeps, whose
// neighbour terms each need one, from being bound by division.
__device__ __forceinline__ double mg_div(double a, double d) { return a / d; }
__device__ __forceinline__ float mg_div(float a, float d) { return a * __builtin_amdgcn_rcpf(d); }
// a * b + c with one rounding
__device__ __forceinline__ double mg_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float mg_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double series2(double a, double b) { return 2.0 * a * b / (a + b); }

// One coarser level from a finer one (FP64 staggered edge arrays and kbar^2
// in the caller's layouts); one thread per output element.
__global__ void k_mg_coarsen(const double* __restrict__ ex, const double* __restrict__ ey,
                             const double* __restrict__ ez, const double* __restrict__ k2, int nx, int ny, int nz,
                             double* __restrict__ cex, double* __restrict__ cey, double* __restrict__ cez,
                             double* __restrict__ ck2, int ncx, int ncy, int ncz) {
    const int64_t nex = (int64_t)(ncx + 1) * ncy * ncz, ney = (int64_t)ncx * (ncy + 1) * ncz;
    const int64_t nez = (int64_t)ncx * ncy * (ncz + 1), nk = (int64_t)ncx * ncy * ncz;
    const int64_t total = nex + ney + nez + nk;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        if (t < nex) {   // x-edges [K][J][E]: lines over (j, k) around (2J+1, 2K+1)
            const int E = (int)(t % (ncx + 1)), J = (int)((t / (ncx + 1)) % ncy), K = (int)(t / ((int64_t)(ncx + 1) * ncy));
            double acc = 0.0, ws = 0.0;
            for (int a = -1; a <= 1; ++a) {
                const int j = 2 * J + 1 + a;
                if (j < 0 || j >= ny) continue;
                for (int b = -1; b <= 1; ++b) {
                    const int k = 2 * K + 1 + b;
                    if (k < 0 || k >= nz) continue;
                    const double* line = ex + (int64_t)(nx + 1) * (j + (int64_t)ny * k);
                    const double e1 = line[2 * E];
                    const double e2 = (2 * E + 1 <= nx) ? line[2 * E + 1] : e1;
                    const double w = w3(a) * w3(b);
                    acc = acc + w * series2(e1, e2);
                    ws = ws + w;
                }
            }
            cex[t] = acc / ws;
        } else if (t < nex + ney) {   // y-edges [K][E][I]: lines over (i, k)
            const int64_t u = t - nex;
            const int I = (int)(u % ncx), E = (int)((u / ncx) % (ncy + 1)), K = (int)(u / ((int64_t)ncx * (ncy + 1)));
            double acc = 0.0, ws = 0.0;
            for (int a = -1; a <= 1; ++a) {
                const int i = 2 * I + 1 + a;
                if (i < 0 || i >= nx) continue;
                for (int b = -1; b <= 1; ++b) {
                    const int k = 2 * K + 1 + b;
                    if (k < 0 || k >= nz) continue;
                    const double e1 = ey[i + (int64_t)nx * (2 * E + (int64_t)(ny + 1) * k)];
                    const double e2 = (2 * E + 1 <= ny) ? ey[i + (int64_t)nx * (2 * E + 1 + (int64_t)(ny + 1) * k)] : e1;
                    const double w = w3(a) * w3(b);
                    acc = acc + w * series2(e1, e2);
                    ws = ws + w;
                }
            }
            cey[u] = acc / ws;
        } else if (t < nex + ney + nez) {   // z-edges [E][J][I]: lines over (i, j)
            const int64_t u = t - nex - ney;
            const int I = (int)(u % ncx), J = (int)((u / ncx) % ncy), E = (int)(u / ((int64_t)ncx * ncy));
            double acc = 0.0, ws = 0.0;
            for (int a = -1; a <= 1; ++a) {
                const int i = 2 * I + 1 + a;
                if (i < 0 || i >= nx) continue;
                for (int b = -1; b <= 1; ++b) {
                    const int j = 2 * J + 1 + b;
                    if (j < 0 || j >= ny) continue;
                    const int64_t plane = (int64_t)nx * ny;
                    const double e1 = ez[i + (int64_t)nx * j + plane * (2 * E)];
                    const double e2 = (2 * E + 1 <= nz) ? ez[i + (int64_t)nx * j + plane * (2 * E + 1)] : e1;
                    const double w = w3(a) * w3(b);
                    acc = acc + w * series2(e1, e2);
                    ws = ws + w;
                }
            }
            cez[u] = acc / ws;
        } else {   // kbar^2 [K][J][I]: full weighting
            const int64_t u = t - nex - ney - nez;
            const int I = (int)(u % ncx), J = (int)((u / ncx) % ncy), K = (int)(u / ((int64_t)ncx * ncy));
            double acc = 0.0, ws = 0.0;
            for (int c = -1; c <= 1; ++c) {
                const int k = 2 * K + 1 + c;
                if (k < 0 || k >= nz) continue;
                for (int b = -1; b <= 1; ++b) {
                    const int j = 2 * J + 1 + b;
                    if (j < 0 || j >= ny) continue;
                    for (int a = -1; a <= 1; ++a) {
                        const int i = 2 * I + 1 + a;
                        if (i < 0 || i >= nx) continue;
                        const double w = w3(a) * w3(b) * w3(c);
                        acc = acc + w * k2[i + (int64_t)nx * (j + (int64_t)ny * k)];
                        ws = ws + w;
                    }
                }
            }
            ck2[u] = acc / ws;
        }
    }
}

// A level's operator in the padded layout (couplings zero across the box
// faces, the diagonal with every edge), rounded to T.
template <typename T>
__global__ void k_mg_op(const double* __restrict__ ex, const double* __restrict__ ey, const double* __restrict__ ez,
                        const double* __restrict__ k2, int nx, int ny, int nz, int64_t sp, double hh, Op<T> op) {
    const int64_t plane = (int64_t)nx * ny, npad = sp * nz;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = t / sp, pp = t - k * sp;
        T* cx = (T*)op.cx;
        T* cy = (T*)op.cy;
        T* cz = (T*)op.cz;
        T* d = (T*)op.d;
        if (pp >= plane) {
            cx[t] = T(0); cy[t] = T(0); cz[t] = T(0); d[t] = T(1);
            continue;
        }
        const int64_t j = pp / nx, i = pp - j * nx, n = pp + plane * k;
        const double exm = ex[i + (int64_t)(nx + 1) * (j + (int64_t)ny * k)];
        const double exp_ = ex[i + 1 + (int64_t)(nx + 1) * (j + (int64_t)ny * k)];
        const double eym = ey[i + (int64_t)nx * (j + (int64_t)(ny + 1) * k)];
        const double eyp = ey[i + (int64_t)nx * (j + 1 + (int64_t)(ny + 1) * k)];
        const double ezm = ez[i + (int64_t)nx * (j + (int64_t)ny * k)];
        const double ezp = ez[i + (int64_t)nx * (j + (int64_t)ny * (k + 1))];
        cx[t] = (T)((i < nx - 1) ? exp_ / hh : 0.0);
        cy[t] = (T)((j < ny - 1) ? eyp / hh : 0.0);
        cz[t] = (T)((k < nz - 1) ? ezp / hh : 0.0);
        d[t] = (T)((((((exm + exp_) + eym) + eyp) + ezm) + ezp) / hh + k2[n]);
    }
}

// Operator readers of the stencil kernels: the four coefficient arrays
// (ArrOp), or one word of dictionary codes per position (CodeOp; level 0 in
// FP32, the words coded.hip builds for the fused solver: byte 0 cx, 1 cy, 2
// cz, 3 d) with the dictionary copied into LDS when the kernel starts. The
// dictionary holds the exact FP32 values, so both give the same results.
// Every thread of a block calls bind() once before the first read.
template <typename T>
struct ArrOp {
    Op<T> op;
    __device__ __forceinline__ void bind() {}
    __device__ __forceinline__ T cx(int64_t t) const { return op.cx[t]; }
    __device__ __forceinline__ T cy(int64_t t) const { return op.cy[t]; }
    __device__ __forceinline__ T cz(int64_t t) const { return op.cz[t]; }
    __device__ __forceinline__ T d(int64_t t) const { return op.d[t]; }
};
struct CodeOp {
    const uint32_t* w;
    const float* dict;   // device dictionary, kCodedTableSize values
    const float* tab;    // its LDS copy (bind)
    __device__ __forceinline__ void bind() {
        __shared__ float s_tab[kCodedTableSize];
        for (int i = threadIdx.x; i < kCodedTableSize; i += blockDim.x) s_tab[i] = dict[i];
        __syncthreads();
        tab = s_tab;
    }
    __device__ __forceinline__ float cx(int64_t t) const { return tab[w[t] & 255u]; }
    __device__ __forceinline__ float cy(int64_t t) const { return tab[(w[t] >> 8) & 255u]; }
    __device__ __forceinline__ float cz(int64_t t) const { return tab[(w[t] >> 16) & 255u]; }
    __device__ __forceinline__ float d(int64_t t) const { return tab[w[t] >> 24]; }
};

// (A v) at padded position t (free-space stencil; zero couplings cut the
// faces and the pad slots).
template <typename T, typename RD>
__device__ __forceinline__ T mg_apply(const RD& op, const T* __restrict__ v, int64_t t, int nx, int64_t sp,
                                      int64_t npad) {
    T nb = op.cx(t) * (t + 1 < npad ? v[t + 1] : T(0));
    nb += (t >= 1 ? op.cx(t - 1) * v[t - 1] : T(0));
    nb += op.cy(t) * (t + nx < npad ? v[t + nx] : T(0));
    nb += (t >= nx ? op.cy(t - nx) * v[t - nx] : T(0));
    nb += op.cz(t) * (t + sp < npad ? v[t + sp] : T(0));
    nb += (t >= sp ? op.cz(t - sp) * v[t - sp] : T(0));
    return op.d(t) * v[t] - nb;
}
template <typename T>
__device__ __forceinline__ T mg_apply(const Op<T>& op, const T* __restrict__ v, int64_t t, int nx, int64_t sp,
                                      int64_t npad) {
    return mg_apply(ArrOp<T>{op}, v, t, nx, sp, npad);
}

// One damped-Jacobi sweep out = in + omega (b - A in)/d; from_zero: in = 0.
template <typename T, typename RD>
__global__ void k_mg_jacobi(RD op, const T* __restrict__ b, const T* __restrict__ in, T* __restrict__ out,
                            int nx, int64_t sp, int64_t npad, T omega, int from_zero, const SyncState* S) {
    if (S && stop(S)) return;
    op.bind();
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x) {
        if (from_zero) {
            out[t] = mg_div(omega * b[t], op.d(t));
        } else {
            const T r = b[t] - mg_apply(op, in, t, nx, sp, npad);
            out[t] = in[t] + mg_div(omega * r, op.d(t));
        }
    }
}

// The first two damped-Jacobi sweeps from zero in one pass. The first
// sweep's output x1 = omega b / d is formed where the second needs it (the
// node and its six neighbours) with the arithmetic of the from_zero sweep, so
// the result equals two k_mg_jacobi launches bit for bit.
template <typename T>
__device__ __forceinline__ T mg_x1(const Op<T>& op, const T* __restrict__ b, int64_t t, T omega) {
    return mg_div(omega * b[t], op.d[t]);
}

template <typename T>
__device__ __forceinline__ T mg_jacobi2z_at(const Op<T>& op, const T* __restrict__ b, int64_t t, int nx, int64_t sp,
                                            int64_t npad, T omega) {
    T nb = op.cx[t] * (t + 1 < npad ? mg_x1(op, b, t + 1, omega) : T(0));
    nb += (t >= 1 ? op.cx[t - 1] * mg_x1(op, b, t - 1, omega) : T(0));
    nb += op.cy[t] * (t + nx < npad ? mg_x1(op, b, t + nx, omega) : T(0));
    nb += (t >= nx ? op.cy[t - nx] * mg_x1(op, b, t - nx, omega) : T(0));
    nb += op.cz[t] * (t + sp < npad ? mg_x1(op, b, t + sp, omega) : T(0));
    nb += (t >= sp ? op.cz[t - sp] * mg_x1(op, b, t - sp, omega) : T(0));
    const T x1 = mg_x1(op, b, t, omega);
    const T r = b[t] - (op.d[t] * x1 - nb);
    return x1 + mg_div(omega * r, op.d[t]);
}
template <typename T>
__global__ void k_mg_jacobi2z(Op<T> op, const T* __restrict__ b, T* __restrict__ out, int nx, int64_t sp,
                              int64_t npad, T omega, const SyncState* S) {
    if (S && stop(S)) return;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x)
        out[t] = mg_jacobi2z_at(op, b, t, nx, sp, npad, omega);
}

// The finest level's last post-smoothing sweep fused with the outer
// iteration's r.z and r.r (the level's right-hand side is the outer residual
// r): block b sweeps positions [b*per, (b+1)*per), threads striding by the
// block size, and stores the block sums in the fixed order of block_sum_store.
template <typename T, typename RD>
__global__ __launch_bounds__(kBS) void k_mg_jacobi_dot2(RD op, const T* __restrict__ b, const T* __restrict__ in,
                                                        T* __restrict__ out, int nx, int64_t sp, int64_t npad,
                                                        T omega, int64_t per, double* __restrict__ partials,
                                                        const SyncState* S) {
    if (stop(S)) return;
    op.bind();
    double acc[2] = {0.0, 0.0};
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(lo + per, npad);
    for (int64_t t = lo + threadIdx.x; t < hi; t += kBS) {
        const T res = b[t] - mg_apply(op, in, t, nx, sp, npad);
        const T z = in[t] + mg_div(omega * res, op.d(t));
        out[t] = z;
        acc[0] += (double)b[t] * (double)z;
        acc[1] += (double)b[t] * (double)b[t];
    }
    block_sum_store<2>(acc, partials + (size_t)blockIdx.x * kMaxPartials);
}

template <typename T, typename RD>
__global__ void k_mg_residual(RD op, const T* __restrict__ b, const T* __restrict__ x, T* __restrict__ r, int nx,
                              int64_t sp, int64_t npad, const SyncState* S) {
    if (S && stop(S)) return;
    op.bind();
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x)
        r[t] = b[t] - mg_apply(op, x, t, nx, sp, npad);
}

// q = A v (the outer iteration's product).
template <typename T>
__global__ void k_mg_apply(Op<T> op, const T* __restrict__ v, T* __restrict__ q, int nx, int64_t sp, int64_t npad,
                           const SyncState* S) {
    if (S && stop(S)) return;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x)
        q[t] = mg_apply(op, v, t, nx, sp, npad);
}

// bc = R r (full weighting; fine nodes outside the grid contribute zero).
// Grid: blockIdx.y is the coarse plane K; the x-dimension strides over the
// coarse plane's positions (pad slots get zero).
template <typename T>
__device__ __forceinline__ T mg_restrict_at(const T* __restrict__ r, int nx, int ny, int nz, int64_t sp, int I, int J,
                                            int K) {
    T acc = T(0);
    for (int c = -1; c <= 1; ++c) {
        const int k = 2 * K + 1 + c;
        if (k < 0 || k >= nz) continue;
        for (int b = -1; b <= 1; ++b) {
            const int j = 2 * J + 1 + b;
            if (j < 0 || j >= ny) continue;
            const T* row = r + (int64_t)k * sp + (int64_t)j * nx;
            for (int a = -1; a <= 1; ++a) {
                const int i = 2 * I + 1 + a;
                if (i < 0 || i >= nx) continue;
                acc += (T)(w3(a) * w3(b) * w3(c)) * row[i];
            }
        }
    }
    return acc;
}
template <typename T>
__global__ void k_mg_restrict(const T* __restrict__ r, int nx, int ny, int nz, int64_t sp, T* __restrict__ bc,
                              int ncx, int ncy, int ncz, int64_t spc, const SyncState* S) {
    if (S && stop(S)) return;
    const int K = blockIdx.y;
    const int pc = ncx * ncy;
    for (int pp = blockIdx.x * blockDim.x + threadIdx.x; pp < (int)spc; pp += gridDim.x * blockDim.x) {
        const int64_t t = (int64_t)K * spc + pp;
        if (pp >= pc) {
            bc[t] = T(0);
            continue;
        }
        const int J = pp / ncx, I = pp - J * ncx;
        bc[t] = mg_restrict_at(r, nx, ny, nz, sp, I, J, K);
    }
}

// x += P xc (trilinear: fine f odd takes coarse (f-1)/2, fine f even the mean
// of coarse f/2-1 and f/2; coarse ghosts are zero). One thread per cell of
// the coarse grid shifted by one fine node: cell (I, J, K), I in -1..ncx-1,
// holds the fine nodes 2I+1 (odd) and 2I+2 (even) of each axis, all of which
// interpolate from the same eight coarse nodes I..I+1 x J..J+1 x K..K+1, read
// once. Each fine node sums its terms in z, y, x order, zero weights skipped.
// Grid: blockIdx.y is K+1; the x-dimension strides over (I, J).
template <typename T>
__device__ __forceinline__ void mg_prolong_cell(const T* __restrict__ xc, int ncx, int ncy, int ncz, int64_t spc,
                                                T* __restrict__ x, int nx, int ny, int nz, int64_t sp, int I, int J,
                                                int K) {
    T v[2][2][2];   // coarse (K+kk, J+jj, I+ii), zero outside the coarse grid
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int ii = 0; ii < 2; ++ii) {
                const int ck = K + kk, cj = J + jj, ci = I + ii;
                const bool in = ck >= 0 && ck < ncz && cj >= 0 && cj < ncy && ci >= 0 && ci < ncx;
                v[kk][jj][ii] = in ? xc[(int64_t)ck * spc + (int64_t)cj * ncx + ci] : T(0);
            }
    // per axis, fine node 2C+1+e (e = 0 odd, 1 even): its terms (coarse
    // offset, weight) in order; n = number of terms
#pragma unroll
    for (int ez = 0; ez < 2; ++ez) {
        const int k = 2 * K + 1 + ez;
        if (k < 0 || k >= nz) continue;
#pragma unroll
        for (int ey = 0; ey < 2; ++ey) {
            const int j = 2 * J + 1 + ey;
            if (j < 0 || j >= ny) continue;
#pragma unroll
            for (int ex = 0; ex < 2; ++ex) {
                const int i = 2 * I + 1 + ex;
                if (i < 0 || i >= nx) continue;
                T add = T(0);
                for (int tz = 0; tz <= ez; ++tz) {
                    const int ck = K + tz;
                    if (ck < 0 || ck >= ncz) continue;
                    const T wz = ez ? T(0.5) : T(1);
                    for (int ty = 0; ty <= ey; ++ty) {
                        const int cj = J + ty;
                        if (cj < 0 || cj >= ncy) continue;
                        const T wy = ey ? T(0.5) : T(1);
                        for (int tx = 0; tx <= ex; ++tx) {
                            const int ci = I + tx;
                            if (ci < 0 || ci >= ncx) continue;
                            const T wx = ex ? T(0.5) : T(1);
                            add += wx * wy * wz * v[tz][ty][tx];
                        }
                    }
                }
                x[(int64_t)k * sp + (int64_t)j * nx + i] += add;
            }
        }
    }
}
template <typename T>
__global__ void k_mg_prolong_add(const T* __restrict__ xc, int ncx, int ncy, int ncz, int64_t spc,
                                 T* __restrict__ x, int nx, int ny, int nz, int64_t sp, const SyncState* S) {
    if (S && stop(S)) return;
    const int K = (int)blockIdx.y - 1;
    const int cw = ncx + 1, cells = cw * (ncy + 1);
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += gridDim.x * blockDim.x) {
        const int J = c / cw - 1, I = c - (J + 1) * cw - 1;
        mg_prolong_cell(xc, ncx, ncy, ncz, spc, x, nx, ny, nz, sp, I, J, K);
    }
}

// Launch shape of the plane-indexed kernels: blockIdx.y = plane.
dim3 plane_grid(int64_t positions, int planes) {
    return dim3((unsigned)std::min<int64_t>(std::max<int64_t>(1, (positions + kBS - 1) / kBS), 1024), (unsigned)planes);
}

// The outer iteration's direction and product in one pass over a block's
// range of rows: p = z + beta p_old (formed wherever the product needs it,
// with one rounding, so neighbours see the value the node's owner stores),
// q = A p, and the block's p.q.
template <typename T, typename RD>
__global__ __launch_bounds__(kBS) void k_mg_direction_apply(RD op, const T* __restrict__ z,
                                                            const T* __restrict__ pold, T* __restrict__ pnew,
                                                            T* __restrict__ q, int nx, int64_t sp, int64_t npad,
                                                            int64_t per, double* __restrict__ partials,
                                                            const SyncState* S) {
    if (stop(S)) return;
    op.bind();
    const T beta = (T)S->beta;
    auto P = [&](int64_t u) { return mg_fma(beta, pold[u], z[u]); };
    double acc[1] = {0.0};
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(lo + per, npad);
    for (int64_t t = lo + threadIdx.x; t < hi; t += kBS) {
        T nb = op.cx(t) * (t + 1 < npad ? P(t + 1) : T(0));
        nb += (t >= 1 ? op.cx(t - 1) * P(t - 1) : T(0));
        nb += op.cy(t) * (t + nx < npad ? P(t + nx) : T(0));
        nb += (t >= nx ? op.cy(t - nx) * P(t - nx) : T(0));
        nb += op.cz(t) * (t + sp < npad ? P(t + sp) : T(0));
        nb += (t >= sp ? op.cz(t - sp) * P(t - sp) : T(0));
        const T pt = P(t);
        const T qt = op.d(t) * pt - nb;
        pnew[t] = pt;
        q[t] = qt;
        acc[0] += (double)pt * (double)qt;
    }
    block_sum_store<1>(acc, partials + (size_t)blockIdx.x * kMaxPartials);
}

// The outer update x += alpha p, rnew = r_old - alpha q, with (given x1)
// level 0's first pre-smoothing sweep from zero on rnew, x1 = omega rnew / d
// (the arithmetic of k_mg_jacobi's first sweep).
template <typename T>
__global__ void k_mg_update(T* __restrict__ x, const T* __restrict__ p, const T* __restrict__ rold,
                            const T* __restrict__ q, T* __restrict__ rnew, const T* __restrict__ d,
                            T* __restrict__ x1, T omega, int64_t npad, const SyncState* S) {
    if (stop(S)) return;
    const T alpha = (T)S->alpha;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x) {
        x[t] = mg_fma(alpha, p[t], x[t]);
        const T r = mg_fma(-alpha, q[t], rold[t]);
        rnew[t] = r;
        if (x1) x1[t] = mg_div(omega * r, d[t]);
    }
}

// The coarsest level: `sweeps` damped-Jacobi sweeps from zero by one
// workgroup (the level is small); buf[(sweeps-1) & 1] holds the result.
// With `lds` set the sweeps run on LDS copies of the operator, right-hand
// side and iterates (the launch brings 7 npad values of dynamic LDS), with
// the same arithmetic, and the result is copied out at the end.
template <typename T>
__device__ __forceinline__ void mg_coarse_sweeps(const Op<T>& o, const T* __restrict__ b, T* __restrict__ u0,
                                                 T* __restrict__ u1, int nx, int64_t sp, int64_t npad, T omega,
                                                 int sweeps) {
    for (int it = 0; it < sweeps; ++it) {
        const T* in = (it & 1) ? u0 : u1;
        T* out = (it & 1) ? u1 : u0;
        for (int64_t t = threadIdx.x; t < npad; t += blockDim.x) {
            if (it == 0) {
                out[t] = mg_div(omega * b[t], o.d[t]);
            } else {
                const T r = b[t] - mg_apply(o, in, t, nx, sp, npad);
                out[t] = in[t] + mg_div(omega * r, o.d[t]);
            }
        }
        __syncthreads();
    }
}
template <typename T>
__global__ __launch_bounds__(1024) void k_mg_coarse(Op<T> op, const T* __restrict__ b, T* __restrict__ buf0,
                                                    T* __restrict__ buf1, int nx, int64_t sp, int64_t npad, T omega,
                                                    int sweeps, int lds, const SyncState* S) {
    if (S && stop(S)) return;
    if (!lds) {
        mg_coarse_sweeps(op, b, buf0, buf1, nx, sp, npad, omega, sweeps);
        return;
    }
    extern __shared__ __align__(16) unsigned char coarse_lds[];
    T* cx = reinterpret_cast<T*>(coarse_lds);
    T* cy = cx + npad;
    T* cz = cy + npad;
    T* d = cz + npad;
    T* bl = d + npad;
    T* u0 = bl + npad;
    T* u1 = u0 + npad;
    for (int64_t t = threadIdx.x; t < npad; t += blockDim.x) {
        cx[t] = op.cx[t];
        cy[t] = op.cy[t];
        cz[t] = op.cz[t];
        d[t] = op.d[t];
        bl[t] = b[t];
    }
    __syncthreads();
    mg_coarse_sweeps(Op<T>{cx, cy, cz, d}, (const T*)bl, u0, u1, nx, sp, npad, omega, sweeps);
    const T* res = ((sweeps - 1) & 1) ? u1 : u0;
    T* dst = ((sweeps - 1) & 1) ? buf1 : buf0;
    for (int64_t t = threadIdx.x; t < npad; t += blockDim.x) dst[t] = res[t];
}

// Outer-iteration pieces: p = z with the sums r.z, r.r, b.b; and r.z, r.r.
template <typename T>
__global__ __launch_bounds__(kBS) void k_mg_init_dots(const T* __restrict__ r, const T* __restrict__ z,
                                                      const T* __restrict__ b, T* __restrict__ p, int64_t npad,
                                                      int64_t per, double* __restrict__ partials) {
    double acc[3] = {0.0, 0.0, 0.0};
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(lo + per, npad);
    for (int64_t t = lo + threadIdx.x; t < hi; t += kBS) {
        p[t] = z[t];
        acc[0] += (double)r[t] * (double)z[t];
        acc[1] += (double)r[t] * (double)r[t];
        acc[2] += (double)b[t] * (double)b[t];
    }
    block_sum_store<3>(acc, partials + (size_t)blockIdx.x * kMaxPartials);
}

// r.z and r.r block sums (the outer iteration's, when the hierarchy has a
// single level and the V-cycle has no post-smoothing sweep to fuse them into).
template <typename T>
__global__ __launch_bounds__(kBS) void k_mg_dot2(const T* __restrict__ r, const T* __restrict__ z, int64_t npad,
                                                 int64_t per, double* __restrict__ partials, const SyncState* S) {
    if (stop(S)) return;
    double acc[2] = {0.0, 0.0};
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(lo + per, npad);
    for (int64_t t = lo + threadIdx.x; t < hi; t += kBS) {
        acc[0] += (double)r[t] * (double)z[t];
        acc[1] += (double)r[t] * (double)r[t];
    }
    block_sum_store<2>(acc, partials + (size_t)blockIdx.x * kMaxPartials);
}

template <typename T>
__global__ void k_mg_sub(const T* __restrict__ b, const T* __restrict__ q, T* __restrict__ r, int64_t npad) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x)
        r[t] = b[t] - q[t];
}

struct LevelShape {
    Layout L;
    double h;
};

std::vector<LevelShape> level_shapes(const Layout& L0, double h) {
    std::vector<LevelShape> v{{L0, h}};
    for (;;) {
        const Layout& L = v.back().L;
        if (std::min(L.nx, std::min(L.ny, L.nz)) / 2 < 3 || L.n <= kMgMinNodes) break;
        v.push_back({make_layout(L.nx / 2, L.ny / 2, L.nz / 2), 2.0 * v.back().h});
    }
    return v;
}

template <typename T>
struct MgLevel {
    Layout L;
    double h;
    Op<T> op;
    T *b, *xa, *xb, *r;                 // right-hand side, two iterate buffers, residual
    double *ex, *ey, *ez, *k2;          // this level's edges and kbar^2 (coarse levels)
    uint32_t* codes;                    // level 0, FP32: code words of the operator
    void* code_scratch;
};

// Workspace carving (nullptr base: sizes only). Level 0 borrows the solve's
// operator, residual and z buffers and needs two more vectors.
template <typename T>
size_t mg_carve(void* base, const Layout& L0, double h, std::vector<MgLevel<T>>* out) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return base ? (void*)((char*)base + o) : nullptr;
    };
    const auto shapes = level_shapes(L0, h);
    for (size_t l = 0; l < shapes.size(); ++l) {
        MgLevel<T> m{};
        m.L = shapes[l].L;
        m.h = shapes[l].h;
        const size_t nT = sizeof(T) * (size_t)m.L.npad;
        if (l > 0) {
            const Layout& L = m.L;
            m.ex = (double*)take(sizeof(double) * (size_t)(L.nx + 1) * L.ny * L.nz);
            m.ey = (double*)take(sizeof(double) * (size_t)L.nx * (L.ny + 1) * L.nz);
            m.ez = (double*)take(sizeof(double) * (size_t)L.nx * L.ny * (L.nz + 1));
            m.k2 = (double*)take(sizeof(double) * (size_t)L.n);
            m.op.cx = (T*)take(nT);
            m.op.cy = (T*)take(nT);
            m.op.cz = (T*)take(nT);
            m.op.d = (T*)take(nT);
            m.b = (T*)take(nT);
            m.xa = (T*)take(nT);
        }
        m.xb = (T*)take(nT);
        m.r = (T*)take(nT);
        if (l == 0 && sizeof(T) == 4) {   // level 0's code words and the dictionary build's scratch
            m.codes = (uint32_t*)take(4 * (size_t)m.L.npad);
            m.code_scratch = take(coded_scratch_bytes());
        }
        if (out) out->push_back(m);
    }
    return off;
}

unsigned mg_grid(int64_t n) { return stream_grid(n); }

// The outer iteration's r.z and r.r taken in the finest level's last sweep.
struct DotFuse {
    double* partials;
    int nblk;
    int64_t per;
};

// ---- level 0 in FP32: four consecutive positions per thread
//
// The same arithmetic as the one-position kernels above (each term rounded
// as written, in the same order), with the neighbour values read as 16-byte
// groups where they are aligned (the node's own group and the planes above
// and below) through raw buffer resources over the whole array: positions
// before the array (one fixed offset past its end) or past its end read as
// zero, as the one-position kernels' range tests make them.
using MgRsrc = __amdgpu_buffer_rsrc_t;
typedef unsigned int mg_u32x4 __attribute__((ext_vector_type(4)));
constexpr uint32_t kMgOutside = 0x80000000u;   // past every array these kernels take (npad < 2^29)
__device__ __forceinline__ MgRsrc mg_rsrc(const void* p, int64_t n) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)(n * 4), 0x00020000);
}
__device__ __forceinline__ uint32_t mg_off(int64_t i) { return i < 0 ? kMgOutside : (uint32_t)(i * 4); }
__device__ __forceinline__ float4 mg_ld4(MgRsrc r, int64_t i) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)mg_off(i), 0, 0));
}
__device__ __forceinline__ float mg_ld1(MgRsrc r, int64_t i) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)mg_off(i), 0, 0));
}
__device__ __forceinline__ mg_u32x4 mg_ldw4(MgRsrc r, int64_t i) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, (int)mg_off(i), 0, 0);
}
__device__ __forceinline__ uint32_t mg_ldw1(MgRsrc r, int64_t i) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)mg_off(i), 0, 0);
}
__device__ __forceinline__ float& g4(float4& v, int u) { return (&v.x)[u]; }

// The couplings a group of four positions t0..t0+3 needs: its own cx, cy,
// cz, d, the x-coupling left of t0, the y-couplings one row down and the
// z-couplings one plane down (zero before the array).
struct Grp4 {
    float cx[4], cy[4], cz[4], d[4], cxl, cyd[4], czd[4];
};
struct ArrGrp {
    const float *pcx, *pcy, *pcz, *pd;
    int64_t n;
    __device__ __forceinline__ void bind() {}
    __device__ __forceinline__ void load(int64_t t0, int nx, int64_t sp, Grp4& g) const {
        const MgRsrc cx = mg_rsrc(pcx, n), cy = mg_rsrc(pcy, n), cz = mg_rsrc(pcz, n), d = mg_rsrc(pd, n);
        const float4 a = mg_ld4(cx, t0), b = mg_ld4(cy, t0), c = mg_ld4(cz, t0), e = mg_ld4(d, t0);
        const float4 zd = mg_ld4(cz, t0 - sp);
        for (int u = 0; u < 4; ++u) {
            g.cx[u] = (&a.x)[u];
            g.cy[u] = (&b.x)[u];
            g.cz[u] = (&c.x)[u];
            g.d[u] = (&e.x)[u];
            g.czd[u] = (&zd.x)[u];
            g.cyd[u] = mg_ld1(cy, t0 + u - nx);
        }
        g.cxl = mg_ld1(cx, t0 - 1);
    }
};
struct CodeGrp {
    const uint32_t* pw;
    int64_t n;
    const float* dict;
    const float* tab;    // the dictionary's LDS copy, set by bind()
    __device__ __forceinline__ void bind() {
        __shared__ float s_tab[kCodedTableSize];
        for (int i = threadIdx.x; i < kCodedTableSize; i += blockDim.x) s_tab[i] = dict[i];
        __syncthreads();
        tab = s_tab;
    }
    __device__ __forceinline__ void load(int64_t t0, int nx, int64_t sp, Grp4& g) const {
        const MgRsrc w = mg_rsrc(pw, n);
        const mg_u32x4 o = mg_ldw4(w, t0), zd = mg_ldw4(w, t0 - sp);
        for (int u = 0; u < 4; ++u) {
            g.cx[u] = tab[o[u] & 255u];
            g.cy[u] = tab[(o[u] >> 8) & 255u];
            g.cz[u] = tab[(o[u] >> 16) & 255u];
            g.d[u] = tab[o[u] >> 24];
            g.czd[u] = tab[(zd[u] >> 16) & 255u];
            g.cyd[u] = tab[(mg_ldw1(w, t0 + u - nx) >> 8) & 255u];
        }
        g.cxl = tab[mg_ldw1(w, t0 - 1) & 255u];
    }
};

// Values of the vector the operator applies to, around a group: the group,
// its x-neighbours, the rows above and below, the planes above and below.
struct Nbr4 {
    float4 c, zu, zd;
    float l, r, yu[4], yd[4];
};
__device__ __forceinline__ void load_nbr(MgRsrc v, int64_t t0, int nx, int64_t sp, Nbr4& n) {
    n.c = mg_ld4(v, t0);
    n.zu = mg_ld4(v, t0 + sp);
    n.zd = mg_ld4(v, t0 - sp);
    n.l = mg_ld1(v, t0 - 1);
    n.r = mg_ld1(v, t0 + 4);
    for (int u = 0; u < 4; ++u) {
        n.yu[u] = mg_ld1(v, t0 + u + nx);
        n.yd[u] = mg_ld1(v, t0 + u - nx);
    }
}
// (A v) for element u of the group, the terms of mg_apply in its order
__device__ __forceinline__ float apply4(const Grp4& g, const Nbr4& n, int u) {
    float c = (&n.c.x)[u];
    float vr = (u == 3) ? n.r : (&n.c.x)[u + 1];
    float vl = (u == 0) ? n.l : (&n.c.x)[u - 1];
    float cl = (u == 0) ? g.cxl : g.cx[u - 1];
    float nb = g.cx[u] * vr;
    nb += cl * vl;
    nb += g.cy[u] * n.yu[u];
    nb += g.cyd[u] * n.yd[u];
    nb += g.cz[u] * (&n.zu.x)[u];
    nb += g.czd[u] * (&n.zd.x)[u];
    return g.d[u] * c - nb;
}

// MODE 0: out = in + (omega (b - A in)) / d (a sweep); MODE 1: r = b - A x.
// Grid-stride over groups of four.
template <int MODE, typename RD>
__global__ __launch_bounds__(kBS) void k_mg4_sweep(RD op, const float* __restrict__ b, const float* __restrict__ in,
                                                   float* __restrict__ out, int nx, int64_t sp, int64_t npad,
                                                   float omega, const SyncState* S) {
    if (S && stop(S)) return;
    op.bind();
    const MgRsrc rin = mg_rsrc(in, npad), rb = mg_rsrc(b, npad), ro = mg_rsrc(out, npad);
    for (int64_t t0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; t0 < npad;
         t0 += (int64_t)gridDim.x * blockDim.x * 4) {
        Grp4 g;
        op.load(t0, nx, sp, g);
        Nbr4 n;
        load_nbr(rin, t0, nx, sp, n);
        const float4 bv = mg_ld4(rb, t0);
        float4 o;
        for (int u = 0; u < 4; ++u) {
            const float r = (&bv.x)[u] - apply4(g, n, u);
            g4(o, u) = MODE == 0 ? (&n.c.x)[u] + mg_div(omega * r, g.d[u]) : r;
        }
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(mg_u32x4, o), ro, (int)mg_off(t0), 0, 0);
    }
}

// The last sweep with the block sums of r.z and r.r (block b: positions
// [b*per, (b+1)*per), per a multiple of 4, groups strided by the block).
template <typename RD>
__global__ __launch_bounds__(kBS) void k_mg4_sweep_dot2(RD op, const float* __restrict__ b,
                                                        const float* __restrict__ in, float* __restrict__ out,
                                                        int nx, int64_t sp, int64_t npad, float omega, int64_t per,
                                                        double* __restrict__ partials, const SyncState* S) {
    if (stop(S)) return;
    op.bind();
    const MgRsrc rin = mg_rsrc(in, npad), rb = mg_rsrc(b, npad), ro = mg_rsrc(out, npad);
    double acc[2] = {0.0, 0.0};
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(lo + per, npad);
    for (int64_t t0 = lo + (int64_t)threadIdx.x * 4; t0 < hi; t0 += kBS * 4) {
        Grp4 g;
        op.load(t0, nx, sp, g);
        Nbr4 n;
        load_nbr(rin, t0, nx, sp, n);
        const float4 bv = mg_ld4(rb, t0);
        float4 o;
        for (int u = 0; u < 4; ++u) {
            const float res = (&bv.x)[u] - apply4(g, n, u);
            const float z = (&n.c.x)[u] + mg_div(omega * res, g.d[u]);
            g4(o, u) = z;
            acc[0] += (double)(&bv.x)[u] * (double)z;
            acc[1] += (double)(&bv.x)[u] * (double)(&bv.x)[u];
        }
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(mg_u32x4, o), ro, (int)mg_off(t0), 0, 0);
    }
    block_sum_store<2>(acc, partials + (size_t)blockIdx.x * kMaxPartials);
}

// p = z + beta p_old, q = A p and the block sums of p.q (as k_mg_direction_apply).
template <typename RD>
__global__ __launch_bounds__(kBS) void k_mg4_direction_apply(RD op, const float* __restrict__ z,
                                                             const float* __restrict__ pold, float* __restrict__ pnew,
                                                             float* __restrict__ q, int nx, int64_t sp, int64_t npad,
                                                             int64_t per, double* __restrict__ partials,
                                                             const SyncState* S) {
    if (stop(S)) return;
    op.bind();
    const float beta = (float)S->beta;
    const MgRsrc rz = mg_rsrc(z, npad), rp = mg_rsrc(pold, npad), rpn = mg_rsrc(pnew, npad), rq = mg_rsrc(q, npad);
    double acc[1] = {0.0};
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(lo + per, npad);
    for (int64_t t0 = lo + (int64_t)threadIdx.x * 4; t0 < hi; t0 += kBS * 4) {
        Grp4 g;
        op.load(t0, nx, sp, g);
        Nbr4 nz, np;
        load_nbr(rz, t0, nx, sp, nz);
        load_nbr(rp, t0, nx, sp, np);
        // the direction at every point the product reads (zero outside the array, as z and p_old are)
        Nbr4 n;
        for (int u = 0; u < 4; ++u) {
            g4(n.c, u) = mg_fma(beta, (&np.c.x)[u], (&nz.c.x)[u]);
            g4(n.zu, u) = mg_fma(beta, (&np.zu.x)[u], (&nz.zu.x)[u]);
            g4(n.zd, u) = mg_fma(beta, (&np.zd.x)[u], (&nz.zd.x)[u]);
            n.yu[u] = mg_fma(beta, np.yu[u], nz.yu[u]);
            n.yd[u] = mg_fma(beta, np.yd[u], nz.yd[u]);
        }
        n.l = mg_fma(beta, np.l, nz.l);
        n.r = mg_fma(beta, np.r, nz.r);
        float4 qv;
        for (int u = 0; u < 4; ++u) {
            const float qt = apply4(g, n, u);
            g4(qv, u) = qt;
            acc[0] += (double)(&n.c.x)[u] * (double)qt;
        }
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(mg_u32x4, n.c), rpn, (int)mg_off(t0), 0, 0);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(mg_u32x4, qv), rq, (int)mg_off(t0), 0, 0);
    }
    block_sum_store<1>(acc, partials + (size_t)blockIdx.x * kMaxPartials);
}

// Runs f with the reader of a level's operator: the code words when `cod` is
// given (FP32 only), else the coefficient arrays.
template <typename T, typename F>
void with_reader(const CodeOp* cod, const Op<T>& op, F&& f) {
    if constexpr (sizeof(T) == 4) {
        if (cod) {
            f(*cod);
            return;
        }
    }
    f(ArrOp<T>{op});
}
// Level 0 in FP32: the four-wide kernels with the code words or the arrays.
struct Vec4Rd {
    bool coded;
    CodeGrp cg;
    ArrGrp ag;
};
template <typename F>
void with_vec4(const Vec4Rd& v, F&& f) {
    if (v.coded) f(v.cg);
    else f(v.ag);
}
unsigned vec4_grid(int64_t npad) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((npad / 4 + kBS - 1) / kBS, 2048));
}

// Blocks of a grid-stride stencil launch: fewer for the coded reader, whose
// blocks each copy the dictionary into LDS first.
template <typename RD>
unsigned reader_grid(unsigned g) {
    return std::is_same<RD, CodeOp>::value ? std::min(g, 2048u) : g;
}

// One V-cycle on level l from zero; returns the buffer holding the result.
// The first two pre-smoothing sweeps run as one pass (k_mg_jacobi2z); with
// `fuse` the finest level's last post-smoothing sweep also stores the block
// sums of r.z and r.r (k_mg_jacobi_dot2). A single-level hierarchy has no
// such sweep; its caller takes those sums with k_mg_dot2. `presmoothed`:
// the caller has already run the first `pre_done` pre-smoothing sweeps of
// level l into that buffer (one of the level's two iterate buffers). `cod`:
// level 0's coded reader (the sweeps and the residual of level 0 read the
// operator through it).
constexpr size_t kMgCoarseLds = 60 * 1024;   // dynamic LDS for the coarsest level's copies

template <typename T>
T* vcycle(std::vector<MgLevel<T>>& lv, size_t l, const SyncState* S, hipStream_t st, const DotFuse* fuse = nullptr,
          T* presmoothed = nullptr, int pre_done = 0, const CodeOp* cod = nullptr, const Vec4Rd* v4 = nullptr) {
    MgLevel<T>& m = lv[l];
    const Layout& L = m.L;
    const T om = (T)kMgOmega;
    const unsigned g = mg_grid(L.npad);
    const CodeOp* rd0 = l == 0 ? cod : nullptr;
    // FP32: level 0 as the caller set it up, the coarser levels with their arrays
    Vec4Rd vl{};
    const Vec4Rd* v40 = nullptr;
    if constexpr (sizeof(T) == 4) {
        if (l == 0) {
            v40 = v4;
        } else if (v4 && L.npad < ((int64_t)1 << 29)) {
            vl.coded = false;
            vl.ag = ArrGrp{(const float*)m.op.cx, (const float*)m.op.cy, (const float*)m.op.cz, (const float*)m.op.d,
                           L.npad};
            v40 = &vl;
        }
    }
    auto jacobi = [&](const T* in, T* out, int from_zero) {
        if constexpr (sizeof(T) == 4) {
            if (v40 && !from_zero) {
                with_vec4(*v40, [&](auto rd) {
                    hipLaunchKernelGGL((k_mg4_sweep<0, decltype(rd)>), dim3(vec4_grid(L.npad)), dim3(kBS), 0, st, rd,
                                       (const float*)m.b, (const float*)in, (float*)out, L.nx, L.sp, L.npad,
                                       (float)om, S);
                });
                return;
            }
        }
        with_reader<T>(rd0, m.op, [&](auto rd) {
            using RD = decltype(rd);
            hipLaunchKernelGGL((k_mg_jacobi<T, RD>), dim3(reader_grid<RD>(g)), dim3(kBS), 0, st, rd, (const T*)m.b,
                               in, out, L.nx, L.sp, L.npad, om, from_zero, S);
        });
    };
    if (l + 1 == lv.size()) {
        const size_t lds = 7 * sizeof(T) * (size_t)L.npad;
        const int use_lds = lds <= kMgCoarseLds ? 1 : 0;
        hipLaunchKernelGGL(k_mg_coarse<T>, dim3(1), dim3(1024), use_lds ? lds : 0, st, m.op, (const T*)m.b, m.xa,
                           m.xb, L.nx, L.sp, L.npad, om, kMgCoarseSweeps, use_lds, S);
        return ((kMgCoarseSweeps - 1) & 1) ? m.xb : m.xa;
    }
    T* cur = m.xa;
    T* oth = m.xb;
    int s0 = 0;
    if (presmoothed) {
        oth = presmoothed;
        cur = (presmoothed == m.xa) ? m.xb : m.xa;
        s0 = pre_done;
    } else if (kMgNu >= 2) {
        hipLaunchKernelGGL(k_mg_jacobi2z<T>, dim3(g), dim3(kBS), 0, st, m.op, (const T*)m.b, cur, L.nx, L.sp, L.npad,
                           om, S);
        std::swap(cur, oth);
        s0 = 2;
    }
    for (int s = s0; s < kMgNu; ++s) {
        jacobi((const T*)oth, cur, s == 0 ? 1 : 0);
        std::swap(cur, oth);
    }
    T* z = oth;   // the last sweep's output
    bool done_res = false;
    if constexpr (sizeof(T) == 4) {
        if (v40) {
            with_vec4(*v40, [&](auto rd) {
                hipLaunchKernelGGL((k_mg4_sweep<1, decltype(rd)>), dim3(vec4_grid(L.npad)), dim3(kBS), 0, st, rd,
                                   (const float*)m.b, (const float*)z, (float*)m.r, L.nx, L.sp, L.npad, (float)om, S);
            });
            done_res = true;
        }
    }
    if (!done_res)
        with_reader<T>(rd0, m.op, [&](auto rd) {
            using RD = decltype(rd);
            hipLaunchKernelGGL((k_mg_residual<T, RD>), dim3(reader_grid<RD>(g)), dim3(kBS), 0, st, rd,
                               (const T*)m.b, (const T*)z, m.r, L.nx, L.sp, L.npad, S);
        });
    MgLevel<T>& c = lv[l + 1];
    hipLaunchKernelGGL(k_mg_restrict<T>, plane_grid(c.L.sp, c.L.nz), dim3(kBS), 0, st, (const T*)m.r, L.nx, L.ny,
                       L.nz, L.sp, c.b, c.L.nx, c.L.ny, c.L.nz, c.L.sp, S);
    T* zc = vcycle<T>(lv, l + 1, S, st, nullptr, nullptr, 0, nullptr, v4);
    hipLaunchKernelGGL(k_mg_prolong_add<T>, plane_grid((int64_t)(c.L.nx + 1) * (c.L.ny + 1), c.L.nz + 1), dim3(kBS),
                       0, st, (const T*)zc, c.L.nx, c.L.ny, c.L.nz, c.L.sp, z, L.nx, L.ny, L.nz, L.sp, S);
    cur = (z == m.xa) ? m.xb : m.xa;
    oth = z;
    for (int s = 0; s < kMgNu; ++s) {
        bool vec_last = false;
        if constexpr (sizeof(T) == 4) vec_last = v40 && fuse && l == 0 && S && s + 1 == kMgNu;
        if (vec_last) {
            if constexpr (sizeof(T) == 4)
                with_vec4(*v40, [&](auto rd) {
                    hipLaunchKernelGGL((k_mg4_sweep_dot2<decltype(rd)>), dim3(fuse->nblk), dim3(kBS), 0, st, rd,
                                       (const float*)m.b, (const float*)oth, (float*)cur, L.nx, L.sp, L.npad,
                                       (float)om, fuse->per, fuse->partials, S);
                });
        } else if (fuse && l == 0 && S && s + 1 == kMgNu)
            with_reader<T>(rd0, m.op, [&](auto rd) {
                using RD = decltype(rd);
                hipLaunchKernelGGL((k_mg_jacobi_dot2<T, RD>), dim3(fuse->nblk), dim3(kBS), 0, st, rd,
                                   (const T*)m.b, (const T*)oth, cur, L.nx, L.sp, L.npad, om, fuse->per,
                                   fuse->partials, S);
            });
        else
            jacobi((const T*)oth, cur, 0);
        std::swap(cur, oth);
    }
    return oth;
}

}  // namespace

size_t mg_workspace_bytes(const Layout& L0, int prec) {
    return prec == PB_F64 ? mg_carve<double>(nullptr, L0, 1.0, nullptr) : mg_carve<float>(nullptr, L0, 1.0, nullptr);
}

// Multigrid-preconditioned CG. `ex..k2` are the caller's FP64 edge arrays
// (level 0 of the hierarchy); s.op is level 0's operator in T.
template <typename T>
pb_status mg_pcg_impl(const Layout& L0, double h, const double* ex, const double* ey, const double* ez,
                      const double* k2, const SolveBufs<T>& s, void* mgws, SyncState* S, double* partials,
                      double tol, int maxiter, hipStream_t st, SolveResult* res) {
    std::vector<MgLevel<T>> lv;
    mg_carve<T>(mgws, L0, h, &lv);
    lv[0].op = s.op;
    lv[0].ex = (double*)ex; lv[0].ey = (double*)ey; lv[0].ez = (double*)ez; lv[0].k2 = (double*)k2;
    lv[0].xa = s.z;      // (lv[0].b, the V-cycle's input, is the outer residual; set per iteration)
    for (size_t l = 1; l < lv.size(); ++l) {
        const MgLevel<T>& f = lv[l - 1];
        MgLevel<T>& c = lv[l];
        const int64_t tot = (int64_t)(c.L.nx + 1) * c.L.ny * c.L.nz + (int64_t)c.L.nx * (c.L.ny + 1) * c.L.nz +
                            (int64_t)c.L.nx * c.L.ny * (c.L.nz + 1) + c.L.n;
        hipLaunchKernelGGL(k_mg_coarsen, dim3(mg_grid(tot)), dim3(kBS), 0, st, (const double*)f.ex, (const double*)f.ey,
                           (const double*)f.ez, (const double*)f.k2, f.L.nx, f.L.ny, f.L.nz, c.ex, c.ey, c.ez, c.k2,
                           c.L.nx, c.L.ny, c.L.nz);
        hipLaunchKernelGGL(k_mg_op<T>, dim3(mg_grid(c.L.npad)), dim3(kBS), 0, st, (const double*)c.ex,
                           (const double*)c.ey, (const double*)c.ez, (const double*)c.k2, c.L.nx, c.L.ny, c.L.nz,
                           c.L.sp, c.h * c.h, c.op);
    }
    PB_HIP(hipGetLastError());
    // level 0 in FP32 reads its operator as code words when the values fit
    // the dictionary (the same words and dictionary as the fused solver's)
    CodeOp cod_{};
    const CodeOp* cod = nullptr;
    if constexpr (sizeof(T) == 4) {
        if (coded_coefficients() && lv[0].codes) {
            bool fits = false;
            const float* tab = nullptr;
            const pb_status e = build_codes(s.op, L0.npad, lv[0].code_scratch, lv[0].codes, st, fits, &tab);
            if (e != PB_OK) return e;
            if (fits) {
                cod_ = CodeOp{lv[0].codes, tab, nullptr};
                cod = &cod_;
            }
        }
    }

    // level 0 in FP32 runs the four-wide kernels (the code words or the arrays)
    Vec4Rd v4_{};
    const Vec4Rd* v4 = nullptr;
    if constexpr (sizeof(T) == 4) {
        if (L0.npad < ((int64_t)1 << 29)) {
            v4_.coded = cod != nullptr;
            if (cod) v4_.cg = CodeGrp{lv[0].codes, L0.npad, cod->dict, nullptr};
            v4_.ag = ArrGrp{(const float*)s.op.cx, (const float*)s.op.cy, (const float*)s.op.cz, (const float*)s.op.d,
                            L0.npad};
            v4 = &v4_;
        }
    }

    const int64_t npad = L0.npad;
    const Ranges R = ranges_for(npad);
    const unsigned g = stream_grid(npad);
    if (launch_fill<int>((int*)S, (int64_t)(sizeof(SyncState) / sizeof(int)), 0, st) != PB_OK) return PB_ERR_HIP;
    hipEvent_t ev[2] = {nullptr, nullptr};
    const bool timed = !(res && res->untimed);
    if (timed) {
        PB_HIP(hipEventCreate(&ev[0]));
        PB_HIP(hipEventCreate(&ev[1]));
    }
    if (timed) PB_HIP(hipEventRecord(ev[0], st));
    // r = b - A x0, z = M r, p = z. The residual and the direction
    // alternate between two buffers each: the fused kernels read the old
    // values around a node while writing the new ones.
    T* rb[2] = {s.r, s.r2};
    T* pb_[2] = {s.p0, s.p1};
    hipLaunchKernelGGL(k_mg_apply<T>, dim3(g), dim3(kBS), 0, st, s.op, (const T*)s.x, s.q, L0.nx, L0.sp, npad,
                       (const SyncState*)nullptr);
    hipLaunchKernelGGL(k_mg_sub<T>, dim3(g), dim3(kBS), 0, st, s.b, (const T*)s.q, rb[0], npad);
    lv[0].b = rb[0];
    T* z = vcycle<T>(lv, 0, nullptr, st);
    hipLaunchKernelGGL(k_mg_init_dots<T>, dim3(R.nblk), dim3(kBS), 0, st, (const T*)rb[0], (const T*)z, s.b, pb_[0],
                       npad, R.per, partials);
    hipLaunchKernelGGL(k_scalar_init, dim3(1), dim3(kBS), 0, st, S, (const double*)partials, R.nblk, tol, maxiter);
    PB_HIP(hipGetLastError());
    // Per iteration: p = z + beta p and q = A p with p.q (beta is 0 before the
    // first); alpha; x and r updated together with level 0's first
    // pre-smoothing sweep; the rest of the V-cycle, its last sweep with r.z
    // and r.r; beta.
    const DotFuse fuse{partials, R.nblk, R.per};
    const T om = (T)kMgOmega;
    int it = 0;
    SyncState hs{};
    for (;;) {
        for (int u = 0; u < kPoll && it < maxiter; ++u, ++it) {
            T* pold = pb_[it & 1];
            T* pnew = pb_[(it + 1) & 1];
            T* rold = rb[it & 1];
            T* rnew = rb[(it + 1) & 1];
            bool vec_dir = false;
            if constexpr (sizeof(T) == 4) {
                if (v4) {
                    with_vec4(*v4, [&](auto rd) {
                        hipLaunchKernelGGL((k_mg4_direction_apply<decltype(rd)>), dim3(R.nblk), dim3(kBS), 0, st, rd,
                                           (const float*)z, (const float*)pold, (float*)pnew, (float*)s.q, L0.nx,
                                           L0.sp, npad, R.per, partials, (const SyncState*)S);
                    });
                    vec_dir = true;
                }
            }
            if (!vec_dir)
                with_reader<T>(cod, s.op, [&](auto rd) {
                    using RD = decltype(rd);
                    hipLaunchKernelGGL((k_mg_direction_apply<T, RD>), dim3(R.nblk), dim3(kBS), 0, st, rd,
                                       (const T*)z, (const T*)pold, pnew, s.q, L0.nx, L0.sp, npad, R.per, partials,
                                       (const SyncState*)S);
                });
            hipLaunchKernelGGL(k_scalar_alpha, dim3(1), dim3(kBS), 0, st, S, (const double*)partials, R.nblk);
            lv[0].b = rnew;
            if (lv.size() > 1) {
                hipLaunchKernelGGL(k_mg_update<T>, dim3(g), dim3(kBS), 0, st, s.x, (const T*)pnew, (const T*)rold,
                                   (const T*)s.q, rnew, s.op.d, lv[0].xa, om, npad, (const SyncState*)S);
                z = vcycle<T>(lv, 0, S, st, &fuse, lv[0].xa, 1, cod, v4);   // also stores the block sums of r.z and r.r
            } else {
                hipLaunchKernelGGL(k_mg_update<T>, dim3(g), dim3(kBS), 0, st, s.x, (const T*)pnew, (const T*)rold,
                                   (const T*)s.q, rnew, s.op.d, (T*)nullptr, om, npad, (const SyncState*)S);
                z = vcycle<T>(lv, 0, S, st, nullptr, nullptr, 0, cod, v4);
                hipLaunchKernelGGL(k_mg_dot2<T>, dim3(R.nblk), dim3(kBS), 0, st, (const T*)rnew, (const T*)z, npad,
                                   R.per, partials, (const SyncState*)S);
            }
            hipLaunchKernelGGL(k_scalar_beta, dim3(1), dim3(kBS), 0, st, S, (const double*)partials, R.nblk, tol,
                               maxiter);
        }
        PB_HIP(hipGetLastError());
        PB_HIP(hipMemcpyAsync(&hs, S, sizeof(SyncState), hipMemcpyDeviceToHost, st));
        PB_HIP(hipStreamSynchronize(st));
        if (hs.done || it >= maxiter) break;
    }
    if (timed) PB_HIP(hipEventRecord(ev[1], st));
    hipLaunchKernelGGL(k_zero_if_zero_rhs<T>, dim3(g), dim3(kBS), 0, st, s.x, npad, (const SyncState*)S);
    PB_HIP(hipGetLastError());
    PB_HIP(hipMemcpyAsync(&hs, S, sizeof(SyncState), hipMemcpyDeviceToHost, st));
    PB_HIP(hipStreamSynchronize(st));
    float ms = 0.0f;
    if (timed) {
        PB_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
    }
    if (res) {
        res->kernel_seconds = 1e-3 * ms;
        res->status = hs.done ? hs.status : (int)PB_NOT_CONVERGED;
        res->iters = hs.iters;
        res->rr = hs.rr;
        res->bb = hs.bb;
    }
    return PB_OK;
}

template pb_status mg_pcg_impl<float>(const Layout&, double, const double*, const double*, const double*,
                                      const double*, const SolveBufs<float>&, void*, SyncState*, double*, double, int,
                                      hipStream_t, SolveResult*);
template pb_status mg_pcg_impl<double>(const Layout&, double, const double*, const double*, const double*,
                                       const double*, const SolveBufs<double>&, void*, SyncState*, double*, double,
                                       int, hipStream_t, SolveResult*);

}  // namespace pb
