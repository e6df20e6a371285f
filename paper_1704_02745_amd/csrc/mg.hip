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

#include <vector>

namespace pb {
namespace {

constexpr int kMgNu = 2;            // Jacobi sweeps before and after the coarse correction
constexpr int kMgCoarseSweeps = 40;  // sweeps on the coarsest level
constexpr int64_t kMgMinNodes = 512;
constexpr double kMgOmega = 0.8;

__device__ __forceinline__ double w3(int a) { return a == 0 ? 0.5 : 0.25; }   // a in -1..1
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

// (A v) at padded position t (free-space stencil; zero couplings cut the
// faces and the pad slots).
template <typename T>
__device__ __forceinline__ T mg_apply(const Op<T>& op, const T* __restrict__ v, int64_t t, int nx, int64_t sp,
                                      int64_t npad) {
    T nb = op.cx[t] * (t + 1 < npad ? v[t + 1] : T(0));
    nb += (t >= 1 ? op.cx[t - 1] * v[t - 1] : T(0));
    nb += op.cy[t] * (t + nx < npad ? v[t + nx] : T(0));
    nb += (t >= nx ? op.cy[t - nx] * v[t - nx] : T(0));
    nb += op.cz[t] * (t + sp < npad ? v[t + sp] : T(0));
    nb += (t >= sp ? op.cz[t - sp] * v[t - sp] : T(0));
    return op.d[t] * v[t] - nb;
}

// One damped-Jacobi sweep out = in + omega (b - A in)/d; from_zero: in = 0.
template <typename T>
__global__ void k_mg_jacobi(Op<T> op, const T* __restrict__ b, const T* __restrict__ in, T* __restrict__ out,
                            int nx, int64_t sp, int64_t npad, T omega, int from_zero, const SyncState* S) {
    if (S && stop(S)) return;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x) {
        if (from_zero) {
            out[t] = omega * b[t] / op.d[t];
        } else {
            const T r = b[t] - mg_apply(op, in, t, nx, sp, npad);
            out[t] = in[t] + omega * r / op.d[t];
        }
    }
}

// The first two damped-Jacobi sweeps from zero in one pass. The first
// sweep's output x1 = omega b / d is formed where the second needs it (the
// node and its six neighbours) with the arithmetic of the from_zero sweep, so
// the result equals two k_mg_jacobi launches bit for bit.
template <typename T>
__device__ __forceinline__ T mg_x1(const Op<T>& op, const T* __restrict__ b, int64_t t, T omega) {
    return omega * b[t] / op.d[t];
}

template <typename T>
__global__ void k_mg_jacobi2z(Op<T> op, const T* __restrict__ b, T* __restrict__ out, int nx, int64_t sp,
                              int64_t npad, T omega, const SyncState* S) {
    if (S && stop(S)) return;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x) {
        T nb = op.cx[t] * (t + 1 < npad ? mg_x1(op, b, t + 1, omega) : T(0));
        nb += (t >= 1 ? op.cx[t - 1] * mg_x1(op, b, t - 1, omega) : T(0));
        nb += op.cy[t] * (t + nx < npad ? mg_x1(op, b, t + nx, omega) : T(0));
        nb += (t >= nx ? op.cy[t - nx] * mg_x1(op, b, t - nx, omega) : T(0));
        nb += op.cz[t] * (t + sp < npad ? mg_x1(op, b, t + sp, omega) : T(0));
        nb += (t >= sp ? op.cz[t - sp] * mg_x1(op, b, t - sp, omega) : T(0));
        const T x1 = mg_x1(op, b, t, omega);
        const T r = b[t] - (op.d[t] * x1 - nb);
        out[t] = x1 + omega * r / op.d[t];
    }
}

// The finest level's last post-smoothing sweep fused with the outer
// iteration's r.z and r.r (the level's right-hand side is the outer residual
// r): block b sweeps positions [b*per, (b+1)*per), threads striding by the
// block size, and stores the block sums in the fixed order of block_sum_store.
template <typename T>
__global__ __launch_bounds__(kBS) void k_mg_jacobi_dot2(Op<T> op, const T* __restrict__ b, const T* __restrict__ in,
                                                        T* __restrict__ out, int nx, int64_t sp, int64_t npad,
                                                        T omega, int64_t per, double* __restrict__ partials,
                                                        const SyncState* S) {
    if (stop(S)) return;
    double acc[2] = {0.0, 0.0};
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(lo + per, npad);
    for (int64_t t = lo + threadIdx.x; t < hi; t += kBS) {
        const T res = b[t] - mg_apply(op, in, t, nx, sp, npad);
        const T z = in[t] + omega * res / op.d[t];
        out[t] = z;
        acc[0] += (double)b[t] * (double)z;
        acc[1] += (double)b[t] * (double)b[t];
    }
    block_sum_store<2>(acc, partials + (size_t)blockIdx.x * kMaxPartials);
}

template <typename T>
__global__ void k_mg_residual(Op<T> op, const T* __restrict__ b, const T* __restrict__ x, T* __restrict__ r, int nx,
                              int64_t sp, int64_t npad, const SyncState* S) {
    if (S && stop(S)) return;
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
template <typename T>
__global__ void k_mg_restrict(const T* __restrict__ r, int nx, int ny, int nz, int64_t sp, T* __restrict__ bc,
                              int ncx, int ncy, int ncz, int64_t spc, const SyncState* S) {
    if (S && stop(S)) return;
    const int64_t pc = (int64_t)ncx * ncy, npc = spc * ncz;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npc;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t K = t / spc, pp = t - K * spc;
        if (pp >= pc) {
            bc[t] = T(0);
            continue;
        }
        const int J = (int)(pp / ncx), I = (int)(pp - (int64_t)J * ncx);
        T acc = T(0);
        for (int c = -1; c <= 1; ++c) {
            const int k = 2 * (int)K + 1 + c;
            if (k < 0 || k >= nz) continue;
            for (int b = -1; b <= 1; ++b) {
                const int j = 2 * J + 1 + b;
                if (j < 0 || j >= ny) continue;
                for (int a = -1; a <= 1; ++a) {
                    const int i = 2 * I + 1 + a;
                    if (i < 0 || i >= nx) continue;
                    acc += (T)(w3(a) * w3(b) * w3(c)) * r[(int64_t)k * sp + (int64_t)j * nx + i];
                }
            }
        }
        bc[t] = acc;
    }
}

// x += P xc (trilinear: fine i odd takes coarse (i-1)/2, fine i even the
// mean of coarse i/2-1 and i/2; coarse ghosts are zero).
template <typename T>
__global__ void k_mg_prolong_add(const T* __restrict__ xc, int ncx, int ncy, int ncz, int64_t spc,
                                 T* __restrict__ x, int nx, int ny, int nz, int64_t sp, const SyncState* S) {
    if (S && stop(S)) return;
    const int64_t plane = (int64_t)nx * ny, npad = sp * nz;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = t / sp, pp = t - k * sp;
        if (pp >= plane) continue;
        const int j = (int)(pp / nx), i = (int)(pp - (int64_t)j * nx);
        int ci[2], cj[2], ck[2];
        T wi[2], wj[2], wk[2];
        auto axis = [](int f, int nc, int (&c)[2], T (&w)[2]) {
            if (f & 1) {
                c[0] = (f - 1) / 2; w[0] = T(1); c[1] = -1; w[1] = T(0);
            } else {
                c[0] = f / 2 - 1; w[0] = T(0.5); c[1] = f / 2; w[1] = T(0.5);
            }
            for (int q = 0; q < 2; ++q)
                if (c[q] < 0 || c[q] >= nc) { c[q] = -1; w[q] = T(0); }
        };
        axis(i, ncx, ci, wi);
        axis(j, ncy, cj, wj);
        axis((int)k, ncz, ck, wk);
        T add = T(0);
        for (int c = 0; c < 2; ++c) {
            if (ck[c] < 0) continue;
            for (int b = 0; b < 2; ++b) {
                if (cj[b] < 0) continue;
                for (int a = 0; a < 2; ++a) {
                    if (ci[a] < 0) continue;
                    add += wi[a] * wj[b] * wk[c] * xc[(int64_t)ck[c] * spc + (int64_t)cj[b] * ncx + ci[a]];
                }
            }
        }
        x[t] += add;
    }
}

// The coarsest level: `sweeps` damped-Jacobi sweeps from zero by one
// workgroup (the level is small); buf[(sweeps-1) & 1] holds the result.
template <typename T>
__global__ __launch_bounds__(1024) void k_mg_coarse(Op<T> op, const T* __restrict__ b, T* __restrict__ buf0,
                                                    T* __restrict__ buf1, int nx, int64_t sp, int64_t npad, T omega,
                                                    int sweeps, const SyncState* S) {
    if (S && stop(S)) return;
    for (int it = 0; it < sweeps; ++it) {
        const T* in = (it & 1) ? buf0 : buf1;
        T* out = (it & 1) ? buf1 : buf0;
        for (int64_t t = threadIdx.x; t < npad; t += blockDim.x) {
            if (it == 0) {
                out[t] = omega * b[t] / op.d[t];
            } else {
                const T r = b[t] - mg_apply(op, in, t, nx, sp, npad);
                out[t] = in[t] + omega * r / op.d[t];
            }
        }
        __syncthreads();
    }
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

// One V-cycle on level l from zero; returns the buffer holding the result.
// The first two pre-smoothing sweeps run as one pass (k_mg_jacobi2z); with
// `fuse` the finest level's last post-smoothing sweep also stores the block
// sums of r.z and r.r (k_mg_jacobi_dot2). A single-level hierarchy has no
// such sweep; its caller takes those sums with k_mg_dot2.
template <typename T>
T* vcycle(std::vector<MgLevel<T>>& lv, size_t l, const SyncState* S, hipStream_t st, const DotFuse* fuse = nullptr) {
    MgLevel<T>& m = lv[l];
    const Layout& L = m.L;
    const T om = (T)kMgOmega;
    const unsigned g = mg_grid(L.npad);
    if (l + 1 == lv.size()) {
        hipLaunchKernelGGL(k_mg_coarse<T>, dim3(1), dim3(1024), 0, st, m.op, (const T*)m.b, m.xa, m.xb, L.nx, L.sp,
                           L.npad, om, kMgCoarseSweeps, S);
        return ((kMgCoarseSweeps - 1) & 1) ? m.xb : m.xa;
    }
    T* cur = m.xa;
    T* oth = m.xb;
    int s0 = 0;
    if (kMgNu >= 2) {
        hipLaunchKernelGGL(k_mg_jacobi2z<T>, dim3(g), dim3(kBS), 0, st, m.op, (const T*)m.b, cur, L.nx, L.sp, L.npad,
                           om, S);
        std::swap(cur, oth);
        s0 = 2;
    }
    for (int s = s0; s < kMgNu; ++s) {
        hipLaunchKernelGGL(k_mg_jacobi<T>, dim3(g), dim3(kBS), 0, st, m.op, (const T*)m.b, (const T*)oth, cur, L.nx,
                           L.sp, L.npad, om, s == 0 ? 1 : 0, S);
        std::swap(cur, oth);
    }
    T* z = oth;   // the last sweep's output
    hipLaunchKernelGGL(k_mg_residual<T>, dim3(g), dim3(kBS), 0, st, m.op, (const T*)m.b, (const T*)z, m.r, L.nx, L.sp,
                       L.npad, S);
    MgLevel<T>& c = lv[l + 1];
    hipLaunchKernelGGL(k_mg_restrict<T>, dim3(mg_grid(c.L.npad)), dim3(kBS), 0, st, (const T*)m.r, L.nx, L.ny, L.nz,
                       L.sp, c.b, c.L.nx, c.L.ny, c.L.nz, c.L.sp, S);
    T* zc = vcycle(lv, l + 1, S, st);
    hipLaunchKernelGGL(k_mg_prolong_add<T>, dim3(g), dim3(kBS), 0, st, (const T*)zc, c.L.nx, c.L.ny, c.L.nz, c.L.sp,
                       z, L.nx, L.ny, L.nz, L.sp, S);
    cur = (z == m.xa) ? m.xb : m.xa;
    oth = z;
    for (int s = 0; s < kMgNu; ++s) {
        if (fuse && l == 0 && S && s + 1 == kMgNu)
            hipLaunchKernelGGL(k_mg_jacobi_dot2<T>, dim3(fuse->nblk), dim3(kBS), 0, st, m.op, (const T*)m.b,
                               (const T*)oth, cur, L.nx, L.sp, L.npad, om, fuse->per, fuse->partials, S);
        else
            hipLaunchKernelGGL(k_mg_jacobi<T>, dim3(g), dim3(kBS), 0, st, m.op, (const T*)m.b, (const T*)oth, cur,
                               L.nx, L.sp, L.npad, om, 0, S);
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
    lv[0].b = s.r;       // the V-cycle's input is the outer residual
    lv[0].xa = s.z;
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
    // r = b - A x0, z = M r, p = z
    hipLaunchKernelGGL(k_mg_apply<T>, dim3(g), dim3(kBS), 0, st, s.op, (const T*)s.x, s.q, L0.nx, L0.sp, npad,
                       (const SyncState*)nullptr);
    hipLaunchKernelGGL(k_mg_sub<T>, dim3(g), dim3(kBS), 0, st, s.b, (const T*)s.q, s.r, npad);
    T* z = vcycle<T>(lv, 0, nullptr, st);
    hipLaunchKernelGGL(k_mg_init_dots<T>, dim3(R.nblk), dim3(kBS), 0, st, (const T*)s.r, (const T*)z, s.b, s.p0, npad,
                       R.per, partials);
    hipLaunchKernelGGL(k_scalar_init, dim3(1), dim3(kBS), 0, st, S, (const double*)partials, R.nblk, tol, maxiter);
    PB_HIP(hipGetLastError());
    const DotFuse fuse{partials, R.nblk, R.per};
    int it = 0;
    SyncState hs{};
    for (;;) {
        for (int u = 0; u < kPoll && it < maxiter; ++u, ++it) {
            hipLaunchKernelGGL(k_mg_apply<T>, dim3(g), dim3(kBS), 0, st, s.op, (const T*)s.p0, s.q, L0.nx, L0.sp, npad,
                               (const SyncState*)S);
            hipLaunchKernelGGL(k_dot<T>, dim3(R.nblk), dim3(kBS), 0, st, (const T*)s.p0, (const T*)s.q, npad, R.per,
                               partials, (const SyncState*)S);
            hipLaunchKernelGGL(k_scalar_alpha, dim3(1), dim3(kBS), 0, st, S, (const double*)partials, R.nblk);
            hipLaunchKernelGGL(k_axpy2<T>, dim3(g), dim3(kBS), 0, st, s.x, (const T*)s.p0, s.r, (const T*)s.q, npad,
                               (const SyncState*)S);
            if (lv.size() > 1) {
                z = vcycle<T>(lv, 0, S, st, &fuse);   // also stores the block sums of r.z and r.r
            } else {
                z = vcycle<T>(lv, 0, S, st);
                hipLaunchKernelGGL(k_mg_dot2<T>, dim3(R.nblk), dim3(kBS), 0, st, (const T*)s.r, (const T*)z, npad,
                                   R.per, partials, (const SyncState*)S);
            }
            hipLaunchKernelGGL(k_scalar_beta, dim3(1), dim3(kBS), 0, st, S, (const double*)partials, R.nblk, tol,
                               maxiter);
            hipLaunchKernelGGL(k_xpay<T>, dim3(g), dim3(kBS), 0, st, (const T*)z, s.p0, npad, (const SyncState*)S);
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
