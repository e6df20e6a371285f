// Fused, persistent Jacobi-preconditioned CG (section 2.2 listing with
// M = diag(A), section 2.4) on the matrix-free 7-point operator of Eq. 3.
//
// One cooperative launch runs the whole iteration. Each workgroup owns a
// fixed set of tiles; a tile is a contiguous range of padded plane positions
// (a "segment", which spans several x-rows) times a run of z-planes. Per
// iteration the kernel makes two passes separated by grid barriers:
//
//   pass A: p = z + beta p_old with z = r/d (recomputed, never stored),
//           q = A p, x += alpha_prev p_old (the previous iteration's x
//           update, deferred to reuse the p_old load), partial p.q
//   -- barrier: alpha = (r.z)/(p.q)
//   pass B: r -= alpha q, partials r.z and r.r
//   -- barrier: beta = (r.z)_new/(r.z)_old, stopping test ||r||/||b|| < tol
//
// Pass A marches in z: the new direction p on the current plane is staged
// in LDS over the segment plus one row of halo on each side (in-plane
// neighbours +-1, +-nx), the planes above and below stay in registers.
// Halo values of p are recomputed from r, d and p_old, so p is written once.
//
// Reductions: every tile reduces its own sums in a fixed order (thread
// order, then a fixed wave/LDS tree) into its own slot; the last workgroup
// to reach a barrier sums the tile slots in tile order. Results therefore do
// not depend on the number of workgroups or on scheduling.
#include "solver.hpp"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

namespace pb {

namespace {

constexpr int kBS = 256;
constexpr int kWaves = kBS / 64;

template <typename T>
struct KArgs {
    Op<T> op;
    const T* b;
    T* x;
    T* r;
    T* p0;
    T* p1;
    T* q;
    int nx, ny, nz;
    int64_t sp;
    int seglen, zchunk, nseg, nzc, ntiles, halo;
    double tol;
    int maxiter;
    int warm;
    SyncState* S;
    double* partials;
    long long timeout_ticks;
};

__device__ __forceinline__ double ld_acquire_d(const double* p) {
    unsigned long long v = __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)v);
}
__device__ __forceinline__ int ld_acquire_i(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reduce acc[0..np) over the workgroup in a fixed order and store the sums
// into dst[0..np) (thread 0). `red` is LDS scratch of kWaves*kMaxPartials.
template <int NP>
__device__ __forceinline__ void tile_reduce_store(double (&acc)[NP], double* red, double* dst) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        double v = acc[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wave * kMaxPartials + i] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            double s = red[i];
            for (int w = 1; w < kWaves; ++w) s += red[w * kMaxPartials + i];
            dst[i] = s;
        }
    }
    __syncthreads();
}

// Sum slot i of all tile partials in tile order (all threads of the last
// workgroup take part); the result is valid in thread 0.
__device__ double sum_tiles(const double* partials, int ntiles, int i, double* buf) {
    double a = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += kBS) a += ld_acquire_d(partials + (size_t)t * kMaxPartials + i);
    buf[threadIdx.x] = a;
    __syncthreads();
    for (int w = kBS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) buf[threadIdx.x] += buf[threadIdx.x + w];
        __syncthreads();
    }
    const double r = buf[0];
    __syncthreads();
    return r;
}

// Grid barrier. The last workgroup to arrive runs `last(buf)` with all its
// threads (it sees every other workgroup's writes) and then releases the
// others. Waits are bounded by timeout_ticks of the constant-rate clock;
// returns false if this workgroup timed out (it must then leave the kernel).
template <typename F>
__device__ bool grid_barrier(SyncState* S, unsigned& gen, long long timeout_ticks, double* buf,
                             int* s_flag, F&& last) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = __hip_atomic_fetch_add(&S->arrive, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        *s_flag = (prev == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    bool ok = true;
    if (*s_flag) {
        last(buf);
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_store(&S->arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&S->generation, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else if (threadIdx.x == 0) {
        const long long t0 = wall_clock64();
        while (__hip_atomic_load(&S->generation, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
            __builtin_amdgcn_s_sleep(2);
            if (wall_clock64() - t0 > timeout_ticks) {
                __hip_atomic_store(&S->status, (int)PB_ERR_TIMEOUT, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                *s_flag = -1;
                break;
            }
        }
    }
    ++gen;
    __syncthreads();
    if (*s_flag == -1) ok = false;
    __syncthreads();
    return ok;
}

template <typename T>
__device__ __forceinline__ typename Vec<T>::type vload(const T* p) {
    return *reinterpret_cast<const typename Vec<T>::type*>(p);
}
template <typename T>
__device__ __forceinline__ void vstore(T* p, const typename Vec<T>::type& v) {
    *reinterpret_cast<typename Vec<T>::type*>(p) = v;
}

// Tile -> (segment, z-chunk). Workgroup w runs on XCD w % 8; the tiles of
// one XCD form a contiguous block of the tile order (z-chunk major), so
// neighbouring tiles share that XCD's L2.
__device__ __forceinline__ void xcd_tile_range(int ntiles, int& first, int& stride, int& end) {
    const int G = gridDim.x;
    const int nx8 = (G >= 8 && G % 8 == 0) ? 8 : 1;
    const int xcd = blockIdx.x % nx8, local = blockIdx.x / nx8, per = G / nx8;
    const int lo = (int)(((long long)xcd * ntiles) / nx8);
    const int hi = (int)(((long long)(xcd + 1) * ntiles) / nx8);
    first = lo + local;
    stride = per;
    end = hi;
}

// ------------------------------------------------------------------ passes

// Initial residual r = b - A x0 (or r = b for a zero guess), p_old = 0,
// partials r.z, r.r, b.b.
template <typename T>
__device__ void init_tile(const KArgs<T>& a, int tile, double (&acc)[3]) {
    constexpr int W = Vec<T>::n;
    using V = typename Vec<T>::type;
    const int seg = tile % a.nseg, zc = tile / a.nseg;
    const int64_t s = (int64_t)seg * a.seglen;
    const int64_t e = min(s + (int64_t)a.seglen, a.sp);
    const int k0 = zc * a.zchunk, k1 = min(k0 + a.zchunk, a.nz);
    const int64_t npad = a.sp * a.nz;
    for (int k = k0; k < k1; ++k) {
        for (int64_t pos = s + (int64_t)threadIdx.x * W; pos < e; pos += (int64_t)kBS * W) {
            const int64_t g = (int64_t)k * a.sp + pos;
            V bv = vload(a.b + g), dv = vload(a.op.d + g), rv;
#pragma unroll
            for (int u = 0; u < W; ++u) {
                T r = vget(bv, u);
                if (a.warm) {
                    const int64_t t = g + u;
                    const T* X = a.x;
                    T nb = a.op.cx[t] * (t + 1 < npad ? X[t + 1] : T(0));
                    nb += (t >= 1 ? a.op.cx[t - 1] * X[t - 1] : T(0));
                    nb += a.op.cy[t] * (t + a.nx < npad ? X[t + a.nx] : T(0));
                    nb += (t >= a.nx ? a.op.cy[t - a.nx] * X[t - a.nx] : T(0));
                    nb += a.op.cz[t] * (t + a.sp < npad ? X[t + a.sp] : T(0));
                    nb += (t >= a.sp ? a.op.cz[t - a.sp] * X[t - a.sp] : T(0));
                    r = r - (vget(dv, u) * X[t] - nb);
                }
                vget(rv, u) = r;
                const T z = r / vget(dv, u);
                acc[0] += (double)r * (double)z;
                acc[1] += (double)r * (double)r;
                acc[2] += (double)vget(bv, u) * (double)vget(bv, u);
            }
            vstore(a.r + g, rv);
            V zero;
#pragma unroll
            for (int u = 0; u < W; ++u) vget(zero, u) = T(0);
            vstore(a.p0 + g, zero);
        }
    }
}

// Pass A on one tile (see the file comment).
template <typename T, int MC>
__device__ void passA_tile(const KArgs<T>& a, int tile, T beta, T alpha_prev, const T* __restrict__ pold,
                           T* __restrict__ pnew, T* lds0, T* lds1, double& pq) {
    constexpr int W = Vec<T>::n;
    using V = typename Vec<T>::type;
    const int seg = tile % a.nseg, zc = tile / a.nseg;
    const int64_t s = (int64_t)seg * a.seglen;
    const int64_t e = min(s + (int64_t)a.seglen, a.sp);
    const int k0 = zc * a.zchunk, k1 = min(k0 + a.zchunk, a.nz);
    const int H = a.halo, nx = a.nx;
    const int64_t sp = a.sp;
    const int64_t lbase = s - H;
    const int hgroups = 2 * H / W;
    const bool do_x = alpha_prev != T(0);

    int64_t pos[MC];
    bool valid[MC];
#pragma unroll
    for (int c = 0; c < MC; ++c) {
        pos[c] = s + (int64_t)(c * kBS + threadIdx.x) * W;
        valid[c] = pos[c] < e;
    }
    V pm[MC], pc[MC], pn[MC], czm[MC], poc[MC], dc[MC];
    const V vzero = [] { V v; for (int u = 0; u < W; ++u) vget(v, u) = T(0); return v; }();

    auto pnew_at = [&](int64_t g, V& po, V& dv) -> V {
        const V rv = vload(a.r + g);
        dv = vload(a.op.d + g);
        po = vload(pold + g);
        V out;
#pragma unroll
        for (int u = 0; u < W; ++u) vget(out, u) = vget(rv, u) / vget(dv, u) + beta * vget(po, u);
        return out;
    };
    auto halo_fill = [&](int k, T* buf) {
        for (int hg = threadIdx.x; hg < hgroups; hg += kBS) {
            const int64_t hp = (hg < H / W) ? (s - H + (int64_t)hg * W) : (e + (int64_t)(hg - H / W) * W);
            V v = vzero;
            if (hp >= 0 && hp < sp) {
                V po, dv;
                v = pnew_at((int64_t)k * sp + hp, po, dv);
            }
            vstore(buf + (hp - lbase), v);
        }
    };

    // prologue: plane k0-1 (own positions only) and plane k0 (with halo)
#pragma unroll
    for (int c = 0; c < MC; ++c) {
        pm[c] = vzero;
        czm[c] = vzero;
        if (valid[c] && k0 > 0) {
            const int64_t g = (int64_t)(k0 - 1) * sp + pos[c];
            V po, dv;
            pm[c] = pnew_at(g, po, dv);
            czm[c] = vload(a.op.cz + g);
        }
    }
    {
        T* buf = (k0 & 1) ? lds1 : lds0;
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            pc[c] = vzero;
            poc[c] = vzero;
            dc[c] = vzero;
            if (valid[c]) {
                pc[c] = pnew_at((int64_t)k0 * sp + pos[c], poc[c], dc[c]);
                vstore(buf + (pos[c] - lbase), pc[c]);
            }
        }
        halo_fill(k0, buf);
    }
    __syncthreads();

    for (int k = k0; k < k1; ++k) {
        const T* cur = (k & 1) ? lds1 : lds0;
        T* nxt = (k & 1) ? lds0 : lds1;
        V pon[MC], dn[MC];
        const bool has_next = k + 1 < a.nz;
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            pn[c] = vzero;
            pon[c] = vzero;
            dn[c] = vzero;
            if (valid[c] && has_next) {
                pn[c] = pnew_at((int64_t)(k + 1) * sp + pos[c], pon[c], dn[c]);
                vstore(nxt + (pos[c] - lbase), pn[c]);
            }
        }
        if (has_next && k + 1 < k1) halo_fill(k + 1, nxt);

#pragma unroll
        for (int c = 0; c < MC; ++c) {
            if (!valid[c]) continue;
            const int64_t g = (int64_t)k * sp + pos[c];
            const int64_t l = pos[c] - lbase;
            const V cxv = vload(a.op.cx + g);
            const V cyv = vload(a.op.cy + g);
            const V czv = vload(a.op.cz + g);
            const T cxm = pos[c] >= 1 ? a.op.cx[g - 1] : T(0);
            const T left = cur[l - 1];
            const T right = cur[l + W];
            V qv;
#pragma unroll
            for (int u = 0; u < W; ++u) {
                const T p = vget(pc[c], u);
                const T pl = (u == 0) ? left : vget(pc[c], u - 1);
                const T pr = (u == W - 1) ? right : vget(pc[c], u + 1);
                const T cl = (u == 0) ? cxm : vget(cxv, u - 1);
                const T cym = (pos[c] + u - nx >= 0) ? a.op.cy[g + u - nx] : T(0);
                T nb = vget(cxv, u) * pr + cl * pl;
                nb += vget(cyv, u) * cur[l + u + nx] + cym * cur[l + u - nx];
                nb += vget(czv, u) * vget(pn[c], u) + vget(czm[c], u) * vget(pm[c], u);
                const T qq = vget(dc[c], u) * p - nb;
                vget(qv, u) = qq;
                pq += (double)p * (double)qq;
            }
            vstore(pnew + g, pc[c]);
            vstore(a.q + g, qv);
            if (do_x) {
                V xv = vload(a.x + g);
#pragma unroll
                for (int u = 0; u < W; ++u) vget(xv, u) = vget(xv, u) + alpha_prev * vget(poc[c], u);
                vstore(a.x + g, xv);
            }
            czm[c] = czv;
        }
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            pm[c] = pc[c];
            pc[c] = pn[c];
            poc[c] = pon[c];
            dc[c] = dn[c];
        }
        __syncthreads();
    }
}

// Pass B on one tile: r -= alpha q; partials r.z and r.r.
template <typename T>
__device__ void passB_tile(const KArgs<T>& a, int tile, T alpha, double& rz, double& rr) {
    constexpr int W = Vec<T>::n;
    using V = typename Vec<T>::type;
    const int seg = tile % a.nseg, zc = tile / a.nseg;
    const int64_t s = (int64_t)seg * a.seglen;
    const int64_t e = min(s + (int64_t)a.seglen, a.sp);
    const int k0 = zc * a.zchunk, k1 = min(k0 + a.zchunk, a.nz);
    for (int k = k0; k < k1; ++k) {
        for (int64_t pos = s + (int64_t)threadIdx.x * W; pos < e; pos += (int64_t)kBS * W) {
            const int64_t g = (int64_t)k * a.sp + pos;
            V rv = vload(a.r + g);
            const V qv = vload(a.q + g);
            const V dv = vload(a.op.d + g);
#pragma unroll
            for (int u = 0; u < W; ++u) {
                const T r = vget(rv, u) - alpha * vget(qv, u);
                vget(rv, u) = r;
                const T z = r / vget(dv, u);
                rz += (double)r * (double)z;
                rr += (double)r * (double)r;
            }
            vstore(a.r + g, rv);
        }
    }
}

// Final pass: x += alpha p (or x = 0 for a zero right-hand side).
template <typename T>
__device__ void final_tile(const KArgs<T>& a, int tile, T alpha, const T* p, bool zero) {
    constexpr int W = Vec<T>::n;
    using V = typename Vec<T>::type;
    const int seg = tile % a.nseg, zc = tile / a.nseg;
    const int64_t s = (int64_t)seg * a.seglen;
    const int64_t e = min(s + (int64_t)a.seglen, a.sp);
    const int k0 = zc * a.zchunk, k1 = min(k0 + a.zchunk, a.nz);
    for (int k = k0; k < k1; ++k) {
        for (int64_t pos = s + (int64_t)threadIdx.x * W; pos < e; pos += (int64_t)kBS * W) {
            const int64_t g = (int64_t)k * a.sp + pos;
            V xv = vload(a.x + g);
            if (zero) {
#pragma unroll
                for (int u = 0; u < W; ++u) vget(xv, u) = T(0);
            } else {
                const V pv = vload(p + g);
#pragma unroll
                for (int u = 0; u < W; ++u) vget(xv, u) = vget(xv, u) + alpha * vget(pv, u);
            }
            vstore(a.x + g, xv);
        }
    }
}

// ------------------------------------------------------------------ kernel

struct Scal {
    double alpha, alpha_prev, beta, rho, rr, bb;
    int iters, done, status, zero;
};

__device__ void read_scalars(SyncState* S, Scal* out) {
    if (threadIdx.x == 0) {
        out->alpha = ld_acquire_d(&S->alpha);
        out->alpha_prev = ld_acquire_d(&S->alpha_prev);
        out->beta = ld_acquire_d(&S->beta);
        out->rho = ld_acquire_d(&S->rho);
        out->rr = ld_acquire_d(&S->rr);
        out->bb = ld_acquire_d(&S->bb);
        out->iters = ld_acquire_i(&S->iters);
        out->done = ld_acquire_i(&S->done);
        out->status = ld_acquire_i(&S->status);
        out->zero = ld_acquire_i(&S->zero_rhs);
    }
    __syncthreads();
}

template <typename T, int MC>
__global__ __launch_bounds__(kBS) void k_jpcg_fused(KArgs<T> a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int lds_len = a.seglen + 2 * a.halo;
    T* lds0 = reinterpret_cast<T*>(lds_raw);
    T* lds1 = lds0 + lds_len;
    __shared__ double red[kWaves * kMaxPartials];
    __shared__ double buf[kBS];
    __shared__ int s_flag;
    __shared__ Scal sc;
    SyncState* S = a.S;
    unsigned gen = 0;
    int first, stride, end;
    xcd_tile_range(a.ntiles, first, stride, end);

    // ---- initial residual
    for (int t = first; t < end; t += stride) {
        double acc[3] = {0.0, 0.0, 0.0};
        init_tile<T>(a, t, acc);
        tile_reduce_store<3>(acc, red, a.partials + (size_t)t * kMaxPartials);
    }
    bool ok = grid_barrier(S, gen, a.timeout_ticks, buf, &s_flag, [&](double* b) {
        const double rz = sum_tiles(a.partials, a.ntiles, 0, b);
        const double rr = sum_tiles(a.partials, a.ntiles, 1, b);
        const double bb = sum_tiles(a.partials, a.ntiles, 2, b);
        if (threadIdx.x == 0) {
            S->rho = rz; S->rr = rr; S->bb = bb;
            S->alpha = 0.0; S->alpha_prev = 0.0; S->beta = 0.0; S->iters = 0;
            int done = 0, status = PB_OK;
            if (!(bb - bb == 0.0) || !(rr - rr == 0.0)) { done = 1; status = PB_ERR_NONFINITE; }
            else if (bb == 0.0) { done = 1; S->zero_rhs = 1; }
            else if (sqrt(rr) / sqrt(bb) < a.tol) { done = 1; }
            else if (a.maxiter <= 0) { done = 1; status = PB_NOT_CONVERGED; }
            S->done = done;
            S->status = status;
        }
    });
    if (!ok) return;
    read_scalars(S, &sc);
    int it = 0;
    bool final_update = false;
    while (!sc.done) {
        const T* pold = (it & 1) ? a.p1 : a.p0;
        T* pnew = (it & 1) ? a.p0 : a.p1;
        const T beta = (T)sc.beta, alpha_prev = (T)sc.alpha_prev;
        for (int t = first; t < end; t += stride) {
            double acc[1] = {0.0};
            passA_tile<T, MC>(a, t, beta, alpha_prev, pold, pnew, lds0, lds1, acc[0]);
            tile_reduce_store<1>(acc, red, a.partials + (size_t)t * kMaxPartials);
        }
        ok = grid_barrier(S, gen, a.timeout_ticks, buf, &s_flag, [&](double* b) {
            const double pq = sum_tiles(a.partials, a.ntiles, 0, b);
            if (threadIdx.x == 0) {
                S->pq = pq;
                if (!(pq > 0.0) || !(pq - pq == 0.0)) {
                    S->done = 1;
                    S->status = PB_ERR_BREAKDOWN;
                    S->alpha = 0.0;
                } else {
                    S->alpha = ld_acquire_d(&S->rho) / pq;
                }
            }
        });
        if (!ok) return;
        read_scalars(S, &sc);
        if (sc.done) break;   // breakdown: x already holds the last good iterate
        const T alpha = (T)sc.alpha;
        for (int t = first; t < end; t += stride) {
            double acc[2] = {0.0, 0.0};
            passB_tile<T>(a, t, alpha, acc[0], acc[1]);
            tile_reduce_store<2>(acc, red, a.partials + (size_t)t * kMaxPartials);
        }
        ok = grid_barrier(S, gen, a.timeout_ticks, buf, &s_flag, [&](double* b) {
            const double rz = sum_tiles(a.partials, a.ntiles, 0, b);
            const double rr = sum_tiles(a.partials, a.ntiles, 1, b);
            if (threadIdx.x == 0) {
                const int iters = ld_acquire_i(&S->iters) + 1;
                S->iters = iters;
                S->beta = rz / ld_acquire_d(&S->rho);
                S->rho = rz;
                S->rr = rr;
                S->alpha_prev = ld_acquire_d(&S->alpha);
                const double rel = sqrt(rr) / sqrt(ld_acquire_d(&S->bb));
                if (!(rel - rel == 0.0)) { S->done = 1; S->status = PB_ERR_BREAKDOWN; }
                else if (rel < a.tol) { S->done = 1; S->status = PB_OK; }
                else if (iters >= a.maxiter) { S->done = 1; S->status = PB_NOT_CONVERGED; }
            }
        });
        if (!ok) return;
        read_scalars(S, &sc);
        ++it;
        final_update = true;
    }
    // ---- final x update with the last alpha and direction (or x = 0)
    if (sc.zero || (final_update && sc.status != PB_ERR_BREAKDOWN)) {
        const T* plast = (it & 1) ? a.p1 : a.p0;
        for (int t = first; t < end; t += stride) final_tile<T>(a, t, (T)sc.alpha, plast, sc.zero != 0);
    }
}

// ------------------------------------------------------------------ host side

struct DevInfo {
    int cus = 0;
    int wallclock_khz = 0;
};

DevInfo dev_info() {
    static std::mutex mu;
    static std::vector<DevInfo> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return DevInfo{};
    std::lock_guard<std::mutex> lk(mu);
    if ((int)cache.size() <= dev) cache.resize(dev + 1);
    if (cache[dev].cus == 0) {
        DevInfo d;
        hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev);
        hipDeviceGetAttribute(&d.wallclock_khz, hipDeviceAttributeWallClockRate, dev);
        cache[dev] = d;
    }
    return cache[dev];
}

template <typename T, int MC>
int max_coresident(size_t lds_bytes) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_jpcg_fused<T, MC>, kBS, lds_bytes) != hipSuccess)
        return 0;
    return nb;
}

template <typename T>
int halo_for(int nx) {
    constexpr int W = Vec<T>::n;
    return (nx + W - 1) / W * W;
}

}  // namespace

// Tile shape: segments of mc*256*VEC positions; z-chunks sized so that every
// workgroup gets at most one tile per pass when possible (balanced work).
template <typename T>
Tiling choose_tiling(const Layout& L) {
    constexpr int W = Vec<T>::n;
    const DevInfo di = dev_info();
    const int cus = di.cus > 0 ? di.cus : 256;
    Tiling best{};
    double best_cost = 1e300;
    for (int mc : {1, 2, 4}) {
        Tiling t{};
        t.mc = mc;
        t.seglen = mc * kBS * W;
        t.halo = halo_for<T>(L.nx);
        const size_t lds = 2 * sizeof(T) * (size_t)(t.seglen + 2 * t.halo);
        int per_cu = 0;
        if (mc == 1) per_cu = max_coresident<T, 1>(lds);
        if (mc == 2) per_cu = max_coresident<T, 2>(lds);
        if (mc == 4) per_cu = max_coresident<T, 4>(lds);
        if (per_cu <= 0) continue;
        int G = per_cu * cus;
        t.nseg = (int)((L.sp + t.seglen - 1) / t.seglen);
        // z-chunk: fill the co-resident workgroups with about one tile each
        int zc = std::max(1, (int)((L.nz * (int64_t)t.nseg + G - 1) / G));
        t.zchunk = zc;
        t.nzc = (L.nz + zc - 1) / zc;
        t.ntiles = t.nseg * t.nzc;
        if (t.ntiles > kMaxTiles) continue;
        if (G > t.ntiles) G = t.ntiles;
        if (G >= 8) G = G / 8 * 8;
        t.grid = G;
        // cost: the busiest workgroup's elements incl. halo and the extra z-plane
        const int tiles_per_wg = (t.ntiles + G - 1) / G;
        const double work = (double)tiles_per_wg * (t.zchunk + 1) * (t.seglen + 2.0 * t.halo * 0.5);
        const double cost = work;
        if (cost < best_cost) {
            best_cost = cost;
            best = t;
        }
    }
    return best;
}
template Tiling choose_tiling<float>(const Layout&);
template Tiling choose_tiling<double>(const Layout&);

template <typename T>
pb_status fused_jpcg(const Layout& L, const SolveBufs<T>& s, SyncState* sync, double* partials, double tol,
                     int maxiter, hipStream_t st, SolveResult* res, Tiling* used) {
    Tiling t = choose_tiling<T>(L);
    if (t.grid <= 0) {
        set_error("fused JPCG: no feasible tiling / occupancy for this grid");
        return PB_ERR_HIP;
    }
    if (used) *used = t;
    const DevInfo di = dev_info();
    KArgs<T> a{};
    a.op = s.op;
    a.b = s.b;
    a.x = s.x;
    a.r = s.r;
    a.p0 = s.p0;
    a.p1 = s.p1;
    a.q = s.q;
    a.nx = L.nx; a.ny = L.ny; a.nz = L.nz;
    a.sp = L.sp;
    a.seglen = t.seglen; a.zchunk = t.zchunk; a.nseg = t.nseg; a.nzc = t.nzc; a.ntiles = t.ntiles;
    a.halo = t.halo;
    a.tol = tol;
    a.maxiter = maxiter;
    a.warm = s.warm;
    a.S = sync;
    a.partials = partials;
    // every wait is bounded: 20 s of the constant-rate clock
    a.timeout_ticks = (long long)(di.wallclock_khz > 0 ? di.wallclock_khz : 100000) * 1000LL * 20LL;
    // the header (barrier counters, scalars) starts cleared
    if (launch_fill<int>((int*)sync, (int64_t)(sizeof(SyncState) / sizeof(int)), 0, st) != PB_OK)
        return PB_ERR_HIP;
    const size_t lds = 2 * sizeof(T) * (size_t)(t.seglen + 2 * t.halo);
    void* args[] = {&a};
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (res) {
        PB_HIP(hipEventCreate(&ev[0]));
        PB_HIP(hipEventCreate(&ev[1]));
        PB_HIP(hipEventRecord(ev[0], st));
    }
    hipError_t e = hipSuccess;
    if (t.mc == 1) e = hipLaunchCooperativeKernel((const void*)k_jpcg_fused<T, 1>, dim3(t.grid), dim3(kBS), args, lds, st);
    else if (t.mc == 2) e = hipLaunchCooperativeKernel((const void*)k_jpcg_fused<T, 2>, dim3(t.grid), dim3(kBS), args, lds, st);
    else e = hipLaunchCooperativeKernel((const void*)k_jpcg_fused<T, 4>, dim3(t.grid), dim3(kBS), args, lds, st);
    if (e != hipSuccess) {
        if (ev[0]) (void)hipEventDestroy(ev[0]);
        if (ev[1]) (void)hipEventDestroy(ev[1]);
        set_error("fused JPCG launch failed: %s (grid %d, lds %zu)", hipGetErrorString(e), t.grid, lds);
        return PB_ERR_HIP;
    }
    if (res) {
        SyncState h;
        PB_HIP(hipEventRecord(ev[1], st));
        PB_HIP(hipMemcpyAsync(&h, sync, sizeof(SyncState), hipMemcpyDeviceToHost, st));
        PB_HIP(hipStreamSynchronize(st));
        float ms = 0.0f;
        PB_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
        res->status = h.status;
        res->iters = h.iters;
        res->rr = h.rr;
        res->bb = h.bb;
        res->kernel_seconds = 1e-3 * ms;
    }
    return PB_OK;
}
template pb_status fused_jpcg<float>(const Layout&, const SolveBufs<float>&, SyncState*, double*, double, int,
                                     hipStream_t, SolveResult*, Tiling*);
template pb_status fused_jpcg<double>(const Layout&, const SolveBufs<double>&, SyncState*, double*, double, int,
                                      hipStream_t, SolveResult*, Tiling*);

}  // namespace pb
