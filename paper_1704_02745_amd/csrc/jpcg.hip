// Fused, persistent Jacobi-preconditioned CG on the matrix-free 7-point
// operator of Eq. 3 (preconditioned CG of section 2.2 with M = diag(A),
// section 2.4), one pass over the grid per iteration.
//
// The listing updates alpha, x, r, then beta, p, and needs two global
// reductions per iteration (p.Ap for alpha, r.z for beta). Here the
// iteration is regrouped so that one pass and one grid barrier suffice:
// pass l receives alpha_{l-1}, beta_{l-1} and the stored q_{l-1} = A p_{l-2},
// and per node computes
//     r_{l-1} = r_{l-2} - alpha_{l-1} q_{l-1}
//     p_{l-1} = r_{l-1}/d + beta_{l-1} p_{l-2}          (z = r/d never stored)
//     x_{l-1} = x_{l-2} + alpha_{l-1} p_{l-2}
//     q_l     = A p_{l-1}
// together with the sums p.q, r.r/d, r.q/d, q.q/d, r.r, r.q, q.q. After the
// barrier: alpha_l = (r.r/d) / (p.q) (the listing's r.z), and because
// r_l = r_{l-1} - alpha_l q_l the next r.z and ||r_l||^2 follow exactly from
// the expansion (r.r/d) - 2 alpha (r.q/d) + alpha^2 (q.q/d), and likewise for
// ||r||^2; beta_l is their ratio. The iterates are those of the listing; only
// the order of the floating-point reductions differs.
//
// Data layout and tiling: arrays use the padded layout of pb_internal.hpp.
// A tile is a contiguous range of padded plane positions (a segment of
// several x-rows) times a run of z-planes. The pass marches up a tile's
// planes: p_{l-1} of the current plane sits in LDS over the segment plus one
// row of halo on each side (in-plane neighbours +-1, +-nx); the planes above
// and below stay in registers. Halo values of p are recomputed pointwise, so
// every array is written once per pass.
//
// Two pass forms compute the same iterates. pass_tile stores q_l for the
// next pass: it reads r, q, d, p_old, cx, cy, cz, x and writes r, p, q, x (48
// bytes per node in FP32). pass_tile40 recomputes q_{l-1} = A p_{l-2} from the
// stored p_{l-2} (in LDS over the segment plus two halo widths), so it reads
// r, p_old, d, cx, cy, cz, x and writes r, p, x: 40 bytes per node, the
// least any schedule of this iteration moves while the operator is four
// arrays (three vectors read and written plus four operator arrays read
// once). Its coded form reads the operator as one word of dictionary codes
// per node instead (28 bytes per node; coded.hip builds the words).
//
// Reductions and the grid barrier: each tile reduces its sums in a fixed
// order into its own slot; workgroups arrive on counters spread over eight
// cache lines, and after the barrier every workgroup sums all tile slots in
// the same fixed order and derives alpha, beta and the stopping test itself.
// Results do not depend on the number of workgroups or on scheduling.
#include "solver.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

namespace pb {

namespace {

constexpr int NPART = 7;   // pq, rrd, rqd, qqd, rr, rq, qq

template <typename T>
struct KArgs {
    Op<T> op;
    const T* b;
    T* x;
    T* r[2];
    T* q[2];
    T* p[2];
    int nx, ny, nz;
    int64_t sp;
    // Owned positions of a plane: [org, org + own). The plain layout owns the
    // whole padded plane (org 0, own sp); the ghost-row layout of the
    // periodic 40-byte pass owns the nx*ny nodes after its two low ghost rows
    // (own rounded up to the vector width; the nodes end at oend).
    int64_t org, own, oend;
    int seglen, zchunk, nseg, nzc, ntiles, halo;
    double tol;
    int maxiter;
    int warm;
    int resume;          // 1: continue from the state and scalars left by an earlier launch
    int chunk;           // > 0: stop after this many iterations in this launch (state stays resumable)
    SyncState* S;
    double* partials;
    long long timeout_ticks;
    const float* cw;     // coded 40-byte pass: one word of coefficient codes per position (bit patterns)
    const float* ctab;   // and the dictionary (kCodedTableSize values)
    const int* fit;      // runtime-checked coded launches: 1 when this problem's dictionary holds its operator
};

__device__ __forceinline__ double ld_agent_d(const double* p) {
    unsigned long long v = __hip_atomic_load((const unsigned long long*)p, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double((long long)v);
}
__device__ __forceinline__ int ld_agent_i(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroup barrier for the LDS hand-off between planes.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Cross-lane moves of a double through DPP (two 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)u, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double readlane_d(double v, int lane) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)u, lane);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kDppXor1 = 0xB1;         // quad permute [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad permute [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane i of 8 reads lane 7-i
constexpr int kDppMirror = 0x140;      // lane i of 16 reads lane 15-i
constexpr int kDppRor8 = 0x128;        // lane i of 16 reads lane (i+8) mod 16

// Sum over the 64 lanes of a wave (every lane active) in a fixed order: a
// butterfly inside each 16-lane row, then (row0 + row1) + (row2 + row3).
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<kDppXor1>(v);
    v += dpp_d<kDppXor2>(v);
    v += dpp_d<kDppHalfMirror>(v);
    v += dpp_d<kDppMirror>(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// LDS scratch of the reductions below, in doubles.
template <int BS>
constexpr int red_len() { return (BS / 64) * 4 * kMaxPartials + kMaxPartials; }

// Reduce acc[0..NP) over the workgroup in a fixed order and store the sums
// into dst. The stores are made by the first NP lanes of wave 0, the wave
// that later publishes them (its release covers its own stores).
template <int BS, int NP>
__device__ __forceinline__ void tile_reduce_store(double (&acc)[NP], double* red, double* dst) {
    constexpr int NW = BS / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const double v = wave_sum(acc[i]);
        if (lane == 0) red[wave * kMaxPartials + i] = v;
    }
    __syncthreads();
    if (threadIdx.x < NP) {
        double v = red[threadIdx.x];
        for (int q = 1; q < NW; ++q) v += red[q * kMaxPartials + threadIdx.x];
        dst[threadIdx.x] = v;
    }
    __syncthreads();
}

// Barrier over the G workgroups that share a problem (the whole grid for a
// single solve, one problem's workgroups in a batch), fused with the
// reduction of the tile sums. Workgroup w adds one release-ordered arrival to
// counter w % 8 (eight cache lines, so arrivals do not serialise on one
// address); for barrier b of this launch it waits (eight lanes polling the
// eight counters together) until every counter holds
// (b+1) times its share of the G workgroups, acquires, and then EVERY
// workgroup reduces all tile sums of slot b & 1 itself in the same fixed
// order (a coalesced sweep over the tiles, then a fixed lane and wave order), so
// all workgroups obtain bitwise identical sums with no second publication
// step. Tile sums are double-buffered by barrier parity: a workgroup can only
// overwrite slot b & 1 after barrier b+1, which every reader of barrier b has
// reached. Waits are bounded by timeout_ticks; returns false on timeout.
// The summation order depends on the block size only, not on G or on which
// workgroup ran which tile.
template <int BS, int NP>
__device__ bool grid_sync_reduce(SyncState* S, int w, int G, int b, const double* __restrict__ tile_sums,
                                 int ntiles, long long timeout_ticks, double* red, int* s_flag,
                                 double (&out)[NP]) {
    constexpr int NW = BS / 64;
    __syncthreads();
    if (threadIdx.x < 64) {
        // wave 0: lane 0 arrives, lanes 0..7 each watch one counter, so one
        // poll costs a single memory round trip
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&S->arrive[w & 7][0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const int c = threadIdx.x & 7;
        const unsigned need = (unsigned)(b + 1) * (unsigned)(G / 8 + (c < G % 8 ? 1 : 0));
        int ok = 1;
        const long long t0 = wall_clock64();
        while (true) {
            const unsigned v = threadIdx.x < 8
                                   ? __hip_atomic_load(&S->arrive[c][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                   : need;
            if (__all(v >= need)) break;
            __builtin_amdgcn_s_sleep(1);
            if (wall_clock64() - t0 > timeout_ticks) {
                ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (threadIdx.x == 0) {
            if (!ok) __hip_atomic_store(&S->status, (int)PB_ERR_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            *s_flag = ok;
        }
    }
    __syncthreads();
    if (!*s_flag) return false;
    // coalesced sweep: thread (j, i) adds slot i of tiles j, j + BS/8, ...
    // Plain loads: after the acquire above they observe every released tile
    // sum, and the workgroups of one XCD then share the lines in its L2.
    constexpr int NJ = BS / 8;
    const int i = threadIdx.x & 7, j = threadIdx.x >> 3;
    constexpr int U = 8;   // loads in flight per thread
    double acc = 0.0;
    if (i < NP) {
        for (int t0 = j; t0 < ntiles; t0 += U * NJ) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u * NJ;
                v[u] = t < ntiles ? tile_sums[(size_t)t * kMaxPartials + i] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc += v[u];
        }
    }
    acc += dpp_d<kDppRor8>(acc);   // lanes i and i+8 of each row hold the same slot
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if ((lane & 15) < 8) red[(wave * 4 + (lane >> 4)) * kMaxPartials + i] = acc;
    __syncthreads();
    double* fin = red + NW * 4 * kMaxPartials;
    if (threadIdx.x < NP) {
        double v = red[threadIdx.x];
        for (int q = 1; q < NW * 4; ++q) v += red[q * kMaxPartials + threadIdx.x];
        fin[threadIdx.x] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NP; ++k) out[k] = fin[k];
    __syncthreads();
    return true;
}

template <typename T>
__device__ __forceinline__ typename Vec<T>::type vload(const T* p) {
    return *reinterpret_cast<const typename Vec<T>::type*>(p);
}
template <typename T>
__device__ __forceinline__ void vstore(T* p, const typename Vec<T>::type& v) {
    *reinterpret_cast<typename Vec<T>::type*>(p) = v;
}
// Streaming forms of vload/vstore with the nontemporal hint. The passes use
// them (kernel variants with NT = true) for the own-position streams that
// nothing reads again within the step: r, p_old, d, cz, x (and q in the
// 48-byte pass) loads; r, p, x (and q) stores. Once the arrays of a pass are
// larger than the last-level cache this is faster on gfx950, even though
// neighbouring tiles re-read the outer rows of these streams as their halo;
// below that size the cached forms win, since the arrays then stay in the
// cache from one iteration to the next. cx and cy are always cached: the x-1
// and y-1 couplings re-read them within the step.
typedef float f4_nt __attribute__((ext_vector_type(4)));
typedef double d2_nt __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float4 vload_nt(const float* p) {
    const f4_nt t = __builtin_nontemporal_load(reinterpret_cast<const f4_nt*>(p));
    return make_float4(t.x, t.y, t.z, t.w);
}
__device__ __forceinline__ double2 vload_nt(const double* p) {
    const d2_nt t = __builtin_nontemporal_load(reinterpret_cast<const d2_nt*>(p));
    return make_double2(t.x, t.y);
}
__device__ __forceinline__ void vstore_nt(float* p, const float4& v) {
    const f4_nt t = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(t, reinterpret_cast<f4_nt*>(p));
}
__device__ __forceinline__ void vstore_nt(double* p, const double2& v) {
    const d2_nt t = {v.x, v.y};
    __builtin_nontemporal_store(t, reinterpret_cast<d2_nt*>(p));
}
template <bool NT, typename T>
__device__ __forceinline__ typename Vec<T>::type sload(const T* p) {
    if constexpr (NT) return vload_nt(p);
    else return vload(p);
}
template <bool NT, typename T>
__device__ __forceinline__ void sstore(T* p, const typename Vec<T>::type& v) {
    if constexpr (NT) vstore_nt(p, v);
    else vstore(p, v);
}
// Jacobi scaling 1/d: the hardware reciprocal in FP32 (about 1 ulp), an
// exact division in FP64. Every use of M^-1 in a solve goes through this one
// function, so the preconditioner is the same fixed positive diagonal in the
// direction update and in the dot products.
__device__ __forceinline__ float jacobi_inv(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ uint32_t bits(float f) { return __float_as_uint(f); }
__device__ __forceinline__ double jacobi_inv(double d) { return 1.0 / d; }

template <typename T>
__device__ __forceinline__ typename Vec<T>::type vzero() {
    typename Vec<T>::type v;
#pragma unroll
    for (int u = 0; u < Vec<T>::n; ++u) vget(v, u) = T(0);
    return v;
}

// Tiles of workgroup `w` out of `G` sharing a problem. With `xcd` set and G a
// multiple of 8, workgroup w runs on XCD w % 8 and each XCD takes a
// contiguous block of the tile order (z-chunk major), so tiles that share
// halos also share that XCD's L2; otherwise tiles are dealt round-robin.
__device__ __forceinline__ void xcd_tile_range(int ntiles, int w, int G, bool xcd_map, int& first, int& stride,
                                               int& end) {
    const int nx8 = (xcd_map && G >= 8 && G % 8 == 0) ? 8 : 1;
    const int xcd = w % nx8, local = w / nx8, per = G / nx8;
    first = (int)(((long long)xcd * ntiles) / nx8) + local;
    stride = per;
    end = (int)(((long long)(xcd + 1) * ntiles) / nx8);
}

struct TileBox {
    int64_t s, e;   // plane positions [s, e)
    int k0, k1;     // planes [k0, k1)
};

template <typename T>
__device__ __forceinline__ TileBox tile_box(const KArgs<T>& a, int tile) {
    TileBox t;
    const int seg = tile % a.nseg, zc = tile / a.nseg;
    t.s = a.org + (int64_t)seg * a.seglen;
    t.e = min(t.s + (int64_t)a.seglen, a.org + a.own);
    t.k0 = zc * a.zchunk;
    t.k1 = min(t.k0 + a.zchunk, a.nz);
    return t;
}

// ------------------------------------------------------------------ passes

// Initial state: r = b - A x0 (r = b for a zero guess), p = 0 and (for the
// pass that reads a stored A.p) q = 0 in buffer 0; sums r.r and b.b.
//
// GL: the ghost-row layout of the periodic 40-byte pass. Every owned node is
// computed with its wrapped neighbours, the elements of the last group past
// the last node (ghost positions) get the values of the nodes nx*ny before
// them, and the ghost copies of rows 0, 1, ny-2, ny-1 are written too.
template <typename T, int BS, bool PER, bool GL = false>
__device__ void init_tile(const KArgs<T>& a, int tile, bool with_q, double (&acc)[2]) {
    constexpr int W = Vec<T>::n;
    using V = typename Vec<T>::type;
    const TileBox tb = tile_box(a, tile);
    const int64_t npad = a.sp * a.nz;
    const V z0 = vzero<T>();
    if constexpr (GL) {
        const int64_t nodes = a.oend - a.org, sp = a.sp;
        const int nx = a.nx, ny = a.ny, nz = a.nz;
        const T* X = a.x;
        for (int k = tb.k0; k < tb.k1; ++k) {
            for (int64_t pos = tb.s + (int64_t)threadIdx.x * W; pos < tb.e; pos += (int64_t)BS * W) {
#pragma unroll
                for (int u = 0; u < W; ++u) {
                    const int64_t q = pos + u;
                    const bool node = q < a.oend;
                    const int64_t rel = node ? q - a.org : q - a.org - nodes;
                    const int64_t t = (int64_t)k * sp + a.org + rel;   // the node whose values q holds
                    const T bv = a.b[t];
                    T rv = bv;
                    if (a.warm) {
                        const int64_t j = rel / nx, i = rel - j * nx;
                        const int64_t xr = (i == nx - 1) ? t - (nx - 1) : t + 1;
                        const int64_t xl = (i == 0) ? t + (nx - 1) : t - 1;
                        const int64_t yu = (j == ny - 1) ? t - (int64_t)(ny - 1) * nx : t + nx;
                        const int64_t yd = (j == 0) ? t + (int64_t)(ny - 1) * nx : t - nx;
                        const int64_t zu = (k == nz - 1) ? t - (int64_t)(nz - 1) * sp : t + sp;
                        const int64_t zd = (k == 0) ? t + (int64_t)(nz - 1) * sp : t - sp;
                        T nb = a.op.cx[t] * X[xr];
                        nb += a.op.cx[xl] * X[xl];
                        nb += a.op.cy[t] * X[yu];
                        nb += a.op.cy[yd] * X[yd];
                        nb += a.op.cz[t] * X[zu];
                        nb += a.op.cz[zd] * X[zd];
                        rv = bv - (a.op.d[t] * X[t] - nb);
                    }
                    const int64_t g = (int64_t)k * sp + q;
                    a.r[0][g] = rv;
                    a.p[0][g] = T(0);
                    if (node) {
                        acc[0] += (double)rv * (double)rv;
                        acc[1] += (double)bv * (double)bv;
                        const int64_t span = (int64_t)nx * ny;
                        const int64_t jq = rel / nx;
                        const int64_t gq = jq < 2 ? q + span : (jq >= ny - 2 ? q - span : -1);
                        if (gq >= 0) {
                            a.r[0][(int64_t)k * sp + gq] = rv;
                            a.p[0][(int64_t)k * sp + gq] = T(0);
                        }
                    }
                }
            }
        }
        return;
    }
    for (int k = tb.k0; k < tb.k1; ++k) {
        for (int64_t pos = tb.s + (int64_t)threadIdx.x * W; pos < tb.e; pos += (int64_t)BS * W) {
            const int64_t g = (int64_t)k * a.sp + pos;
            const V bv = vload(a.b + g);
            V rv = bv;
            if (a.warm) {
                const V dv = vload(a.op.d + g);
#pragma unroll
                for (int u = 0; u < W; ++u) {
                    const int64_t t = g + u;
                    const T* X = a.x;
                    T nb;
                    if constexpr (PER) {
                        const int64_t q = pos + u;
                        if (q >= (int64_t)a.nx * a.ny) {
                            nb = T(0);
                        } else {
                            const int64_t j = q / a.nx, i = q - j * a.nx;
                            const int64_t ys = (int64_t)(a.ny - 1) * a.nx, zs = (int64_t)(a.nz - 1) * a.sp;
                            const int64_t xr = (i == a.nx - 1) ? t - (a.nx - 1) : t + 1;
                            const int64_t xl = (i == 0) ? t + (a.nx - 1) : t - 1;
                            const int64_t yu = (j == a.ny - 1) ? t - ys : t + a.nx;
                            const int64_t yd = (j == 0) ? t + ys : t - a.nx;
                            const int64_t zu = (k == a.nz - 1) ? t - zs : t + a.sp;
                            const int64_t zd = (k == 0) ? t + zs : t - a.sp;
                            nb = a.op.cx[t] * X[xr];
                            nb += a.op.cx[xl] * X[xl];
                            nb += a.op.cy[t] * X[yu];
                            nb += a.op.cy[yd] * X[yd];
                            nb += a.op.cz[t] * X[zu];
                            nb += a.op.cz[zd] * X[zd];
                        }
                    } else {
                        nb = a.op.cx[t] * (t + 1 < npad ? X[t + 1] : T(0));
                        nb += (t >= 1 ? a.op.cx[t - 1] * X[t - 1] : T(0));
                        nb += a.op.cy[t] * (t + a.nx < npad ? X[t + a.nx] : T(0));
                        nb += (t >= a.nx ? a.op.cy[t - a.nx] * X[t - a.nx] : T(0));
                        nb += a.op.cz[t] * (t + a.sp < npad ? X[t + a.sp] : T(0));
                        nb += (t >= a.sp ? a.op.cz[t - a.sp] * X[t - a.sp] : T(0));
                    }
                    vget(rv, u) = vget(bv, u) - (vget(dv, u) * X[t] - nb);
                }
            }
#pragma unroll
            for (int u = 0; u < W; ++u) {
                acc[0] += (double)vget(rv, u) * (double)vget(rv, u);
                acc[1] += (double)vget(bv, u) * (double)vget(bv, u);
            }
            vstore(a.r[0] + g, rv);
            if (with_q) vstore(a.q[0] + g, z0);
            vstore(a.p[0] + g, z0);
        }
    }
}

// One pass on one tile (see the file comment). `o`/`n` index the old and new
// buffers; alpha, beta are alpha_{l-1}, beta_{l-1}. PER: periodic boundary
// (one vector group per thread): neighbours across the x ends come from the
// LDS row, across the y ends from p recomputed pointwise at the partner node
// of the far row (one plane ahead, with the other loads), across the z ends
// from the wrapped plane of the march.
template <typename T, int BS, int MC, bool PER, bool NT>
__device__ void pass_tile(const KArgs<T>& a, int tile, int o, int n, T alpha, T beta, T* lds0, T* lds1,
                          double (&acc)[NPART]) {
    static_assert(!PER || MC == 1, "the periodic pass takes one vector group per thread");
    constexpr int W = Vec<T>::n;
    using V = typename Vec<T>::type;
    const TileBox tb = tile_box(a, tile);
    const int64_t s = tb.s, e = tb.e, sp = a.sp;
    const int k0 = tb.k0, k1 = tb.k1;
    const int H = a.halo, nx = a.nx;
    const int64_t lbase = s - H;
    const int hgroups = 2 * H / W;
    // ping-pong buffers chosen by select (no runtime array indexing, which
    // would put a private copy of the arguments in scratch memory)
    const T* __restrict__ rold = o ? a.r[1] : a.r[0];
    const T* __restrict__ qold = o ? a.q[1] : a.q[0];
    const T* __restrict__ pold = o ? a.p[1] : a.p[0];
    T* __restrict__ rnew = n ? a.r[1] : a.r[0];
    T* __restrict__ pnew = n ? a.p[1] : a.p[0];
    T* __restrict__ qnew = n ? a.q[1] : a.q[0];
    const bool do_x = alpha != T(0);
    const V z0 = vzero<T>();

    int64_t pos[MC];
    bool valid[MC];
#pragma unroll
    for (int c = 0; c < MC; ++c) {
        pos[c] = s + (int64_t)(c * BS + (int)threadIdx.x) * W;
        valid[c] = pos[c] < e;
    }
    // periodic: per element of this thread's group, bit u set when element u
    // is at i = 0 (wl), i = nx-1 (wr), j = 0 (wd) or j = ny-1 (wu), or is a
    // pad slot after the plane (wpad: the last real node's wrap couplings
    // would otherwise reach it through cx[n-1], cy[n-nx])
    unsigned wl = 0, wr = 0, wd = 0, wu = 0, wpad = 0;
    const int64_t yspan = (int64_t)(a.ny - 1) * nx;   // offset of the partner row
    if constexpr (PER) {
        const int64_t plane = (int64_t)nx * a.ny;
        if (valid[0]) {
#pragma unroll
            for (int u = 0; u < W; ++u) {
                const int64_t q = pos[0] + u;
                if (q >= plane) {
                    wpad |= 1u << u;
                    continue;
                }
                const int64_t j = q / nx, i = q - j * nx;
                if (i == 0) wl |= 1u << u;
                if (i == nx - 1) wr |= 1u << u;
                if (j == 0) wd |= 1u << u;
                if (j == a.ny - 1) wu |= 1u << u;
            }
        }
    }
    // p_{l-1} at one node from the old state (the arithmetic of p_at below)
    auto p_point = [&](int64_t g) -> T {
        const T r = rold[g] - alpha * qold[g];
        return r * jacobi_inv(a.op.d[g]) + beta * pold[g];
    };
    // p_{l-1} at a position from the old state (pointwise); also returns
    // r_{l-1}, p_{l-2} and d there.
    auto p_at = [&](int64_t g, V& rv, V& po, V& dv) -> V {
        rv = vload(rold + g);
        const V qv = vload(qold + g);
        dv = vload(a.op.d + g);
        po = vload(pold + g);
        V out;
#pragma unroll
        for (int u = 0; u < W; ++u) {
            const T r = vget(rv, u) - alpha * vget(qv, u);
            vget(rv, u) = r;
            vget(out, u) = r * jacobi_inv(vget(dv, u)) + beta * vget(po, u);
        }
        return out;
    };
    auto halo_fill = [&](int k, T* buf) {
        for (int hg = threadIdx.x; hg < hgroups; hg += BS) {
            const int64_t hp = (hg < H / W) ? (s - H + (int64_t)hg * W) : (e + (int64_t)(hg - H / W) * W);
            V v = z0;
            if (hp >= 0 && hp < sp) {
                V rv, po, dv;
                v = p_at((int64_t)k * sp + hp, rv, po, dv);
            }
            vstore(buf + (hp - lbase), v);
        }
    };
    // Own positions of plane k: the new p (also into LDS when `buf` is
    // given); for an owned plane also r_{l-1} and the x update are written.
    V pc[MC], pm[MC], pn[MC], czm[MC], rc[MC], dc[MC];
    auto own_plane = [&](int k, T* buf, bool owned, V (&pv)[MC], V (&rv)[MC], V (&dv)[MC]) {
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            pv[c] = z0;
            rv[c] = z0;
            dv[c] = z0;
            if (!valid[c]) continue;
            const int64_t g = (int64_t)k * sp + pos[c];
            V po;
            pv[c] = p_at(g, rv[c], po, dv[c]);
            if (buf) vstore(buf + (pos[c] - lbase), pv[c]);
            if (owned) {
                vstore(rnew + g, rv[c]);
                if (do_x) {
                    V xv = vload(a.x + g);
#pragma unroll
                    for (int u = 0; u < W; ++u) vget(xv, u) = vget(xv, u) + alpha * vget(po, u);
                    vstore(a.x + g, xv);
                }
            }
        }
    };

    // y-wrap partners of plane k (periodic): p_{l-1} at the far row
    T pw[W];
#pragma unroll
    for (int u = 0; u < W; ++u) pw[u] = T(0);
    auto partners = [&](int k, T (&out)[W]) {
#pragma unroll
        for (int u = 0; u < W; ++u) {
            out[u] = T(0);
            if ((wd >> u) & 1u) out[u] = p_point((int64_t)k * sp + pos[0] + u + yspan);
            if ((wu >> u) & 1u) out[u] = p_point((int64_t)k * sp + pos[0] + u - yspan);
        }
    };

    // prologue: plane k0-1 (own positions, z-neighbour only) and plane k0
    {
        V rdummy[MC], ddummy[MC];
        if (k0 > 0 || PER) {
            const int km = k0 > 0 ? k0 - 1 : a.nz - 1;   // periodic: the top plane wraps below plane 0
            own_plane(km, nullptr, false, pm, rdummy, ddummy);
#pragma unroll
            for (int c = 0; c < MC; ++c) czm[c] = valid[c] ? vload(a.op.cz + (int64_t)km * sp + pos[c]) : z0;
        } else {
#pragma unroll
            for (int c = 0; c < MC; ++c) {
                pm[c] = z0;
                czm[c] = z0;
            }
        }
        T* buf = (k0 & 1) ? lds1 : lds0;
        own_plane(k0, buf, true, pc, rc, dc);
        halo_fill(k0, buf);
        if constexpr (PER) partners(k0, pw);
    }
    lds_barrier();

    // Each plane step first issues every global load it needs (the next
    // plane's r, q, d, p_old and x, this thread's halo group of the next
    // plane, and the current plane's couplings), then computes: one memory
    // round trip per step. The tiling guarantees at most one halo group per
    // thread (2*halo/VEC <= block size).
    const int hg = threadIdx.x;
    const int64_t hp = (hg < H / W) ? (s - H + (int64_t)hg * W) : (e + (int64_t)(hg - H / W) * W);
    const bool h_in_range = hg < hgroups && hp >= 0 && hp < sp;
    // The global loads of step k depend on k only (the next plane's r, q, d,
    // p_old and x, this thread's halo group of it, the current plane's
    // couplings); they are issued one step ahead, before the previous step's
    // LDS barrier, so their latency overlaps it.
    struct Ld {
        V in_r[MC], in_q[MC], in_d[MC], in_po[MC], in_x[MC];
        V cxv[MC], cyv[MC], czv[MC];
        T cxm[MC], cym[MC][W];
        T cxw[W], cyw[W];   // periodic: wrap couplings of plane k
        // periodic: r, q, d, p_old at the y-wrap partners of the next plane
        T pr_r[W], pr_q[W], pr_d[W], pr_po[W];
        V h_r, h_q, h_d, h_po;
    };
    auto issue = [&](int k, Ld& L) {
        const bool has_next = PER || k + 1 < a.nz;
        const int kn = (PER && k + 1 == a.nz) ? 0 : k + 1;
        const bool owned = k + 1 < k1;
        const bool x_upd = owned && do_x;
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            L.in_r[c] = L.in_q[c] = L.in_po[c] = L.in_x[c] = z0;
            L.in_d[c] = z0;
            L.cxv[c] = L.cyv[c] = L.czv[c] = z0;
            L.cxm[c] = T(0);
#pragma unroll
            for (int u = 0; u < W; ++u) L.cym[c][u] = T(0);
            if (!valid[c]) continue;
            if (has_next) {
                const int64_t g1 = (int64_t)kn * sp + pos[c];
                L.in_r[c] = sload<NT>(rold + g1);
                L.in_q[c] = sload<NT>(qold + g1);
                L.in_d[c] = sload<NT>(a.op.d + g1);
                L.in_po[c] = sload<NT>(pold + g1);
                if (x_upd) L.in_x[c] = sload<NT>(a.x + g1);
            }
            const int64_t g = (int64_t)k * sp + pos[c];
            L.cxv[c] = vload(a.op.cx + g);
            L.cyv[c] = vload(a.op.cy + g);
            L.czv[c] = sload<NT>(a.op.cz + g);
            L.cxm[c] = pos[c] >= 1 ? a.op.cx[g - 1] : T(0);
#pragma unroll
            for (int u = 0; u < W; ++u) L.cym[c][u] = (pos[c] + u - nx >= 0) ? a.op.cy[g + u - nx] : T(0);
        }
#pragma unroll
        for (int u = 0; u < W; ++u) L.cxw[u] = L.cyw[u] = T(0);
#pragma unroll
        for (int u = 0; u < W; ++u) L.pr_r[u] = L.pr_q[u] = L.pr_d[u] = L.pr_po[u] = T(0);
        if constexpr (PER) {
            const int64_t g = (int64_t)k * sp + pos[0];
            const int64_t gn = (int64_t)kn * sp + pos[0];
#pragma unroll
            for (int u = 0; u < W; ++u) {
                L.cxw[u] = ((wl >> u) & 1u) ? a.op.cx[g + u + nx - 1] : T(0);
                L.cyw[u] = ((wd >> u) & 1u) ? a.op.cy[g + u + yspan] : T(0);
                if (((wd | wu) >> u) & 1u) {
                    const int64_t gq = gn + u + (((wu >> u) & 1u) ? -yspan : yspan);
                    L.pr_r[u] = rold[gq];
                    L.pr_q[u] = qold[gq];
                    L.pr_d[u] = a.op.d[gq];
                    L.pr_po[u] = pold[gq];
                }
            }
        }
        L.h_r = L.h_q = L.h_d = L.h_po = z0;
        if (has_next && owned && h_in_range) {
            const int64_t gh = (int64_t)(k + 1) * sp + hp;
            L.h_r = vload(rold + gh);
            L.h_q = vload(qold + gh);
            L.h_d = vload(a.op.d + gh);
            L.h_po = vload(pold + gh);
        }
    };
    Ld ldc;
    issue(k0, ldc);
    for (int k = k0; k < k1; ++k) {
        const T* cur = (k & 1) ? lds1 : lds0;
        T* nxt = (k & 1) ? lds0 : lds1;
        const bool has_next = PER || k + 1 < a.nz;
        const int kn = (PER && k + 1 == a.nz) ? 0 : k + 1;   // the next plane (wrapped when periodic)
        const bool owned = k + 1 < k1;
        const bool x_upd = owned && do_x;
        V (&in_r)[MC] = ldc.in_r; V (&in_q)[MC] = ldc.in_q; V (&in_d)[MC] = ldc.in_d;
        V (&in_po)[MC] = ldc.in_po; V (&in_x)[MC] = ldc.in_x;
        const V (&cxv)[MC] = ldc.cxv; const V (&cyv)[MC] = ldc.cyv; const V (&czv)[MC] = ldc.czv;
        const T (&cxm)[MC] = ldc.cxm; const T (&cym)[MC][W] = ldc.cym;
        const T (&cxw)[W] = ldc.cxw; const T (&cyw)[W] = ldc.cyw;
        const V& h_r = ldc.h_r; const V& h_q = ldc.h_q; const V& h_d = ldc.h_d; const V& h_po = ldc.h_po;
        T pwn[W];   // periodic: p_{l-1} at the y-wrap partners of the next plane (p_point's arithmetic)
        if constexpr (PER) {
#pragma unroll
            for (int u = 0; u < W; ++u) {
                pwn[u] = T(0);
                if (((wd | wu) >> u) & 1u) {
                    const T r = ldc.pr_r[u] - alpha * ldc.pr_q[u];
                    pwn[u] = r * jacobi_inv(ldc.pr_d[u]) + beta * ldc.pr_po[u];
                }
            }
        }
        // ---- next plane: new p (own and halo), r_{l-1}, x update
        V rn[MC], dn[MC];
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            pn[c] = z0;
            rn[c] = z0;
            dn[c] = in_d[c];
            if (!valid[c] || !has_next) continue;
            const int64_t g1 = (int64_t)kn * sp + pos[c];
#pragma unroll
            for (int u = 0; u < W; ++u) {
                const T r = vget(in_r[c], u) - alpha * vget(in_q[c], u);
                vget(rn[c], u) = r;
                vget(pn[c], u) = r * jacobi_inv(vget(in_d[c], u)) + beta * vget(in_po[c], u);
            }
            if (owned) {
                vstore(nxt + (pos[c] - lbase), pn[c]);
                sstore<NT>(rnew + g1, rn[c]);
                if (x_upd) {
#pragma unroll
                    for (int u = 0; u < W; ++u) vget(in_x[c], u) = vget(in_x[c], u) + alpha * vget(in_po[c], u);
                    sstore<NT>(a.x + g1, in_x[c]);
                }
            }
        }
        if (has_next && owned && hg < hgroups) {
            V hv = z0;
            if (h_in_range) {
#pragma unroll
                for (int u = 0; u < W; ++u) {
                    const T r = vget(h_r, u) - alpha * vget(h_q, u);
                    vget(hv, u) = r * jacobi_inv(vget(h_d, u)) + beta * vget(h_po, u);
                }
            }
            vstore(nxt + (hp - lbase), hv);
        }
        // ---- current plane: q = A p and the partial sums
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            if (!valid[c]) continue;
            const int64_t g = (int64_t)k * sp + pos[c];
            const int64_t l = pos[c] - lbase;
            const T left = cur[l - 1];
            const T right = cur[l + W];
            V qv;
#pragma unroll
            for (int u = 0; u < W; ++u) {
                const T p = vget(pc[c], u);
                T pl = (u == 0) ? left : vget(pc[c], u - 1);
                T pr = (u == W - 1) ? right : vget(pc[c], u + 1);
                T cl = (u == 0) ? cxm[c] : vget(cxv[c], u - 1);
                T vup = cur[l + u + nx], vdn = cur[l + u - nx], cdn = cym[c][u];
                if constexpr (PER) {
                    if ((wr >> u) & 1u) pr = cur[l + u - (nx - 1)];
                    if ((wl >> u) & 1u) {
                        pl = cur[l + u + (nx - 1)];
                        cl = cxw[u];
                    }
                    if ((wu >> u) & 1u) vup = pw[u];
                    if ((wd >> u) & 1u) {
                        vdn = pw[u];
                        cdn = cyw[u];
                    }
                }
                T nb = vget(cxv[c], u) * pr + cl * pl;
                nb += vget(cyv[c], u) * vup + cdn * vdn;
                nb += vget(czv[c], u) * vget(pn[c], u) + vget(czm[c], u) * vget(pm[c], u);
                T qq = vget(dc[c], u) * p - nb;
                if constexpr (PER) {
                    if ((wpad >> u) & 1u) qq = T(0);
                }
                vget(qv, u) = qq;
                const T iv = jacobi_inv(vget(dc[c], u));
                const double pd = (double)p, qd = (double)qq, rd = (double)vget(rc[c], u);
                const double zd = (double)(vget(rc[c], u) * iv), wd = (double)(qq * iv);
                acc[0] += pd * qd;
                acc[1] += rd * zd;
                acc[2] += rd * wd;
                acc[3] += qd * wd;
                acc[4] += rd * rd;
                acc[5] += rd * qd;
                acc[6] += qd * qd;
            }
            sstore<NT>(pnew + g, pc[c]);
            sstore<NT>(qnew + g, qv);
            czm[c] = czv[c];
        }
#pragma unroll
        for (int c = 0; c < MC; ++c) {
            pm[c] = pc[c];
            pc[c] = pn[c];
            rc[c] = rn[c];
            dc[c] = dn[c];
        }
        if constexpr (PER) {
#pragma unroll
            for (int u = 0; u < W; ++u) pw[u] = pwn[u];
        }
        if (k + 1 < k1) {
            Ld ldn;
            issue(k + 1, ldn);
            lds_barrier();
            ldc = ldn;
        } else {
            lds_barrier();
        }
    }
}

// Final update x += alpha p (or x = 0 for a zero right-hand side).
// (A v) at one node: d v minus the six couplings times the neighbour values,
// summed in one fixed order (x, then y, then z). Every evaluation of the
// operator in the 40-byte pass goes through this function, so a node's value
// recomputed in a tile's halo is the one its own tile computes.
// (A v)_n at one node. The rounding is fixed by explicit fused multiply-adds
// (no compiler contraction), so every kernel variant computes the same value.
template <typename T>
__device__ __forceinline__ T apply_point(T d, T v, T cr, T vr, T cl, T vl, T cu, T vu, T cd, T vd, T ca, T va, T cb,
                                         T vb) {
#pragma clang fp contract(off)
    T nb = cr * vr;
    nb = fma(cl, vl, nb);
    nb = fma(cu, vu, nb);
    nb = fma(cd, vd, nb);
    nb = fma(ca, va, nb);
    nb = fma(cb, vb, nb);
    return fma(d, v, -nb);
}

// ---- periodic boundary in the ghost-row layout (40-byte pass)
//
// Each plane holds two ghost rows below row 0 (copies of rows ny-2, ny-1) and
// two above row ny-1 (copies of rows 0, 1), so that every y-neighbour of a
// node, wrapped or not, sits one row away as in the free-boundary layout.
// The owner of a node of rows 0, 1, ny-2, ny-1 stores its r and p also into
// the ghost copy, and a ghost node recomputed in a tile's halo sees the same
// inputs as its original and gets the same value. Planes wrap in z; across
// the x ends a group takes the neighbour from the other end of the row (one
// row is shorter than the in-plane halo, so it is in LDS).
template <bool PER>
__device__ __forceinline__ int wrap_plane(int k, int nz) {
    if constexpr (!PER) return k;
    return k < 0 ? k + nz : (k >= nz ? k - nz : k);
}
struct XWrap {
    int wl, wr;   // element of the group in column 0 / column nx-1, -1 if none
};
// Row and column of plane position q relative to row 0 (32-bit: planes of
// the ghost-row layout hold fewer than 2^31 positions, checked on the host).
struct RowCol {
    int j, i;
};
template <typename T>
__device__ __forceinline__ RowCol row_col(const KArgs<T>& a, int64_t q) {
    const int rel = (int)(q - a.org) + 4 * a.nx;   // >= 0 for every position a pass touches
    const int j = rel / a.nx;
    return RowCol{j - 4, rel - j * a.nx};
}
// Only positions of the node and ghost rows (rows -2 .. ny+1) count.
template <int W, typename T>
__device__ __forceinline__ XWrap x_wrap(const KArgs<T>& a, int64_t q0) {
    XWrap w{-1, -1};
    const RowCol rc = row_col(a, q0);
#pragma unroll
    for (int u = 0; u < W; ++u) {
        const bool next = rc.i + u >= a.nx;   // nx > W: the group crosses at most one row end
        const int i = next ? rc.i + u - a.nx : rc.i + u;
        const int j = next ? rc.j + 1 : rc.j;
        const bool in = j >= -2 && j < a.ny + 2;
        if (in && i == 0) w.wl = u;
        if (in && i == a.nx - 1) w.wr = u;
    }
    return w;
}
// The row end inside a group as one number: the element in column 0, W when
// the last element is in column nx-1 and the next row starts after the
// group, -1 when the group holds no row end. Element u takes its left
// neighbour across the row end when u == brk, its right one when u + 1 == brk.
template <int W, typename T>
__device__ __forceinline__ int x_break(const KArgs<T>& a, int64_t q0) {
    const XWrap w = x_wrap<W>(a, q0);
    return w.wl >= 0 ? w.wl : (w.wr == W - 1 ? W : -1);
}
// The value, unknown to the optimizer: compares against it are made where
// they are used (in the plane loop) instead of being hoisted and kept as
// scalar lane masks.
__device__ __forceinline__ int opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}
// Plane positions of the ghost copies of the owned nodes q0 .. q0+W-1 (the
// first nv of them): -1 for nodes of rows 2 .. ny-3.
template <int W, typename T>
__device__ __forceinline__ void ghost_of(const KArgs<T>& a, int64_t q0, int nv, int64_t (&gd)[W]) {
    const RowCol rc = row_col(a, q0);
    const int64_t span = (int64_t)a.nx * a.ny;
#pragma unroll
    for (int u = 0; u < W; ++u) {
        const int j = rc.j + (rc.i + u >= a.nx ? 1 : 0);
        gd[u] = -1;
        if (u < nv && j < 2) gd[u] = q0 + u + span;
        if (u < nv && j >= a.ny - 2) gd[u] = q0 + u - span;
    }
}

// One pass on one tile, 40-byte form: the same iteration as pass_tile, but
// q_{l-1} = A p_{l-2} is recomputed from the stored p_{l-2} instead of being
// stored by the previous pass. Per node the pass reads r, p_old, d, cx, cy,
// cz, x and writes r, p, x: 40 bytes in FP32 against 48.
//
// The march keeps p_{l-2} on planes k, k+1, k+2 and p_{l-1} on planes k-1,
// k, k+1. Plane k+1 of p_{l-2} is in LDS over the segment widened by two
// halo widths (the in-plane neighbours of the inner halo ring); plane k of
// p_{l-1} is in LDS over the segment widened by one. Step k evaluates
// q_{l-1} and p_{l-1} on plane k+1 (own positions and the inner ring), then
// q_l = A p_{l-1} and the sums on plane k. Two warm-up steps below the tile
// build planes k0-1 and k0 of p_{l-1}. Threads: own positions s + tid*VEC,
// inner ring groups on the first 2*halo/VEC threads, outer ring groups on the
// last 2*halo/VEC threads (the tiling guarantees 2*halo/VEC <= BS).
template <typename T, int BS, bool NT, bool PER>
__device__ void pass_tile40(const KArgs<T>& a, int tile, int o, int n, T alpha, T beta, T* lds,
                            double (&acc)[NPART]) {
#pragma clang fp contract(off)
    constexpr int W = Vec<T>::n;
    using V = typename Vec<T>::type;
    const TileBox tb = tile_box(a, tile);
    const int64_t s = tb.s, e = tb.e, sp = a.sp;
    const int k0 = tb.k0, k1 = tb.k1, nz = a.nz;
    const int H = a.halo, nx = a.nx;
    const int lo_len = a.seglen + 4 * H, ln_len = a.seglen + 2 * H;
    T* const PO0 = lds;
    T* const PO1 = lds + lo_len;
    T* const PN0 = lds + 2 * lo_len;
    T* const PN1 = PN0 + ln_len;
    T* const CX0 = PN1 + ln_len;   // x/y couplings of a plane over the segment +- halo
    T* const CX1 = CX0 + ln_len;
    T* const CY0 = CX1 + ln_len;
    T* const CY1 = CY0 + ln_len;
    const int64_t obase = s - 2 * H, nbase = s - H;
    const T* __restrict__ rold = o ? a.r[1] : a.r[0];
    const T* __restrict__ pold = o ? a.p[1] : a.p[0];
    T* __restrict__ rnew = n ? a.r[1] : a.r[0];
    T* __restrict__ pnew = n ? a.p[1] : a.p[0];
    const T* __restrict__ CX = a.op.cx;
    const T* __restrict__ CY = a.op.cy;
    const T* __restrict__ CZ = a.op.cz;
    const T* __restrict__ DD = a.op.d;
    const bool do_x = alpha != T(0);
    const V z0 = vzero<T>();

    const int tid = threadIdx.x;
    const int64_t pos = s + (int64_t)tid * W;
    const bool valid = pos < e;
    const int ring = 2 * H / W;   // vector groups per ring (both sides)
    const bool is_h = tid < ring;
    const int64_t hp = (tid < H / W) ? (s - H + (int64_t)tid * W) : (e + (int64_t)(tid - H / W) * W);
    const bool h_in = is_h && hp >= 0 && hp < sp;
    const int og = tid - (BS - ring);
    const bool is_o = og >= 0;
    const int64_t op = (og < H / W) ? (s - 2 * H + (int64_t)og * W) : (e + H + (int64_t)(og - H / W) * W);
    const bool o_in = is_o && op >= 0 && op < sp;
    // periodic (ghost-row layout): planes wrap, the column-0 and column-nx-1
    // elements of a group take their x-neighbour from the other end of the
    // row, owned nodes of the first and last two rows are also stored into
    // their ghost copies, and only the owned elements of the last group
    // (nv of them) enter the sums
    const int nv = valid ? (int)min((int64_t)W, a.oend - pos) : 0;
    const int brk = PER && valid ? x_break<W>(a, pos) : -1;
    const int hbrk = PER && h_in ? x_break<W>(a, hp) : -1;
    // the elements whose neighbour across a row end is read (any element when
    // there is none: the value read is then unused)
    const int kl = min(max(brk, 0), W - 1), kr = min(max(brk - 1, 0), W - 1);
    const int hkl = min(max(hbrk, 0), W - 1), hkr = min(max(hbrk - 1, 0), W - 1);
    int64_t gd[W];
    if constexpr (PER) ghost_of<W>(a, pos, nv, gd);
    else
#pragma unroll
        for (int u = 0; u < W; ++u) gd[u] = -1;
    // a group copied whole to consecutive positions takes one 16-byte store
    bool g_vec = gd[0] >= 0;
#pragma unroll
    for (int u = 1; u < W; ++u) g_vec = g_vec && gd[u] == gd[0] + u;
    auto pl_of = [&](int k) { return (int64_t)wrap_plane<PER>(k, nz) * sp; };

    // State at the start of step k (k = k0-2 first): p_{l-2} of planes k and
    // k+1 lives in the two p_old LDS slots (plane k until the step's end),
    // p_{l-1} of plane k in its LDS slot, the couplings of plane k in the
    // coupling slots; in registers stay cz of plane k (own, ring), and p_{l-1},
    // r_{l-1}, d of the planes the z-stencil and the sums need.
    V cz_c, hcz_c;    // cz on plane k (own, ring)
    {
        V po_m, po_c, hpo_m, hpo_c;
        const int km = k0 - 2, kc = k0 - 1;
        const bool vm = PER || km >= 0, vc = PER || kc >= 0;
        po_m = (valid && vm) ? vload(pold + pl_of(km) + pos) : z0;
        po_c = (valid && vc) ? vload(pold + pl_of(kc) + pos) : z0;
        cz_c = (valid && vm) ? vload(CZ + pl_of(km) + pos) : z0;
        hpo_m = (h_in && vm) ? vload(pold + pl_of(km) + hp) : z0;
        hpo_c = (h_in && vc) ? vload(pold + pl_of(kc) + hp) : z0;
        hcz_c = (h_in && vm) ? vload(CZ + pl_of(km) + hp) : z0;
        const V o_po = (o_in && vc) ? vload(pold + pl_of(kc) + op) : z0;
        T* P = (kc & 1) ? PO1 : PO0;
        if (valid) vstore(P + (pos - obase), po_c);
        if (is_h) vstore(P + (hp - obase), hpo_c);
        if (is_o) vstore(P + (op - obase), o_po);
        T* Pm = (km & 1) ? PO1 : PO0;
        if (valid) vstore(Pm + (pos - obase), po_m);
        if (is_h) vstore(Pm + (hp - obase), hpo_m);
    }
    // The global loads of step k depend on k only: p_{l-2} of plane k+2; r,
    // d, x and the couplings of plane k+1 (own positions and the inner ring);
    // p_{l-2} of plane k+2 on the outer ring. They are issued one step ahead,
    // before the previous step's LDS barrier, so their latency overlaps it.
    struct Ld {
        V po_n, r_o, d_n, x_n, cx_n, cy_n, cz_n;
        T cxm_n, cym_n[W], cxw_n;
        V hpo_n, h_r, h_d, h_cx, h_cy, h_cz;
        T h_cxm, h_cym[W], h_cxw;
        V o_po;
    };
    auto issue = [&](int k, Ld& L) {
        const int kn = k + 1, kf = k + 2;
        const bool v1 = PER || (kn >= 0 && kn < nz);
        const bool v2 = PER || (kf >= 0 && kf < nz);
        const bool own1 = kn >= k0 && kn < k1;
        const bool xu = own1 && do_x;
        const int64_t g1 = pl_of(kn) + pos;
        L.po_n = z0; L.r_o = z0; L.d_n = z0; L.x_n = z0; L.cx_n = z0; L.cy_n = z0; L.cz_n = z0;
        L.cxm_n = T(0);
        L.cxw_n = T(0);
        L.h_cxw = T(0);
#pragma unroll
        for (int u = 0; u < W; ++u) L.cym_n[u] = T(0);
        if (valid) {
            if (v2) L.po_n = sload<NT>(pold + pl_of(kf) + pos);
            if (v1) {
                L.r_o = sload<NT>(rold + g1);
                L.d_n = sload<NT>(DD + g1);
                if (xu) L.x_n = sload<NT>(a.x + g1);
                L.cx_n = vload(CX + g1);
                L.cy_n = vload(CY + g1);
                L.cz_n = sload<NT>(CZ + g1);
                L.cxm_n = pos >= 1 ? CX[g1 - 1] : T(0);
#pragma unroll
                for (int u = 0; u < W; ++u) L.cym_n[u] = (pos + u - nx >= 0) ? CY[g1 + u - nx] : T(0);
                if (PER) L.cxw_n = CX[g1 + kl + nx - 1];
            }
        }
        L.hpo_n = z0; L.h_r = z0; L.h_d = z0; L.h_cx = z0; L.h_cy = z0; L.h_cz = z0;
        L.h_cxm = T(0);
#pragma unroll
        for (int u = 0; u < W; ++u) L.h_cym[u] = T(0);
        if (h_in) {
            if (v2) L.hpo_n = vload(pold + pl_of(kf) + hp);
            if (v1) {
                const int64_t gh = pl_of(kn) + hp;
                L.h_cz = vload(CZ + gh);
                if (own1) {
                    L.h_r = vload(rold + gh);
                    L.h_d = vload(DD + gh);
                    L.h_cx = vload(CX + gh);
                    L.h_cy = vload(CY + gh);
                    L.h_cxm = hp >= 1 ? CX[gh - 1] : T(0);
#pragma unroll
                    for (int u = 0; u < W; ++u) L.h_cym[u] = (hp + u - nx >= 0) ? CY[gh + u - nx] : T(0);
                    if (PER && hbrk >= 0 && hbrk < W) L.h_cxw = CX[gh + hkl + nx - 1];
                }
            }
        }
        L.o_po = (o_in && v2) ? vload(pold + pl_of(kf) + op) : z0;
    };
    Ld cur;
    issue(k0 - 2, cur);
    lds_barrier();

    V pn_m = z0, rn_c = z0, d_c = z0;   // p_{l-1} on k-1; r_{l-1}, d on k (own)
    V cz_m = z0;                        // cz of plane k-1

    for (int k = k0 - 2; k < k1; ++k) {
        const int kn = k + 1, kf = k + 2;
        const bool v1 = PER || (kn >= 0 && kn < nz);
        const bool own1 = kn >= k0 && kn < k1;   // plane k+1 belongs to this tile
        const bool xu = own1 && do_x;
        T* const POc = (kn & 1) ? PO1 : PO0;
        T* const POn = (kf & 1) ? PO1 : PO0;
        const T* const PNc = (k & 1) ? PN1 : PN0;
        T* const PNn = (kn & 1) ? PN1 : PN0;
        const T* const CXc = (k & 1) ? CX1 : CX0;
        const T* const CYc = (k & 1) ? CY1 : CY0;
        T* const CXn = (kn & 1) ? CX1 : CX0;
        T* const CYn = (kn & 1) ? CY1 : CY0;
        const int64_t g1 = pl_of(kn) + pos;
        const V po_c = valid ? vload(POc + (pos - obase)) : z0;    // p_{l-2}, plane k+1
        const V po_m = valid ? vload(POn + (pos - obase)) : z0;    // p_{l-2}, plane k

        V& po_n = cur.po_n; V& r_o = cur.r_o; V& d_n = cur.d_n; V& x_n = cur.x_n;
        V& cx_n = cur.cx_n; V& cy_n = cur.cy_n; V& cz_n = cur.cz_n;
        T& cxm_n = cur.cxm_n; T (&cym_n)[W] = cur.cym_n; const T cxw_n = cur.cxw_n;
        V& hpo_n = cur.hpo_n; V& h_r = cur.h_r; V& h_d = cur.h_d; V& h_cx = cur.h_cx; V& h_cy = cur.h_cy;
        V& h_cz = cur.h_cz; T& h_cxm = cur.h_cxm; T (&h_cym)[W] = cur.h_cym; const T h_cxw = cur.h_cxw;
        const V& o_po = cur.o_po;
        // ---- q_{l-1}, r_{l-1}, p_{l-1} (and x) on plane k+1, own positions
        V pn_n = z0, rn_n = z0;
        if (valid && v1) {
            const int64_t l = pos - obase;
            const T left = POc[l - 1], right = POc[l + W];
            const T wl_v = PER ? POc[l + kl + nx - 1] : T(0);
            const T wr_v = PER ? POc[l + kr - (nx - 1)] : T(0);
            const int bk = PER ? opaque(brk) : -1;
#pragma unroll
            for (int u = 0; u < W; ++u) {
                const bool ul = PER && u == bk, ur = PER && u + 1 == bk;
                const T pr = ur ? wr_v : (u == W - 1) ? right : vget(po_c, u + 1);
                const T pl = ul ? wl_v : (u == 0) ? left : vget(po_c, u - 1);
                const T cl = ul ? cxw_n : (u == 0) ? cxm_n : vget(cx_n, u - 1);
                const T qo = apply_point(vget(d_n, u), vget(po_c, u), vget(cx_n, u), pr, cl, pl, vget(cy_n, u),
                                         POc[l + u + nx], cym_n[u], POc[l + u - nx], vget(cz_n, u), vget(po_n, u),
                                         vget(cz_c, u), vget(po_m, u));
                const T r = fma(-alpha, qo, vget(r_o, u));
                vget(rn_n, u) = r;
                vget(pn_n, u) = fma(beta, vget(po_c, u), r * jacobi_inv(vget(d_n, u)));
                if (xu) vget(x_n, u) = fma(alpha, vget(po_c, u), vget(x_n, u));
            }
            vstore(PNn + (pos - nbase), pn_n);
            if (own1) {
                sstore<NT>(rnew + g1, rn_n);
                sstore<NT>(pnew + g1, pn_n);
                if (xu) sstore<NT>(a.x + g1, x_n);
                if constexpr (PER) {
                    const int64_t pk = g1 - pos;
                    if (g_vec) {   // element-aligned only: copied bytewise
                        __builtin_memcpy(rnew + pk + gd[0], &rn_n, sizeof(V));
                        __builtin_memcpy(pnew + pk + gd[0], &pn_n, sizeof(V));
                    } else {
#pragma unroll
                        for (int u = 0; u < W; ++u)
                            if (gd[u] >= 0) {
                                rnew[pk + gd[u]] = vget(rn_n, u);
                                pnew[pk + gd[u]] = vget(pn_n, u);
                            }
                    }
                }
            }
        }
        // ---- the same on the inner ring (LDS only; needed on owned planes)
        if (is_h && own1) {
            V hv = z0;
            if (h_in) {
                const V hpo_c = vload(POc + (hp - obase));
                const V hpo_m = vload(POn + (hp - obase));
                const int64_t l = hp - obase;
                const T left = POc[l - 1], right = POc[l + W];
                const T wl_v = PER ? POc[l + hkl + nx - 1] : T(0);
                const T wr_v = PER ? POc[l + hkr - (nx - 1)] : T(0);
                const int bk = PER ? opaque(hbrk) : -1;
#pragma unroll
                for (int u = 0; u < W; ++u) {
                    const bool ul = PER && u == bk, ur = PER && u + 1 == bk;
                    const T pr = ur ? wr_v : (u == W - 1) ? right : vget(hpo_c, u + 1);
                    const T pl = ul ? wl_v : (u == 0) ? left : vget(hpo_c, u - 1);
                    const T cl = ul ? h_cxw : (u == 0) ? h_cxm : vget(h_cx, u - 1);
                    const T qo = apply_point(vget(h_d, u), vget(hpo_c, u), vget(h_cx, u), pr, cl, pl, vget(h_cy, u),
                                             POc[l + u + nx], h_cym[u], POc[l + u - nx], vget(h_cz, u),
                                             vget(hpo_n, u), vget(hcz_c, u), vget(hpo_m, u));
                    const T r = fma(-alpha, qo, vget(h_r, u));
                    vget(hv, u) = fma(beta, vget(hpo_c, u), r * jacobi_inv(vget(h_d, u)));
                }
            }
            vstore(PNn + (hp - nbase), hv);
        }
        // ---- q_l = A p_{l-1} on plane k and the partial sums
        // p_{l-1} of plane k (own): the z-neighbour of the next step's q_l
        // (its LDS slot was written at step k-1; zero below the grid)
        const V pn_c = (valid && k >= k0 - 1 && (PER || k >= 0)) ? vload(PNc + (pos - nbase)) : z0;
        if (k >= k0 && valid) {
            const int64_t l = pos - nbase;
            const V cxv = vload(CXc + l), cyv = vload(CYc + l);
            const T left = PNc[l - 1], right = PNc[l + W];
            const T wl_v = PER ? PNc[l + kl + nx - 1] : T(0);
            const T wl_c = PER ? CXc[l + kl + nx - 1] : T(0);
            const T wr_v = PER ? PNc[l + kr - (nx - 1)] : T(0);
            const int bk = PER ? opaque(brk) : -1;
            const int nvk = PER ? opaque(nv) : W;
#pragma unroll
            for (int u = 0; u < W; ++u) {
                const bool ul = PER && u == bk, ur = PER && u + 1 == bk;
                const T p = vget(pn_c, u);
                const T pr = ur ? wr_v : (u == W - 1) ? right : vget(pn_c, u + 1);
                const T pl = ul ? wl_v : (u == 0) ? left : vget(pn_c, u - 1);
                const T cl = ul ? wl_c : (u == 0) ? CXc[l - 1] : vget(cxv, u - 1);
                const T qq = apply_point(vget(d_c, u), p, vget(cxv, u), pr, cl, pl, vget(cyv, u), PNc[l + u + nx],
                                         CYc[l + u - nx], PNc[l + u - nx], vget(cz_c, u), vget(pn_n, u), vget(cz_m, u),
                                         vget(pn_m, u));
                if (u >= nvk) continue;   // a ghost position past the last owned node
                const T iv = jacobi_inv(vget(d_c, u));
                const double pd = (double)p, qd = (double)qq, rd = (double)vget(rn_c, u);
                const double zd = (double)(vget(rn_c, u) * iv), wd = (double)(qq * iv);
                acc[0] = fma(pd, qd, acc[0]);
                acc[1] = fma(rd, zd, acc[1]);
                acc[2] = fma(rd, wd, acc[2]);
                acc[3] = fma(qd, wd, acc[3]);
                acc[4] = fma(rd, rd, acc[4]);
                acc[5] = fma(rd, qd, acc[5]);
                acc[6] = fma(qd, qd, acc[6]);
            }
        }
        // ---- p_{l-2} of plane k+2 and the couplings of plane k+1 into LDS
        // for the next step (the p_old slot of plane k is free from here on)
        if (valid) {
            vstore(POn + (pos - obase), po_n);
            vstore(CXn + (pos - nbase), cx_n);
            vstore(CYn + (pos - nbase), cy_n);
        }
        if (is_h) {
            vstore(POn + (hp - obase), hpo_n);
            vstore(CXn + (hp - nbase), h_cx);
            vstore(CYn + (hp - nbase), h_cy);
        }
        if (is_o) vstore(POn + (op - obase), o_po);
        // ---- advance one plane
        hcz_c = h_cz;
        pn_m = pn_c;
        rn_c = rn_n;
        d_c = d_n;
        cz_m = cz_c;
        cz_c = cz_n;
        if (k + 1 < k1) {
            Ld nxt;
            issue(k + 1, nxt);
            lds_barrier();
            cur = nxt;
        } else {
            lds_barrier();
        }
    }
}

// ------------------------------------------------------------------ coded 40-byte pass

// Raw buffer resources (stride 0): a load at a byte offset at or past
// num_records returns 0 and a store there is dropped. The coded pass gives
// each plane of an array a resource one plane long (zero long outside the
// grid), so neighbours before a plane's first position, past its end or on
// planes beyond the grid read as the zeros the iteration needs there, with
// no test or select in the plane loop; the per-thread offsets are fixed for
// the whole march.
constexpr int kRawBufferWord3 = 0x00020000;
// An offset past the end of every plane resource (planes hold fewer than
// 2^29 positions, checked on the host). Offsets are only ever formed from
// in-plane positions or this value: the bounds check compares the unsigned
// sum of offset and access size, so an offset meant to be negative would
// wrap around it and read the bytes before the plane.
constexpr uint32_t kOutOfPlane = 0x80000000u;
using Rsrc = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ Rsrc plane_rsrc(const void* base, int k, int nz, int64_t sp) {
    const bool in = k >= 0 && k < nz;
    const char* p = static_cast<const char*>(base) + (in ? (int64_t)k * sp * 4 : 0);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(p), 0, in ? (int)(sp * 4) : 0, kRawBufferWord3);
}
template <bool NT>
__device__ __forceinline__ float4 bload4(Rsrc r, uint32_t off) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, NT ? 2 : 0));
}
template <bool NT>
__device__ __forceinline__ u32x4 bload4w(Rsrc r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, NT ? 2 : 0);
}
__device__ __forceinline__ uint32_t bload1(Rsrc r, uint32_t off) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
}
template <bool NT>
__device__ __forceinline__ void bstore4(Rsrc r, uint32_t off, const float4& v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, (int)off, 0, NT ? 2 : 0);
}
__device__ __forceinline__ void bstore1(Rsrc r, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)off, 0, 0);
}
__device__ __forceinline__ float4 lds4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ void lds4(float* p, const float4& v) { *reinterpret_cast<float4*>(p) = v; }

// One pass on one tile of the 40-byte form with the operator read as one
// word of dictionary codes per position (byte 0: cx, 1: cy, 2: cz, 3: d). The
// iteration, the LDS planes and the order of every floating-point operation
// are those of pass_tile40, so the iterates are bit for bit the uncoded
// pass's. `tv` is the dictionary and `ti` the Jacobi scaling of each entry
// (jacobi_inv of the value), both in static LDS, so that a lookup is one
// shift of a code byte and one LDS read.
//
// Threads past the segment's end work on a copy of the last group (their
// loads stay in bounds) and store nothing and add nothing to the sums.
template <int BS, bool NT, bool PER>
__device__ void pass_tile_coded(const KArgs<float>& a, int tile, int o, int n, float alpha, float beta, float* lds,
                                const float* tv, double (&acc)[NPART]) {
#pragma clang fp contract(off)
    constexpr int W = 4;
    using V = float4;
    const float* ti = tv + kCodedTableSize;
    const TileBox tb = tile_box(a, tile);
    const int64_t s = tb.s, e = tb.e, sp = a.sp;
    const int k0 = tb.k0, k1 = tb.k1, nz = a.nz;
    const int H = a.halo, nx = a.nx;
    const int lo_len = a.seglen + 4 * H, ln_len = a.seglen + 2 * H;
    float* const PO0 = lds;
    float* const PO1 = lds + lo_len;
    float* const PN0 = lds + 2 * lo_len;
    float* const PN1 = PN0 + ln_len;
    float* const CX0 = PN1 + ln_len;
    float* const CX1 = CX0 + ln_len;
    float* const CY0 = CX1 + ln_len;
    float* const CY1 = CY0 + ln_len;
    const int64_t obase = s - 2 * H, nbase = s - H;
    const float* rold = o ? a.r[1] : a.r[0];
    const float* pold = o ? a.p[1] : a.p[0];
    float* rnew = n ? a.r[1] : a.r[0];
    float* pnew = n ? a.p[1] : a.p[0];
    const float* CW = a.cw;
    const bool do_x = alpha != 0.0f;
    const V z0 = make_float4(0.f, 0.f, 0.f, 0.f);

    const int tid = threadIdx.x;
    const int64_t pos = s + (int64_t)tid * W;
    const bool valid = pos < e;
    const int64_t posc = valid ? pos : e - W;
    const int ring = 2 * H / W;
    const bool is_h = tid < ring;
    const int64_t hp = (tid < H / W) ? (s - H + (int64_t)tid * W) : (e + (int64_t)(tid - H / W) * W);
    const bool h_in = is_h && hp >= 0 && hp < sp;
    const int og = tid - (BS - ring);
    const bool is_o = og >= 0;
    const int64_t op = (og < H / W) ? (s - 2 * H + (int64_t)og * W) : (e + H + (int64_t)(og - H / W) * W);
    // byte offsets in a plane; positions outside it get kOutOfPlane, which
    // lies past every plane resource, so their loads return 0
    auto off = [&](int64_t q) { return (q >= 0 && q < sp) ? (uint32_t)q * 4u : kOutOfPlane; };
    const uint32_t oo = off(posc), oxm = off(posc - 1);
    uint32_t oym[W];
#pragma unroll
    for (int u = 0; u < W; ++u) oym[u] = off(posc + u - nx);
    const uint32_t oh = off(hp), ohxm = off(hp - 1);
    uint32_t ohym[W];
#pragma unroll
    for (int u = 0; u < W; ++u) ohym[u] = off(hp + u - nx);
    const uint32_t oop = off(op);
    // periodic (ghost-row layout; see wrap_plane): wrapped planes, the
    // x-wrap elements and their coupling words, the ghost copies of the
    // owned nodes of the first and last two rows, and the owned elements of
    // the last group (nv) that enter the sums
    auto prs = [&](const void* base, int k) { return plane_rsrc(base, wrap_plane<PER>(k, nz), nz, sp); };
    const int nv = valid ? (int)min((int64_t)W, a.oend - pos) : 0;
    const int brk = PER ? x_break<W>(a, posc) : -1;
    const int hbrk = PER && h_in ? x_break<W>(a, hp) : -1;
    // the elements whose neighbour across a row end is read (any element when
    // there is none: the value read is then unused)
    const int kl = min(max(brk, 0), W - 1), kr = min(max(brk - 1, 0), W - 1);
    const int hkl = min(max(hbrk, 0), W - 1), hkr = min(max(hbrk - 1, 0), W - 1);
    const uint32_t oxw = PER ? off(posc + kl + nx - 1) : kOutOfPlane;
    const uint32_t ohxw = (hbrk >= 0 && hbrk < W) ? off(hp + hkl + nx - 1) : kOutOfPlane;
    // ghost copies: one 16-byte store (dword-aligned, which buffer stores
    // allow) when the whole group is copied to consecutive positions, else one
    // store per element
    uint32_t ogh[W];
    bool has_g = false, g_vec = false;
    {
        int64_t gd[W];
#pragma unroll
        for (int u = 0; u < W; ++u) gd[u] = -1;
        if constexpr (PER) ghost_of<W>(a, pos, nv, gd);
        g_vec = gd[0] >= 0;
#pragma unroll
        for (int u = 0; u < W; ++u) {
            ogh[u] = gd[u] >= 0 ? off(gd[u]) : kOutOfPlane;
            has_g = has_g || gd[u] >= 0;
            g_vec = g_vec && gd[u] == gd[0] + u;
        }
    }
    const int lo = (int)(posc - obase), ln = (int)(posc - nbase);
    const int lho = (int)(hp - obase), lhn = (int)(hp - nbase), loo = (int)(op - obase);

    auto val = [&](uint32_t w, int byte) { return tv[(w >> (8 * byte)) & 255u]; };
    auto inv = [&](uint32_t w) { return ti[w >> 24]; };

    // cz of plane k (own, ring) and p_{l-2} of planes k0-2, k0-1 into LDS
    V cz_c, hcz_c;
    {
        const int km = k0 - 2, kc = k0 - 1;
        const Rsrc pm = prs(pold, km), pc = prs(pold, kc);
        const Rsrc wm = prs(CW, km);
        const V po_m = bload4<false>(pm, oo), po_c = bload4<false>(pc, oo);
        const u32x4 w = bload4w<false>(wm, oo);
#pragma unroll
        for (int u = 0; u < W; ++u) vget(cz_c, u) = val(w[u], 2);
        float* P = (kc & 1) ? PO1 : PO0;
        float* Pm = (km & 1) ? PO1 : PO0;
        if (valid) {
            lds4(P + lo, po_c);
            lds4(Pm + lo, po_m);
        }
        if (is_h) {
            const V hpo_m = bload4<false>(pm, oh), hpo_c = bload4<false>(pc, oh);
            const u32x4 hw = bload4w<false>(wm, oh);
#pragma unroll
            for (int u = 0; u < W; ++u) vget(hcz_c, u) = val(hw[u], 2);
            lds4(P + lho, hpo_c);
            lds4(Pm + lho, hpo_m);
        }
        if (is_o) lds4(P + loo, bload4<false>(pc, oop));
    }

    // The global loads of step k: p_{l-2} of plane k+2; r, x and the code
    // words (own, x-1 and y-1 neighbours) of plane k+1; the same on the inner
    // ring, p_{l-2} of plane k+2 on the outer ring. They are issued during the
    // previous step, after the last use of that step's values.
    struct Ld {
        V po, r, x;
        u32x4 w;
        uint32_t wxm, wym[W], wxw;
        V hpo, hr;
        u32x4 hw;
        uint32_t hwxm, hwym[W], hwxw;
        V opo;
    };
    auto issue = [&](int k, Ld& L) {
        const int kn = k + 1, kf = k + 2;
        const bool own1 = kn >= k0 && kn < k1;
        const Rsrc pf = prs(pold, kf);
        const Rsrc rn = prs(rold, kn);
        const Rsrc wn = prs(CW, kn);
        L.po = bload4<NT>(pf, oo);
        L.r = bload4<NT>(rn, oo);
        if (own1 && do_x) L.x = bload4<NT>(prs(a.x, kn), oo);
        L.w = bload4w<NT>(wn, oo);
        L.wxm = bload1(wn, oxm);
#pragma unroll
        for (int u = 0; u < W; ++u) L.wym[u] = bload1(wn, oym[u]);
        if constexpr (PER) L.wxw = bload1(wn, oxw);
        if (is_h) {
            L.hpo = bload4<false>(pf, oh);
            L.hw = bload4w<false>(wn, oh);
            if (own1) {
                L.hr = bload4<false>(rn, oh);
                L.hwxm = bload1(wn, ohxm);
#pragma unroll
                for (int u = 0; u < W; ++u) L.hwym[u] = bload1(wn, ohym[u]);
                if constexpr (PER) L.hwxw = bload1(wn, ohxw);
            }
        }
        if (is_o) L.opo = bload4<false>(pf, oop);
    };
    Ld cur;
    issue(k0 - 2, cur);
    lds_barrier();

    V pn_m = z0, rn_c = z0, d_c = z0, iv_c = z0;   // p_{l-1} on k-1; r_{l-1}, d, 1/d on k (own)
    V cz_m = z0;                                   // cz of plane k-1

    for (int k = k0 - 2; k < k1; ++k) {
        const int kn = k + 1, kf = k + 2;
        const bool v1 = PER || (kn >= 0 && kn < nz);
        const bool own1 = kn >= k0 && kn < k1;   // plane k+1 belongs to this tile
        const bool xu = own1 && do_x;
        float* const POc = (kn & 1) ? PO1 : PO0;
        float* const POn = (kf & 1) ? PO1 : PO0;
        const float* const PNc = (k & 1) ? PN1 : PN0;
        float* const PNn = (kn & 1) ? PN1 : PN0;
        const float* const CXc = (k & 1) ? CX1 : CX0;
        const float* const CYc = (k & 1) ? CY1 : CY0;
        float* const CXn = (kn & 1) ? CX1 : CX0;
        float* const CYn = (kn & 1) ? CY1 : CY0;

        // decode plane k+1's words: own positions, the left x-coupling and
        // the y-couplings one row down
        V cx_n, cy_n, cz_n, d_n, iv_n;
        float cym_n[W];
#pragma unroll
        for (int u = 0; u < W; ++u) {
            const uint32_t c = cur.w[u];
            vget(cx_n, u) = val(c, 0);
            vget(cy_n, u) = val(c, 1);
            vget(cz_n, u) = val(c, 2);
            vget(d_n, u) = val(c, 3);
            vget(iv_n, u) = inv(c);
            cym_n[u] = val(cur.wym[u], 1);
        }
        const float cxm_n = val(cur.wxm, 0);
        const float cxw_n = PER ? val(cur.wxw, 0) : 0.0f;

        // ---- q_{l-1}, r_{l-1}, p_{l-1} (and x) on plane k+1, own positions
        const V po_c = lds4(POc + lo);    // p_{l-2}, plane k+1
        const V po_m = lds4(POn + lo);    // p_{l-2}, plane k
        V pn_n = z0, rn_n = z0, xv = cur.x;
        if (v1) {
            const float left = POc[lo - 1], right = POc[lo + W];
            const float wl_v = PER ? POc[lo + kl + nx - 1] : 0.0f;
            const float wr_v = PER ? POc[lo + kr - (nx - 1)] : 0.0f;
            const int bk = PER ? opaque(brk) : -1;
#pragma unroll
            for (int u = 0; u < W; ++u) {
                const bool ul = PER && u == bk, ur = PER && u + 1 == bk;
                const float pr = ur ? wr_v : (u == W - 1) ? right : vget(po_c, u + 1);
                const float pl = ul ? wl_v : (u == 0) ? left : vget(po_c, u - 1);
                const float cl = ul ? cxw_n : (u == 0) ? cxm_n : vget(cx_n, u - 1);
                const float qo = apply_point(vget(d_n, u), vget(po_c, u), vget(cx_n, u), pr, cl, pl, vget(cy_n, u),
                                             POc[lo + u + nx], cym_n[u], POc[lo + u - nx], vget(cz_n, u),
                                             vget(cur.po, u), vget(cz_c, u), vget(po_m, u));
                const float r = fmaf(-alpha, qo, vget(cur.r, u));
                vget(rn_n, u) = r;
                vget(pn_n, u) = fmaf(beta, vget(po_c, u), r * vget(iv_n, u));
                if (xu) vget(xv, u) = fmaf(alpha, vget(po_c, u), vget(xv, u));
            }
            if (valid) lds4(PNn + ln, pn_n);
        }
        // ---- the inner ring: decode, and p_{l-1} on owned planes (LDS only)
        V h_cx, h_cy, h_cz;
        if (is_h) {
#pragma unroll
            for (int u = 0; u < W; ++u) {
                const uint32_t c = cur.hw[u];
                vget(h_cx, u) = val(c, 0);
                vget(h_cy, u) = val(c, 1);
                vget(h_cz, u) = val(c, 2);
            }
            if (own1) {
                V hv = z0;
                if (h_in) {
                    const V hpo_c = lds4(POc + lho);
                    const V hpo_m = lds4(POn + lho);
                    const float left = POc[lho - 1], right = POc[lho + W];
                    const float h_cxm = val(cur.hwxm, 0);
                    const float h_cxw = PER ? val(cur.hwxw, 0) : 0.0f;
                    const float wl_v = PER ? POc[lho + hkl + nx - 1] : 0.0f;
                    const float wr_v = PER ? POc[lho + hkr - (nx - 1)] : 0.0f;
                    const int bk = PER ? opaque(hbrk) : -1;
#pragma unroll
                    for (int u = 0; u < W; ++u) {
                        const uint32_t c = cur.hw[u];
                        const bool ul = PER && u == bk, ur = PER && u + 1 == bk;
                        const float pr = ur ? wr_v : (u == W - 1) ? right : vget(hpo_c, u + 1);
                        const float pl = ul ? wl_v : (u == 0) ? left : vget(hpo_c, u - 1);
                        const float cl = ul ? h_cxw : (u == 0) ? h_cxm : vget(h_cx, u - 1);
                        const float qo = apply_point(val(c, 3), vget(hpo_c, u), vget(h_cx, u), pr, cl, pl,
                                                     vget(h_cy, u), POc[lho + u + nx], val(cur.hwym[u], 1),
                                                     POc[lho + u - nx], vget(h_cz, u), vget(cur.hpo, u),
                                                     vget(hcz_c, u), vget(hpo_m, u));
                        const float r = fmaf(-alpha, qo, vget(cur.hr, u));
                        vget(hv, u) = fmaf(beta, vget(hpo_c, u), r * inv(c));
                    }
                }
                lds4(PNn + lhn, hv);
            }
        }
        // ---- p_{l-2} of plane k+2 and the couplings of plane k+1 into LDS
        // for the next step (the p_old slot of plane k is free from here on)
        if (valid) {
            lds4(POn + lo, cur.po);
            lds4(CXn + ln, cx_n);
            lds4(CYn + ln, cy_n);
        }
        if (is_h) {
            lds4(POn + lho, cur.hpo);
            lds4(CXn + lhn, h_cx);
            lds4(CYn + lhn, h_cy);
            hcz_c = h_cz;
        }
        if (is_o) lds4(POn + loo, cur.opo);
        // ---- r, p, x of plane k+1 to memory, once every load of this step
        // has been used (a store in flight would make the wait for a load
        // wait for the store too), then the loads of the next step, which
        // land while q_l and the sums below are computed
        if (valid && v1 && own1) {
            bstore4<NT>(prs(rnew, kn), oo, rn_n);
            bstore4<NT>(prs(pnew, kn), oo, pn_n);
            if (xu) bstore4<NT>(prs(a.x, kn), oo, xv);
            if (PER && has_g) {
                const Rsrc gr = prs(rnew, kn), gp = prs(pnew, kn);
                if (g_vec) {
                    bstore4<false>(gr, ogh[0], rn_n);
                    bstore4<false>(gp, ogh[0], pn_n);
                } else {
#pragma unroll
                    for (int u = 0; u < W; ++u) {
                        bstore1(gr, ogh[u], vget(rn_n, u));
                        bstore1(gp, ogh[u], vget(pn_n, u));
                    }
                }
            }
        }
        if (k + 1 < k1) issue(k + 1, cur);
        // ---- q_l = A p_{l-1} on plane k and the partial sums
        const V pn_c = (PER || k >= 0) ? lds4(PNc + ln) : z0;   // p_{l-1}, plane k (zero below the grid)
        if (k >= k0) {
            const V cxv = lds4(CXc + ln), cyv = lds4(CYc + ln);
            const float left = PNc[ln - 1], right = PNc[ln + W];
            const float wl_v = PER ? PNc[ln + kl + nx - 1] : 0.0f;
            const float wl_c = PER ? CXc[ln + kl + nx - 1] : 0.0f;
            const float wr_v = PER ? PNc[ln + kr - (nx - 1)] : 0.0f;
            const int bk = PER ? opaque(brk) : -1;
            const int nvk = PER ? opaque(nv) : W;
#pragma unroll
            for (int u = 0; u < W; ++u) {
                const bool ul = PER && u == bk, ur = PER && u + 1 == bk;
                const float p = vget(pn_c, u);
                const float pr = ur ? wr_v : (u == W - 1) ? right : vget(pn_c, u + 1);
                const float pl = ul ? wl_v : (u == 0) ? left : vget(pn_c, u - 1);
                const float cl = ul ? wl_c : (u == 0) ? CXc[ln - 1] : vget(cxv, u - 1);
                const float qq = apply_point(vget(d_c, u), p, vget(cxv, u), pr, cl, pl, vget(cyv, u),
                                             PNc[ln + u + nx], CYc[ln + u - nx], PNc[ln + u - nx], vget(cz_c, u),
                                             vget(pn_n, u), vget(cz_m, u), vget(pn_m, u));
                if (valid && u < nvk) {
                    const float iv = vget(iv_c, u);
                    const double pd = (double)p, qd = (double)qq, rd = (double)vget(rn_c, u);
                    const double zd = (double)(vget(rn_c, u) * iv), wd = (double)(qq * iv);
                    acc[0] = fma(pd, qd, acc[0]);
                    acc[1] = fma(rd, zd, acc[1]);
                    acc[2] = fma(rd, wd, acc[2]);
                    acc[3] = fma(qd, wd, acc[3]);
                    acc[4] = fma(rd, rd, acc[4]);
                    acc[5] = fma(rd, qd, acc[5]);
                    acc[6] = fma(qd, qd, acc[6]);
                }
            }
        }
        // ---- advance one plane
        pn_m = pn_c;
        rn_c = rn_n;
        d_c = d_n;
        iv_c = iv_n;
        cz_m = cz_c;
        cz_c = cz_n;
        lds_barrier();
    }
}

template <typename T, int BS>
__device__ void final_tile(const KArgs<T>& a, int tile, T alpha, const T* p, bool zero) {
    constexpr int W = Vec<T>::n;
    using V = typename Vec<T>::type;
    const TileBox tb = tile_box(a, tile);
    for (int k = tb.k0; k < tb.k1; ++k) {
        for (int64_t pos = tb.s + (int64_t)threadIdx.x * W; pos < tb.e; pos += (int64_t)BS * W) {
            const int64_t g = (int64_t)k * a.sp + pos;
            V xv = vload(a.x + g);
            if (zero) {
                xv = vzero<T>();
            } else {
                const V pv = vload(p + g);
#pragma unroll
                for (int u = 0; u < Vec<T>::n; ++u) vget(xv, u) = vget(xv, u) + alpha * vget(pv, u);
            }
            vstore(a.x + g, xv);
        }
    }
}

// ------------------------------------------------------------------ kernel

struct Scal {
    double alpha, beta, rr, bb;
    int iters, done, status, zero;
};

// The whole solve of one problem by workgroup `w` of the `G` workgroups
// assigned to it with pass form SCH (0: pass_tile, 48 bytes per node; 1:
// pass_tile40); `lds_raw` holds that form's plane buffers.
// Every workgroup derives the scalars (alpha, beta, stopping test) itself
// from the identically reduced tile sums; workgroup 0 also persists them in
// S for the host and for a resumed launch.
//
// CD: the 40-byte pass reads coded coefficients. RT (with CD): whether it
// does is read per problem from *a.fit at the start of the launch (written
// by the dictionary build enqueued before it), so one launch serves problems
// whose operators fit the dictionary and problems whose operators do not.
template <typename T, int BS, int MC, int SCH, bool PER, bool NT, bool CD, bool RT = false>
__device__ void run_problem(const KArgs<T>& a, int w, int G, bool xcd_map, unsigned char* lds_raw) {
    static_assert(SCH == 0 || MC == 1, "the 40-byte pass takes one vector group per thread");
    static_assert(!CD || SCH == 1, "coded coefficients are read by the 40-byte pass");
    const int lds_len = a.seglen + 2 * a.halo;
    T* lds0 = reinterpret_cast<T*>(lds_raw);
    T* lds1 = lds0 + lds_len;
    // coded form: the dictionary and the Jacobi scaling of each entry, in
    // static LDS (their addresses are then constants of the kernel)
    bool use_codes = CD;
    float* dict = nullptr;
    if constexpr (CD) {
        __shared__ float s_dict[2 * kCodedTableSize];
        dict = s_dict;
        if constexpr (RT) use_codes = a.fit[0] == 1;
        if (use_codes) {
            for (int i = threadIdx.x; i < kCodedTableSize; i += BS) {
                const float v = a.ctab[i];
                s_dict[i] = v;
                s_dict[kCodedTableSize + i] = jacobi_inv(v);
            }
        }
        __syncthreads();
    }
    __shared__ double red[red_len<BS>()];
    __shared__ int s_flag;
    __shared__ Scal sc;
    SyncState* S = a.S;
    const bool lead = (w == 0) && (threadIdx.x == 0);
    int first, stride, end;
    xcd_tile_range(a.ntiles, w, G, xcd_map, first, stride, end);
    int b = 0;   // barrier index within this launch (arrival counters start at zero)
    auto sums = [&](int bb) { return a.partials + (size_t)(bb & 1) * a.ntiles * kMaxPartials; };

    if (!a.resume) {
        // ---- initial residual
        for (int t = first; t < end; t += stride) {
            double acc[2] = {0.0, 0.0};
            init_tile<T, BS, PER, PER && SCH == 1>(a, t, SCH == 0, acc);
            tile_reduce_store<BS, 2>(acc, red, sums(b) + (size_t)t * kMaxPartials);
        }
        double v[2];
        if (!grid_sync_reduce<BS, 2>(S, w, G, b, sums(b), a.ntiles, a.timeout_ticks, red, &s_flag, v)) return;
        ++b;
        if (threadIdx.x == 0) {
            const double rr = v[0], bb = v[1];
            int done = 0, status = PB_OK, zero = 0;
            if (!(bb - bb == 0.0) || !(rr - rr == 0.0)) { done = 1; status = PB_ERR_NONFINITE; }
            else if (bb == 0.0) { done = 1; zero = 1; }
            else if (sqrt(rr) / sqrt(bb) < a.tol) { done = 1; }
            else if (a.maxiter <= 0) { done = 1; status = PB_NOT_CONVERGED; }
            sc.alpha = 0.0; sc.beta = 0.0; sc.rr = rr; sc.bb = bb;
            sc.iters = 0; sc.done = done; sc.status = status; sc.zero = zero;
            if (lead) {
                S->rr = rr; S->bb = bb; S->alpha = 0.0; S->beta = 0.0; S->iters = 0;
                S->done = done; S->status = status; S->zero_rhs = zero;
            }
        }
        __syncthreads();
    } else {
        if (threadIdx.x == 0) {
            sc.alpha = ld_agent_d(&S->alpha); sc.beta = ld_agent_d(&S->beta);
            sc.rr = ld_agent_d(&S->rr); sc.bb = ld_agent_d(&S->bb);
            sc.iters = ld_agent_i(&S->iters); sc.done = ld_agent_i(&S->done);
            sc.status = ld_agent_i(&S->status); sc.zero = ld_agent_i(&S->zero_rhs);
        }
        __syncthreads();
    }

    int it = sc.iters, this_launch = 0;
    bool final_update = false;
    while (!sc.done && (a.chunk <= 0 || this_launch < a.chunk)) {
        const int o = it & 1, n = (it + 1) & 1;
        const T alpha = (T)sc.alpha, beta = (T)sc.beta;
        for (int t = first; t < end; t += stride) {
            double acc[NPART] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            if constexpr (SCH == 1)
            {
                if constexpr (CD) {
                    if (use_codes) pass_tile_coded<BS, NT, PER>(a, t, o, n, alpha, beta, lds0, dict, acc);
                    else pass_tile40<T, BS, NT, PER>(a, t, o, n, alpha, beta, lds0, acc);
                } else {
                    pass_tile40<T, BS, NT, PER>(a, t, o, n, alpha, beta, lds0, acc);
                }
            }
            else
                pass_tile<T, BS, MC, PER, NT>(a, t, o, n, alpha, beta, lds0, lds1, acc);
            tile_reduce_store<BS, NPART>(acc, red, sums(b) + (size_t)t * kMaxPartials);
        }
        double v[NPART];
        if (!grid_sync_reduce<BS, NPART>(S, w, G, b, sums(b), a.ntiles, a.timeout_ticks, red, &s_flag, v)) return;
        ++b;
        if (threadIdx.x == 0) {
            const double pq = v[0], rrd = v[1], rqd = v[2], qqd = v[3], rr0 = v[4], rq = v[5], qq = v[6];
            if (!(pq > 0.0) || !(pq - pq == 0.0) || !(rrd > 0.0)) {
                sc.done = 1;
                sc.status = PB_ERR_BREAKDOWN;
                sc.alpha = 0.0;
            } else {
                const double al = rrd / pq;
                const double rho = fmax(rrd - 2.0 * al * rqd + al * al * qqd, 0.0);
                const double rr = fmax(rr0 - 2.0 * al * rq + al * al * qq, 0.0);
                const int iters = sc.iters + 1;
                sc.alpha = al;
                sc.beta = rho / rrd;
                sc.rr = rr;
                sc.iters = iters;
                const double rel = sqrt(rr) / sqrt(sc.bb);
                if (!(rel - rel == 0.0)) { sc.done = 1; sc.status = PB_ERR_BREAKDOWN; }
                else if (rel < a.tol) { sc.done = 1; sc.status = PB_OK; }
                else if (iters >= a.maxiter) { sc.done = 1; sc.status = PB_NOT_CONVERGED; }
                if (lead) S->rho = rho;
            }
            if (lead) {
                S->pq = pq;
                S->alpha = sc.alpha; S->beta = sc.beta; S->rr = sc.rr; S->iters = sc.iters;
                S->done = sc.done; S->status = sc.status;
            }
        }
        __syncthreads();
        ++it;
        ++this_launch;
        if (sc.status == PB_ERR_BREAKDOWN) break;   // x holds the last good iterate
        final_update = true;
    }
    // ---- last x update with the final alpha and direction (or x = 0); a
    // chunk that stops before convergence leaves the state to be resumed
    if (sc.zero || (sc.done && final_update && sc.status != PB_ERR_BREAKDOWN)) {
        const T* plast = (it & 1) ? a.p[1] : a.p[0];
        for (int t = first; t < end; t += stride) final_tile<T, BS>(a, t, (T)sc.alpha, plast, sc.zero != 0);
    }
}

template <typename T, int BS, int MC, int SCH, bool PER, bool NT, bool CD = false>
__global__ __launch_bounds__(BS) void k_jpcg_fused(KArgs<T> a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    run_problem<T, BS, MC, SCH, PER, NT, CD>(a, blockIdx.x, gridDim.x, true, lds_raw);
}

// Many independent problems in one launch: workgroups [first[p], first[p+1])
// solve problem p with their own barrier state; problems never wait for
// each other, and each problem's tiling and reduction order depend only on
// its own shape.
template <typename T, int BS, int MC, int SCH, bool NT, bool CD = false, bool RT = false>
__global__ __launch_bounds__(BS) void k_jpcg_batch(const KArgs<T>* __restrict__ probs,
                                                   const int* __restrict__ first, int nprob) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    int lo = 0, hi = nprob;   // last p with first[p] <= blockIdx.x
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (first[mid] <= (int)blockIdx.x) lo = mid; else hi = mid;
    }
    const KArgs<T> a = probs[lo];
    // coded launches: every problem's arguments carry its code words and
    // dictionary (and, runtime-checked, its fit flag)
    run_problem<T, BS, MC, SCH, false, NT, CD, RT>(a, blockIdx.x - first[lo], first[lo + 1] - first[lo], false,
                                                   lds_raw);
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
        if (hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) d.cus = 0;
        if (hipDeviceGetAttribute(&d.wallclock_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
            d.wallclock_khz = 0;
        cache[dev] = d;
    }
    return cache[dev];
}

using KernelFn = const void*;

struct Variant {
    int bs, mc, scheme, per, nt;
    KernelFn fn;
    int cd = 0;   // 1: reads coded coefficients (chosen per solve, never by the tiling search)
};

// Coded forms of the 40-byte pass (FP32 only).
template <typename T>
std::vector<Variant> coded_variants() {
    return {};
}
template <>
std::vector<Variant> coded_variants<float>() {
    return {
        {256, 1, 1, 0, 0, (KernelFn)k_jpcg_fused<float, 256, 1, 1, false, false, true>, 1},
        {512, 1, 1, 0, 0, (KernelFn)k_jpcg_fused<float, 512, 1, 1, false, false, true>, 1},
        {256, 1, 1, 0, 1, (KernelFn)k_jpcg_fused<float, 256, 1, 1, false, true, true>, 1},
        {512, 1, 1, 0, 1, (KernelFn)k_jpcg_fused<float, 512, 1, 1, false, true, true>, 1},
        {256, 1, 1, 1, 0, (KernelFn)k_jpcg_fused<float, 256, 1, 1, true, false, true>, 1},
        {512, 1, 1, 1, 0, (KernelFn)k_jpcg_fused<float, 512, 1, 1, true, false, true>, 1},
        {256, 1, 1, 1, 1, (KernelFn)k_jpcg_fused<float, 256, 1, 1, true, true, true>, 1},
        {512, 1, 1, 1, 1, (KernelFn)k_jpcg_fused<float, 512, 1, 1, true, true, true>, 1},
    };
}

template <typename T>
std::vector<Variant> base_variants() {
    return {
        {256, 1, 0, 0, 0, (KernelFn)k_jpcg_fused<T, 256, 1, 0, false, false>},
        {256, 2, 0, 0, 0, (KernelFn)k_jpcg_fused<T, 256, 2, 0, false, false>},
        {512, 1, 0, 0, 0, (KernelFn)k_jpcg_fused<T, 512, 1, 0, false, false>},
        {512, 2, 0, 0, 0, (KernelFn)k_jpcg_fused<T, 512, 2, 0, false, false>},
        {256, 1, 1, 0, 0, (KernelFn)k_jpcg_fused<T, 256, 1, 1, false, false>},
        {512, 1, 1, 0, 0, (KernelFn)k_jpcg_fused<T, 512, 1, 1, false, false>},
        {256, 1, 0, 1, 0, (KernelFn)k_jpcg_fused<T, 256, 1, 0, true, false>},
        {512, 1, 0, 1, 0, (KernelFn)k_jpcg_fused<T, 512, 1, 0, true, false>},
        {256, 1, 0, 0, 1, (KernelFn)k_jpcg_fused<T, 256, 1, 0, false, true>},
        {256, 2, 0, 0, 1, (KernelFn)k_jpcg_fused<T, 256, 2, 0, false, true>},
        {512, 1, 0, 0, 1, (KernelFn)k_jpcg_fused<T, 512, 1, 0, false, true>},
        {512, 2, 0, 0, 1, (KernelFn)k_jpcg_fused<T, 512, 2, 0, false, true>},
        {256, 1, 1, 0, 1, (KernelFn)k_jpcg_fused<T, 256, 1, 1, false, true>},
        {512, 1, 1, 0, 1, (KernelFn)k_jpcg_fused<T, 512, 1, 1, false, true>},
        {256, 1, 0, 1, 1, (KernelFn)k_jpcg_fused<T, 256, 1, 0, true, true>},
        {512, 1, 0, 1, 1, (KernelFn)k_jpcg_fused<T, 512, 1, 0, true, true>},
        // periodic boundary, 40-byte pass (ghost-row layout)
        {256, 1, 1, 1, 0, (KernelFn)k_jpcg_fused<T, 256, 1, 1, true, false>},
        {512, 1, 1, 1, 0, (KernelFn)k_jpcg_fused<T, 512, 1, 1, true, false>},
        {256, 1, 1, 1, 1, (KernelFn)k_jpcg_fused<T, 256, 1, 1, true, true>},
        {512, 1, 1, 1, 1, (KernelFn)k_jpcg_fused<T, 512, 1, 1, true, true>},
    };
}

template <typename T>
const std::vector<Variant>& variants() {
    static const std::vector<Variant> v = [] {
        std::vector<Variant> all = base_variants<T>();
        for (const Variant& c : coded_variants<T>()) all.push_back(c);
        return all;
    }();
    return v;
}

int max_coresident(KernelFn fn, int bs, size_t lds_bytes) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, bs, lds_bytes) != hipSuccess) return 0;
    return nb;
}

// Segment length for at most `cap` positions per plane step: the fewest
// segments that cover a padded plane, split evenly (rounded up to 64 bytes,
// so segments start aligned and none is empty once nseg is recomputed).
template <typename T>
int balanced_seglen(const Layout& L, int cap) {
    constexpr int A = 64 / (int)sizeof(T);
    const int64_t nseg = (L.sp + cap - 1) / cap;
    const int64_t even = (L.sp + nseg - 1) / nseg;
    return (int)std::min<int64_t>(cap, (even + A - 1) / A * A);
}

// Dynamic LDS of one workgroup: two planes of p over the segment +- halo
// (48-byte pass); two planes of p_old over the segment +- 2 halo, and two
// planes each of p, cx and cy over the segment +- halo (40-byte pass).
template <typename T>
size_t lds_bytes(int scheme, int seglen, int halo) {
    const size_t elems = scheme == 1 ? 2 * (size_t)(seglen + 4 * halo) + 6 * (size_t)(seglen + 2 * halo)
                                     : 2 * (size_t)(seglen + 2 * halo);
    return sizeof(T) * elems;
}

template <typename T>
int halo_for(int nx) {
    constexpr int W = Vec<T>::n;
    return (nx + W - 1) / W * W;
}

// Tiling for one kernel variant: z-chunks chosen so that the tile count
// fits the co-resident workgroups (each workgroup owns at most one tile, so
// a pass takes the time of one tile). `extra_seg` splits each plane into
// that many more segments than the fewest the block covers (shorter tiles
// that can fill more of the device). Returns grid = 0 when infeasible.
template <typename T>
Tiling tiling_for(const Layout& L, const Variant& v, int cus, int max_per_cu, int extra_seg = 0) {
    constexpr int W = Vec<T>::n;
    Tiling t{};
    t.mc = v.mc;
    t.bs = v.bs;
    t.scheme = v.scheme;
    t.per = v.per;
    t.nt = v.nt;
    t.seglen = balanced_seglen<T>(L, v.mc * v.bs * W);
    if (extra_seg > 0) {
        // an even split into nseg0 + extra_seg segments, each rounded up to
        // 64 bytes so that every segment starts aligned
        constexpr int A = 64 / (int)sizeof(T);
        const int64_t nseg0 = (L.sp + t.seglen - 1) / t.seglen;
        const int64_t even = (L.sp + nseg0 + extra_seg - 1) / (nseg0 + extra_seg);
        const int seglen = (int)((even + A - 1) / A * A);
        if ((L.sp + seglen - 1) / seglen <= nseg0) return t;   // no more segments than without
        t.seglen = seglen;
    }
    t.halo = halo_for<T>(L.nx);
    if (2 * t.halo / W > v.bs) return t;   // halo groups must fit one per thread
    const size_t lds = lds_bytes<T>(t.scheme, t.seglen, t.halo);
    int per_cu = max_coresident(v.fn, v.bs, lds);
    if (max_per_cu > 0) per_cu = std::min(per_cu, max_per_cu);
    if (per_cu <= 0) return t;
    const int G = per_cu * cus;
    t.nseg = (int)((L.sp + t.seglen - 1) / t.seglen);
    const int max_chunks = G / t.nseg;
    if (max_chunks < 1) return t;
    t.zchunk = (L.nz + max_chunks - 1) / max_chunks;
    t.nzc = (L.nz + t.zchunk - 1) / t.zchunk;
    t.ntiles = t.nseg * t.nzc;
    if (t.ntiles > kMaxTiles || t.ntiles > G) return t;
    int grid = (t.ntiles + 7) / 8 * 8;
    if (grid > G) grid = t.ntiles;
    t.grid = grid;
    t.lds = lds;
    return t;
}

// Streaming (nontemporal) variants are the default once the arrays one pass
// touches (about 12 per node: r, p and q in two copies, x, d, cx, cy, cz)
// exceed 1.75 times the last-level cache (256 MiB of Infinity Cache on
// MI355X). Measured crossover: cached wins at 161^3 FP32/FP64 and 193^3 FP32
// (201-402 MB), streaming at 193^3 FP64, 225^3 FP32 and 257^3 FP32 (549 MB and
// up); part of a working set somewhat above the cache still survives between
// iterations.
constexpr double kLastLevelCacheBytes = 256.0 * 1024 * 1024;
constexpr double kStreamingFactor = 1.75;
template <typename T>
int streaming_default(const Layout& L) {
    return (double)L.sp * L.nz * sizeof(T) * 12.0 > kStreamingFactor * kLastLevelCacheBytes ? 1 : 0;
}

constexpr int kMaxExtraSegments = 8;

template <typename T>
Tiling choose_tiling_impl(const Layout& L, int want_bs, int want_mc, int max_per_cu, int want_scheme = -1,
                          int want_per = 0, int want_nt = -1, int want_extra = -1) {
    const DevInfo di = dev_info();
    const int cus = di.cus > 0 ? di.cus : 256;
    if (want_nt < 0) want_nt = streaming_default<T>(L);
    Tiling best{};
    double best_cost = 1e300;
    for (const auto& v : variants<T>())
    for (int extra = 0; extra <= kMaxExtraSegments; ++extra) {
        if (want_extra >= 0 && extra != want_extra) continue;
        if ((want_bs > 0 && v.bs != want_bs) || (want_mc > 0 && v.mc != want_mc)) continue;
        if (want_scheme >= 0 && v.scheme != want_scheme) continue;
        if (v.per != want_per || v.nt != want_nt || v.cd) continue;
        // the periodic 40-byte pass tiles the owned range of the ghost-row layout
        if (v.per && v.scheme == 1 && !ghost_layout_ok(L)) continue;
        Layout Lt = L;
        if (v.per && v.scheme == 1) Lt.sp = ghost_layout(L).own;
        Tiling t = tiling_for<T>(Lt, v, cus, max_per_cu, extra);
        if (t.grid <= 0) continue;
        // model: bytes of one tile (planes incl. the extra ones below, segment
        // incl. halo work) times the tiles that share a CU, plus a
        // per-workgroup barrier cost; ties go to one vector group per thread
        const double tile = t.scheme == 1 ? 40.0 * (t.zchunk + 2) * (t.seglen + 1.5 * t.halo)
                                          : 48.0 * (t.zchunk + 1) * (t.seglen + t.halo);
        const double cost = tile * ((t.grid + cus - 1) / cus) + 1920.0 * t.grid;
        if (cost < best_cost || (cost == best_cost && t.mc < best.mc)) {
            best_cost = cost;
            best = t;
        }
    }
    return best;
}

// Tilings recorded by the autotuner, per device, grid shape and precision.
using TuneKey = std::tuple<int, int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, Tiling> g_tuned;

template <typename T>
TuneKey tune_key(const Layout& L) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    return TuneKey(dev, L.nx, L.ny, L.nz, (int)sizeof(T));
}

}  // namespace

template <typename T>
Tiling choose_tiling(const Layout& L) {
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(tune_key<T>(L));
        if (it != g_tuned.end()) return it->second;
    }
    return choose_tiling_impl<T>(L, 0, 0, 0);
}

template <typename T>
void record_tiling(const Layout& L, const Tiling& t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[tune_key<T>(L)] = t;
}
template void record_tiling<float>(const Layout&, const Tiling&);
template void record_tiling<double>(const Layout&, const Tiling&);

// Every distinct feasible tiling over block sizes, vector groups, pass forms,
// cached and streaming accesses and workgroups-per-CU caps (the autotuner's
// search space).
template <typename T>
std::vector<Tiling> tiling_candidates(const Layout& L) {
    std::vector<Tiling> out;
    for (const auto& v : variants<T>()) {
        if (v.per || v.cd) continue;   // periodic solves use their own default tiling; coding is per solve
        for (int cap : {1, 2, 3, 4, 0})
            for (int extra = 0; extra <= kMaxExtraSegments; ++extra) {
                const Tiling t = choose_tiling_impl<T>(L, v.bs, v.mc, cap, v.scheme, 0, v.nt, extra);
                if (t.grid <= 0) continue;
                bool dup = false;
                for (const auto& u : out)
                    dup = dup || (u.bs == t.bs && u.mc == t.mc && u.scheme == t.scheme && u.nt == t.nt &&
                                  u.grid == t.grid && u.zchunk == t.zchunk && u.nseg == t.nseg);
                if (!dup) out.push_back(t);
            }
    }
    return out;
}
template std::vector<Tiling> tiling_candidates<float>(const Layout&);
template std::vector<Tiling> tiling_candidates<double>(const Layout&);
template Tiling choose_tiling<float>(const Layout&);
template Tiling choose_tiling<double>(const Layout&);

namespace {
std::atomic<int> g_periodic_pass{-1};
}
void set_periodic_pass(int form) { g_periodic_pass.store(form); }
int periodic_pass() { return g_periodic_pass.load(); }

template <typename T>
Tiling solve_tiling(const Layout& L, int periodic) {
    if (!periodic) return choose_tiling<T>(L);
    const int form = periodic_pass();
    if (form != 0 && ghost_layout_ok(L)) {
        // a 40-byte tiling recorded for this shape (autotuner, pb_set_tuning)
        // carries over to the periodic pass: the same block size, access
        // kind, workgroups per CU, segment count and z-chunk on the owned
        // range of the ghost-row layout
        Tiling rec{};
        bool have = false;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tuned.find(tune_key<T>(L));
            if (it != g_tuned.end()) {
                rec = it->second;
                have = true;
            }
        }
        if (have && rec.scheme == 1 && rec.grid > 0) {
            const DevInfo di = dev_info();
            const int cus = di.cus > 0 ? di.cus : 256;
            const int per_cu = (rec.grid + cus - 1) / cus;
            for (int extra = 0; extra <= kMaxExtraSegments; ++extra) {
                const Tiling t = choose_tiling_impl<T>(L, rec.bs, rec.mc, per_cu, 1, 1, rec.nt, extra);
                if (t.grid > 0 && t.nseg == rec.nseg && t.zchunk == rec.zchunk) return t;
            }
        }
    }
    Tiling t = choose_tiling_impl<T>(L, 0, 0, 0, form, 1);
    if (t.grid <= 0 && form >= 0) t = choose_tiling_impl<T>(L, 0, 0, 0, -1, 1);
    return t;
}
template Tiling solve_tiling<float>(const Layout&, int);
template Tiling solve_tiling<double>(const Layout&, int);

template <typename T>
int streaming_for(const Layout& L) {
    return streaming_default<T>(L);
}
template int streaming_for<float>(const Layout&);
template int streaming_for<double>(const Layout&);

template <typename T>
Tiling tiling_with(const Layout& L, int bs, int mc, int max_per_cu) {
    return choose_tiling_impl<T>(L, bs, mc, max_per_cu);
}
template Tiling tiling_with<float>(const Layout&, int, int, int);
template Tiling tiling_with<double>(const Layout&, int, int, int);

namespace {

// Into the ghost-row layout (ghost_layout): position q of plane k holds the
// node of row (q - org) / nx modulo ny of the plain layout's plane k (rows -2,
// -1 and ny, ny+1 are the ghost copies), or no node (zero couplings, unit
// diagonal, zero vectors). The operator is copied when gcx is given; the
// iteration vectors start at zero.
template <typename T>
__global__ void k_ghost_in(const T* __restrict__ cx, const T* __restrict__ cy, const T* __restrict__ cz,
                           const T* __restrict__ d, T* __restrict__ gcx, T* __restrict__ gcy, T* __restrict__ gcz,
                           T* __restrict__ gd, const T* __restrict__ b, const T* __restrict__ x, T* __restrict__ gb,
                           T* __restrict__ gx, T* __restrict__ gr, T* __restrict__ gr2, T* __restrict__ gp0,
                           T* __restrict__ gp1, int nx, int ny, int64_t sp, int64_t org, int64_t gsp, int64_t gnpad) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < gnpad;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = t / gsp, q = t - k * gsp;
        const int64_t rel = q - (org - 2 * (int64_t)nx);
        const bool in = rel >= 0 && rel < (int64_t)(ny + 4) * nx;
        int64_t src = 0;
        bool node = false;
        if (in) {
            const int64_t j = rel / nx - 2, i = rel % nx;
            node = j >= 0 && j < ny;
            src = k * sp + ((j + ny) % ny) * nx + i;
        }
        if (gcx) {
            gcx[t] = in ? cx[src] : T(0);
            gcy[t] = in ? cy[src] : T(0);
            gcz[t] = in ? cz[src] : T(0);
            gd[t] = in ? d[src] : T(1);
        }
        gb[t] = node ? b[src] : T(0);
        gx[t] = node ? x[src] : T(0);
        gr[t] = T(0);
        gr2[t] = T(0);
        gp0[t] = T(0);
        gp1[t] = T(0);
    }
}

// Back to the plain layout: x at the nodes, zero in the pad slots.
template <typename T>
__global__ void k_ghost_out(const T* __restrict__ gx, T* __restrict__ x, int64_t plane, int64_t sp, int64_t npad,
                            int64_t org, int64_t gsp) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < npad;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = t / sp, q = t - k * sp;
        x[t] = q < plane ? gx[k * gsp + org + q] : T(0);
    }
}

unsigned copy_grid(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 8192); }

}  // namespace

template <typename T>
pb_status fused_jpcg(const Layout& L, const SolveBufs<T>& s, SyncState* sync, double* partials, double tol,
                     int maxiter, hipStream_t st, SolveResult* res, const Tiling* force, int periodic) {
    const Tiling t = !periodic && force && force->grid > 0 ? *force : solve_tiling<T>(L, periodic);
    if (t.grid <= 0) {
        set_error("fused JPCG: no feasible tiling for this grid (nx too large for the in-plane halo)");
        return PB_ERR_ARG;
    }
    // the periodic 40-byte pass runs on ghost-row copies of the operator and
    // the state (the operator's copy is kept while the code words built from
    // it are valid)
    const bool gl = t.per && t.scheme == 1;
    GhostLayout G{};
    if (gl) {
        if (!s.gop.cx || !s.gop.cy || !s.gop.cz || !s.gop.d || !s.gb || !s.gx || !s.gr || !s.gr2 || !s.gp0 ||
            !s.gp1) {
            set_error("fused JPCG: the periodic 40-byte pass needs the ghost-row arrays of the workspace");
            return PB_ERR_ARG;
        }
        G = ghost_layout(L);
        const bool with_op = !s.codes_valid;
        hipLaunchKernelGGL(k_ghost_in<T>, dim3(copy_grid(G.npad)), dim3(256), 0, st, s.op.cx, s.op.cy, s.op.cz,
                           s.op.d, with_op ? (T*)s.gop.cx : nullptr, (T*)s.gop.cy, (T*)s.gop.cz, (T*)s.gop.d, s.b,
                           (const T*)s.x, s.gb, s.gx, s.gr, s.gr2, s.gp0, s.gp1, L.nx, L.ny, L.sp, G.org, G.sp,
                           G.npad);
        PB_HIP(hipGetLastError());
    }
    KernelFn fn = nullptr;
    for (const auto& v : variants<T>())
        if (!v.cd && v.bs == t.bs && v.mc == t.mc && v.scheme == t.scheme && v.per == t.per && v.nt == t.nt)
            fn = v.fn;
    if (!fn) {
        set_error("fused JPCG: unknown kernel variant bs=%d mc=%d scheme=%d periodic=%d streaming=%d", t.bs, t.mc,
                  t.scheme, t.per, t.nt);
        return PB_ERR_ARG;
    }
    const DevInfo di = dev_info();
    // Coded coefficients (40-byte FP32 pass): the same tiling with the
    // operator read as code words, when the operator's values fit the
    // dictionary and the coded kernel keeps the grid co-resident. The code
    // words go to q2 and the dictionary to q, which this pass form leaves
    // unused.
    size_t lds = t.lds;
    const float* cw = nullptr;
    const float* ctab = nullptr;
    int coded = 0;
    if constexpr (sizeof(T) == 4) {
        if (t.scheme == 1 && coded_coefficients() && s.q && (gl ? s.gcodes != nullptr : s.q2 != nullptr) &&
            coded_layout_ok(L) && (!gl || G.sp < ((int64_t)1 << 29))) {
            KernelFn cfn = nullptr;
            for (const auto& v : variants<T>())
                if (v.cd && v.bs == t.bs && v.mc == t.mc && v.per == t.per && v.nt == t.nt) cfn = v.fn;
            const size_t clds = t.lds + kCodedLdsBytes;
            const int cus = di.cus > 0 ? di.cus : 256;
            if (cfn && (int64_t)max_coresident(cfn, t.bs, clds) * cus >= t.grid) {
                bool fits = s.codes_valid != 0;
                const float* tab = s.ctab;
                uint32_t* words = gl ? s.gcodes : (uint32_t*)s.q2;
                if (!fits) {
                    const pb_status e = gl ? build_codes(s.gop, G.npad, (void*)s.q, words, st, fits, &tab)
                                           : build_codes(s.op, L.npad, (void*)s.q, words, st, fits, &tab);
                    if (e != PB_OK) return e;
                }
                if (fits) {
                    fn = cfn;
                    lds = clds;
                    cw = (const float*)words;
                    ctab = tab;
                    coded = 1;
                }
            }
        }
    }
    KArgs<T> a{};
    a.op = s.op;
    a.b = s.b;
    a.x = s.x;
    a.r[0] = s.r;
    a.r[1] = s.r2;
    a.q[0] = s.q;
    a.q[1] = s.q2;
    a.p[0] = s.p0;
    a.p[1] = s.p1;
    a.nx = L.nx; a.ny = L.ny; a.nz = L.nz;
    a.sp = L.sp;
    a.org = 0;
    a.own = L.sp;
    a.oend = L.sp;
    if (gl) {
        a.op = s.gop;
        a.b = s.gb;
        a.x = s.gx;
        a.r[0] = s.gr;
        a.r[1] = s.gr2;
        a.p[0] = s.gp0;
        a.p[1] = s.gp1;
        a.sp = G.sp;
        a.org = G.org;
        a.own = G.own;
        a.oend = G.org + L.plane;
    }
    a.seglen = t.seglen; a.zchunk = t.zchunk; a.nseg = t.nseg; a.nzc = t.nzc; a.ntiles = t.ntiles;
    a.halo = t.halo;
    a.tol = tol;
    a.maxiter = maxiter;
    a.warm = s.warm;
    a.S = sync;
    a.partials = partials;
    a.cw = cw;
    a.ctab = ctab;
    // every wait is bounded: 20 s of the constant-rate clock
    a.timeout_ticks = (long long)(di.wallclock_khz > 0 ? di.wallclock_khz : 100000) * 1000LL * 20LL;
    // the header (barrier counters, scalars) starts cleared
    if (launch_fill<int>((int*)sync, (int64_t)(sizeof(SyncState) / sizeof(int)), 0, st) != PB_OK)
        return PB_ERR_HIP;
    void* args[] = {&a};
    hipEvent_t ev[2] = {nullptr, nullptr};
    const bool timed = res && !res->untimed;
    if (timed) {
        PB_HIP(hipEventCreate(&ev[0]));
        PB_HIP(hipEventCreate(&ev[1]));
        PB_HIP(hipEventRecord(ev[0], st));
    }
    const hipError_t e = hipLaunchCooperativeKernel(fn, dim3(t.grid), dim3(t.bs), args, lds, st);
    if (e != hipSuccess) {
        if (ev[0]) (void)hipEventDestroy(ev[0]);
        if (ev[1]) (void)hipEventDestroy(ev[1]);
        set_error("fused JPCG launch failed: %s (grid %d, block %d, lds %zu, coded %d)", hipGetErrorString(e),
                  t.grid, t.bs, lds, coded);
        return PB_ERR_HIP;
    }
    if (timed) PB_HIP(hipEventRecord(ev[1], st));
    if (gl) {
        hipLaunchKernelGGL(k_ghost_out<T>, dim3(copy_grid(L.npad)), dim3(256), 0, st, (const T*)s.gx, s.x, L.plane,
                           L.sp, L.npad, G.org, G.sp);
        PB_HIP(hipGetLastError());
    }
    if (res) {
        SyncState h;
        PB_HIP(hipMemcpyAsync(&h, sync, sizeof(SyncState), hipMemcpyDeviceToHost, st));
        PB_HIP(hipStreamSynchronize(st));
        float ms = 0.0f;
        if (timed) {
            PB_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
            (void)hipEventDestroy(ev[0]);
            (void)hipEventDestroy(ev[1]);
        }
        res->status = h.status;
        res->iters = h.iters;
        res->rr = h.rr;
        res->bb = h.bb;
        res->kernel_seconds = 1e-3 * ms;
        res->tiling = t;
        res->coded = coded;
        res->ctab = ctab;
    }
    return PB_OK;
}

// ------------------------------------------------------------------ coded-coefficient switch

namespace {
std::atomic<int> g_coded{1};
}
void set_coded_coefficients(int on) { g_coded.store(on ? 1 : 0); }
int coded_coefficients() { return g_coded.load(); }
template pb_status fused_jpcg<float>(const Layout&, const SolveBufs<float>&, SyncState*, double*, double, int,
                                     hipStream_t, SolveResult*, const Tiling*, int);

// ------------------------------------------------------------------ batch support

namespace {
constexpr int kBatchBS = 256;
constexpr int kBatchMC = 1;
constexpr int kBatchZ = 32;   // default z-chunk; pb_batch_autotune / pb_batch_set_zchunk change it per device
constexpr int kBatchScheme = 1;
constexpr bool kBatchNT = false;
// coded: 0 uncoded, 1 coded (every problem fits), 2 coded where each problem's fit flag says so.
template <typename T>
KernelFn batch_kernel(int coded = 0) {
    if constexpr (sizeof(T) == 4) {
        if (coded == 1) return (KernelFn)k_jpcg_batch<float, kBatchBS, kBatchMC, kBatchScheme, kBatchNT, true>;
        if (coded == 2) return (KernelFn)k_jpcg_batch<float, kBatchBS, kBatchMC, kBatchScheme, kBatchNT, true, true>;
    }
    return (KernelFn)k_jpcg_batch<T, kBatchBS, kBatchMC, kBatchScheme, kBatchNT>;
}
}  // namespace

// The batched and served kernels' z-chunk, per device.
std::map<int, int> g_batch_z;

int batch_zchunk() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_batch_z.find(dev);
    return it == g_batch_z.end() ? kBatchZ : it->second;
}

void set_batch_zchunk(int z) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_batch_z[dev] = z;
}

// Tiling used for a problem inside a batch: a fixed kernel variant and the
// device's batch z-chunk, so under one setting it depends on the problem's
// shape alone (the same problem gives bitwise the same result alone and in
// any mix). grid is left 0.
template <typename T>
Tiling batch_tiling(const Layout& L, int zchunk) {
    constexpr int W = Vec<T>::n;
    Tiling t{};
    t.bs = kBatchBS;
    t.mc = kBatchMC;
    t.seglen = balanced_seglen<T>(L, kBatchMC * kBatchBS * W);
    t.halo = halo_for<T>(L.nx);
    if (2 * t.halo / W > kBatchBS) return t;   // infeasible: ntiles stays 0
    t.zchunk = zchunk > 0 ? zchunk : batch_zchunk();
    t.nseg = (int)((L.sp + t.seglen - 1) / t.seglen);
    t.nzc = (L.nz + t.zchunk - 1) / t.zchunk;
    t.ntiles = t.nseg * t.nzc;
    t.scheme = kBatchScheme;
    t.nt = kBatchNT ? 1 : 0;
    t.lds = lds_bytes<T>(kBatchScheme, t.seglen, t.halo);
    return t;
}
template Tiling batch_tiling<float>(const Layout&, int);
template Tiling batch_tiling<double>(const Layout&, int);

template <typename T>
size_t batch_kargs_bytes() {
    return sizeof(KArgs<T>);
}
template size_t batch_kargs_bytes<float>();
template size_t batch_kargs_bytes<double>();

// Host-side record of one problem's kernel arguments (written to `dst`).
template <typename T>
void batch_fill_kargs(void* dst, const Layout& L, const SolveBufs<T>& s, SyncState* S, double* partials,
                      const Tiling& t, double tol, int maxiter, int resume, int chunk, const float* cw,
                      const float* ctab, const int* fit) {
    const DevInfo di = dev_info();
    KArgs<T> a{};
    a.op = s.op;
    a.b = s.b;
    a.x = s.x;
    a.r[0] = s.r; a.r[1] = s.r2;
    a.q[0] = s.q; a.q[1] = s.q2;
    a.p[0] = s.p0; a.p[1] = s.p1;
    a.nx = L.nx; a.ny = L.ny; a.nz = L.nz;
    a.sp = L.sp;
    a.org = 0;
    a.own = L.sp;
    a.oend = L.sp;
    a.seglen = t.seglen; a.zchunk = t.zchunk; a.nseg = t.nseg; a.nzc = t.nzc; a.ntiles = t.ntiles;
    a.halo = t.halo;
    a.tol = tol;
    a.maxiter = maxiter;
    a.warm = s.warm;
    a.resume = resume;
    a.chunk = chunk;
    a.S = S;
    a.partials = partials;
    a.timeout_ticks = (long long)(di.wallclock_khz > 0 ? di.wallclock_khz : 100000) * 1000LL * 20LL;
    a.cw = cw;
    a.ctab = ctab;
    a.fit = fit;
    std::memcpy(dst, &a, sizeof(a));
}
template void batch_fill_kargs<float>(void*, const Layout&, const SolveBufs<float>&, SyncState*, double*,
                                      const Tiling&, double, int, int, int, const float*, const float*,
                                      const int*);
template void batch_fill_kargs<double>(void*, const Layout&, const SolveBufs<double>&, SyncState*, double*,
                                       const Tiling&, double, int, int, int, const float*, const float*,
                                       const int*);

// Co-resident workgroups of the batch kernel with `lds` bytes of dynamic LDS.
template <typename T>
int batch_capacity(size_t lds, int coded) {
    const DevInfo di = dev_info();
    const int per_cu = max_coresident(batch_kernel<T>(coded), kBatchBS, lds);
    return per_cu * (di.cus > 0 ? di.cus : 256);
}
template int batch_capacity<float>(size_t, int);
template int batch_capacity<double>(size_t, int);

template <typename T>
__global__ void k_reset_arrivals(const KArgs<T>* __restrict__ probs, int nprob) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nprob * 8) probs[i / 8].S->arrive[i % 8][0] = 0u;
}

// Clear the arrival counters of every problem in a device argument table
// (needed before a launch that resumes problems whose state is kept).
template <typename T>
pb_status batch_reset_arrivals(const void* d_kargs, int nprob, hipStream_t st) {
    hipLaunchKernelGGL(k_reset_arrivals<T>, dim3((nprob * 8 + 255) / 256), dim3(256), 0, st,
                       (const KArgs<T>*)d_kargs, nprob);
    PB_HIP(hipGetLastError());
    return PB_OK;
}
template pb_status batch_reset_arrivals<float>(const void*, int, hipStream_t);
template pb_status batch_reset_arrivals<double>(const void*, int, hipStream_t);

template <typename T>
__global__ void k_state_digests(const KArgs<T>* __restrict__ probs, int nprob, StateDigest* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nprob) return;
    const SyncState* S = probs[i].S;
    StateDigest d;
    d.rr = S->rr;
    d.bb = S->bb;
    d.iters = S->iters;
    d.done = S->done;
    d.status = S->status;
    d.pad = 0;
    out[i] = d;
}

template <typename T>
pb_status batch_state_digests(const void* d_kargs, int nprob, StateDigest* out, hipStream_t st) {
    hipLaunchKernelGGL(k_state_digests<T>, dim3((nprob + 255) / 256), dim3(256), 0, st, (const KArgs<T>*)d_kargs,
                       nprob, out);
    PB_HIP(hipGetLastError());
    return PB_OK;
}
template pb_status batch_state_digests<float>(const void*, int, StateDigest*, hipStream_t);
template pb_status batch_state_digests<double>(const void*, int, StateDigest*, hipStream_t);

template <typename T>
pb_status batch_launch(const void* d_kargs, const int* d_first, int nprob, int grid, size_t lds, hipStream_t st,
                       bool cooperative, int coded) {
    const KArgs<T>* kp = (const KArgs<T>*)d_kargs;
    void* args[] = {&kp, &d_first, &nprob};
    hipError_t e;
    if (cooperative)
        e = hipLaunchCooperativeKernel(batch_kernel<T>(coded), dim3(grid), dim3(kBatchBS), args, lds, st);
    else
        e = hipLaunchKernel(batch_kernel<T>(coded), dim3(grid), dim3(kBatchBS), args, lds, st);
    if (e != hipSuccess) {
        set_error("batch JPCG launch failed: %s (grid %d, lds %zu)", hipGetErrorString(e), grid, lds);
        return PB_ERR_HIP;
    }
    return PB_OK;
}
template pb_status batch_launch<float>(const void*, const int*, int, int, size_t, hipStream_t, bool, int);
template pb_status batch_launch<double>(const void*, const int*, int, int, size_t, hipStream_t, bool, int);
template pb_status fused_jpcg<double>(const Layout&, const SolveBufs<double>&, SyncState*, double*, double, int,
                                      hipStream_t, SolveResult*, const Tiling*, int);

}  // namespace pb
