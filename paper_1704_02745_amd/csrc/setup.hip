// System setup on the GPU (section 2.7 of the paper; Eq. 3 right-hand side).
//
// This file is compiled with -ffp-contract=off: the node classification,
// the edge means and the charge weights must round exactly as the plain
// (unfused) arithmetic they are defined by.
#include "solver.hpp"

#include <cmath>
#include <vector>

namespace pb {

namespace {

constexpr double kFourPi = 12.566370614359172;   // 4*pi rounded to double
constexpr double kCoulombKcal = 332.0637133;     // e^2/(4 pi eps0), kcal A/mol
constexpr int kMaxAtoms = (1 << 21) - 1;          // pair id = 8*atom + corner < 2^24
constexpr double kPeriodicMaxIndex = 268435456.0;  // 2^28: bound on |(c - o)/h| with the periodic boundary

__global__ void k_fill_u8(uint8_t* p, int64_t n, uint8_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_i32(int* p, int64_t n, int v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// Node classification: one workgroup per atom walks the atom's bounding
// window of padded nodes and marks the ones strictly inside the sphere.
// Concurrent writers only ever store 1, so the result is order independent.
__global__ void k_classify(const double* __restrict__ xyz, const double* __restrict__ radius,
                           int64_t natoms, int nx, int ny, int nz, double h,
                           double ox, double oy, double oz, int per, uint8_t* __restrict__ mask) {
    const int64_t a = blockIdx.x;
    if (a >= natoms) return;
    const double cx = xyz[3 * a], cy = xyz[3 * a + 1], cz = xyz[3 * a + 2];
    const double r = radius[a];
    const double rr = r * r;
    const double o[3] = {ox, oy, oz};
    const double c[3] = {cx, cy, cz};
    const int n3[3] = {nx, ny, nz};
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        double l = floor((c[d] - r - o[d]) / h) - 1.0;
        double u = ceil((c[d] + r - o[d]) / h) + 1.0;
        if (per) {
            // periodic: the unwrapped window around the sphere (the nodes it
            // covers are marked at their wrapped index)
            if (!(fabs(l) < kPeriodicMaxIndex && fabs(u) < kPeriodicMaxIndex)) return;
        } else {
            l = fmin(fmax(l, -1.0), (double)n3[d]);
            u = fmin(fmax(u, -1.0), (double)n3[d]);
        }
        lo[d] = (int)l;
        hi[d] = (int)u;   // inclusive
    }
    const int wx = hi[0] - lo[0] + 1, wy = hi[1] - lo[1] + 1, wz = hi[2] - lo[2] + 1;
    if (wx <= 0 || wy <= 0 || wz <= 0) return;
    const int64_t total = (int64_t)wx * wy * wz;
    const int64_t px = nx + 2, py = ny + 2;
    for (int64_t t = threadIdx.x; t < total; t += blockDim.x) {
        const int i = lo[0] + (int)(t % wx);
        const int j = lo[1] + (int)((t / wx) % wy);
        const int k = lo[2] + (int)(t / ((int64_t)wx * wy));
        const double x = ox + h * (double)i;
        const double y = oy + h * (double)j;
        const double z = oz + h * (double)k;
        const double dx = x - cx, dy = y - cy, dz = z - cz;
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 < rr) {
            if (per) {
                const int iw = ((i % nx) + nx) % nx, jw = ((j % ny) + ny) % ny, kw = ((k % nz) + nz) % nz;
                mask[(iw + 1) + px * ((jw + 1) + py * (int64_t)(kw + 1))] = 1;
            } else {
                mask[(i + 1) + px * ((j + 1) + py * (int64_t)(k + 1))] = 1;
            }
        }
    }
}

// Periodic: fill the ghost layer of the padded mask with the wrapped nodes,
// one axis at a time (x, then y over whole padded rows, then z over whole
// padded planes) so edges and corners wrap too.
__global__ void k_wrap_ghosts(uint8_t* __restrict__ m, int nx, int ny, int nz, int axis) {
    const int64_t px = nx + 2, py = ny + 2, pz = nz + 2;
    const int64_t n = axis == 0 ? (int64_t)ny * nz : axis == 1 ? px * nz : px * py;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        if (axis == 0) {
            const int64_t j = 1 + t % ny, k = 1 + t / ny;
            uint8_t* row = m + px * (j + py * k);
            row[0] = row[nx];
            row[nx + 1] = row[1];
        } else if (axis == 1) {
            const int64_t i = t % px, k = 1 + t / px;
            uint8_t* col = m + i + px * py * k;
            col[0] = col[px * ny];
            col[px * (ny + 1)] = col[px];
        } else {
            const int64_t i = t % px, j = t / px;
            uint8_t* line = m + i + px * j;
            line[0] = line[px * py * nz];
            line[px * py * (pz - 1)] = line[px * py];
        }
    }
}

__device__ __forceinline__ double node_eps(uint8_t m, double ein, double eout) {
    return m ? ein : eout;
}

__device__ __forceinline__ double harmonic(double a, double b) {
    return 2.0 * a * b / (a + b);
}

// Staggered edge dielectrics and the salt term, one thread per element.
__global__ void k_edges(const uint8_t* __restrict__ mask, int nx, int ny, int nz,
                        double ein, double eout, double kbar2,
                        double* __restrict__ ex, double* __restrict__ ey,
                        double* __restrict__ ez, double* __restrict__ k2) {
    const int64_t px = nx + 2, py = ny + 2;
    const int64_t nex = (int64_t)(nx + 1) * ny * nz;
    const int64_t ney = (int64_t)nx * (ny + 1) * nz;
    const int64_t nez = (int64_t)nx * ny * (nz + 1);
    const int64_t nn = (int64_t)nx * ny * nz;
    const int64_t total = nex + ney + nez + nn;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        if (t < nex) {
            const int64_t e = t % (nx + 1);
            const int64_t j = (t / (nx + 1)) % ny;
            const int64_t k = t / ((int64_t)(nx + 1) * ny);
            const int64_t base = px * ((j + 1) + py * (k + 1));
            ex[t] = harmonic(node_eps(mask[base + e], ein, eout), node_eps(mask[base + e + 1], ein, eout));
        } else if (t < nex + ney) {
            const int64_t u = t - nex;
            const int64_t i = u % nx;
            const int64_t e = (u / nx) % (ny + 1);
            const int64_t k = u / ((int64_t)nx * (ny + 1));
            const int64_t a = (i + 1) + px * (e + py * (k + 1));
            ey[u] = harmonic(node_eps(mask[a], ein, eout), node_eps(mask[a + px], ein, eout));
        } else if (t < nex + ney + nez) {
            const int64_t u = t - nex - ney;
            const int64_t i = u % nx;
            const int64_t j = (u / nx) % ny;
            const int64_t e = u / ((int64_t)nx * ny);
            const int64_t a = (i + 1) + px * ((j + 1) + py * e);
            ez[u] = harmonic(node_eps(mask[a], ein, eout), node_eps(mask[a + px * py], ein, eout));
        } else {
            const int64_t u = t - nex - ney - nez;
            const int64_t i = u % nx;
            const int64_t j = (u / nx) % ny;
            const int64_t k = u / ((int64_t)nx * ny);
            const uint8_t m = mask[(i + 1) + px * ((j + 1) + py * (k + 1))];
            k2[u] = m ? 0.0 : kbar2;
        }
    }
}

// ---------------------------------------------------------------- fractional edges
//
// Weighted harmonic edge dielectric 1/(f/eps_in + (1-f)/eps_out), f the
// fraction of the edge segment inside the union of the spheres. Atoms are
// binned into cells of m*h (m = ceil(R_max/h)) over the padded node range;
// each edge visits the cells within R_max of its segment, clips each
// sphere's chord to [0,1] and keeps the union as a sorted list of disjoint
// segments (intervals that overlap or touch merge), whose lengths are summed
// in increasing order.
constexpr int kMaxSegments = 16;
// The device path of the fractional model is switched off: its first device
// run ended in a memory fault whose cause is not yet found (the same kernel
// text compiled for the host stays in bounds and matches the FP64 model bit
// for bit). pb_setup_ex refuses PB_EDGE_FRACTION while this is false.
constexpr bool kFractionEdgesEnabled = false;

__global__ __launch_bounds__(1024) void k_max_radius(const double* __restrict__ r, int64_t n, double* __restrict__ out) {
    __shared__ double s[1024];
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) m = fmax(m, r[i]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

__device__ __forceinline__ int padded_cell(double c, double o, double h, int n, int m) {
    double g = floor((c - o) / h) + 1.0;
    g = fmin(fmax(g, 0.0), (double)(n + 1));
    return (int)g / m;
}

// key = cell << 24 | atom (cells in x-fastest order over the padded nodes)
__global__ void k_cell_keys(const double* __restrict__ xyz, int64_t natoms, int nx, int ny, int nz, double h,
                            double ox, double oy, double oz, int m, int ncx, int ncy, uint64_t* __restrict__ keys) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= natoms) return;
    const int cx = padded_cell(xyz[3 * a], ox, h, nx, m);
    const int cy = padded_cell(xyz[3 * a + 1], oy, h, ny, m);
    const int cz = padded_cell(xyz[3 * a + 2], oz, h, nz, m);
    const uint64_t cell = (uint64_t)cx + (uint64_t)ncx * ((uint64_t)cy + (uint64_t)ncy * (uint64_t)cz);
    keys[a] = (cell << 24) | (uint64_t)a;
}

// first/last+1 sorted position of each cell's atoms (cells start empty)
__global__ void k_cell_bounds(const uint64_t* __restrict__ keys, int64_t natoms, int* __restrict__ start,
                              int* __restrict__ end) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= natoms) return;
    const uint64_t c = keys[p] >> 24;
    if (p == 0 || (keys[p - 1] >> 24) != c) start[c] = (int)p;
    if (p == natoms - 1 || (keys[p + 1] >> 24) != c) end[c] = (int)(p + 1);
}

__global__ void k_edges_fraction(const double* __restrict__ xyz, const double* __restrict__ radius,
                                 const uint64_t* __restrict__ keys, const int* __restrict__ cstart,
                                 const int* __restrict__ cend, int nx, int ny, int nz, double h, double ox, double oy,
                                 double oz, double rmax, int m, int ncx, int ncy, int ncz, double ein, double eout,
                                 double* __restrict__ ex, double* __restrict__ ey, double* __restrict__ ez,
                                 int* __restrict__ flags) {
    const int64_t nex = (int64_t)(nx + 1) * ny * nz;
    const int64_t ney = (int64_t)nx * (ny + 1) * nz;
    const int64_t nez = (int64_t)nx * ny * (nz + 1);
    const int64_t total = nex + ney + nez;
    const double o[3] = {ox, oy, oz};
    const int n3[3] = {nx, ny, nz};
    const int nc[3] = {ncx, ncy, ncz};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        int axis, idx[3];
        double* outp;
        if (t < nex) {
            axis = 0;
            idx[0] = (int)(t % (nx + 1)) - 1; idx[1] = (int)((t / (nx + 1)) % ny); idx[2] = (int)(t / ((int64_t)(nx + 1) * ny));
            outp = ex + t;
        } else if (t < nex + ney) {
            const int64_t u = t - nex;
            axis = 1;
            idx[0] = (int)(u % nx); idx[1] = (int)((u / nx) % (ny + 1)) - 1; idx[2] = (int)(u / ((int64_t)nx * (ny + 1)));
            outp = ey + u;
        } else {
            const int64_t u = t - nex - ney;
            axis = 2;
            idx[0] = (int)(u % nx); idx[1] = (int)((u / nx) % ny); idx[2] = (int)(u / ((int64_t)nx * ny)) - 1;
            outp = ez + u;
        }
        double p[3];
        for (int d = 0; d < 3; ++d) p[d] = o[d] + h * (double)idx[d];   // the edge's first node
        int clo[3], chi[3];
        for (int d = 0; d < 3; ++d) {
            const double lo = p[d] - rmax, hi = p[d] + (d == axis ? h : 0.0) + rmax;
            clo[d] = padded_cell(lo, o[d], h, n3[d], m);
            chi[d] = min(padded_cell(hi, o[d], h, n3[d], m), nc[d] - 1);
        }
        double s0[kMaxSegments], s1[kMaxSegments];
        int ns = 0;
        bool overflow = false;
        for (int cz = clo[2]; cz <= chi[2]; ++cz)
            for (int cy = clo[1]; cy <= chi[1]; ++cy)
                for (int cx = clo[0]; cx <= chi[0]; ++cx) {
                    const int64_t cell = (int64_t)cx + (int64_t)ncx * ((int64_t)cy + (int64_t)ncy * cz);
                    for (int q = cstart[cell]; q < cend[cell]; ++q) {
                        const int64_t a = (int64_t)(keys[q] & 0xFFFFFFull);
                        const double c[3] = {xyz[3 * a], xyz[3 * a + 1], xyz[3 * a + 2]};
                        const double R = radius[a];
                        const double RR = R * R;
                        double d2 = 0.0;
                        for (int d = 0; d < 3; ++d) {
                            if (d == axis) continue;
                            const double dd = p[d] - c[d];
                            d2 = d2 + dd * dd;
                        }
                        if (!(d2 < RR)) continue;
                        const double w = sqrt(RR - d2);
                        double t0 = ((c[axis] - w) - p[axis]) / h;
                        double t1 = ((c[axis] + w) - p[axis]) / h;
                        t0 = fmax(t0, 0.0);
                        t1 = fmin(t1, 1.0);
                        if (!(t1 > t0)) continue;
                        // insert into the sorted disjoint union (merge what overlaps or touches)
                        int i = 0;
                        while (i < ns && s1[i] < t0) ++i;          // segments entirely before
                        int j = i;
                        double a0 = t0, a1 = t1;
                        while (j < ns && s0[j] <= a1) {            // segments touching [a0, a1]
                            a0 = fmin(a0, s0[j]);
                            a1 = fmax(a1, s1[j]);
                            ++j;
                        }
                        const int removed = j - i;
                        if (removed == 0) {
                            if (ns == kMaxSegments) { overflow = true; continue; }
                            for (int k = ns; k > i; --k) { s0[k] = s0[k - 1]; s1[k] = s1[k - 1]; }
                            ++ns;
                        } else if (removed > 1) {
                            for (int k = i + 1; k + removed - 1 < ns; ++k) {
                                s0[k] = s0[k + removed - 1];
                                s1[k] = s1[k + removed - 1];
                            }
                            ns -= removed - 1;
                        }
                        s0[i] = a0;
                        s1[i] = a1;
                    }
                }
        if (overflow) atomicOr(flags, 4);
        double f = 0.0;
        for (int i = 0; i < ns; ++i) f = f + (s1[i] - s0[i]);
        *outp = (f == 0.0) ? eout : (f == 1.0) ? ein : 1.0 / (f / ein + (1.0 - f) / eout);
    }
}

// Trilinear cell of one atom along one axis: i0 = clamp(floor(g), 0, n-2),
// f = g - i0. Periodic: i0 = floor(g) mod n, f = g - floor(g) (the second
// node of the cell is (i0 + 1) mod n).
__device__ __forceinline__ bool cell_axis(double c, double o, double h, int n, int per, int& i0, double& f) {
    const double g = (c - o) / h;
    if (per) {
        if (!(fabs(g) < kPeriodicMaxIndex)) return false;
        const double fl = floor(g);
        f = g - fl;
        const long long w = (long long)fl % n;
        i0 = (int)(w < 0 ? w + n : w);
        return true;
    }
    if (!(g >= 0.0) || !(g <= (double)(n - 1))) return false;
    double fl = floor(g);
    fl = fmin(fmax(fl, 0.0), (double)(n - 2));
    i0 = (int)fl;
    f = g - fl;
    return true;
}

// Node index of corner c (bit 0: +x, bit 1: +y, bit 2: +z) of a cell.
__device__ __forceinline__ int64_t corner_node(int i0, int j0, int k0, int c, int nx, int ny, int nz) {
    int i = i0 + (c & 1), j = j0 + ((c >> 1) & 1), k = k0 + ((c >> 2) & 1);
    if (i == nx) i = 0;   // only reached with the periodic cell
    if (j == ny) j = 0;
    if (k == nz) k = 0;
    return (int64_t)i + (int64_t)nx * ((int64_t)j + (int64_t)ny * k);
}

// Charge spreading, step 1: one sort key per (atom, corner) pair,
// key = node_index << 24 | (8*atom + corner). Sorting the keys groups the
// contributions of each node in increasing atom order.
__global__ void k_spread_keys(const double* __restrict__ xyz, int64_t natoms, int nx, int ny, int nz,
                              double h, double ox, double oy, double oz, int per,
                              uint64_t* __restrict__ keys, int* __restrict__ flags) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= 8 * natoms) return;
    const int64_t a = p >> 3;
    const int c = (int)(p & 7);
    int i0, j0, k0;
    double fx, fy, fz;
    bool ok = cell_axis(xyz[3 * a], ox, h, nx, per, i0, fx);
    ok = cell_axis(xyz[3 * a + 1], oy, h, ny, per, j0, fy) && ok;
    ok = cell_axis(xyz[3 * a + 2], oz, h, nz, per, k0, fz) && ok;
    if (!ok) {
        atomicOr(flags, 1);
        keys[p] = ~0ull;
        return;
    }
    const int64_t node = corner_node(i0, j0, k0, c, nx, ny, nz);
    keys[p] = ((uint64_t)node << 24) | (uint64_t)p;
}

// One compare-exchange step of a bitonic sorting network (ascending).
__global__ void k_bitonic_step(uint64_t* __restrict__ a, int64_t n, int64_t j, int64_t k) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t l = i ^ j;
    if (l > i) {
        const uint64_t x = a[i], y = a[l];
        const bool up = (i & k) == 0;
        if ((x > y) == up) {
            a[i] = y;
            a[l] = x;
        }
    }
}

// The steps of the same network whose pairs lie within one aligned chunk of
// kSortChunk keys (j < kSortChunk), in LDS: block b sorts chunk b through
// stages k_first..k_last (powers of two), starting stage k_first at j_first.
// The keys are distinct, so any correct sort leaves the same order.
constexpr int kSortChunk = 2048;
__global__ __launch_bounds__(1024) void k_bitonic_local(uint64_t* __restrict__ a, int64_t n, int64_t k_first,
                                                        int64_t k_last, int64_t j_first) {
    __shared__ uint64_t s[kSortChunk];
    const int chunk = (int)min<int64_t>(n, kSortChunk);
    const int64_t base = (int64_t)blockIdx.x * chunk;
    for (int e = threadIdx.x; e < chunk; e += blockDim.x) s[e] = a[base + e];
    __syncthreads();
    for (int64_t k = k_first; k <= k_last; k <<= 1) {
        for (int64_t j = (k == k_first) ? j_first : (k >> 1); j > 0; j >>= 1) {
            for (int e = threadIdx.x; e < chunk; e += blockDim.x) {
                const int le = e ^ (int)j;
                if (le > e) {
                    const uint64_t x = s[e], y = s[le];
                    const bool up = ((base + e) & k) == 0;
                    if ((x > y) == up) {
                        s[e] = y;
                        s[le] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int e = threadIdx.x; e < chunk; e += blockDim.x) a[base + e] = s[e];
}

// Charge spreading, step 2: the first key of each node's run sums the run in
// key order (increasing atom index), starting from zero, and stores q_node.
__global__ void k_spread_sum(const uint64_t* __restrict__ keys, int64_t npairs,
                             const double* __restrict__ xyz, const double* __restrict__ charge,
                             int nx, int ny, int nz, double h, double ox, double oy, double oz, int per,
                             double* __restrict__ q) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npairs) return;
    const uint64_t key = keys[i];
    if (key == ~0ull) return;
    const uint64_t node = key >> 24;
    if (i > 0 && (keys[i - 1] >> 24) == node) return;
    double s = 0.0;
    for (int64_t t = i; t < npairs; ++t) {
        const uint64_t kt = keys[t];
        if (kt == ~0ull || (kt >> 24) != node) break;
        const int64_t p = (int64_t)(kt & 0xFFFFFFull);
        const int64_t a = p >> 3;
        const int c = (int)(p & 7);
        int i0, j0, k0;
        double fx, fy, fz;
        cell_axis(xyz[3 * a], ox, h, nx, per, i0, fx);
        cell_axis(xyz[3 * a + 1], oy, h, ny, per, j0, fy);
        cell_axis(xyz[3 * a + 2], oz, h, nz, per, k0, fz);
        const double wx = (c & 1) ? fx : 1.0 - fx;
        const double wy = (c & 2) ? fy : 1.0 - fy;
        const double wz = (c & 4) ? fz : 1.0 - fz;
        s = s + charge[a] * wx * wy * wz;
    }
    q[node] = s;
}

// Ghost point `t` of the six faces (x-, x+, y-, y+, z-, z+), in that order;
// within a face the faster index comes first (y then z, x then z, x then y).
__device__ __forceinline__ void ghost_point(int64_t t, int nx, int ny, int nz, double h,
                                            double ox, double oy, double oz,
                                            double& px, double& py, double& pz) {
    const int64_t fx = (int64_t)ny * nz, fy = (int64_t)nx * nz;
    if (t < 2 * fx) {
        const int side = t >= fx;
        const int64_t u = t - side * fx;
        px = ox + h * (side ? (double)nx : -1.0);
        py = oy + h * (double)(u % ny);
        pz = oz + h * (double)(u / ny);
    } else if (t < 2 * fx + 2 * fy) {
        const int64_t v = t - 2 * fx;
        const int side = v >= fy;
        const int64_t u = v - side * fy;
        px = ox + h * (double)(u % nx);
        py = oy + h * (side ? (double)ny : -1.0);
        pz = oz + h * (double)(u / nx);
    } else {
        const int64_t fz = (int64_t)nx * ny;
        const int64_t v = t - 2 * fx - 2 * fy;
        const int side = v >= fz;
        const int64_t u = v - side * fz;
        px = ox + h * (double)(u % nx);
        py = oy + h * (double)(u / nx);
        pz = oz + h * (side ? (double)nz : -1.0);
    }
}

// Debye-Hueckel potential on the face ghosts: each thread owns one ghost
// point and sums over all atoms in index order; atoms are staged in LDS.
// This is the arithmetic-bound part of setup (6 n^2 points x natoms terms).
constexpr int kDhBlock = 256;
// 1/sqrt(r2) for r2 > 0: the hardware estimate and two Newton steps,
// y <- y (1 + (1 - r2 y^2)/2), each roughly doubling the correct bits.
__device__ __forceinline__ double rsqrt_nr(double r2) {
    // the hardware estimate, then two Newton steps y += y (1/2 - (r2/2) y^2)
    const double h = 0.5 * r2;
    double y = __builtin_amdgcn_rsq(r2);
    y = fma(y, fma(-(h * y), y, 0.5), y);
    y = fma(y, fma(-(h * y), y, 0.5), y);
    return y;
}

// 2^(j/64), j = 0..63, each the double nearest to the exact value.
constexpr int kExpTab = 64;
__constant__ double kExp2Frac[kExpTab] = {
    0x1.0000000000000p+0, 0x1.02c9a3e778061p+0, 0x1.059b0d3158574p+0, 0x1.0874518759bc8p+0,
    0x1.0b5586cf9890fp+0, 0x1.0e3ec32d3d1a2p+0, 0x1.11301d0125b51p+0, 0x1.1429aaea92de0p+0,
    0x1.172b83c7d517bp+0, 0x1.1a35beb6fcb75p+0, 0x1.1d4873168b9aap+0, 0x1.2063b88628cd6p+0,
    0x1.2387a6e756238p+0, 0x1.26b4565e27cddp+0, 0x1.29e9df51fdee1p+0, 0x1.2d285a6e4030bp+0,
    0x1.306fe0a31b715p+0, 0x1.33c08b26416ffp+0, 0x1.371a7373aa9cbp+0, 0x1.3a7db34e59ff7p+0,
    0x1.3dea64c123422p+0, 0x1.4160a21f72e2ap+0, 0x1.44e086061892dp+0, 0x1.486a2b5c13cd0p+0,
    0x1.4bfdad5362a27p+0, 0x1.4f9b2769d2ca7p+0, 0x1.5342b569d4f82p+0, 0x1.56f4736b527dap+0,
    0x1.5ab07dd485429p+0, 0x1.5e76f15ad2148p+0, 0x1.6247eb03a5585p+0, 0x1.6623882552225p+0,
    0x1.6a09e667f3bcdp+0, 0x1.6dfb23c651a2fp+0, 0x1.71f75e8ec5f74p+0, 0x1.75feb564267c9p+0,
    0x1.7a11473eb0187p+0, 0x1.7e2f336cf4e62p+0, 0x1.82589994cce13p+0, 0x1.868d99b4492edp+0,
    0x1.8ace5422aa0dbp+0, 0x1.8f1ae99157736p+0, 0x1.93737b0cdc5e5p+0, 0x1.97d829fde4e50p+0,
    0x1.9c49182a3f090p+0, 0x1.a0c667b5de565p+0, 0x1.a5503b23e255dp+0, 0x1.a9e6b5579fdbfp+0,
    0x1.ae89f995ad3adp+0, 0x1.b33a2b84f15fbp+0, 0x1.b7f76f2fb5e47p+0, 0x1.bcc1e904bc1d2p+0,
    0x1.c199bdd85529cp+0, 0x1.c67f12e57d14bp+0, 0x1.cb720dcef9069p+0, 0x1.d072d4a07897cp+0,
    0x1.d5818dcfba487p+0, 0x1.da9e603db3285p+0, 0x1.dfc97337b9b5fp+0, 0x1.e502ee78b3ff6p+0,
    0x1.ea4afa2a490dap+0, 0x1.efa1bee615a27p+0, 0x1.f50765b6e4540p+0, 0x1.fa7c1819e90d8p+0,
};

// e^x for x <= 0 (the screening factor e^(-kappa d)), without the range
// checks of a general exponential, with `tab` the table above (an LDS copy
// on the device). Tang's table-driven reduction: x = (64 n + j) ln2/64 + r,
// |r| <= ln2/128, so e^x = 2^n 2^(j/64) e^r. ln2/64 is taken in two parts, a
// head with 32 significant bits (n * head is exact for any n this range
// gives) and the rounded remainder. e^r - 1 is the Taylor series to degree
// 5, whose truncation is below 4e-17 relative on that interval; the result
// is 2^(j/64) + 2^(j/64) (e^r - 1) in one rounding, and ldexp applies 2^n
// (rounding results below the normal range as they underflow).
__device__ __forceinline__ double exp_nonpos(double x, const double* tab) {
    constexpr double k64InvLn2 = 92.332482616893658;
    constexpr double kHead = 0x1.62e42fee00000p-7;
    constexpr double kTail = 0x1.a39ef35793c76p-39;
    const double fk = rint(x * k64InvLn2);
    const int k = (int)fk;
    const double r = fma(-fk, kTail, fma(-fk, kHead, x));
    const double r2 = r * r;
    double p = fma(r, 1.0 / 120.0, 1.0 / 24.0);
    p = fma(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    const double em1 = fma(p, r2, r);
    const double t = tab[k & (kExpTab - 1)];
    return ldexp(fma(t, em1, t), k >> 6);
}

// Screened Coulomb sum of every atom at each ghost-face point, atoms in
// index order through LDS records (x, y, z, q): phi = (1/eps_out) sum q e^(-kd)/d.
// Ghost points lie one node outside the box and atoms inside it, so d >= h > 0.
__global__ __launch_bounds__(kDhBlock) void k_dh_faces(
        const double* __restrict__ xyz, const double* __restrict__ charge, int64_t natoms,
        int nx, int ny, int nz, double h, double ox, double oy, double oz,
        double kd, double eout, double* __restrict__ ghost, int64_t nghost) {
    __shared__ double4 sa[kDhBlock];
    __shared__ double s_tab[kExpTab];
    if (threadIdx.x < kExpTab) s_tab[threadIdx.x] = kExp2Frac[threadIdx.x];
    const int64_t t = (int64_t)blockIdx.x * kDhBlock + threadIdx.x;
    double px = 0, py = 0, pz = 0;
    if (t < nghost) ghost_point(t, nx, ny, nz, h, ox, oy, oz, px, py, pz);
    double s = 0.0;
    for (int64_t a0 = 0; a0 < natoms; a0 += kDhBlock) {
        __syncthreads();
        const int64_t a = a0 + threadIdx.x;
        if (a < natoms) sa[threadIdx.x] = make_double4(xyz[3 * a], xyz[3 * a + 1], xyz[3 * a + 2], charge[a]);
        __syncthreads();
        const int m = (int)min<int64_t>(kDhBlock, natoms - a0);
        if (kd == 0.0) {
#pragma unroll 4
            for (int b = 0; b < m; ++b) {
                const double4 c = sa[b];
                const double dx = px - c.x, dy = py - c.y, dz = pz - c.z;
                const double y = rsqrt_nr(dx * dx + dy * dy + dz * dz);
                s = fma(c.w, y, s);
            }
        } else {
#pragma unroll 4
            for (int b = 0; b < m; ++b) {
                const double4 c = sa[b];
                const double dx = px - c.x, dy = py - c.y, dz = pz - c.z;
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double y = rsqrt_nr(r2);
                s = fma(c.w * exp_nonpos(-kd * (r2 * y), s_tab), y, s);
            }
        }
    }
    if (t < nghost) ghost[t] = s / eout;
}

// Right-hand side: 4*pi*q/h^3 plus, for nodes on the box faces, the ghost
// potential times the ghost-side edge dielectric over h^2 (x-, x+, y-, y+,
// z-, z+ in that order).
__global__ void k_rhs(const double* __restrict__ q, const double* __restrict__ ex,
                      const double* __restrict__ ey, const double* __restrict__ ez,
                      const double* __restrict__ ghost, int nx, int ny, int nz,
                      double h3, double ih2, int per, double* __restrict__ b) {
    const int64_t nn = (int64_t)nx * ny * nz;
    const int64_t fx = (int64_t)ny * nz, fy = (int64_t)nx * nz, fz = (int64_t)nx * ny;
    const double* gxm = ghost;
    const double* gxp = ghost + fx;
    const double* gym = ghost + 2 * fx;
    const double* gyp = gym + fy;
    const double* gzm = gym + 2 * fy;
    const double* gzp = gzm + fz;
    for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < nn;
         n += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = n % nx, j = (n / nx) % ny, k = n / fz;
        double fold = 0.0;
        if (per) {   // no boundary values: the box repeats
            b[n] = kFourPi * q[n] / h3;
            continue;
        }
        if (i == 0) fold = fold + ex[(nx + 1) * (j + ny * k)] * ih2 * gxm[j + ny * k];
        if (i == nx - 1) fold = fold + ex[nx + (nx + 1) * (j + ny * k)] * ih2 * gxp[j + ny * k];
        if (j == 0) fold = fold + ey[i + (int64_t)nx * ((ny + 1) * k)] * ih2 * gym[i + nx * k];
        if (j == ny - 1) fold = fold + ey[i + (int64_t)nx * (ny + (ny + 1) * k)] * ih2 * gyp[i + nx * k];
        if (k == 0) fold = fold + ez[i + nx * j] * ih2 * gzm[i + nx * j];
        if (k == nz - 1) fold = fold + ez[i + nx * j + fz * nz] * ih2 * gzp[i + nx * j];
        b[n] = kFourPi * q[n] / h3 + fold;
    }
}

// Potential at each atom centre by the spreading weights; product q_a*phi_a.
__global__ void k_energy_atoms(const double* __restrict__ xyz, const double* __restrict__ charge,
                               int64_t natoms, int nx, int ny, int nz, double h,
                               double ox, double oy, double oz, int per, const double* __restrict__ x,
                               double* __restrict__ atom_phi, double* __restrict__ qphi,
                               int* __restrict__ flags) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= natoms) return;
    int i0, j0, k0;
    double fx, fy, fz;
    bool ok = cell_axis(xyz[3 * a], ox, h, nx, per, i0, fx);
    ok = cell_axis(xyz[3 * a + 1], oy, h, ny, per, j0, fy) && ok;
    ok = cell_axis(xyz[3 * a + 2], oz, h, nz, per, k0, fz) && ok;
    if (!ok) {
        atomicOr(flags, 1);
        qphi[a] = 0.0;
        if (atom_phi) atom_phi[a] = 0.0;
        return;
    }
    double t[8];
    for (int c = 0; c < 8; ++c) {
        const double wx = (c & 1) ? fx : 1.0 - fx;
        const double wy = (c & 2) ? fy : 1.0 - fy;
        const double wz = (c & 4) ? fz : 1.0 - fz;
        t[c] = wx * wy * wz * x[corner_node(i0, j0, k0, c, nx, ny, nz)];
    }
    const double phi = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
    if (atom_phi) atom_phi[a] = phi;
    qphi[a] = charge[a] * phi;
}

// Fixed-order sum of n doubles by one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_sum_fixed(const double* __restrict__ v, int64_t n,
                                                    double* __restrict__ out) {
    __shared__ double s[1024];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) acc += v[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

// b -= sums[0] / n when sums[1] == 0 (periodic boundary without salt: the
// operator annihilates constants, b gets a uniform neutralising background).
__global__ void k_neutralise(double* __restrict__ b, int64_t n, const double* __restrict__ sums) {
    if (sums[1] != 0.0) return;
    const double m = sums[0] / (double)n;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        b[t] = b[t] - m;
}

inline int64_t next_pow2(int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

inline unsigned blocks_for(int64_t n, int bs, int64_t cap = 65536) {
    int64_t b = (n + bs - 1) / bs;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

// Ascending sort of n keys (n a power of two >= 2): the stages up to the
// chunk size in one LDS launch; each later stage k takes its steps with
// j >= kSortChunk one launch each, then the rest in one LDS launch.
pb_status bitonic_sort(uint64_t* keys, int64_t n, hipStream_t st) {
    const int64_t chunk = std::min<int64_t>(n, kSortChunk);
    const unsigned nb = (unsigned)(n / chunk);
    hipLaunchKernelGGL(k_bitonic_local, dim3(nb), dim3(1024), 0, st, keys, n, (int64_t)2, chunk, (int64_t)1);
    for (int64_t k = 2 * chunk; k <= n; k <<= 1) {
        for (int64_t j = k >> 1; j >= chunk; j >>= 1)
            hipLaunchKernelGGL(k_bitonic_step, dim3(blocks_for(n, 256, 1 << 30)), dim3(256), 0, st, keys, n, j, k);
        hipLaunchKernelGGL(k_bitonic_local, dim3(nb), dim3(1024), 0, st, keys, n, k, k, chunk >> 1);
    }
    PB_HIP(hipGetLastError());
    return PB_OK;
}


}  // namespace

SetupWs carve_setup(void* base, int nx, int ny, int nz, int64_t natoms, bool frac) {
    SetupWs w{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    const int64_t npairs = next_pow2(std::max<int64_t>(2, 8 * natoms));
    const int64_t nn = (int64_t)nx * ny * nz;
    const int64_t nmask = (int64_t)(nx + 2) * (ny + 2) * (nz + 2);
    const int64_t ngh = 2 * ((int64_t)ny * nz + (int64_t)nx * nz + (int64_t)nx * ny);
    size_t o_flags = take(256);
    size_t o_keys = take(sizeof(uint64_t) * npairs);
    size_t o_q = take(sizeof(double) * nn);
    size_t o_mask = take((size_t)nmask);
    size_t o_gh = take(sizeof(double) * ngh);
    size_t o_cs = 0, o_ce = 0;
    if (frac) {
        o_cs = take(sizeof(int) * (size_t)nmask);
        o_ce = take(sizeof(int) * (size_t)nmask);
    }
    w.bytes = off;
    if (base) {
        char* b = (char*)base;
        w.flags = (int*)(b + o_flags);
        w.keys = (uint64_t*)(b + o_keys);
        w.qgrid = (double*)(b + o_q);
        w.mask = (uint8_t*)(b + o_mask);
        w.ghost = (double*)(b + o_gh);
        w.cell_start = frac ? (int*)(b + o_cs) : nullptr;
        w.cell_end = frac ? (int*)(b + o_ce) : nullptr;
    }
    return w;
}

namespace {

bool setup_opts_ok(const pb_setup_opts* o) {
    return o && (o->edge_model == PB_EDGE_NODE || o->edge_model == PB_EDGE_FRACTION);
}

bool grid_ok(const pb_grid* g) {
    const int m = (g && g->boundary == PB_BOUNDARY_PERIODIC) ? 3 : 2;
    return g && (g->boundary == PB_BOUNDARY_FREE || g->boundary == PB_BOUNDARY_PERIODIC) && g->nx >= m &&
           g->ny >= m && g->nz >= m && std::isfinite(g->h) && g->h > 0.0 &&
           std::isfinite(g->origin[0]) && std::isfinite(g->origin[1]) && std::isfinite(g->origin[2]) &&
           (int64_t)(g->nx + 2) * (g->ny + 2) * (int64_t)(g->nz + 2) < (int64_t(1) << 40);
}

}  // namespace

// Every launch of the setup on `st` (the outputs and the flags in w.flags
// are final once the stream reaches this point). The fractional-edge model
// reads the largest radius back to size its cell list, so it synchronises
// once; the two-point model never does.
pb_status setup_enqueue(const pb_grid* g, int64_t natoms, const double* xyz, const double* radius,
                        const double* charge, double eps_in, double eps_out, double kappa_d2, bool frac,
                        double* eps_x, double* eps_y, double* eps_z, double* kappa2, double* rhs, double* qgrid,
                        uint8_t* mask, const SetupWs& w, hipStream_t st) {
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    const double h = g->h, ox = g->origin[0], oy = g->origin[1], oz = g->origin[2];
    const int64_t nn = (int64_t)nx * ny * nz;
    const int64_t nmask = (int64_t)(nx + 2) * (ny + 2) * (nz + 2);
    const int64_t ngh = 2 * ((int64_t)ny * nz + (int64_t)nx * nz + (int64_t)nx * ny);
    uint8_t* m = mask ? mask : w.mask;
    double* q = qgrid ? qgrid : w.qgrid;
    const int per = g->boundary == PB_BOUNDARY_PERIODIC ? 1 : 0;

    hipLaunchKernelGGL(k_fill_u8, dim3(1), dim3(64), 0, st, (uint8_t*)w.flags, (int64_t)256, (uint8_t)0);
    hipLaunchKernelGGL(k_fill_u8, dim3(blocks_for(nmask, 256)), dim3(256), 0, st, m, nmask, (uint8_t)0);
    if (natoms > 0)
        hipLaunchKernelGGL(k_classify, dim3((unsigned)natoms), dim3(256), 0, st, xyz, radius, natoms,
                           nx, ny, nz, h, ox, oy, oz, per, m);
    if (per) {
        hipLaunchKernelGGL(k_wrap_ghosts, dim3(blocks_for((int64_t)ny * nz, 256)), dim3(256), 0, st, m, nx, ny,
                           nz, 0);
        hipLaunchKernelGGL(k_wrap_ghosts, dim3(blocks_for((int64_t)(nx + 2) * nz, 256)), dim3(256), 0, st, m,
                           nx, ny, nz, 1);
        hipLaunchKernelGGL(k_wrap_ghosts, dim3(blocks_for((int64_t)(nx + 2) * (ny + 2), 256)), dim3(256), 0, st,
                           m, nx, ny, nz, 2);
    }
    const int64_t nedge = (int64_t)(nx + 1) * ny * nz + (int64_t)nx * (ny + 1) * nz +
                          (int64_t)nx * ny * (nz + 1) + nn;
    hipLaunchKernelGGL(k_edges, dim3(blocks_for(nedge, 256)), dim3(256), 0, st, m, nx, ny, nz,
                       eps_in, eps_out, eps_out * kappa_d2, eps_x, eps_y, eps_z, kappa2);
    if (frac && natoms > 0) {
        // cell list of the atoms, then the fractional edges over the two-point ones
        double* rmax_d = (double*)w.ghost;   // the boundary buffer is free until the face sums
        hipLaunchKernelGGL(k_max_radius, dim3(1), dim3(1024), 0, st, radius, natoms, rmax_d);
        double rmax = 0.0;
        PB_HIP(hipMemcpyAsync(&rmax, rmax_d, sizeof(double), hipMemcpyDeviceToHost, st));
        PB_HIP(hipStreamSynchronize(st));
        PB_ARG(std::isfinite(rmax) && rmax >= 0.0, "pb_setup: non-finite atom radius");
        const int mcell = std::max(1, (int)std::ceil(rmax / h));
        const int ncx = (nx + 2 + mcell - 1) / mcell, ncy = (ny + 2 + mcell - 1) / mcell, ncz = (nz + 2 + mcell - 1) / mcell;
        const int64_t ncells = (int64_t)ncx * ncy * ncz;
        const int64_t P = next_pow2(std::max<int64_t>(2, natoms));
        hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(P, 256)), dim3(256), 0, st, w.keys, P, ~0ull);
        hipLaunchKernelGGL(k_cell_keys, dim3(blocks_for(natoms, 256, 1 << 30)), dim3(256), 0, st, xyz, natoms, nx, ny,
                           nz, h, ox, oy, oz, mcell, ncx, ncy, w.keys);
        for (int64_t k = 2; k <= P; k <<= 1)
            for (int64_t j = k >> 1; j > 0; j >>= 1)
                hipLaunchKernelGGL(k_bitonic_step, dim3(blocks_for(P, 256, 1 << 30)), dim3(256), 0, st, w.keys, P,
                                   j, k);
        hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(ncells, 256)), dim3(256), 0, st, w.cell_start, ncells, 0);
        hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(ncells, 256)), dim3(256), 0, st, w.cell_end, ncells, 0);
        hipLaunchKernelGGL(k_cell_bounds, dim3(blocks_for(natoms, 256, 1 << 30)), dim3(256), 0, st,
                           (const uint64_t*)w.keys, natoms, w.cell_start, w.cell_end);
        const int64_t nedge3 = nedge - nn;
        hipLaunchKernelGGL(k_edges_fraction, dim3(blocks_for(nedge3, 256)), dim3(256), 0, st, xyz, radius,
                           (const uint64_t*)w.keys, (const int*)w.cell_start, (const int*)w.cell_end, nx, ny, nz, h,
                           ox, oy, oz, rmax, mcell, ncx, ncy, ncz, eps_in, eps_out, eps_x, eps_y, eps_z, w.flags);
    }

    // charges: keys, sort, per-node run sums
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(nn, 256)), dim3(256), 0, st, q, nn, 0.0);
    if (natoms > 0) {
        const int64_t np = 8 * natoms;
        const int64_t P = next_pow2(std::max<int64_t>(2, np));
        hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(P, 256)), dim3(256), 0, st, w.keys, P, ~0ull);
        hipLaunchKernelGGL(k_spread_keys, dim3(blocks_for(np, 256, 1 << 30)), dim3(256), 0, st, xyz,
                           natoms, nx, ny, nz, h, ox, oy, oz, per, w.keys, w.flags);
        const pb_status es = bitonic_sort(w.keys, P, st);
        if (es != PB_OK) return es;
        hipLaunchKernelGGL(k_spread_sum, dim3(blocks_for(np, 256, 1 << 30)), dim3(256), 0, st, w.keys,
                           np, xyz, charge, nx, ny, nz, h, ox, oy, oz, per, q);
    }
    // boundary potential on the face ghosts (free space only)
    if (!per)
        hipLaunchKernelGGL(k_dh_faces, dim3(blocks_for(ngh, kDhBlock, 1 << 30)), dim3(kDhBlock), 0, st,
                           xyz, charge, natoms, nx, ny, nz, h, ox, oy, oz, std::sqrt(kappa_d2), eps_out,
                           w.ghost, ngh);
    hipLaunchKernelGGL(k_rhs, dim3(blocks_for(nn, 256)), dim3(256), 0, st, q, eps_x, eps_y, eps_z,
                       w.ghost, nx, ny, nz, std::pow(h, 3.0), 1.0 / (h * h), per, rhs);
    if (per) {   // sums of b and kbar^2 (fixed order) into the unused ghost buffer, then the background
        hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(1024), 0, st, (const double*)rhs, nn, w.ghost);
        hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(1024), 0, st, (const double*)kappa2, nn, w.ghost + 1);
        hipLaunchKernelGGL(k_neutralise, dim3(blocks_for(nn, 256)), dim3(256), 0, st, rhs, nn,
                           (const double*)w.ghost);
    }
    PB_HIP(hipGetLastError());
    return PB_OK;
}

size_t energy_scratch_bytes(int64_t natoms) { return sizeof(double) * (size_t)std::max<int64_t>(natoms, 1); }

pb_status energy_enqueue(const pb_grid* g, int64_t natoms, const double* xyz, const double* charge, const double* x,
                         double* qphi, int* flags, double* sum, hipStream_t st) {
    if (natoms > 0)
        hipLaunchKernelGGL(k_energy_atoms, dim3(blocks_for(natoms, 256, 1 << 30)), dim3(256), 0, st, xyz, charge,
                           natoms, g->nx, g->ny, g->nz, g->h, g->origin[0], g->origin[1], g->origin[2],
                           g->boundary == PB_BOUNDARY_PERIODIC ? 1 : 0, x, (double*)nullptr, qphi, flags);
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(1024), 0, st, (const double*)qphi, natoms, sum);
    PB_HIP(hipGetLastError());
    return PB_OK;
}

double energy_kcal(double sum_q_phi) { return 0.5 * sum_q_phi * kCoulombKcal; }

namespace {

}  // namespace

}  // namespace pb

using namespace pb;

extern "C" size_t pb_setup_workspace_bytes(const pb_grid* g, int64_t natoms) {
    if (!grid_ok(g) || natoms < 0 || natoms > kMaxAtoms) return 0;
    return carve_setup(nullptr, g->nx, g->ny, g->nz, natoms).bytes;
}

extern "C" size_t pb_setup_ex_workspace_bytes(const pb_grid* g, int64_t natoms, const pb_setup_opts* opts) {
    if (!grid_ok(g) || natoms < 0 || natoms > kMaxAtoms || !setup_opts_ok(opts)) return 0;
    return carve_setup(nullptr, g->nx, g->ny, g->nz, natoms, opts->edge_model == PB_EDGE_FRACTION).bytes;
}

extern "C" pb_status pb_setup(const pb_grid* g, int64_t natoms, const double* xyz,
                              const double* radius, const double* charge, double eps_in,
                              double eps_out, double kappa_d2, double* eps_x, double* eps_y,
                              double* eps_z, double* kappa2, double* rhs, double* qgrid,
                              uint8_t* mask, void* workspace, size_t workspace_bytes,
                              void* stream_) {
    pb_setup_opts o{};
    o.edge_model = PB_EDGE_NODE;
    return pb_setup_ex(g, natoms, xyz, radius, charge, eps_in, eps_out, kappa_d2, &o, eps_x, eps_y, eps_z, kappa2,
                       rhs, qgrid, mask, workspace, workspace_bytes, stream_);
}

extern "C" pb_status pb_setup_ex(const pb_grid* g, int64_t natoms, const double* xyz,
                                 const double* radius, const double* charge, double eps_in,
                                 double eps_out, double kappa_d2, const pb_setup_opts* opts, double* eps_x,
                                 double* eps_y, double* eps_z, double* kappa2, double* rhs, double* qgrid,
                                 uint8_t* mask, void* workspace, size_t workspace_bytes, void* stream_) {
    PB_ARG(setup_opts_ok(opts), "pb_setup: invalid options (edge_model)");
    const bool frac = opts->edge_model == PB_EDGE_FRACTION;
    PB_ARG(!frac || (g && g->boundary == PB_BOUNDARY_FREE),
           "pb_setup: the fractional-edge dielectric is available with the free-space boundary only");
    PB_ARG(!frac || kFractionEdgesEnabled,
           "pb_setup: the fractional-edge dielectric (PB_EDGE_FRACTION) is switched off in this library");
    PB_ARG(grid_ok(g), "pb_setup: grid needs a valid boundary, nx,ny,nz >= 2 (>= 3 periodic), finite h > 0 "
                       "and a finite origin");
    PB_ARG(natoms >= 0 && natoms <= kMaxAtoms, "pb_setup: natoms must be in [0, 2^21-1]");
    PB_ARG(natoms == 0 || (xyz && radius && charge), "pb_setup: null atom array");
    PB_ARG(eps_x && eps_y && eps_z && kappa2 && rhs, "pb_setup: null output array");
    PB_ARG(std::isfinite(eps_in) && std::isfinite(eps_out) && eps_in > 0 && eps_out > 0,
           "pb_setup: dielectric constants must be finite and > 0");
    PB_ARG(std::isfinite(kappa_d2) && kappa_d2 >= 0, "pb_setup: kappa_d2 must be finite and >= 0");
    PB_ARG(workspace != nullptr, "pb_setup: null workspace");
    const int nx = g->nx, ny = g->ny, nz = g->nz;
    SetupWs w = carve_setup(workspace, nx, ny, nz, natoms, frac);
    if (workspace_bytes < w.bytes) {
        set_error("pb_setup: workspace of %zu bytes, %zu needed", workspace_bytes, w.bytes);
        return PB_ERR_NOMEM;
    }
    hipStream_t st = (hipStream_t)stream_;
    const pb_status e = setup_enqueue(g, natoms, xyz, radius, charge, eps_in, eps_out, kappa_d2, frac, eps_x, eps_y,
                                      eps_z, kappa2, rhs, qgrid, mask, w, st);
    if (e != PB_OK) return e;
    const int per = g->boundary == PB_BOUNDARY_PERIODIC ? 1 : 0;
    PB_HIP(hipGetLastError());
    int flags = 0;
    PB_HIP(hipMemcpyAsync(&flags, w.flags, sizeof(int), hipMemcpyDeviceToHost, st));
    PB_HIP(hipStreamSynchronize(st));
    if (flags & 4) {
        set_error("pb_setup: more than 16 separate inside pieces on one edge (fractional edges)");
        return PB_ERR_ARG;
    }
    if (flags) {
        set_error(per ? "pb_setup: an atom centre lies beyond 2^28 nodes from the origin"
                      : "pb_setup: an atom centre lies outside the node box");
        return PB_ERR_ARG;
    }
    return PB_OK;
}

extern "C" size_t pb_energy_workspace_bytes(int64_t natoms) {
    if (natoms < 0 || natoms > kMaxAtoms) return 0;
    return 512 + align_up(sizeof(double) * (size_t)std::max<int64_t>(natoms, 1), 256);
}

extern "C" pb_status pb_energy(const pb_grid* g, int64_t natoms, const double* xyz,
                               const double* charge, const double* x, double* atom_phi,
                               double* energy, void* workspace, size_t workspace_bytes,
                               void* stream_) {
    PB_ARG(grid_ok(g), "pb_energy: grid needs a valid boundary, nx,ny,nz >= 2 (>= 3 periodic), finite h > 0 "
                       "and a finite origin");
    PB_ARG(natoms >= 0 && natoms <= kMaxAtoms, "pb_energy: natoms must be in [0, 2^21-1]");
    PB_ARG(natoms == 0 || (xyz && charge), "pb_energy: null atom array");
    PB_ARG(x && energy && workspace, "pb_energy: null x, energy or workspace");
    const size_t need = pb_energy_workspace_bytes(natoms);
    if (workspace_bytes < need) {
        set_error("pb_energy: workspace of %zu bytes, %zu needed", workspace_bytes, need);
        return PB_ERR_NOMEM;
    }
    hipStream_t st = (hipStream_t)stream_;
    char* b = (char*)workspace;
    int* flags = (int*)b;
    double* out = (double*)(b + 256);
    double* qphi = (double*)(b + 512);
    hipLaunchKernelGGL(k_fill_u8, dim3(1), dim3(64), 0, st, (uint8_t*)flags, (int64_t)256, (uint8_t)0);
    if (natoms > 0)
        hipLaunchKernelGGL(k_energy_atoms, dim3(blocks_for(natoms, 256, 1 << 30)), dim3(256), 0, st, xyz,
                           charge, natoms, g->nx, g->ny, g->nz, g->h, g->origin[0], g->origin[1],
                           g->origin[2], g->boundary == PB_BOUNDARY_PERIODIC ? 1 : 0, x, atom_phi, qphi, flags);
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(1024), 0, st, qphi, natoms, out);
    PB_HIP(hipGetLastError());
    double host[2];
    int hflags = 0;
    PB_HIP(hipMemcpyAsync(host, out, sizeof(double), hipMemcpyDeviceToHost, st));
    PB_HIP(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, st));
    PB_HIP(hipStreamSynchronize(st));
    if (hflags) {
        set_error("pb_energy: an atom centre lies outside the node box");
        return PB_ERR_ARG;
    }
    *energy = 0.5 * host[0] * kCoulombKcal;
    return PB_OK;
}
