// Host build of the fractional-edge device kernels (their text is extracted
// from setup.hip into kernels.inc by the test), run through the same host
// steps as pb_setup_ex: cell keys, bitonic sort, cell bounds, edges. Every
// buffer has its exact size, so AddressSanitizer sees any access outside it.
// Input file: int32 nx,ny,nz; f64 h, ox, oy, oz, eps_in, eps_out; int64
// natoms; f64 xyz[3n], radius[n]; f64 expected eps_x, eps_y, eps_z.
// Prints the number of edges that differ from the expected values.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>
struct D3 { unsigned x = 0, y = 0, z = 0; };
static D3 blockIdx, threadIdx, blockDim, gridDim;
#define __global__
#define __device__
#define __forceinline__ inline
#define __restrict__
using std::max;
using std::min;
static inline int atomicOr(int* p, int v) { const int o = *p; *p |= v; return o; }
#include "kernels.inc"

template <class F>
static void launch(unsigned nb, unsigned bs, F f) {
    gridDim.x = nb;
    blockDim.x = bs;
    for (unsigned b = 0; b < nb; ++b)
        for (unsigned t = 0; t < bs; ++t) {
            blockIdx.x = b;
            threadIdx.x = t;
            f();
        }
}
static int64_t next_pow2(int64_t v) { int64_t p = 1; while (p < v) p <<= 1; return p; }
static unsigned blocks_for(int64_t n, int bs, int64_t cap = 65536) {
    int64_t b = (n + bs - 1) / bs;
    return (unsigned)std::min<int64_t>(std::max<int64_t>(b, 1), cap);
}
static bool rd(FILE* f, void* p, size_t sz, size_t n) { return fread(p, sz, n, f) == n; }

int main(int argc, char** argv) {
    if (argc != 2) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int dims[3];
    double hv[6];
    int64_t natoms = 0;
    if (!rd(f, dims, 4, 3) || !rd(f, hv, 8, 6) || !rd(f, &natoms, 8, 1) || natoms < 1) return 2;
    const int nx = dims[0], ny = dims[1], nz = dims[2];
    const double h = hv[0], ox = hv[1], oy = hv[2], oz = hv[3], ein = hv[4], eout = hv[5];
    std::vector<double> xyz_v(3 * natoms), rad_v(natoms);
    const int64_t nex = (int64_t)(nx + 1) * ny * nz, ney = (int64_t)nx * (ny + 1) * nz,
                  nez = (int64_t)nx * ny * (nz + 1);
    std::vector<double> ref(nex + ney + nez);
    if (!rd(f, xyz_v.data(), 8, xyz_v.size()) || !rd(f, rad_v.data(), 8, rad_v.size()) ||
        !rd(f, ref.data(), 8, ref.size()))
        return 2;
    fclose(f);
    double rmax = 0.0;
    for (double r : rad_v) rmax = std::max(rmax, r);
    const int mcell = std::max(1, (int)std::ceil(rmax / h));
    const int ncx = (nx + 2 + mcell - 1) / mcell, ncy = (ny + 2 + mcell - 1) / mcell,
              ncz = (nz + 2 + mcell - 1) / mcell;
    const int64_t ncells = (int64_t)ncx * ncy * ncz;
    const int64_t P = next_pow2(std::max<int64_t>(2, natoms));
    // exact-size heap buffers
    double* xyz = new double[3 * natoms];
    double* radius = new double[natoms];
    std::copy(xyz_v.begin(), xyz_v.end(), xyz);
    std::copy(rad_v.begin(), rad_v.end(), radius);
    uint64_t* keys = new uint64_t[P];
    int* cs = new int[ncells];
    int* ce = new int[ncells];
    double* ex = new double[nex];
    double* ey = new double[ney];
    double* ez = new double[nez];
    int* flags = new int[1]();
    for (int64_t i = 0; i < P; ++i) keys[i] = ~0ull;
    launch(blocks_for(natoms, 256, 1 << 30), 256,
           [&] { k_cell_keys(xyz, natoms, nx, ny, nz, h, ox, oy, oz, mcell, ncx, ncy, keys); });
    for (int64_t k = 2; k <= P; k <<= 1)
        for (int64_t j = k >> 1; j > 0; j >>= 1)
            launch(blocks_for(P, 256, 1 << 30), 256, [&] { k_bitonic_step(keys, P, j, k); });
    for (int64_t i = 0; i < ncells; ++i) cs[i] = ce[i] = 0;
    launch(blocks_for(natoms, 256, 1 << 30), 256, [&] { k_cell_bounds(keys, natoms, cs, ce); });
    launch(blocks_for(nex + ney + nez, 256), 256, [&] {
        k_edges_fraction(xyz, radius, keys, cs, ce, nx, ny, nz, h, ox, oy, oz, rmax, mcell, ncx, ncy, ncz, ein,
                         eout, ex, ey, ez, flags);
    });
    const int fl = flags[0];
    int64_t bad = 0;
    for (int64_t i = 0; i < nex; ++i) bad += ex[i] != ref[i];
    for (int64_t i = 0; i < ney; ++i) bad += ey[i] != ref[nex + i];
    for (int64_t i = 0; i < nez; ++i) bad += ez[i] != ref[nex + ney + i];
    printf("flags %d cells %lld mismatching %lld of %lld\n", fl, (long long)ncells, (long long)bad,
           (long long)(nex + ney + nez));
    delete[] xyz; delete[] radius; delete[] keys; delete[] cs; delete[] ce;
    delete[] ex; delete[] ey; delete[] ez; delete[] flags;
    return bad == 0 && fl == 0 ? 0 : 1;
}
