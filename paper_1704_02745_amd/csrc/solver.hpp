// Host-side declarations of the solver building blocks.
#pragma once

#include "pb_internal.hpp"

#include <vector>

namespace pb {

// operator.hip
pb_status launch_prepare64(const double* ex, const double* ey, const double* ez, const double* k2,
                           const double* rhs, const double* xin, int warm, int periodic, const Layout& L,
                           double h, Op<double> op, double* b, double* x, int* flags, hipStream_t st);
pb_status launch_round32(Op<double> op64, const double* b, const double* x, int64_t npad, Op<float> op32,
                         float* b32, float* x32, hipStream_t st);
int residual_blocks(const Layout& L);
pb_status launch_residual64(Op<double> op, const double* b, const double* x, const Layout& L, int periodic,
                            double* r64, float* r32, double* partials, double* out2, hipStream_t st);
// v -= mean(v) over the real nodes of a padded FP64 array (fixed-order sum).
pb_status launch_remove_mean(double* v, const Layout& L, double* partials, double* out2, hipStream_t st);
pb_status launch_add_correction(double* x, const float* dx, int64_t npad, hipStream_t st);
pb_status launch_f32_to_f64(const float* a, double* b, int64_t n, hipStream_t st);
template <typename T>
pb_status launch_unpad(const T* xp, const Layout& L, double* out, hipStream_t st);
template <typename T>
pb_status launch_fill(T* p, int64_t n, T v, hipStream_t st);

// Tiling of the fused kernel: a tile is a contiguous range of `seglen`
// padded plane positions times a run of `zchunk` planes.
struct Tiling {
    int bs;          // threads per workgroup
    int mc;          // 16-byte vector groups per thread per plane (segment = mc*bs*VEC)
    int scheme;      // 0: pass stores A.p (48 B/node FP32); 1: recomputes it (40 B/node)
    int per;         // 1: periodic-boundary kernel (scheme 0 only)
    int nt;          // 1: streaming (nontemporal) accesses for the own-position streams
    size_t lds;      // dynamic LDS bytes
    int seglen;      // elements per segment
    int zchunk;      // planes per tile
    int nseg, nzc, ntiles;
    int halo;        // in-plane halo, >= nx, multiple of the vector width
    int grid;        // workgroups of the cooperative launch
};

constexpr int kMaxTiles = 65536;
constexpr int kMaxPartials = 8;   // doubles per tile (tile sums are double-buffered: 2 slots)

// Solver state arrays for one fused or DIA solve in precision T.
template <typename T>
struct SolveBufs {
    Op<T> op;
    const T* b;
    T* x;
    T* r;
    T* r2;         // fused form: second residual buffer (ping-pong)
    T* p0;
    T* p1;
    T* q;
    T* q2;         // fused form: second A.p buffer (ping-pong)
    T* z;          // multigrid form only
    T* dia;        // DIA form only: 7 diagonals x npad
    int warm;      // 1: x holds a nonzero initial guess
    // fused FP32 40-byte form: the code words in q2 and the dictionary (ctab,
    // inside q) were built for this operator by an earlier inner solve (with
    // the periodic boundary: the code words in gcodes, the dictionary in q)
    int codes_valid;
    const float* ctab;
    // periodic boundary, 40-byte pass: the operator and the state in the
    // ghost-row layout (ghost_layout); null when the workspace holds none
    Op<T> gop;
    T* gb;
    T* gx;
    T* gr;
    T* gr2;
    T* gp0;
    T* gp1;
    uint32_t* gcodes;   // FP32 only
};

// Ghost-row layout of the periodic 40-byte pass: per plane, two ghost rows
// (copies of rows ny-2, ny-1), the nx*ny nodes from position org (a multiple
// of 64 elements), then two ghost rows (copies of rows 0, 1); planes of sp
// positions (a multiple of 64). Tiles own [org, org + own), own being nx*ny
// rounded up to 4 (the last group runs into the upper ghost rows).
struct GhostLayout {
    int64_t org, own, sp, npad;
};
inline GhostLayout ghost_layout(const Layout& L) {
    GhostLayout g;
    g.org = (int64_t)align_up((size_t)(2 * L.nx), 64);
    g.own = (int64_t)align_up((size_t)L.plane, 4);
    g.sp = (int64_t)align_up((size_t)(g.org + L.plane + 2 * (int64_t)L.nx), 64);
    g.npad = g.sp * L.nz;
    return g;
}
// Whether the periodic 40-byte pass takes this grid: a group of four
// consecutive nodes holds at most one row end (nx > 4), the four ghost rows
// copy four distinct rows, and in-plane positions fit 32-bit arithmetic.
inline bool ghost_layout_ok(const Layout& L) {
    return L.nx >= 5 && L.ny >= 4 && L.nz >= 3 && ghost_layout(L).sp + 4 * (int64_t)L.nx < ((int64_t)1 << 31);
}

struct SolveResult {
    int status;
    int iters;
    double rr;     // ||r||^2 (recurrence) at exit
    double bb;     // ||b||^2
    double kernel_seconds;   // duration of the iteration kernel / loop (HIP events)
    Tiling tiling;           // fused form: the tiling used
    int coded;               // fused form: 1 when the pass read coded coefficients
    const float* ctab;       // and the dictionary it used (device)
    int untimed;             // input: 1 = record no HIP events (kernel_seconds stays 0)
};

// jpcg.hip: one persistent cooperative launch running the whole iteration.
template <typename T>
pb_status fused_jpcg(const Layout& L, const SolveBufs<T>& s, SyncState* sync, double* partials,
                     double tol, int maxiter, hipStream_t st, SolveResult* res, const Tiling* force,
                     int periodic = 0);

template <typename T>
Tiling choose_tiling(const Layout& L);
// The tiling a fused solve of this shape launches (free or periodic boundary);
// grid = 0 when no kernel variant fits the row width.
template <typename T>
Tiling solve_tiling(const Layout& L, int periodic);
// 1 when the shape's default is the streaming (nontemporal) kernel variant.
template <typename T>
int streaming_for(const Layout& L);

// coded.hip: coded operator coefficients for the 40-byte FP32 pass. Up to
// kCodedTableSize distinct values over cx, cy, cz and d; one 4-byte word of
// codes per padded position (byte 0: cx, 1: cy, 2: cz, 3: d).
constexpr int kCodedTableSize = 256;
size_t coded_scratch_bytes();
// Whether a problem of this layout can run the coded pass: its code words and
// dictionary fit the arrays the pass leaves unused, and its planes are short
// enough for the pass's 32-bit in-plane byte offsets.
inline bool coded_layout_ok(const Layout& L) {
    return (size_t)L.npad * sizeof(float) >= coded_scratch_bytes() && L.sp < ((int64_t)1 << 29);
}
// Builds the dictionary in `scratch` (coded_scratch_bytes()) and, when the
// values fit, the code words; fits = false leaves `codes` untouched. Reads one
// flag back to the host (synchronises `st`). *table: the device dictionary.
pb_status build_codes(const Op<float>& op, int64_t npad, void* scratch, uint32_t* codes, hipStream_t st,
                      bool& fits, const float** table);
// The same in two asynchronous halves: the dictionary (writes 1 to *ok_out
// when the values fit, 0 otherwise) and, once that is known, the code words.
pb_status enqueue_dictionary(const Op<float>& op, int64_t npad, void* scratch, int* ok_out, hipStream_t st);
pb_status enqueue_encode(const Op<float>& op, int64_t npad, const void* scratch, uint32_t* codes, hipStream_t st,
                         const int* fit = nullptr);   // fit: skip unless *fit == 1 (device flag)
const float* dictionary_table(const void* scratch);
// Extra dynamic LDS of the coded kernels: none, since the dictionary sits in
// static LDS, which the kernels' own group segment size already counts.
constexpr size_t kCodedLdsBytes = 0;
// Process-wide switch (default on): 0 keeps every fused FP32 solve uncoded.
void set_coded_coefficients(int on);
int coded_coefficients();
// Process-wide pass form of periodic fused solves: -1 the model's choice, 0
// or 1 that scheme (1 falls back to 0 where the ghost-row layout does not fit).
void set_periodic_pass(int form);
int periodic_pass();

// mg.hip: multigrid-preconditioned CG (workspace for the coarse levels and
// level 0's extra vectors; ex..k2 are the caller's FP64 edge arrays).
size_t mg_workspace_bytes(const Layout& L0, int prec);
template <typename T>
pb_status mg_pcg_impl(const Layout& L0, double h, const double* ex, const double* ey, const double* ez,
                      const double* k2, const SolveBufs<T>& s, void* mgws, SyncState* S, double* partials,
                      double tol, int maxiter, hipStream_t st, SolveResult* res);

// Tiling restricted to a block size / vector-group count (0 = any) and a
// cap on workgroups per CU (0 = occupancy limit).
template <typename T>
Tiling tiling_with(const Layout& L, int bs, int mc, int max_per_cu);

// Autotuner support: the search space, and recording the winner for later solves.
template <typename T>
std::vector<Tiling> tiling_candidates(const Layout& L);
template <typename T>
void record_tiling(const Layout& L, const Tiling& t);

// dia.hip: DIA SpMV plus separate vector kernels, host-driven loop.
template <typename T>
pb_status dia_jpcg_impl(const Layout& L, const SolveBufs<T>& s, SyncState* S, double* partials,
                        double tol, int maxiter, hipStream_t st, SolveResult* res);

// Batch support (jpcg.hip): shape-only tiling, per-problem kernel arguments,
// capacity and launch of the multi-problem persistent kernel.
template <typename T>
Tiling batch_tiling(const Layout& L, int zchunk = 0);   // zchunk 0: the device's batch z-chunk
// The batched and served kernels' z-chunk on the current device (default 32).
int batch_zchunk();
void set_batch_zchunk(int z);
template <typename T>
size_t batch_kargs_bytes();
template <typename T>
void batch_fill_kargs(void* dst, const Layout& L, const SolveBufs<T>& s, SyncState* S, double* partials,
                      const Tiling& t, double tol, int maxiter, int resume, int chunk, const float* cw = nullptr,
                      const float* ctab = nullptr, const int* fit = nullptr);
// Co-resident workgroups of the batch kernel. coded: 0 uncoded, 1 coded (every
// problem's operator fits), 2 coded per problem as its fit flag says; for 1
// and 2, lds includes kCodedLdsBytes.
template <typename T>
int batch_capacity(size_t lds, int coded = 0);
template <typename T>
pb_status batch_reset_arrivals(const void* d_kargs, int nprob, hipStream_t st);
// The scalars the host needs from each problem's barrier state, gathered
// into one device array (one read-back for a whole launch).
struct StateDigest {
    double rr, bb;
    int iters, done, status, pad;
};
template <typename T>
pb_status batch_state_digests(const void* d_kargs, int nprob, StateDigest* out, hipStream_t st);
template <typename T>
pb_status batch_launch(const void* d_kargs, const int* d_first, int nprob, int grid, size_t lds, hipStream_t st,
                       bool cooperative, int coded = 0);

// setup.hip: the setup's kernels without the host checks, for callers that
// sequence them themselves (the served form).
struct SetupWs {
    int* flags;
    uint64_t* keys;
    double* qgrid;
    uint8_t* mask;
    double* ghost;
    int* cell_start;   // fractional edges: atom ranges per cell
    int* cell_end;
    size_t bytes;
};
SetupWs carve_setup(void* base, int nx, int ny, int nz, int64_t natoms, bool frac = false);
// Enqueues the whole setup of pb_setup_ex on `st`; validation is the
// caller's. The atom-range flags land in w.flags (nonzero: an atom outside
// the node box).
pb_status setup_enqueue(const pb_grid* g, int64_t natoms, const double* xyz, const double* radius,
                        const double* charge, double eps_in, double eps_out, double kappa_d2, bool frac,
                        double* eps_x, double* eps_y, double* eps_z, double* kappa2, double* rhs, double* qgrid,
                        uint8_t* mask, const SetupWs& w, hipStream_t st);
// Enqueues sum_a q_a phi(c_a) into *sum (device); qphi holds natoms doubles.
size_t energy_scratch_bytes(int64_t natoms);
pb_status energy_enqueue(const pb_grid* g, int64_t natoms, const double* xyz, const double* charge, const double* x,
                         double* qphi, int* flags, double* sum, hipStream_t st);
// The energy 1/2 sum_a q_a phi(c_a) in kcal/mol from that sum.
double energy_kcal(double sum_q_phi);

}  // namespace pb
