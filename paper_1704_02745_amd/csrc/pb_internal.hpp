// Internal declarations shared by the pbgpu HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/pbgpu.h"

namespace pb {

// ---------------------------------------------------------------- errors

void set_error(const char* fmt, ...);

#define PB_HIP(call)                                                          \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess) {                                               \
            ::pb::set_error("%s failed: %s (%s:%d)", #call,                   \
                            hipGetErrorString(e_), __FILE__, __LINE__);       \
            return PB_ERR_HIP;                                                \
        }                                                                     \
    } while (0)

#define PB_ARG(cond, ...)                                                     \
    do {                                                                      \
        if (!(cond)) {                                                        \
            ::pb::set_error(__VA_ARGS__);                                     \
            return PB_ERR_ARG;                                                \
        }                                                                     \
    } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// ---------------------------------------------------------------- layout
//
// Internal (workspace) arrays use a padded layout: each z-plane of nx*ny
// nodes is stored with a stride `sp` rounded up to 64 elements, so that every
// plane starts on a 256-byte boundary and 16-byte vector loads stay aligned.
// Pad slots hold zero coefficients, a unit diagonal and a zero right-hand
// side, so they stay exactly zero through the iteration.
struct Layout {
    int nx, ny, nz;
    int64_t plane;   // nx*ny
    int64_t sp;      // padded plane stride (multiple of 64)
    int64_t npad;    // nz*sp
    int64_t n;       // nx*ny*nz
};

inline Layout make_layout(int nx, int ny, int nz) {
    Layout L;
    L.nx = nx; L.ny = ny; L.nz = nz;
    L.plane = (int64_t)nx * ny;
    L.sp = (int64_t)align_up((size_t)L.plane, 64);
    L.npad = L.sp * nz;
    L.n = L.plane * nz;
    return L;
}

// Operator in the padded layout: (A p)_n = d_n p_n - sum over the six
// neighbours of c * p_nb, where cx[n] couples n to n+1 (0 when n+1 is a ghost),
// cy[n] couples n to n+nx, cz[n] couples n to n+sp. All values already carry
// the 1/h^2 factor; d includes the ghost-side edges and kbar^2.
template <typename T>
struct Op {
    const T* cx;
    const T* cy;
    const T* cz;
    const T* d;
};

// ---------------------------------------------------------------- device sync
//
// Barrier state of the persistent solver and the scalars it persists. One
// instance per problem (at the head of the solve workspace for a single
// solve). The arrival counters are cleared before every launch; the scalars
// are written by workgroup 0 after every iteration so the host can read
// them and a later launch can resume.
struct alignas(256) SyncState {
    unsigned int arrive[8][64];   // arrivals of this launch, spread over 8 cache lines
    double alpha;                 // alpha of the last completed iteration
    double alpha_prev;
    double beta;
    double rho;                   // r.z
    double rr;                    // ||r||^2 (recurrence)
    double bb;                    // ||b||^2
    double pq;
    double rq, qq, rqd, qqd;
    int iters;
    int done;                     // 1: stop iterating
    int status;                   // pb_status
    int zero_rhs;                 // 1: ||b|| == 0
    int flags;
    int pad2[59];
};

enum PrepFlags {
    FLAG_BAD_COEF = 1,    // negative / non-finite coefficient or non-positive diagonal
    FLAG_BAD_RHS = 2,     // NaN / Inf in the right-hand side
    FLAG_BAD_GUESS = 4,   // NaN / Inf in the initial guess
    FLAG_HAS_SALT = 8,    // some node has kbar^2 > 0 (the periodic operator is then definite)
};

// ---------------------------------------------------------------- helpers

template <typename T> struct Vec;
template <> struct Vec<float>  { using type = float4;  static constexpr int n = 4; };
template <> struct Vec<double> { using type = double2; static constexpr int n = 2; };

// elementwise access into the 16-byte vector types
__device__ __forceinline__ float& vget(float4& v, int i) { return (&v.x)[i]; }
__device__ __forceinline__ double& vget(double2& v, int i) { return (&v.x)[i]; }
__device__ __forceinline__ float vget(const float4& v, int i) { return (&v.x)[i]; }
__device__ __forceinline__ double vget(const double2& v, int i) { return (&v.x)[i]; }

}  // namespace pb
