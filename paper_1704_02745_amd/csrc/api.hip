// C-ABI entry points of the solve, argument checking and error reporting.
#include "solver.hpp"

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>

namespace pb {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

namespace {

struct SolveWs {
    SyncState* sync;
    double* partials;
    double* small;        // 16 doubles of device scratch
    Op<double> op64;
    double* b64;
    double* x64;
    double* res64;        // residual partials / scratch (npad)
    // FP64 state (PB_F64)
    SolveBufs<double> s64;
    // FP32 state (PB_F32, PB_F32_REFINE64)
    SolveBufs<float> s32;
    SyncState* dia_sync;
    void* mg;             // multigrid levels (PB_OP_MG)
    // the caller's arrays (level 0 of the multigrid hierarchy)
    double h;
    const double *ex, *ey, *ez, *k2;
    size_t bytes;
};

// per: periodic boundary; the fused solve then also holds the ghost-row
// copies of the operator and state for the 40-byte pass (ghost_layout).
SolveWs carve_solve(void* base, const Layout& L, int prec, int op, int per) {
    SolveWs w{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return base ? (void*)((char*)base + o) : nullptr;
    };
    const size_t n8 = sizeof(double) * (size_t)L.npad;
    const size_t n4 = sizeof(float) * (size_t)L.npad;
    w.sync = (SyncState*)take(sizeof(SyncState));
    w.dia_sync = (SyncState*)take(sizeof(SyncState));
    w.small = (double*)take(16 * sizeof(double));
    w.partials = (double*)take(2 * sizeof(double) * kMaxPartials * (size_t)kMaxTiles);
    w.op64.cx = (double*)take(n8);
    w.op64.cy = (double*)take(n8);
    w.op64.cz = (double*)take(n8);
    w.op64.d = (double*)take(n8);
    w.b64 = (double*)take(n8);
    w.x64 = (double*)take(n8);
    w.res64 = (double*)take(n8);
    if (prec == PB_F64) {
        SolveBufs<double>& s = w.s64;
        s.op = w.op64;
        s.b = w.b64;
        s.x = w.x64;
        s.r = (double*)take(n8);
        s.p0 = (double*)take(n8);
        s.p1 = (double*)take(n8);
        s.q = (double*)take(n8);
        if (op == PB_OP_DIA) {
            s.dia = (double*)take(7 * n8);
        } else if (op == PB_OP_MG) {
            s.z = (double*)take(n8);
            s.r2 = (double*)take(n8);
        } else {
            s.r2 = (double*)take(n8);
            s.q2 = (double*)take(n8);
            if (per && ghost_layout_ok(L)) {
                const size_t g8 = sizeof(double) * (size_t)ghost_layout(L).npad;
                s.gop.cx = (double*)take(g8);
                s.gop.cy = (double*)take(g8);
                s.gop.cz = (double*)take(g8);
                s.gop.d = (double*)take(g8);
                s.gb = (double*)take(g8);
                s.gx = (double*)take(g8);
                s.gr = (double*)take(g8);
                s.gr2 = (double*)take(g8);
                s.gp0 = (double*)take(g8);
                s.gp1 = (double*)take(g8);
            }
        }
    } else {
        SolveBufs<float>& s = w.s32;
        s.op.cx = (float*)take(n4);
        s.op.cy = (float*)take(n4);
        s.op.cz = (float*)take(n4);
        s.op.d = (float*)take(n4);
        s.b = (float*)take(n4);
        s.x = (float*)take(n4);
        s.r = (float*)take(n4);
        s.p0 = (float*)take(n4);
        s.p1 = (float*)take(n4);
        s.q = (float*)take(n4);
        if (op == PB_OP_DIA) {
            s.dia = (float*)take(7 * n4);
        } else if (op == PB_OP_MG) {
            s.z = (float*)take(n4);
            s.r2 = (float*)take(n4);
        } else {
            s.r2 = (float*)take(n4);
            s.q2 = (float*)take(n4);
            if (per && ghost_layout_ok(L)) {
                const size_t g4 = sizeof(float) * (size_t)ghost_layout(L).npad;
                s.gop.cx = (float*)take(g4);
                s.gop.cy = (float*)take(g4);
                s.gop.cz = (float*)take(g4);
                s.gop.d = (float*)take(g4);
                s.gb = (float*)take(g4);
                s.gx = (float*)take(g4);
                s.gr = (float*)take(g4);
                s.gr2 = (float*)take(g4);
                s.gp0 = (float*)take(g4);
                s.gp1 = (float*)take(g4);
                s.gcodes = (uint32_t*)take(g4);
            }
        }
    }
    if (op == PB_OP_MG) w.mg = take(mg_workspace_bytes(L, prec));
    w.bytes = off;
    return w;
}

bool opts_ok(const pb_solve_opts* o) {
    return o && std::isfinite(o->tol) && o->tol > 0 && o->precision >= PB_F64 &&
           o->precision <= PB_F32_REFINE64 && (o->op == PB_OP_STENCIL || o->op == PB_OP_DIA || o->op == PB_OP_MG) &&
           o->inner_tol >= 0 && o->inner_tol < 1 && o->max_outer >= 0 &&
           (o->boundary == PB_BOUNDARY_FREE || (o->boundary == PB_BOUNDARY_PERIODIC && o->op == PB_OP_STENCIL));
}

bool dims_ok(int nx, int ny, int nz) {
    return nx >= 1 && ny >= 1 && nz >= 1 && (int64_t)nx * ny * nz < (int64_t(1) << 36);
}

template <typename T>
pb_status run_inner(const Layout& L, const SolveBufs<T>& s, const SolveWs& w, int op, int periodic, double tol,
                    int maxiter, hipStream_t st, SolveResult* r) {
    if (op == PB_OP_DIA) return dia_jpcg_impl<T>(L, s, w.dia_sync, w.partials, tol, maxiter, st, r);
    if (op == PB_OP_MG)
        return mg_pcg_impl<T>(L, w.h, w.ex, w.ey, w.ez, w.k2, s, w.mg, w.dia_sync, w.partials, tol, maxiter, st, r);
    return fused_jpcg<T>(L, s, w.sync, w.partials, tol, maxiter, st, r, nullptr, periodic);
}

// FP64 residual r = b - A x; returns ||r||^2 and ||b||^2 on the host.
pb_status residual(const Layout& L, const SolveWs& w, int periodic, float* r32, double& rr, double& bb,
                   hipStream_t st) {
    pb_status e = launch_residual64(w.op64, w.b64, w.x64, L, periodic, nullptr, r32, w.res64, w.small, st);
    if (e != PB_OK) return e;
    double h[2];
    PB_HIP(hipMemcpyAsync(h, w.small, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    PB_HIP(hipStreamSynchronize(st));
    rr = h[0];
    bb = h[1];
    return PB_OK;
}

// Convert the caller's arrays into the padded FP64 operator and check them.
// `singular` (out): periodic boundary with kbar^2 = 0 at every node, where
// the operator annihilates constants; b then has its mean removed here.
pb_status prepare(const Layout& L, double h, const double* eps_x, const double* eps_y, const double* eps_z,
                  const double* kappa2, const double* rhs, const double* x, int warm, int periodic,
                  const SolveWs& w, hipStream_t st, bool* singular) {
    int* flags = (int*)w.small;
    pb_status e = launch_fill<int>(flags, 1, 0, st);
    if (e != PB_OK) return e;
    e = launch_prepare64(eps_x, eps_y, eps_z, kappa2, rhs, x, warm, periodic, L, h, w.op64, w.b64, w.x64, flags,
                         st);
    if (e != PB_OK) return e;
    int hflags = 0;
    PB_HIP(hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, st));
    PB_HIP(hipStreamSynchronize(st));
    if (hflags & FLAG_BAD_COEF) {
        set_error("negative or non-finite coefficient, or non-positive diagonal");
        return PB_ERR_ARG;
    }
    if (hflags & (FLAG_BAD_RHS | FLAG_BAD_GUESS)) {
        set_error("NaN/Inf in the right-hand side or the initial guess");
        return PB_ERR_NONFINITE;
    }
    const bool sing = periodic && !(hflags & FLAG_HAS_SALT);
    if (singular) *singular = sing;
    if (sing) return launch_remove_mean(w.b64, L, w.res64, w.small + 8, st);
    return PB_OK;
}

// Time `iters` iterations of the fused kernel with tiling t (second of two runs).
template <typename T>
pb_status time_tiling(const Layout& L, const SolveBufs<T>& s, const SolveWs& w, const Tiling& t, int iters,
                      hipStream_t st, double& us_per_iter) {
    SolveResult r{};
    for (int rep = 0; rep < 2; ++rep) {
        pb_status e = fused_jpcg<T>(L, s, w.sync, w.partials, 1e-300, iters, st, &r, &t, 0);
        if (e != PB_OK) return e;
        if (r.status < 0) {
            set_error("autotune trial failed with status %d", r.status);
            return (pb_status)r.status;
        }
    }
    if (r.iters <= 0) {
        set_error("autotune: the system converged before any timed iteration (zero right-hand side?)");
        return PB_ERR_ARG;
    }
    us_per_iter = 1e6 * r.kernel_seconds / r.iters;
    return PB_OK;
}

template <typename T>
pb_status autotune_impl(const Layout& L, const SolveBufs<T>& s, const SolveWs& w, int iters, hipStream_t st,
                        pb_tuning* best) {
    const std::vector<Tiling> cand = tiling_candidates<T>(L);
    if (cand.empty()) {
        set_error("autotune: no feasible tiling for this grid");
        return PB_ERR_ARG;
    }
    double best_us = 1e300;
    Tiling best_t{};
    for (const Tiling& t : cand) {
        double us = 0.0;
        pb_status e = time_tiling<T>(L, s, w, t, iters, st, us);
        if (e != PB_OK) return e;
        if (us < best_us) {
            best_us = us;
            best_t = t;
        }
    }
    record_tiling<T>(L, best_t);
    if (best) {
        best->block = best_t.bs;
        best->groups = best_t.mc;
        best->scheme = best_t.scheme;
        best->streaming = best_t.nt;
        best->zchunk = best_t.zchunk;
        best->grid = best_t.grid;
        best->segments = best_t.nseg;
        best->us_per_iter = best_us;
        best->candidates = (int)cand.size();
    }
    return PB_OK;
}

}  // namespace

}  // namespace pb

using namespace pb;

extern "C" const char* pb_version(void) { return "pbgpu 0.1 (gfx950)"; }

extern "C" const char* pb_last_error(void) { return g_err; }

extern "C" size_t pb_solve_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, const pb_solve_opts* opts) {
    if (!dims_ok(nx, ny, nz) || !opts_ok(opts)) return 0;
    return carve_solve(nullptr, make_layout(nx, ny, nz), opts->precision, opts->op,
                       opts->boundary == PB_BOUNDARY_PERIODIC).bytes;
}

namespace {

// The whole of pb_solve on a given workspace. `untimed`: record no HIP events
// (pb_info.kernel_seconds stays 0), so that nothing in the call allocates.
pb_status solve_impl(int32_t nx, int32_t ny, int32_t nz, double h, const double* eps_x, const double* eps_y,
                     const double* eps_z, const double* kappa2, const double* rhs, double* x,
                     const pb_solve_opts* opts, void* workspace, size_t workspace_bytes, void* stream_,
                     pb_info* info, bool untimed) {
    const auto t0 = std::chrono::steady_clock::now();
    if (info) std::memset(info, 0, sizeof(*info));
    PB_ARG(dims_ok(nx, ny, nz), "pb_solve: dims must be >= 1 (and below 2^36 nodes)");
    PB_ARG(std::isfinite(h) && h > 0, "pb_solve: h must be finite and > 0");
    PB_ARG(opts_ok(opts), "pb_solve: invalid options (tol > 0, precision, operator, inner_tol in [0,1), max_outer >= 0)");
    PB_ARG(eps_x && eps_y && eps_z && kappa2 && rhs && x, "pb_solve: null array");
    PB_ARG(workspace != nullptr, "pb_solve: null workspace");
    PB_ARG(((uintptr_t)workspace & 255) == 0, "pb_solve: workspace must be 256-byte aligned");
    const Layout L = make_layout(nx, ny, nz);
    const int prec = opts->precision, op = opts->op;
    SolveWs w = carve_solve(workspace, L, prec, op, opts->boundary == PB_BOUNDARY_PERIODIC);
    if (workspace_bytes < w.bytes) {
        set_error("pb_solve: workspace of %zu bytes, %zu needed", workspace_bytes, w.bytes);
        return PB_ERR_NOMEM;
    }
    w.h = h;
    w.ex = eps_x; w.ey = eps_y; w.ez = eps_z; w.k2 = kappa2;
    const int maxiter = opts->maxiter > 0 ? opts->maxiter : 10 * std::max(nx, std::max(ny, nz));
    const int per = opts->boundary == PB_BOUNDARY_PERIODIC ? 1 : 0;
    PB_ARG(!per || (nx >= 3 && ny >= 3 && nz >= 3), "pb_solve: the periodic boundary needs nx, ny, nz >= 3");
    if (opts->op == PB_OP_STENCIL) {
        const Tiling t = opts->precision == PB_F64 ? solve_tiling<double>(L, per) : solve_tiling<float>(L, per);
        PB_ARG(t.grid > 0, "pb_solve: no tiling of the fused kernel fits this row width (nx at most 1024 in "
                           "FP32, 512 in FP64)");
    }
    hipStream_t st = (hipStream_t)stream_;
    bool singular = false;
    pb_status e = prepare(L, h, eps_x, eps_y, eps_z, kappa2, rhs, x, opts->warm_start ? 1 : 0, per, w, st,
                          &singular);
    if (e != PB_OK) return e;

    SolveResult r{};
    r.untimed = untimed ? 1 : 0;
    int total_iters = 0, outer = 0, launches = 0, coded_launches = 0;
    double ksec = 0.0;
    double relres_recur = 0.0;
    pb_status status = PB_OK;
    if (prec == PB_F64) {
        SolveBufs<double> s = w.s64;
        s.warm = opts->warm_start ? 1 : 0;
        e = run_inner<double>(L, s, w, op, per, opts->tol, maxiter, st, &r);
        if (e != PB_OK) return e;
        ++launches;
        ksec += r.kernel_seconds;
        status = (pb_status)r.status;
        total_iters = r.iters;
        relres_recur = r.bb > 0 ? std::sqrt(r.rr) / std::sqrt(r.bb) : 0.0;
    } else if (prec == PB_F32) {
        SolveBufs<float> s = w.s32;
        s.warm = opts->warm_start ? 1 : 0;
        e = launch_round32(w.op64, w.b64, w.x64, L.npad, s.op, (float*)s.b, s.x, st);
        if (e != PB_OK) return e;
        e = run_inner<float>(L, s, w, op, per, opts->tol, maxiter, st, &r);
        if (e != PB_OK) return e;
        ++launches;
        coded_launches += r.coded;
        ksec += r.kernel_seconds;
        status = (pb_status)r.status;
        total_iters = r.iters;
        relres_recur = r.bb > 0 ? std::sqrt(r.rr) / std::sqrt(r.bb) : 0.0;
        e = launch_f32_to_f64(s.x, w.x64, L.npad, st);
        if (e != PB_OK) return e;
    } else {
        // iterative refinement: FP64 residual, FP32 correction solve, FP64 update
        SolveBufs<float> s = w.s32;
        s.warm = 0;
        e = launch_round32(w.op64, w.b64, w.x64, L.npad, s.op, nullptr, nullptr, st);
        if (e != PB_OK) return e;
        const double inner_tol = opts->inner_tol > 0 ? opts->inner_tol : 1e-4;
        const int max_outer = opts->max_outer > 0 ? opts->max_outer : 20;
        double rr = 0, bb = 0, rr_prev = -1;
        status = PB_NOT_CONVERGED;
        for (outer = 0;; ++outer) {
            e = residual(L, w, per, (float*)s.b, rr, bb, st);
            if (e != PB_OK) return e;
            if (bb == 0.0) {
                e = launch_fill<double>(w.x64, L.npad, 0.0, st);
                if (e != PB_OK) return e;
                relres_recur = 0.0;
                status = PB_OK;
                break;
            }
            relres_recur = std::sqrt(rr) / std::sqrt(bb);
            if (!std::isfinite(relres_recur)) { status = PB_ERR_BREAKDOWN; break; }
            if (relres_recur < opts->tol) { status = PB_OK; break; }
            if (outer >= max_outer) break;
            if (rr_prev >= 0 && rr > 0.25 * rr_prev) break;   // fell by less than 2x: stagnation
            rr_prev = rr;
            e = launch_fill<float>(s.x, L.npad, 0.0f, st);
            if (e != PB_OK) return e;
            e = run_inner<float>(L, s, w, op, per, inner_tol, maxiter, st, &r);
            if (e != PB_OK) return e;
            ++launches;
            coded_launches += r.coded;
            if (r.coded && op == PB_OP_STENCIL) {   // the operator is the same for every inner solve
                s.codes_valid = 1;
                s.ctab = r.ctab;
            }
            ksec += r.kernel_seconds;
            total_iters += r.iters;
            if (r.status < 0) { status = (pb_status)r.status; break; }
            e = launch_add_correction(w.x64, s.x, L.npad, st);
            if (e != PB_OK) return e;
        }
    }
    if (status == PB_ERR_TIMEOUT) set_error("pb_solve: a device-side wait timed out");
    if (status == PB_ERR_BREAKDOWN) set_error("pb_solve: CG breakdown (p.Ap <= 0 or non-finite)");
    if (status == PB_NOT_CONVERGED) set_error("pb_solve: not converged within the iteration limit");

    // singular periodic system: report the zero-mean potential
    if (singular) {
        e = launch_remove_mean(w.x64, L, w.res64, w.small + 8, st);
        if (e != PB_OK) return e;
    }
    // true FP64 residual of the returned potential, then hand x back
    double rr = 0, bb = 0;
    e = residual(L, w, per, nullptr, rr, bb, st);
    if (e != PB_OK) return e;
    e = launch_unpad<double>(w.x64, L, x, st);
    if (e != PB_OK) return e;
    PB_HIP(hipStreamSynchronize(st));
    if (info) {
        info->iters = total_iters;
        info->outer_iters = outer;
        info->status = status;
        info->relres_recur = relres_recur;
        info->relres_true = bb > 0 ? std::sqrt(rr) / std::sqrt(bb) : 0.0;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->kernel_launches = launches;
        info->kernel_seconds = ksec;
        info->coded_launches = coded_launches;
        info->reserved = 0;
    }
    return status;
}

// Scratch of pb_solve_noalloc: one copy per GPU, for the process lifetime.
// Host code reaches it only through the per-device address that
// hipGetSymbolAddress returns (the symbol itself is not a device address).
constexpr size_t kNoAllocScratchBytes = (size_t)256 << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

pb_status scratch_for_current_device(void** out) {
    int dev = 0;
    PB_HIP(hipGetDevice(&dev));
    PB_ARG(dev >= 0 && dev < kMaxDevices, "pb_solve_noalloc: device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        PB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PB_OK;
}

}  // namespace

extern "C" pb_status pb_solve(int32_t nx, int32_t ny, int32_t nz, double h, const double* eps_x,
                              const double* eps_y, const double* eps_z, const double* kappa2, const double* rhs,
                              double* x, const pb_solve_opts* opts, void* workspace, size_t workspace_bytes,
                              void* stream_, pb_info* info) {
    return solve_impl(nx, ny, nz, h, eps_x, eps_y, eps_z, kappa2, rhs, x, opts, workspace, workspace_bytes, stream_,
                      info, false);
}

extern "C" size_t pb_solve_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

extern "C" pb_status pb_solve_noalloc(int32_t nx, int32_t ny, int32_t nz, double h, const double* eps_x,
                                      const double* eps_y, const double* eps_z, const double* kappa2,
                                      const double* rhs, double* x, const pb_solve_opts* opts, void* stream_,
                                      pb_info* info) {
    if (info) std::memset(info, 0, sizeof(*info));
    PB_ARG(dims_ok(nx, ny, nz), "pb_solve_noalloc: dims must be >= 1 (and below 2^36 nodes)");
    PB_ARG(opts_ok(opts), "pb_solve_noalloc: invalid options");
    const size_t need = carve_solve(nullptr, make_layout(nx, ny, nz), opts->precision, opts->op,
                                    opts->boundary == PB_BOUNDARY_PERIODIC).bytes;
    if (need > kNoAllocScratchBytes) {
        set_error("pb_solve_noalloc: this grid needs %zu bytes of scratch and the library holds %zu per GPU "
                  "(about 2.2M nodes); use pb_solve with a workspace",
                  need, kNoAllocScratchBytes);
        return PB_ERR_NOMEM;
    }
    void* ws = nullptr;
    const pb_status e = scratch_for_current_device(&ws);
    if (e != PB_OK) return e;
    return solve_impl(nx, ny, nz, h, eps_x, eps_y, eps_z, kappa2, rhs, x, opts, ws, kNoAllocScratchBytes, stream_,
                      info, true);
}

extern "C" pb_status pb_autotune(int32_t nx, int32_t ny, int32_t nz, double h, const double* eps_x,
                                 const double* eps_y, const double* eps_z, const double* kappa2,
                                 const double* rhs, const pb_solve_opts* opts, int32_t iters_per_trial,
                                 void* workspace, size_t workspace_bytes, void* stream_, pb_tuning* best) {
    if (best) std::memset(best, 0, sizeof(*best));
    PB_ARG(dims_ok(nx, ny, nz), "pb_autotune: dims must be >= 1 (and below 2^36 nodes)");
    PB_ARG(std::isfinite(h) && h > 0, "pb_autotune: h must be finite and > 0");
    PB_ARG(opts_ok(opts) && opts->op == PB_OP_STENCIL && opts->boundary == PB_BOUNDARY_FREE,
           "pb_autotune: invalid options (stencil operator and free-space boundary only)");
    PB_ARG(iters_per_trial >= 1 && iters_per_trial <= 10000, "pb_autotune: iters_per_trial in [1, 10000]");
    PB_ARG(eps_x && eps_y && eps_z && kappa2 && rhs, "pb_autotune: null array");
    PB_ARG(workspace != nullptr && ((uintptr_t)workspace & 255) == 0, "pb_autotune: null or misaligned workspace");
    const Layout L = make_layout(nx, ny, nz);
    SolveWs w = carve_solve(workspace, L, opts->precision, PB_OP_STENCIL, 0);
    if (workspace_bytes < w.bytes) {
        set_error("pb_autotune: workspace of %zu bytes, %zu needed", workspace_bytes, w.bytes);
        return PB_ERR_NOMEM;
    }
    hipStream_t st = (hipStream_t)stream_;
    pb_status e = prepare(L, h, eps_x, eps_y, eps_z, kappa2, rhs, nullptr, 0, 0, w, st, nullptr);
    if (e != PB_OK) return e;
    if (opts->precision == PB_F64) {
        SolveBufs<double> s = w.s64;
        s.warm = 0;
        return autotune_impl<double>(L, s, w, iters_per_trial, st, best);
    }
    SolveBufs<float> s = w.s32;
    s.warm = 0;
    e = launch_round32(w.op64, w.b64, w.x64, L.npad, s.op, (float*)s.b, s.x, st);
    if (e != PB_OK) return e;
    return autotune_impl<float>(L, s, w, iters_per_trial, st, best);
}

extern "C" void pb_set_coded_coefficients(int32_t on) { set_coded_coefficients(on); }
extern "C" int32_t pb_get_coded_coefficients(void) { return coded_coefficients(); }
extern "C" void pb_set_periodic_pass(int32_t form) {
    if (form >= -1 && form <= 1) set_periodic_pass(form);
}
extern "C" int32_t pb_get_periodic_pass(void) { return periodic_pass(); }

extern "C" pb_status pb_get_tuning(int32_t nx, int32_t ny, int32_t nz, int32_t precision, pb_tuning* out) {
    PB_ARG(dims_ok(nx, ny, nz) && out, "pb_get_tuning: bad dims or null output");
    PB_ARG(precision >= PB_F64 && precision <= PB_F32_REFINE64, "pb_get_tuning: bad precision");
    const Layout L = make_layout(nx, ny, nz);
    const Tiling c = precision == PB_F64 ? choose_tiling<double>(L) : choose_tiling<float>(L);
    PB_ARG(c.grid > 0, "pb_get_tuning: no feasible tiling for this grid (nx too large for the in-plane halo)");
    pb_tuning t{};
    t.block = c.bs;
    t.groups = c.mc;
    t.zchunk = c.zchunk;
    t.grid = c.grid;
    t.scheme = c.scheme;
    t.streaming = c.nt;
    t.segments = c.nseg;
    *out = t;
    return PB_OK;
}

extern "C" pb_status pb_tiling_candidates(int32_t nx, int32_t ny, int32_t nz, int32_t precision, pb_tuning* out,
                                         int32_t max, int32_t* count) {
    PB_ARG(dims_ok(nx, ny, nz) && count, "pb_tiling_candidates: bad dims or null count");
    PB_ARG(precision >= PB_F64 && precision <= PB_F32_REFINE64, "pb_tiling_candidates: bad precision");
    PB_ARG(max >= 0 && (max == 0 || out), "pb_tiling_candidates: bad output array");
    const Layout L = make_layout(nx, ny, nz);
    const std::vector<Tiling> c =
        precision == PB_F64 ? tiling_candidates<double>(L) : tiling_candidates<float>(L);
    *count = (int32_t)c.size();
    for (int i = 0; i < (int)c.size() && i < max; ++i) {
        pb_tuning t{};
        t.block = c[i].bs;
        t.groups = c[i].mc;
        t.zchunk = c[i].zchunk;
        t.grid = c[i].grid;
        t.us_per_iter = 0.0;
        t.candidates = (int32_t)c.size();
        t.scheme = c[i].scheme;
        t.streaming = c[i].nt;
        t.segments = c[i].nseg;
        out[i] = t;
    }
    return PB_OK;
}

extern "C" pb_status pb_set_tuning(int32_t nx, int32_t ny, int32_t nz, int32_t precision, const pb_tuning* t) {
    PB_ARG(dims_ok(nx, ny, nz) && t, "pb_set_tuning: bad dims or null tuning");
    PB_ARG(precision >= PB_F64 && precision <= PB_F32_REFINE64, "pb_set_tuning: bad precision");
    const Layout L = make_layout(nx, ny, nz);
    PB_ARG(t->streaming >= -1 && t->streaming <= 1, "pb_set_tuning: streaming must be -1, 0 or 1");
    auto apply = [&](auto tag) -> pb_status {
        using T = decltype(tag);
        const int nt = t->streaming >= 0 ? t->streaming : streaming_for<T>(L);
        for (const Tiling& c : tiling_candidates<T>(L)) {
            if (c.bs == t->block && c.mc == t->groups && c.scheme == t->scheme && c.nt == nt &&
                c.zchunk == t->zchunk && c.grid == t->grid && (t->segments <= 0 || c.nseg == t->segments)) {
                record_tiling<T>(L, c);
                return PB_OK;
            }
        }
        set_error("pb_set_tuning: (block %d, groups %d, scheme %d, streaming %d, zchunk %d, grid %d) is not a "
                  "feasible tiling here",
                  t->block, t->groups, t->scheme, t->streaming, t->zchunk, t->grid);
        return PB_ERR_ARG;
    };
    return precision == PB_F64 ? apply(double{}) : apply(float{});
}
