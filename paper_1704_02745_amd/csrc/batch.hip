// Batched solves: many independent systems of uneven size in one persistent
// launch (and the same work recorded once in a HIP graph for replay).
//
// Each problem is prepared into its own padded operator and state, gets a
// tiling that depends on its shape only, and a share of the co-resident
// workgroups proportional to its expected work (nodes x max edge, since the
// Jacobi-CG iteration count grows with the grid edge). Workgroups of one
// problem synchronise only with each other, so problems never wait for one
// another, and every problem's result is bitwise the same alone or in any mix.
#include "solver.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

namespace pb {
namespace {

struct ProbRec {            // per-problem host-visible results in the workspace
    int flags;
    int pad;
    double rr, bb;          // true FP64 residual sums
    double pad2[5];
};

template <typename T>
struct Plan {
    int nprob = 0;
    size_t bytes = 0;
    size_t lds = 0;
    char* table = nullptr;          // device: KArgs records
    int* first = nullptr;           // device: workgroup offsets (nprob + 1)
    SyncState* sync = nullptr;      // device: one per problem
    ProbRec* rec = nullptr;         // device: one per problem
    int* fit = nullptr;             // device: one per problem (coded coefficients fit the dictionary)
    std::vector<Layout> L;
    std::vector<Tiling> t;
    std::vector<SolveBufs<T>> s;
    std::vector<Op<double>> op64;
    std::vector<double*> b64, x64, resp;
    std::vector<double*> partials;
};

bool problem_ok(const pb_problem& p) {
    return p.nx >= 1 && p.ny >= 1 && p.nz >= 1 && (int64_t)p.nx * p.ny * p.nz < (int64_t(1) << 36) &&
           std::isfinite(p.h) && p.h > 0 && std::isfinite(p.tol) && p.tol > 0 && p.eps_x && p.eps_y &&
           p.eps_z && p.kappa2 && p.rhs && p.x;
}

// Carve the workspace (base may be null to size it). Returns false with an
// error set if a problem cannot be tiled.
template <typename T>
bool carve_batch(void* base, int nprob, const pb_problem* probs, Plan<T>& P, int zchunk = 0) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> void* {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return base ? (void*)((char*)base + o) : nullptr;
    };
    P.nprob = nprob;
    P.table = (char*)take(batch_kargs_bytes<T>() * (size_t)nprob);
    P.first = (int*)take(sizeof(int) * (size_t)(nprob + 1));
    P.sync = (SyncState*)take(sizeof(SyncState) * (size_t)nprob);
    P.rec = (ProbRec*)take(sizeof(ProbRec) * (size_t)nprob);
    P.fit = (int*)take(sizeof(int) * (size_t)nprob);
    P.lds = 0;
    for (int i = 0; i < nprob; ++i) {
        const Layout L = make_layout(probs[i].nx, probs[i].ny, probs[i].nz);
        const Tiling t = batch_tiling<T>(L, zchunk);
        if (t.ntiles <= 0) {
            set_error("batch: problem %d (nx = %d) is too wide for the batch kernel's in-plane halo", i, L.nx);
            return false;
        }
        P.lds = std::max(P.lds, t.lds);
        const size_t n8 = sizeof(double) * (size_t)L.npad, nT = sizeof(T) * (size_t)L.npad;
        P.L.push_back(L);
        P.t.push_back(t);
        P.partials.push_back((double*)take(2 * sizeof(double) * kMaxPartials * (size_t)t.ntiles));
        P.resp.push_back((double*)take(sizeof(double) * 2 * (size_t)residual_blocks(L)));
        Op<double> o64;
        o64.cx = (double*)take(n8);
        o64.cy = (double*)take(n8);
        o64.cz = (double*)take(n8);
        o64.d = (double*)take(n8);
        P.op64.push_back(o64);
        P.b64.push_back((double*)take(n8));
        P.x64.push_back((double*)take(n8));
        SolveBufs<T> s{};
        if constexpr (sizeof(T) == sizeof(double)) {
            s.op = o64;
            s.b = P.b64.back();
            s.x = P.x64.back();
        } else {
            s.op.cx = (T*)take(nT); s.op.cy = (T*)take(nT); s.op.cz = (T*)take(nT); s.op.d = (T*)take(nT);
            s.b = (T*)take(nT);
            s.x = (T*)take(nT);
        }
        s.r = (T*)take(nT); s.r2 = (T*)take(nT);
        s.q = (T*)take(nT); s.q2 = (T*)take(nT);
        s.p0 = (T*)take(nT); s.p1 = (T*)take(nT);
        s.warm = probs[i].warm_start ? 1 : 0;
        P.s.push_back(s);
    }
    P.bytes = off;
    return true;
}

// Workgroups per problem, proportional to nodes x max edge, at least one,
// at most the problem's tile count; returns the offsets (size nprob + 1).
std::vector<int> share_workgroups(const std::vector<Layout>& L, const std::vector<Tiling>& t, int capacity) {
    const int n = (int)L.size();
    std::vector<double> w(n);
    double tot = 0;
    for (int i = 0; i < n; ++i) {
        w[i] = (double)L[i].n * std::max(L[i].nx, std::max(L[i].ny, L[i].nz));
        tot += w[i];
    }
    std::vector<int> g(n, 1);
    int used = n;
    // hand out the remaining workgroups one at a time to the problem with the
    // largest work per workgroup that can still take one
    std::vector<double> load(n);
    for (int i = 0; i < n; ++i) load[i] = w[i] / g[i];
    while (used < capacity) {
        int best = -1;
        for (int i = 0; i < n; ++i)
            if (g[i] < t[i].ntiles && (best < 0 || load[i] > load[best])) best = i;
        if (best < 0) break;
        ++g[best];
        ++used;
        load[best] = w[best] / g[best];
    }
    std::vector<int> first(n + 1, 0);
    for (int i = 0; i < n; ++i) first[i + 1] = first[i] + g[i];
    (void)tot;
    return first;
}

template <typename T>
pb_status enqueue_prepare(const Plan<T>& P, const pb_problem* probs, hipStream_t st) {
    for (int i = 0; i < P.nprob; ++i) {
        pb_status e = launch_prepare64(probs[i].eps_x, probs[i].eps_y, probs[i].eps_z, probs[i].kappa2, probs[i].rhs,
                                       probs[i].x, probs[i].warm_start ? 1 : 0, 0, P.L[i], probs[i].h, P.op64[i],
                                       P.b64[i], P.x64[i], &P.rec[i].flags, st);
        if (e != PB_OK) return e;
        if constexpr (sizeof(T) == sizeof(float)) {
            e = launch_round32(P.op64[i], P.b64[i], P.x64[i], P.L[i].npad, P.s[i].op, (float*)P.s[i].b, P.s[i].x, st);
            if (e != PB_OK) return e;
        }
    }
    return PB_OK;
}

template <typename T>
pb_status enqueue_finish(const Plan<T>& P, const pb_problem* probs, hipStream_t st) {
    for (int i = 0; i < P.nprob; ++i) {
        pb_status e = PB_OK;
        if constexpr (sizeof(T) == sizeof(float)) e = launch_f32_to_f64(P.s[i].x, P.x64[i], P.L[i].npad, st);
        if (e != PB_OK) return e;
        e = launch_residual64(P.op64[i], P.b64[i], P.x64[i], P.L[i], 0, nullptr, nullptr, P.resp[i], &P.rec[i].rr, st);
        if (e != PB_OK) return e;
        e = launch_unpad<double>(P.x64[i], P.L[i], probs[i].x, st);
        if (e != PB_OK) return e;
    }
    return PB_OK;
}

// The whole batch on `st`: clear flags and barrier state, prepare, solve,
// finish; nothing is read back to the host, so it can be recorded in a graph.
// coded == 2 (FP32): every problem's dictionary, fit flag and code words are
// rebuilt on the device before the launch, whose kernel reads each problem's
// fit flag (the arguments table must carry the code words, dictionaries and
// flags).
template <typename T>
pb_status enqueue_batch(const Plan<T>& P, const pb_problem* probs, int grid, bool cooperative, hipStream_t st,
                        int coded = 0) {
    pb_status e = launch_fill<int>((int*)P.rec, (int64_t)(sizeof(ProbRec) / sizeof(int)) * P.nprob, 0, st);
    if (e != PB_OK) return e;
    e = launch_fill<int>((int*)P.sync, (int64_t)(sizeof(SyncState) / sizeof(int)) * P.nprob, 0, st);
    if (e != PB_OK) return e;
    e = enqueue_prepare<T>(P, probs, st);
    if (e != PB_OK) return e;
    if constexpr (sizeof(T) == sizeof(float)) {
        if (coded == 2)
            for (int i = 0; i < P.nprob; ++i) {
                e = enqueue_dictionary(P.s[i].op, P.L[i].npad, (void*)P.s[i].q, P.fit + i, st);
                if (e != PB_OK) return e;
                e = enqueue_encode(P.s[i].op, P.L[i].npad, P.s[i].q, (uint32_t*)P.s[i].q2, st, P.fit + i);
                if (e != PB_OK) return e;
            }
    }
    e = batch_launch<T>(P.table, P.first, P.nprob, grid, coded ? P.lds + kCodedLdsBytes : P.lds, st, cooperative,
                        coded);
    if (e != PB_OK) return e;
    return enqueue_finish<T>(P, probs, st);
}

// Write the per-problem kernel arguments (with each problem's code words and
// dictionary when `coded`, and its fit flag when coded == 2).
template <typename T>
pb_status fill_table(const Plan<T>& P, const pb_problem* probs, int coded, hipStream_t st) {
    std::vector<char> host(batch_kargs_bytes<T>() * (size_t)P.nprob);
    for (int i = 0; i < P.nprob; ++i) {
        const int maxiter = probs[i].maxiter > 0 ? probs[i].maxiter
                                                 : 10 * std::max(probs[i].nx, std::max(probs[i].ny, probs[i].nz));
        const float* cw = coded ? (const float*)P.s[i].q2 : nullptr;
        const float* tab = coded ? dictionary_table(P.s[i].q) : nullptr;
        batch_fill_kargs<T>(host.data() + batch_kargs_bytes<T>() * i, P.L[i], P.s[i], &P.sync[i], P.partials[i],
                            P.t[i], probs[i].tol, maxiter, 0, 0, cw, tab, coded == 2 ? P.fit + i : nullptr);
    }
    PB_HIP(hipMemcpyAsync(P.table, host.data(), host.size(), hipMemcpyHostToDevice, st));
    PB_HIP(hipStreamSynchronize(st));
    return PB_OK;
}

// Upload the per-problem kernel arguments and workgroup offsets.
template <typename T>
pb_status upload_table(const Plan<T>& P, const pb_problem* probs, int& grid, hipStream_t st) {
    const int cap = batch_capacity<T>(P.lds);
    if (cap < P.nprob) {
        set_error("batch: %d problems but only %d co-resident workgroups; split the batch", P.nprob, cap);
        return PB_ERR_ARG;
    }
    const std::vector<int> first = share_workgroups(P.L, P.t, cap);
    grid = first.back();
    PB_HIP(hipMemcpyAsync(P.first, first.data(), sizeof(int) * first.size(), hipMemcpyHostToDevice, st));
    return fill_table<T>(P, probs, 0, st);
}

// The direct (not graph-recorded) batch: as enqueue_batch, with coded
// coefficients when every problem's FP32 operator fits its dictionary and
// the coded kernel keeps the grid co-resident. The fit flags are read back
// to the host once, after the preparation; the code words go to each
// problem's q2 and the dictionary to its q (the batch's pass form uses
// neither).
template <typename T>
pb_status enqueue_batch_direct(const Plan<T>& P, const pb_problem* probs, int grid, hipStream_t st, bool& coded) {
    coded = false;
    pb_status e = launch_fill<int>((int*)P.rec, (int64_t)(sizeof(ProbRec) / sizeof(int)) * P.nprob, 0, st);
    if (e != PB_OK) return e;
    e = launch_fill<int>((int*)P.sync, (int64_t)(sizeof(SyncState) / sizeof(int)) * P.nprob, 0, st);
    if (e != PB_OK) return e;
    e = enqueue_prepare<T>(P, probs, st);
    if (e != PB_OK) return e;
    if constexpr (sizeof(T) == sizeof(float)) {
        bool can = coded_coefficients() != 0 && batch_capacity<T>(P.lds + kCodedLdsBytes, true) >= grid;
        for (int i = 0; i < P.nprob && can; ++i) can = coded_layout_ok(P.L[i]);
        if (can) {
            for (int i = 0; i < P.nprob; ++i) {
                e = enqueue_dictionary(P.s[i].op, P.L[i].npad, (void*)P.s[i].q, P.fit + i, st);
                if (e != PB_OK) return e;
            }
            std::vector<int> fit(P.nprob, 0);
            PB_HIP(hipMemcpyAsync(fit.data(), P.fit, sizeof(int) * P.nprob, hipMemcpyDeviceToHost, st));
            PB_HIP(hipStreamSynchronize(st));
            for (int i = 0; i < P.nprob; ++i) can = can && fit[i] == 1;
        }
        if (can) {
            for (int i = 0; i < P.nprob; ++i) {
                e = enqueue_encode(P.s[i].op, P.L[i].npad, P.s[i].q, (uint32_t*)P.s[i].q2, st);
                if (e != PB_OK) return e;
            }
            e = fill_table<T>(P, probs, 1, st);
            if (e != PB_OK) return e;
            coded = true;
        }
    }
    e = batch_launch<T>(P.table, P.first, P.nprob, grid, coded ? P.lds + kCodedLdsBytes : P.lds, st, true, coded);
    if (e != PB_OK) return e;
    return enqueue_finish<T>(P, probs, st);
}

// Read back per-problem results; returns the batch status (first error, else
// PB_NOT_CONVERGED if any problem did not converge, else PB_OK).
template <typename T>
pb_status collect(const Plan<T>& P, hipStream_t st, pb_info* infos, double seconds) {
    std::vector<SyncState> S(P.nprob);
    std::vector<ProbRec> R(P.nprob);
    PB_HIP(hipMemcpyAsync(S.data(), P.sync, sizeof(SyncState) * P.nprob, hipMemcpyDeviceToHost, st));
    PB_HIP(hipMemcpyAsync(R.data(), P.rec, sizeof(ProbRec) * P.nprob, hipMemcpyDeviceToHost, st));
    PB_HIP(hipStreamSynchronize(st));
    pb_status worst = PB_OK;
    for (int i = 0; i < P.nprob; ++i) {
        int status = S[i].status;
        if (R[i].flags & FLAG_BAD_COEF) status = PB_ERR_ARG;
        else if (R[i].flags & (FLAG_BAD_RHS | FLAG_BAD_GUESS)) status = PB_ERR_NONFINITE;
        if (infos) {
            pb_info& f = infos[i];
            std::memset(&f, 0, sizeof(f));
            f.iters = S[i].iters;
            f.status = status;
            f.kernel_launches = 1;
            f.relres_recur = S[i].bb > 0 ? std::sqrt(S[i].rr) / std::sqrt(S[i].bb) : 0.0;
            f.relres_true = R[i].bb > 0 ? std::sqrt(R[i].rr) / std::sqrt(R[i].bb) : 0.0;
            f.seconds = seconds;
        }
        if (status < 0 && worst >= 0) worst = (pb_status)status;
        if (status == PB_NOT_CONVERGED && worst == PB_OK) worst = PB_NOT_CONVERGED;
    }
    if (worst < 0) set_error("batch: at least one problem failed (see its pb_info.status)");
    return worst;
}

template <typename T>
pb_status solve_batch_impl(int nprob, const pb_problem* probs, void* ws, size_t wsb, hipStream_t st, pb_info* infos) {
    const auto t0 = std::chrono::steady_clock::now();
    Plan<T> P;
    if (!carve_batch<T>(ws, nprob, probs, P)) return PB_ERR_ARG;
    if (wsb < P.bytes) {
        set_error("pb_solve_batch: workspace of %zu bytes, %zu needed", wsb, P.bytes);
        return PB_ERR_NOMEM;
    }
    int grid = 0;
    pb_status e = upload_table<T>(P, probs, grid, st);
    if (e != PB_OK) return e;
    hipEvent_t ev[2];
    PB_HIP(hipEventCreate(&ev[0]));
    PB_HIP(hipEventCreate(&ev[1]));
    PB_HIP(hipEventRecord(ev[0], st));
    bool coded = false;
    e = enqueue_batch_direct<T>(P, probs, grid, st, coded);
    if (e != PB_OK) {
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
        return e;
    }
    PB_HIP(hipEventRecord(ev[1], st));
    PB_HIP(hipStreamSynchronize(st));
    float ms = 0;
    PB_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    const pb_status st_all = collect<T>(P, st, infos, secs);
    if (infos)
        for (int i = 0; i < nprob; ++i) {
            infos[i].kernel_seconds = 1e-3 * ms;
            infos[i].coded_launches = coded ? 1 : 0;
        }
    return st_all;
}

// z-chunks the batch autotuner times.
constexpr int kBatchZCandidates[] = {16, 24, 32, 48, 64};

// Time the batch kernel for each candidate z-chunk on these problems, each
// capped at `iters` iterations (state cleared and prepared as for a solve,
// but no hand-back: the problems' x arrays are not written), and make the
// fastest the device's batch z-chunk.
template <typename T>
pb_status batch_autotune_impl(int nprob, const pb_problem* probs, int iters, void* ws, size_t wsb, hipStream_t st,
                              int* best_z, double* best_seconds) {
    std::vector<pb_problem> trial(probs, probs + nprob);
    for (auto& p : trial) p.maxiter = iters;
    hipEvent_t ev[2];
    PB_HIP(hipEventCreate(&ev[0]));
    PB_HIP(hipEventCreate(&ev[1]));
    double best = 1e300;
    int bz = 0;
    pb_status e = PB_OK;
    for (int z : kBatchZCandidates) {
        Plan<T> P;
        if (!carve_batch<T>(ws, nprob, trial.data(), P, z)) { e = PB_ERR_ARG; break; }
        if (wsb < P.bytes) {
            set_error("pb_batch_autotune: workspace of %zu bytes, %zu needed", wsb, P.bytes);
            e = PB_ERR_NOMEM;
            break;
        }
        int grid = 0;
        if ((e = upload_table<T>(P, trial.data(), grid, st)) != PB_OK) break;
        if ((e = launch_fill<int>((int*)P.rec, (int64_t)(sizeof(ProbRec) / sizeof(int)) * nprob, 0, st)) != PB_OK) break;
        if ((e = launch_fill<int>((int*)P.sync, (int64_t)(sizeof(SyncState) / sizeof(int)) * nprob, 0, st)) != PB_OK) break;
        if ((e = enqueue_prepare<T>(P, trial.data(), st)) != PB_OK) break;
        // solves run coded where they can: time the kernel they will run (the
        // per-problem checked form, which needs no read-back here)
        int coded = 0;
        if constexpr (sizeof(T) == sizeof(float)) {
            bool can = coded_coefficients() != 0 && batch_capacity<T>(P.lds + kCodedLdsBytes, 2) >= grid;
            for (int i = 0; i < nprob && can; ++i) can = coded_layout_ok(P.L[i]);
            if (can) {
                for (int i = 0; i < nprob && e == PB_OK; ++i) {
                    e = enqueue_dictionary(P.s[i].op, P.L[i].npad, (void*)P.s[i].q, P.fit + i, st);
                    if (e == PB_OK) e = enqueue_encode(P.s[i].op, P.L[i].npad, P.s[i].q, (uint32_t*)P.s[i].q2, st,
                                                       P.fit + i);
                }
                if (e != PB_OK || (e = fill_table<T>(P, trial.data(), 2, st)) != PB_OK) break;
                coded = 2;
            }
        }
        if (hipEventRecord(ev[0], st) != hipSuccess) { e = PB_ERR_HIP; break; }
        if ((e = batch_launch<T>(P.table, P.first, nprob, grid, coded ? P.lds + kCodedLdsBytes : P.lds, st, true,
                                 coded)) != PB_OK)
            break;
        if (hipEventRecord(ev[1], st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) { e = PB_ERR_HIP; break; }
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) { e = PB_ERR_HIP; break; }
        if (ms < best) {
            best = ms;
            bz = z;
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (e != PB_OK) return e;
    set_batch_zchunk(bz);
    if (best_z) *best_z = bz;
    if (best_seconds) *best_seconds = 1e-3 * best;
    return PB_OK;
}

bool batch_args_ok(int nprob, const pb_problem* probs, int precision) {
    if (nprob < 1 || !probs || (precision != PB_F32 && precision != PB_F64)) return false;
    for (int i = 0; i < nprob; ++i)
        if (!problem_ok(probs[i])) return false;
    return true;
}

}  // namespace

struct BatchGraph {
    int precision = 0;
    int nprob = 0;
    std::vector<pb_problem> probs;
    std::unique_ptr<Plan<float>> p32;
    std::unique_ptr<Plan<double>> p64;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool cooperative = true;
    int coded = 0;   // 2: the recorded batch builds dictionaries and its kernel reads each problem's fit flag
    hipEvent_t ev[2] = {nullptr, nullptr};
};

}  // namespace pb

using namespace pb;

struct pb_batch_graph : public pb::BatchGraph {};

extern "C" size_t pb_batch_workspace_bytes(int32_t nprob, const pb_problem* probs, int32_t precision) {
    if (!batch_args_ok(nprob, probs, precision)) return 0;
    if (precision == PB_F64) {
        Plan<double> P;
        return carve_batch<double>(nullptr, nprob, probs, P) ? P.bytes : 0;
    }
    Plan<float> P;
    return carve_batch<float>(nullptr, nprob, probs, P) ? P.bytes : 0;
}

extern "C" pb_status pb_solve_batch(int32_t nprob, const pb_problem* probs, int32_t precision, void* workspace,
                                    size_t workspace_bytes, void* stream, pb_info* infos) {
    PB_ARG(batch_args_ok(nprob, probs, precision),
           "pb_solve_batch: need nprob >= 1, valid problems (dims >= 1, h > 0, tol > 0, non-null arrays), "
           "precision PB_F32 or PB_F64");
    PB_ARG(workspace != nullptr && ((uintptr_t)workspace & 255) == 0, "pb_solve_batch: null or misaligned workspace");
    hipStream_t st = (hipStream_t)stream;
    if (precision == PB_F64) return solve_batch_impl<double>(nprob, probs, workspace, workspace_bytes, st, infos);
    return solve_batch_impl<float>(nprob, probs, workspace, workspace_bytes, st, infos);
}

extern "C" pb_status pb_batch_set_zchunk(int32_t zchunk) {
    PB_ARG(zchunk >= 1 && zchunk <= 4096, "pb_batch_set_zchunk: zchunk in [1, 4096]");
    set_batch_zchunk(zchunk);
    return PB_OK;
}

extern "C" int32_t pb_batch_get_zchunk(void) { return batch_zchunk(); }

extern "C" size_t pb_batch_autotune_workspace_bytes(int32_t nprob, const pb_problem* probs, int32_t precision) {
    if (!batch_args_ok(nprob, probs, precision)) return 0;
    size_t most = 0;
    for (int z : kBatchZCandidates) {
        size_t b = 0;
        if (precision == PB_F64) {
            Plan<double> P;
            b = carve_batch<double>(nullptr, nprob, probs, P, z) ? P.bytes : 0;
        } else {
            Plan<float> P;
            b = carve_batch<float>(nullptr, nprob, probs, P, z) ? P.bytes : 0;
        }
        if (b == 0) return 0;
        most = std::max(most, b);
    }
    return most;
}

extern "C" pb_status pb_batch_autotune(int32_t nprob, const pb_problem* probs, int32_t precision,
                                       int32_t iters_per_trial, void* workspace, size_t workspace_bytes, void* stream,
                                       int32_t* best_zchunk, double* best_seconds) {
    PB_ARG(batch_args_ok(nprob, probs, precision),
           "pb_batch_autotune: need nprob >= 1, valid problems, precision PB_F32 or PB_F64");
    PB_ARG(iters_per_trial >= 1, "pb_batch_autotune: iters_per_trial >= 1");
    PB_ARG(workspace != nullptr && ((uintptr_t)workspace & 255) == 0,
           "pb_batch_autotune: null or misaligned workspace");
    hipStream_t st = (hipStream_t)stream;
    if (precision == PB_F64)
        return batch_autotune_impl<double>(nprob, probs, iters_per_trial, workspace, workspace_bytes, st,
                                           best_zchunk, best_seconds);
    return batch_autotune_impl<float>(nprob, probs, iters_per_trial, workspace, workspace_bytes, st, best_zchunk,
                                      best_seconds);
}

namespace {

template <typename T>
pb_status graph_build(pb_batch_graph* G, Plan<T>& P, void* ws, size_t wsb, hipStream_t st) {
    if (!carve_batch<T>(ws, G->nprob, G->probs.data(), P)) return PB_ERR_ARG;
    if (wsb < P.bytes) {
        set_error("pb_batch_graph_create: workspace of %zu bytes, %zu needed", wsb, P.bytes);
        return PB_ERR_NOMEM;
    }
    int grid = 0;
    pb_status e = upload_table<T>(P, G->probs.data(), grid, st);
    if (e != PB_OK) return e;
    // coded coefficients, decided on the device at every replay (the
    // coefficients may change between replays)
    G->coded = 0;
    if constexpr (sizeof(T) == sizeof(float)) {
        bool can = coded_coefficients() != 0 && batch_capacity<T>(P.lds + kCodedLdsBytes, 2) >= grid;
        for (int i = 0; i < P.nprob && can; ++i) can = coded_layout_ok(P.L[i]);
        if (can) {
            e = fill_table<T>(P, G->probs.data(), 2, st);
            if (e != PB_OK) return e;
            G->coded = 2;
        }
    }
    hipStream_t cs;
    PB_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    for (int attempt = 0; attempt < 2; ++attempt) {
        const bool coop = attempt == 0;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) break;
        const pb_status ee = enqueue_batch<T>(P, G->probs.data(), grid, coop, cs, G->coded);
        hipGraph_t g = nullptr;
        const hipError_t he = hipStreamEndCapture(cs, &g);
        if (ee == PB_OK && he == hipSuccess && g) {
            if (hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0) == hipSuccess) {
                G->graph = g;
                G->cooperative = coop;
                break;
            }
        }
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
    }
    (void)hipStreamDestroy(cs);
    if (!G->exec) {
        set_error("pb_batch_graph_create: could not capture the batch into a graph");
        return PB_ERR_HIP;
    }
    PB_HIP(hipEventCreate(&G->ev[0]));
    PB_HIP(hipEventCreate(&G->ev[1]));
    return PB_OK;
}

}  // namespace

extern "C" pb_status pb_batch_graph_create(int32_t nprob, const pb_problem* probs, int32_t precision, void* workspace,
                                           size_t workspace_bytes, void* stream, pb_batch_graph** out) {
    PB_ARG(out != nullptr, "pb_batch_graph_create: null output handle");
    *out = nullptr;
    PB_ARG(batch_args_ok(nprob, probs, precision), "pb_batch_graph_create: invalid problems or precision");
    PB_ARG(workspace != nullptr && ((uintptr_t)workspace & 255) == 0,
           "pb_batch_graph_create: null or misaligned workspace");
    std::unique_ptr<pb_batch_graph> G(new pb_batch_graph());
    G->precision = precision;
    G->nprob = nprob;
    G->probs.assign(probs, probs + nprob);
    hipStream_t st = (hipStream_t)stream;
    pb_status e;
    if (precision == PB_F64) {
        G->p64.reset(new Plan<double>());
        e = graph_build<double>(G.get(), *G->p64, workspace, workspace_bytes, st);
    } else {
        G->p32.reset(new Plan<float>());
        e = graph_build<float>(G.get(), *G->p32, workspace, workspace_bytes, st);
    }
    if (e != PB_OK) {
        if (G->exec) (void)hipGraphExecDestroy(G->exec);
        if (G->graph) (void)hipGraphDestroy(G->graph);
        return e;
    }
    *out = G.release();
    return PB_OK;
}

extern "C" pb_status pb_batch_graph_launch(pb_batch_graph* G, void* stream) {
    PB_ARG(G && G->exec, "pb_batch_graph_launch: null graph");
    hipStream_t st = (hipStream_t)stream;
    PB_HIP(hipEventRecord(G->ev[0], st));
    PB_HIP(hipGraphLaunch(G->exec, st));
    PB_HIP(hipEventRecord(G->ev[1], st));
    return PB_OK;
}

extern "C" pb_status pb_batch_graph_results(pb_batch_graph* G, void* stream, pb_info* infos) {
    PB_ARG(G && G->exec, "pb_batch_graph_results: null graph");
    hipStream_t st = (hipStream_t)stream;
    PB_HIP(hipStreamSynchronize(st));
    float ms = 0;
    PB_HIP(hipEventElapsedTime(&ms, G->ev[0], G->ev[1]));
    const pb_status s = G->precision == PB_F64 ? collect<double>(*G->p64, st, infos, 1e-3 * ms)
                                               : collect<float>(*G->p32, st, infos, 1e-3 * ms);
    std::vector<int> fit(G->nprob, 0);
    if (infos && G->coded == 2) {
        PB_HIP(hipMemcpyAsync(fit.data(), G->p32->fit, sizeof(int) * G->nprob, hipMemcpyDeviceToHost, st));
        PB_HIP(hipStreamSynchronize(st));
    }
    if (infos)
        for (int i = 0; i < G->nprob; ++i) {
            infos[i].kernel_seconds = 1e-3 * ms;
            infos[i].coded_launches = fit[i] == 1 ? 1 : 0;
        }
    return s;
}

extern "C" int32_t pb_batch_graph_is_cooperative(const pb_batch_graph* G) { return G && G->cooperative ? 1 : 0; }

extern "C" void pb_batch_graph_destroy(pb_batch_graph* G) {
    if (!G) return;
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->graph) (void)hipGraphDestroy(G->graph);
    if (G->ev[0]) (void)hipEventDestroy(G->ev[0]);
    if (G->ev[1]) (void)hipEventDestroy(G->ev[1]);
    delete G;
}
