// Continuous-batching solve server.
//
// Requests (systems of any supported size and tolerance) are queued by
// pb_server_submit. Each pb_server_step admits queued requests in arrival
// order while slots and the caller's HBM arena allow, advances every active
// request by up to `chunk` Jacobi-PCG iterations in ONE persistent batch
// launch (the requests' work overlaps on the device), retires requests that
// converged or failed, and frees their memory for the next admissions. The
// CG state of an unfinished request stays resident between steps and the
// next launch resumes it exactly, so chunking and the mix of co-running
// requests do not change any request's arithmetic.
//
// PB_F32 requests run FP32 JPCG to their tolerance. PB_F32_REFINE64 requests
// cycle: FP64 residual -> FP32 JPCG correction to a relative 1e-4 -> FP64
// update, until the FP64 residual is below their tolerance.
//
// A request is either an assembled system (pb_server_submit) or a molecule
// (pb_server_submit_atoms: atoms, radii, charges and a grid, as the paper's
// user supplies them): then the setup runs at admission inside the
// request's arena memory and the energy 1/2 sum q phi when it finishes.
//
// Every slot's host-visible results (flags, residual sums, energy sum) sit
// in one device array of records, read back with one copy per step phase.
#include "solver.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <memory>
#include <vector>

namespace pb {
namespace {

constexpr double kInnerTol = 1e-4;
constexpr int kMaxOuter = 20;

// A request's tiling: the batch kernel's, with the z-chunk cut (down to
// kServeMinZ planes) until the request has kServeTiles tiles, so that a
// small or mid-size grid spreads over enough workgroups to iterate quickly
// when the server is lightly loaded. It depends on the request's grid only
// (and the device's batch z-chunk), so a request's arithmetic is the same
// whatever else is in flight.
constexpr int kServeTiles = 128;
constexpr int kServeMinZ = 8;

Tiling serve_tiling(const Layout& L) {
    Tiling t = batch_tiling<float>(L);
    if (t.ntiles <= 0 || t.ntiles >= kServeTiles || t.zchunk <= kServeMinZ) return t;
    const int nzc = (kServeTiles + t.nseg - 1) / t.nseg;
    const int z = std::max(kServeMinZ, (L.nz + nzc - 1) / nzc);
    return z < t.zchunk ? batch_tiling<float>(L, z) : t;
}

// Per-iteration cost of one running request, in node updates of its busiest
// workgroup: the tiles that workgroup owns (tiles are whole, so the count is
// a ceiling) each take zchunk + 2 plane steps of one segment, plus the
// request's grid barrier and reductions, about 5.5 us, which the fused pass
// at 257^3 spends on about 3,500 node updates per workgroup (1.6 ns each).
constexpr double kBarrierNodes = 3500.0;
// A request advances by at most this many times the caller's chunk per launch.
constexpr int kMaxChunkScale = 16;

double iter_cost(const Tiling& t, int g) {
    const int per = (t.ntiles + g - 1) / g;
    return (double)per * (double)t.seglen * (double)(t.zchunk + 2) + kBarrierNodes;
}

// Workgroups and iteration counts of one launch over the running requests.
// Workgroups go, one useful step at a time, to the request whose iterations
// are the slowest (a step is the fewest extra workgroups that take one tile
// off its busiest workgroup), so the launch's slowest iteration is as short
// as the co-resident capacity allows. Every request then runs as many
// iterations as fit into the slowest request's `chunk` iterations (at least
// `chunk`, at most kMaxChunkScale times it): cheap requests (small grids, or
// the ones that got all the workgroups they can use) do not idle while the
// slow ones finish, and finish in fewer launches. Neither the workgroup
// count nor the iteration count of a launch changes a request's arithmetic.
void share_launch(const std::vector<Tiling>& Ts, int cap, int chunk, std::vector<int>& first,
                  std::vector<int>& chunks) {
    const int n = (int)Ts.size();
    std::vector<int> g(n, 1);
    std::vector<char> stuck(n, 0);
    int used = n;
    for (;;) {
        int best = -1;
        for (int i = 0; i < n; ++i)
            if (!stuck[i] && g[i] < Ts[i].ntiles && (best < 0 || iter_cost(Ts[i], g[i]) > iter_cost(Ts[best], g[best])))
                best = i;
        if (best < 0) break;
        const int nt = Ts[best].ntiles, per = (nt + g[best] - 1) / g[best];
        const int want = (nt + per - 2) / (per - 1);   // fewest workgroups with per - 1 tiles each
        if (used + (want - g[best]) > cap) {
            stuck[best] = 1;
            continue;
        }
        used += want - g[best];
        g[best] = want;
    }
    double cmax = 0.0;
    for (int i = 0; i < n; ++i) cmax = std::max(cmax, iter_cost(Ts[i], g[i]));
    for (int i = 0; i < n; ++i) {
        first[i + 1] = first[i] + g[i];
        const double scale = std::min<double>(kMaxChunkScale, cmax / iter_cost(Ts[i], g[i]));
        chunks[i] = std::max(chunk, (int)std::min<double>(2e9, std::floor(chunk * scale)));
    }
}

struct SlotRec {   // per-slot results written by kernels and read by the host
    int flags;
    int fit;       // 1: the FP32 operator fits the coded-coefficient dictionary
    double rr, bb;
    double esum;   // molecule requests: sum_a q_a phi(c_a)
    int setup_flags;   // molecule requests: nonzero when an atom lies outside the node box
    int energy_flags;
    double pad2[3];
};

struct Slot {
    int64_t id = 0;
    pb_problem req{};
    int precision = PB_F32;
    Layout L{};
    Tiling t{};
    size_t off = 0, bytes = 0;       // arena range
    SyncState* S = nullptr;
    SlotRec* rec = nullptr;
    double* partials = nullptr;
    double* resp = nullptr;
    Op<double> op64{};
    double* b64 = nullptr;
    double* x64 = nullptr;
    SolveBufs<float> s{};
    bool coded = false;              // code words in s.q2, dictionary in s.q (the pass form uses neither)
    int maxiter = 0;
    bool resume = false;             // inner solve already initialised
    bool solving = false;            // inner solve in progress
    bool ready = false;              // admission's read-back processed: the slot may join a launch
    int outer = 0, iters = 0;
    double rr_prev = -1.0;
    int status = PB_OK;
    double relres = 0.0, relres_true = 0.0;
    double t_submit = 0.0;
    int rec_idx = -1;                // index of this slot's record while admitted
    // molecule requests (pb_server_submit_atoms)
    bool from_atoms = false;
    pb_grid grid{};
    int64_t natoms = 0;
    const double* xyz = nullptr;
    const double* radius = nullptr;
    const double* charge = nullptr;
    double eps_in = 1.0, eps_out = 80.0, kappa_d2 = 0.0;
    double* energy_host = nullptr;
    SetupWs sw{};
    double* qphi = nullptr;
    bool energy_enqueued = false;
};

// Carve one slot's device memory at `base` (null to size it).
size_t carve_slot(char* base, Slot& s) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return base ? base + o : nullptr;
    };
    const size_t n8 = sizeof(double) * (size_t)s.L.npad, n4 = sizeof(float) * (size_t)s.L.npad;
    s.S = (SyncState*)take(sizeof(SyncState));
    s.partials = (double*)take(2 * sizeof(double) * kMaxPartials * (size_t)s.t.ntiles);
    s.resp = (double*)take(sizeof(double) * 2 * (size_t)residual_blocks(s.L));
    s.op64.cx = (double*)take(n8);
    s.op64.cy = (double*)take(n8);
    s.op64.cz = (double*)take(n8);
    s.op64.d = (double*)take(n8);
    s.b64 = (double*)take(n8);
    s.x64 = (double*)take(n8);
    s.s.op.cx = (float*)take(n4);
    s.s.op.cy = (float*)take(n4);
    s.s.op.cz = (float*)take(n4);
    s.s.op.d = (float*)take(n4);
    s.s.b = (float*)take(n4);
    s.s.x = (float*)take(n4);
    s.s.r = (float*)take(n4);
    s.s.r2 = (float*)take(n4);
    s.s.q = (float*)take(n4);
    s.s.q2 = (float*)take(n4);
    s.s.p0 = (float*)take(n4);
    s.s.p1 = (float*)take(n4);
    if (s.from_atoms) {   // the system the setup writes, its workspace and the energy's
        const int nx = s.L.nx, ny = s.L.ny, nz = s.L.nz;
        const size_t N = (size_t)nx * ny * nz;
        s.req.eps_x = (const double*)take(sizeof(double) * (size_t)(nx + 1) * ny * nz);
        s.req.eps_y = (const double*)take(sizeof(double) * (size_t)nx * (ny + 1) * nz);
        s.req.eps_z = (const double*)take(sizeof(double) * (size_t)nx * ny * (nz + 1));
        s.req.kappa2 = (const double*)take(sizeof(double) * N);
        s.req.rhs = (const double*)take(sizeof(double) * N);
        char* ws = take(carve_setup(nullptr, nx, ny, nz, s.natoms).bytes);
        if (base) s.sw = carve_setup(ws, nx, ny, nz, s.natoms);
        s.qphi = (double*)take(energy_scratch_bytes(s.natoms));
    }
    return off;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct Server {
    char* arena = nullptr;
    size_t arena_bytes = 0;
    int max_slots = 0;
    char* table = nullptr;        // device: kernel-argument records for max_slots
    int* first = nullptr;         // device: workgroup offsets
    StateDigest* digests = nullptr;   // device: each running request's scalars after a launch
    SlotRec* recs = nullptr;      // device: one record per admitted slot (max_slots)
    size_t reserved = 0;          // arena bytes used by the table, offsets, digests and records
    std::vector<std::pair<size_t, size_t>> free_list;   // (offset, bytes), sorted by offset
    std::deque<std::unique_ptr<Slot>> pending;
    std::vector<std::unique_ptr<Slot>> active;
    int64_t next_id = 1;
    int64_t launches = 0;
    int64_t coded_launches = 0;
    double device_seconds = 0.0;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t ev_in = nullptr;      // the caller's stream at the start of a step
    hipStream_t adm = nullptr;       // admissions (setup, preparation), overlapping the running launch
    std::vector<char> host_table;
    std::vector<int> host_first;
    std::vector<StateDigest> host_digests;
    std::vector<SlotRec> host_recs;
    std::vector<int> free_recs;   // unused record indices

    // one copy of every record, on the stream (the caller synchronises)
    pb_status read_recs(hipStream_t st) {
        PB_HIP(hipMemcpyAsync(host_recs.data(), recs, sizeof(SlotRec) * host_recs.size(), hipMemcpyDeviceToHost,
                              st));
        return PB_OK;
    }

    bool alloc(size_t bytes, size_t& off) {
        for (size_t i = 0; i < free_list.size(); ++i) {
            if (free_list[i].second >= bytes) {
                off = free_list[i].first;
                free_list[i].first += bytes;
                free_list[i].second -= bytes;
                if (free_list[i].second == 0) free_list.erase(free_list.begin() + i);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = std::lower_bound(free_list.begin(), free_list.end(), std::make_pair(off, (size_t)0));
        it = free_list.insert(it, {off, bytes});
        // merge with neighbours
        size_t i = it - free_list.begin();
        if (i + 1 < free_list.size() && free_list[i].first + free_list[i].second == free_list[i + 1].first) {
            free_list[i].second += free_list[i + 1].second;
            free_list.erase(free_list.begin() + i + 1);
        }
        if (i > 0 && free_list[i - 1].first + free_list[i - 1].second == free_list[i].first) {
            free_list[i - 1].second += free_list[i].second;
            free_list.erase(free_list.begin() + i);
        }
    }
    size_t used() const {
        size_t f = 0;
        for (auto& p : free_list) f += p.second;
        return arena_bytes - f;
    }
};

namespace {

// Enqueue the FP64 residual of a refinement slot: r (FP32) into the inner
// right-hand side, sums into rec.
pb_status enqueue_outer_residual(Slot& s, hipStream_t st) {
    return launch_residual64(s.op64, s.b64, s.x64, s.L, 0, nullptr, (float*)s.s.b, s.resp, &s.rec->rr, st);
}

// Reset the inner FP32 solve of a slot (zero guess, cleared barrier state).
pb_status enqueue_inner_reset(Slot& s, hipStream_t st) {
    pb_status e = launch_fill<int>((int*)s.S, (int64_t)(sizeof(SyncState) / sizeof(int)), 0, st);
    if (e != PB_OK) return e;
    e = launch_fill<float>(s.s.x, s.L.npad, 0.0f, st);
    s.resume = false;
    s.solving = true;
    return e;
}

}  // namespace
}  // namespace pb

using namespace pb;

struct pb_server : public pb::Server {};

extern "C" size_t pb_server_request_bytes(const pb_problem* req) {
    if (!req || req->nx < 1 || req->ny < 1 || req->nz < 1) return 0;
    Slot s;
    s.L = make_layout(req->nx, req->ny, req->nz);
    s.t = serve_tiling(s.L);
    if (s.t.ntiles <= 0) return 0;
    return carve_slot(nullptr, s);
}

extern "C" pb_status pb_server_create(void* arena, size_t arena_bytes, int32_t max_slots, pb_server** out) {
    PB_ARG(out != nullptr, "pb_server_create: null output handle");
    *out = nullptr;
    PB_ARG(arena != nullptr && ((uintptr_t)arena & 255) == 0, "pb_server_create: null or misaligned arena");
    PB_ARG(max_slots >= 1 && max_slots <= 4096, "pb_server_create: max_slots in [1, 4096]");
    std::unique_ptr<pb_server> S(new pb_server());
    S->arena = (char*)arena;
    S->arena_bytes = arena_bytes;
    S->max_slots = max_slots;
    const size_t tb = align_up(batch_kargs_bytes<float>() * (size_t)max_slots, 256);
    const size_t fb = align_up(sizeof(int) * (size_t)(max_slots + 1), 256);
    const size_t db = align_up(sizeof(StateDigest) * (size_t)max_slots, 256);
    const size_t rb = align_up(sizeof(SlotRec) * (size_t)max_slots, 256);
    PB_ARG(arena_bytes > tb + fb + db + rb, "pb_server_create: arena too small");
    S->table = S->arena;
    S->first = (int*)(S->arena + tb);
    S->digests = (StateDigest*)(S->arena + tb + fb);
    S->recs = (SlotRec*)(S->arena + tb + fb + db);
    S->reserved = tb + fb + db + rb;
    S->host_digests.resize(max_slots);
    S->host_recs.resize(max_slots);
    for (int i = max_slots - 1; i >= 0; --i) S->free_recs.push_back(i);
    S->free_list.push_back({S->reserved, arena_bytes - S->reserved});
    S->host_table.resize(batch_kargs_bytes<float>() * (size_t)max_slots);
    S->host_first.resize(max_slots + 1);
    PB_HIP(hipEventCreate(&S->ev[0]));
    PB_HIP(hipEventCreate(&S->ev[1]));
    PB_HIP(hipEventCreateWithFlags(&S->ev_in, hipEventDisableTiming));
    PB_HIP(hipStreamCreateWithFlags(&S->adm, hipStreamNonBlocking));
    *out = S.release();
    return PB_OK;
}

extern "C" pb_status pb_server_submit(pb_server* S, const pb_problem* req, int32_t precision, int64_t* id) {
    PB_ARG(S && req && id, "pb_server_submit: null argument");
    PB_ARG(precision == PB_F32 || precision == PB_F32_REFINE64, "pb_server_submit: precision PB_F32 or PB_F32_REFINE64");
    PB_ARG(req->nx >= 1 && req->ny >= 1 && req->nz >= 1 && std::isfinite(req->h) && req->h > 0 &&
               std::isfinite(req->tol) && req->tol > 0 && req->eps_x && req->eps_y && req->eps_z && req->kappa2 &&
               req->rhs && req->x,
           "pb_server_submit: invalid request");
    std::unique_ptr<Slot> s(new Slot());
    s->req = *req;
    s->precision = precision;
    s->L = make_layout(req->nx, req->ny, req->nz);
    s->t = serve_tiling(s->L);
    PB_ARG(s->t.ntiles > 0, "pb_server_submit: grid too wide for the batch kernel (nx <= 512)");
    s->bytes = carve_slot(nullptr, *s);
    PB_ARG(s->bytes <= S->arena_bytes - S->reserved, "pb_server_submit: request larger than the whole arena");
    s->maxiter = req->maxiter > 0 ? req->maxiter : 10 * std::max(req->nx, std::max(req->ny, req->nz));
    s->id = S->next_id++;
    s->t_submit = now_s();
    *id = s->id;
    S->pending.push_back(std::move(s));
    return PB_OK;
}

extern "C" size_t pb_server_request_bytes_atoms(const pb_grid* grid, int64_t natoms) {
    if (!grid || grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || natoms < 0) return 0;
    Slot s;
    s.from_atoms = true;
    s.natoms = natoms;
    s.L = make_layout(grid->nx, grid->ny, grid->nz);
    s.t = serve_tiling(s.L);
    if (s.t.ntiles <= 0) return 0;
    return carve_slot(nullptr, s);
}

extern "C" pb_status pb_server_submit_atoms(pb_server* S, const pb_grid* grid, int64_t natoms, const double* xyz,
                                            const double* radius, const double* charge, double eps_in,
                                            double eps_out, double kappa_d2, double tol, int32_t maxiter,
                                            int32_t precision, double* x, double* energy, int64_t* id) {
    PB_ARG(S && grid && id && x, "pb_server_submit_atoms: null argument");
    PB_ARG(precision == PB_F32 || precision == PB_F32_REFINE64,
           "pb_server_submit_atoms: precision PB_F32 or PB_F32_REFINE64");
    PB_ARG(grid->boundary == PB_BOUNDARY_FREE && grid->nx >= 2 && grid->ny >= 2 && grid->nz >= 2 &&
               std::isfinite(grid->h) && grid->h > 0 && std::isfinite(grid->origin[0]) &&
               std::isfinite(grid->origin[1]) && std::isfinite(grid->origin[2]),
           "pb_server_submit_atoms: the grid needs the free-space boundary, nx,ny,nz >= 2, finite h > 0 and a "
           "finite origin");
    PB_ARG(natoms >= 0 && natoms < (1 << 21) && (natoms == 0 || (xyz && radius && charge)),
           "pb_server_submit_atoms: natoms in [0, 2^21) with non-null atom arrays");
    PB_ARG(std::isfinite(eps_in) && std::isfinite(eps_out) && eps_in > 0 && eps_out > 0 && std::isfinite(kappa_d2) &&
               kappa_d2 >= 0,
           "pb_server_submit_atoms: dielectrics finite and > 0, kappa_d2 finite and >= 0");
    PB_ARG(std::isfinite(tol) && tol > 0, "pb_server_submit_atoms: tol must be finite and > 0");
    std::unique_ptr<Slot> s(new Slot());
    s->from_atoms = true;
    s->grid = *grid;
    s->natoms = natoms;
    s->xyz = xyz;
    s->radius = radius;
    s->charge = charge;
    s->eps_in = eps_in;
    s->eps_out = eps_out;
    s->kappa_d2 = kappa_d2;
    s->energy_host = energy;
    s->req.nx = grid->nx;
    s->req.ny = grid->ny;
    s->req.nz = grid->nz;
    s->req.h = grid->h;
    s->req.tol = tol;
    s->req.maxiter = maxiter;
    s->req.x = x;
    s->precision = precision;
    s->L = make_layout(grid->nx, grid->ny, grid->nz);
    s->t = serve_tiling(s->L);
    PB_ARG(s->t.ntiles > 0, "pb_server_submit_atoms: grid too wide for the batch kernel (nx <= 512)");
    s->bytes = carve_slot(nullptr, *s);
    PB_ARG(s->bytes <= S->arena_bytes - S->reserved, "pb_server_submit_atoms: request larger than the whole arena");
    s->maxiter = maxiter > 0 ? maxiter : 10 * std::max(grid->nx, std::max(grid->ny, grid->nz));
    s->id = S->next_id++;
    s->t_submit = now_s();
    *id = s->id;
    S->pending.push_back(std::move(s));
    return PB_OK;
}

namespace {

// Mark a slot finished and hand its potential back to the caller (enqueued).
pb_status finish_slot(Slot& s, int status, hipStream_t st) {
    s.status = status;
    s.solving = false;
    return launch_unpad<double>(s.x64, s.L, s.req.x, st);
}

}  // namespace

extern "C" pb_status pb_server_step(pb_server* S, int32_t chunk, void* stream, int32_t max_done, int32_t* n_done,
                                    int64_t* done_ids, pb_info* done_infos) {
    PB_ARG(S && n_done, "pb_server_step: null argument");
    PB_ARG(chunk >= 1, "pb_server_step: chunk >= 1");
    PB_ARG(max_done >= 0 && (max_done == 0 || (done_ids && done_infos)), "pb_server_step: bad output arrays");
    *n_done = 0;
    hipStream_t st = (hipStream_t)stream;
    pb_status e;

    // ---- admission (arrival order; stops at the first request that does not fit)
    // Admissions run on the server's own stream (after everything the caller
    // enqueued before this step), overlapping this step's launch; a request
    // admitted here joins the launch of the next step, or of this one when
    // no other request is running.
    std::vector<Slot*> admitted;
    hipStream_t ad = S->adm;
    if (!S->pending.empty()) {
        PB_HIP(hipEventRecord(S->ev_in, st));
        PB_HIP(hipStreamWaitEvent(ad, S->ev_in, 0));
    }
    while (!S->pending.empty() && (int)S->active.size() < S->max_slots) {
        Slot& s = *S->pending.front();
        size_t off = 0;
        if (!S->alloc(s.bytes, off)) break;
        s.off = off;
        carve_slot(S->arena + off, s);
        s.rec_idx = S->free_recs.back();
        S->free_recs.pop_back();
        s.rec = S->recs + s.rec_idx;
        e = launch_fill<int>((int*)s.rec, (int64_t)(sizeof(SlotRec) / sizeof(int)), 0, ad);
        if (e != PB_OK) return e;
        if (s.from_atoms) {
            e = setup_enqueue(&s.grid, s.natoms, s.xyz, s.radius, s.charge, s.eps_in, s.eps_out, s.kappa_d2, false,
                              (double*)s.req.eps_x, (double*)s.req.eps_y, (double*)s.req.eps_z,
                              (double*)s.req.kappa2, (double*)s.req.rhs, nullptr, nullptr, s.sw, ad);
            if (e != PB_OK) return e;
            PB_HIP(hipMemcpyAsync(&s.rec->setup_flags, s.sw.flags, sizeof(int), hipMemcpyDeviceToDevice, ad));
        }
        e = launch_prepare64(s.req.eps_x, s.req.eps_y, s.req.eps_z, s.req.kappa2, s.req.rhs, s.req.x,
                             s.req.warm_start ? 1 : 0, 0, s.L, s.req.h, s.op64, s.b64, s.x64, &s.rec->flags, ad);
        if (e != PB_OK) return e;
        if (s.precision == PB_F32) {
            e = launch_round32(s.op64, s.b64, s.x64, s.L.npad, s.s.op, (float*)s.s.b, s.s.x, ad);
            if (e != PB_OK) return e;
            e = launch_fill<int>((int*)s.S, (int64_t)(sizeof(SyncState) / sizeof(int)), 0, ad);
            if (e != PB_OK) return e;
            s.s.warm = s.req.warm_start ? 1 : 0;
            s.resume = false;
            s.solving = true;
        } else {
            e = launch_round32(s.op64, s.b64, s.x64, s.L.npad, s.s.op, nullptr, nullptr, ad);
            if (e != PB_OK) return e;
            s.s.warm = 0;
            e = enqueue_outer_residual(s, ad);
            if (e != PB_OK) return e;
        }
        // coded coefficients: the dictionary now, the code words once the fit flag is read back
        if (coded_coefficients() && coded_layout_ok(s.L)) {
            e = enqueue_dictionary(s.s.op, s.L.npad, (void*)s.s.q, &s.rec->fit, ad);
            if (e != PB_OK) return e;
        }
        admitted.push_back(&s);
        S->active.push_back(std::move(S->pending.front()));
        S->pending.pop_front();
    }
    // the admissions' read-back: setup and coefficient flags, the fit flag,
    // the first FP64 residual of refinement requests; their follow-up work
    // goes to the caller's stream
    auto process_admitted = [&]() -> pb_status {
        PB_HIP(hipStreamSynchronize(ad));
        if ((e = S->read_recs(ad)) != PB_OK) return e;
        PB_HIP(hipStreamSynchronize(ad));
        for (Slot* sp : admitted) {
            Slot& s = *sp;
            const SlotRec r = S->host_recs[s.rec_idx];
            if (r.setup_flags || (r.flags & FLAG_BAD_COEF)) {
                e = finish_slot(s, PB_ERR_ARG, st);
                if (e != PB_OK) return e;
                continue;
            }
            if (r.fit == 1) {
                e = enqueue_encode(s.s.op, s.L.npad, s.s.q, (uint32_t*)s.s.q2, st);
                if (e != PB_OK) return e;
                s.coded = true;
            }
            if (r.flags & (FLAG_BAD_RHS | FLAG_BAD_GUESS)) {
                e = finish_slot(s, PB_ERR_NONFINITE, st);
                if (e != PB_OK) return e;
                continue;
            }
            if (s.precision == PB_F32_REFINE64) {
                if (r.bb == 0.0) {
                    e = launch_fill<double>(s.x64, s.L.npad, 0.0, st);
                    if (e != PB_OK) return e;
                    s.relres = s.relres_true = 0.0;
                    e = finish_slot(s, PB_OK, st);
                } else {
                    s.relres = s.relres_true = std::sqrt(r.rr) / std::sqrt(r.bb);
                    if (s.relres < s.req.tol) e = finish_slot(s, PB_OK, st);
                    else {
                        s.rr_prev = r.rr;
                        e = enqueue_inner_reset(s, st);
                    }
                }
                if (e != PB_OK) return e;
            }
        }
        for (Slot* sp : admitted) sp->ready = true;
        admitted.clear();
        return PB_OK;
    };
    bool running = false;
    for (auto& up : S->active)
        if (up->solving && up->ready) running = true;
    if (!admitted.empty() && !running && (e = process_admitted()) != PB_OK) return e;

    // ---- one persistent launch over every slot with an inner solve in progress
    std::vector<Slot*> run;
    for (auto& up : S->active)
        if (up->solving && up->ready) run.push_back(up.get());
    if (!run.empty()) {
        std::vector<Layout> Ls;
        std::vector<Tiling> Ts;
        size_t lds = 0;
        for (Slot* sp : run) {
            Ls.push_back(sp->L);
            Ts.push_back(sp->t);
            lds = std::max(lds, sp->t.lds);
        }
        // the coded kernel when every running request has its code words
        bool coded = coded_coefficients() != 0;
        for (Slot* sp : run) coded = coded && sp->coded;
        int cap = coded ? batch_capacity<float>(lds + kCodedLdsBytes, true) : 0;
        if (coded && cap >= (int)run.size()) lds += kCodedLdsBytes;
        else {
            coded = false;
            cap = batch_capacity<float>(lds);
        }
        if (cap < (int)run.size()) {
            set_error("pb_server_step: %zu active solves exceed %d co-resident workgroups", run.size(), cap);
            return PB_ERR_ARG;
        }
        std::vector<int> first(run.size() + 1, 0), chunks(run.size(), chunk);
        share_launch(Ts, cap, chunk, first, chunks);
        const size_t kb = batch_kargs_bytes<float>();
        for (size_t i = 0; i < run.size(); ++i) {
            Slot& s = *run[i];
            const double tol = s.precision == PB_F32 ? s.req.tol : kInnerTol;
            batch_fill_kargs<float>(S->host_table.data() + kb * i, s.L, s.s, s.S, s.partials, s.t, tol, s.maxiter,
                                    s.resume ? 1 : 0, chunks[i], coded ? (const float*)s.s.q2 : nullptr,
                                    coded ? dictionary_table(s.s.q) : nullptr);
        }
        PB_HIP(hipMemcpyAsync(S->table, S->host_table.data(), kb * run.size(), hipMemcpyHostToDevice, st));
        PB_HIP(hipMemcpyAsync(S->first, first.data(), sizeof(int) * first.size(), hipMemcpyHostToDevice, st));
        e = batch_reset_arrivals<float>(S->table, (int)run.size(), st);
        if (e != PB_OK) return e;
        PB_HIP(hipEventRecord(S->ev[0], st));
        // a plain launch sized to co-residency (a cooperative launch would
        // keep the admissions from running beside it): workgroups still
        // waiting for a slot get one as the admissions' kernels finish
        e = batch_launch<float>(S->table, S->first, (int)run.size(), first.back(), lds, st, false, coded);
        if (e != PB_OK) return e;
        PB_HIP(hipEventRecord(S->ev[1], st));
        // every running request's scalars in one read-back
        e = batch_state_digests<float>(S->table, (int)run.size(), S->digests, st);
        if (e != PB_OK) return e;
        PB_HIP(hipMemcpyAsync(S->host_digests.data(), S->digests, sizeof(StateDigest) * run.size(),
                              hipMemcpyDeviceToHost, st));
        // this step's admissions, while the launch runs
        if (!admitted.empty() && (e = process_admitted()) != PB_OK) return e;
        PB_HIP(hipStreamSynchronize(st));
        float ms = 0;
        PB_HIP(hipEventElapsedTime(&ms, S->ev[0], S->ev[1]));
        S->device_seconds += 1e-3 * ms;
        ++S->launches;
        if (coded) ++S->coded_launches;
        // ---- inner solves that finished in this chunk
        std::vector<Slot*> outer_check;
        for (size_t ri = 0; ri < run.size(); ++ri) {
            Slot& s = *run[ri];
            s.resume = true;
            const StateDigest& h = S->host_digests[ri];
            if (!h.done) continue;
            if (s.precision == PB_F32) {
                s.iters = h.iters;
                s.relres = h.bb > 0 ? std::sqrt(h.rr) / std::sqrt(h.bb) : 0.0;
                e = launch_f32_to_f64(s.s.x, s.x64, s.L.npad, st);
                if (e != PB_OK) return e;
                e = launch_residual64(s.op64, s.b64, s.x64, s.L, 0, nullptr, nullptr, s.resp, &s.rec->rr, st);
                if (e != PB_OK) return e;
                e = finish_slot(s, h.status, st);
                if (e != PB_OK) return e;
                outer_check.push_back(&s);
            } else {
                s.iters += h.iters;
                if (h.status < 0) {
                    e = finish_slot(s, h.status, st);
                    if (e != PB_OK) return e;
                    continue;
                }
                ++s.outer;
                e = launch_add_correction(s.x64, s.s.x, s.L.npad, st);
                if (e != PB_OK) return e;
                e = enqueue_outer_residual(s, st);
                if (e != PB_OK) return e;
                e = launch_unpad<double>(s.x64, s.L, s.req.x, st);
                if (e != PB_OK) return e;
                s.solving = false;
                outer_check.push_back(&s);
            }
        }
        if (!outer_check.empty()) {
            if ((e = S->read_recs(st)) != PB_OK) return e;
            PB_HIP(hipStreamSynchronize(st));
            for (Slot* sp : outer_check) {
                Slot& s = *sp;
                const SlotRec r = S->host_recs[s.rec_idx];
                const double rel = r.bb > 0 ? std::sqrt(r.rr) / std::sqrt(r.bb) : 0.0;
                if (s.precision == PB_F32) {
                    s.relres_true = rel;
                    continue;
                }
                s.relres = s.relres_true = rel;
                if (!(rel - rel == 0.0)) s.status = PB_ERR_BREAKDOWN;
                else if (rel < s.req.tol) s.status = PB_OK;
                else if (s.outer >= kMaxOuter || r.rr > 0.25 * s.rr_prev) s.status = PB_NOT_CONVERGED;
                else {
                    s.rr_prev = r.rr;
                    e = enqueue_inner_reset(s, st);
                    if (e != PB_OK) return e;
                    continue;
                }
            }
        }
    }

    if (!admitted.empty() && (e = process_admitted()) != PB_OK) return e;

    // ---- retire finished slots (their potential was handed back on the
    // stream); molecule requests first get their energy from that potential
    bool energies = false;
    for (auto& up : S->active) {
        Slot& s = *up;
        if (s.solving || !s.from_atoms || s.energy_enqueued || !s.energy_host || s.status < 0) continue;
        e = energy_enqueue(&s.grid, s.natoms, s.xyz, s.charge, s.req.x, s.qphi, &s.rec->energy_flags, &s.rec->esum,
                           st);
        if (e != PB_OK) return e;
        s.energy_enqueued = true;
        energies = true;
    }
    if (energies && (e = S->read_recs(st)) != PB_OK) return e;
    PB_HIP(hipStreamSynchronize(st));
    const double tnow = now_s();
    std::vector<std::unique_ptr<Slot>> keep;
    for (auto& up : S->active) {
        Slot& s = *up;
        if (s.solving) {
            keep.push_back(std::move(up));
            continue;
        }
        if (*n_done < max_done) {
            done_ids[*n_done] = s.id;
            pb_info& f = done_infos[*n_done];
            std::memset(&f, 0, sizeof(f));
            f.iters = s.iters;
            f.outer_iters = s.outer;
            f.status = s.status;
            f.relres_recur = s.relres;
            f.relres_true = s.relres_true;
            f.seconds = tnow - s.t_submit;
            ++*n_done;
            if (s.energy_enqueued) *s.energy_host = energy_kcal(S->host_recs[s.rec_idx].esum);
            S->release(s.off, s.bytes);
            S->free_recs.push_back(s.rec_idx);
        } else {
            keep.push_back(std::move(up));   // reported by a later step
        }
    }
    S->active = std::move(keep);
    return PB_OK;
}

extern "C" pb_status pb_server_stats(const pb_server* S, pb_server_stats_t* out) {
    PB_ARG(S && out, "pb_server_stats: null argument");
    out->pending = (int32_t)S->pending.size();
    out->active = (int32_t)S->active.size();
    out->arena_used = S->used();
    out->arena_bytes = S->arena_bytes;
    out->launches = S->launches;
    out->device_seconds = S->device_seconds;
    out->coded_launches = S->coded_launches;
    return PB_OK;
}

extern "C" void pb_server_destroy(pb_server* S) {
    if (!S) return;
    if (S->adm) (void)hipStreamSynchronize(S->adm);
    if (S->ev[0]) (void)hipEventDestroy(S->ev[0]);
    if (S->ev[1]) (void)hipEventDestroy(S->ev[1]);
    if (S->ev_in) (void)hipEventDestroy(S->ev_in);
    if (S->adm) (void)hipStreamDestroy(S->adm);
    delete S;
}
