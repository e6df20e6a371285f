/*
 * pbgpu: MI355X (gfx950) solver for the linear finite-difference
 * Poisson-Boltzmann equation by Jacobi-preconditioned conjugate gradient.
 *
 * The system is Eq. 3 of Qi, Botello-Smith and Luo, "Acceleration of Linear
 * Finite-Difference Poisson-Boltzmann Methods on Graphics Processing Units"
 * (section 2.1): the 7-point stencil with edge dielectrics eps_i, eps_j,
 * eps_k between neighbouring nodes, a diagonal salt term kappa^2 and a
 * right-hand side h^-3 q(i,j,k). It is solved by the preconditioned CG of
 * section 2.2 with M = diag(A) (section 2.4).
 *
 * Conventions shared by every entry point:
 *   - Grid nx*ny*nz; every node is an unknown. Node (i,j,k) sits at
 *     origin + h*(i,j,k) (Angstrom) and has flat index i + nx*(j + ny*k)
 *     (x fastest). Dirichlet values live on a ghost layer one h outside.
 *   - Units are Gaussian: the operator is -div(eps grad phi) + kbar^2 phi
 *     and the right-hand side is 4*pi*q_node/h^3 plus the boundary terms, so
 *     phi is in e/Angstrom; energies are returned in kcal/mol.
 *   - Every array argument is a DEVICE pointer owned by the caller, 8-byte
 *     aligned, unless marked "host". The library never frees caller memory.
 *     Workspaces are caller-allocated device memory of at least the size
 *     the matching *_workspace_bytes query returns (256-byte aligned).
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Work is enqueued on that stream. Entry points that return results to
 *     the host (pb_solve with info, pb_energy) synchronise the stream.
 *   - Arguments are validated before any launch; a bad argument returns
 *     PB_ERR_ARG and touches no memory. pb_last_error() then describes it.
 *   - All reductions run in a fixed order: the same inputs give bitwise
 *     identical outputs on every call.
 */
#ifndef PBGPU_H
#define PBGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PB_OK = 0,
    PB_NOT_CONVERGED = 1,   /* maxiter (or refinement stagnation) reached; x holds the last iterate */
    PB_ERR_ARG = -1,        /* invalid argument (dims, pointers, sizes, negative dielectric, ...) */
    PB_ERR_BREAKDOWN = -2,  /* p.Ap <= 0 or non-finite during CG; x holds the last good iterate */
    PB_ERR_NONFINITE = -3,  /* NaN/Inf in the right-hand side or the initial guess */
    PB_ERR_NOMEM = -4,      /* workspace smaller than required */
    PB_ERR_HIP = -5,        /* a HIP runtime call failed */
    PB_ERR_TIMEOUT = -6     /* a device-side wait exceeded its bound (the kernel exited cleanly) */
} pb_status;

typedef enum {
    PB_F64 = 0,             /* FP64 coefficients, state and arithmetic */
    PB_F32 = 1,             /* FP32 coefficients and state; dot products accumulated in FP64 */
    PB_F32_REFINE64 = 2     /* FP32 inner JPCG inside an FP64 iterative-refinement loop */
} pb_precision;

typedef enum {
    PB_OP_STENCIL = 0,      /* matrix-free stencil fused into one persistent JPCG kernel */
    PB_OP_DIA = 1,          /* 7-diagonal (DIA) SpMV and separate vector kernels, host-driven loop */
    PB_OP_MG = 2            /* CG preconditioned by one geometric-multigrid V-cycle instead of diag(A)
                               (free-space boundary): vertex coarsening by two, coarse edge
                               dielectrics by series/transverse averaging, trilinear transfer,
                               damped-Jacobi smoothing; iterations nearly independent of n */
} pb_operator;

typedef enum {
    PB_BOUNDARY_FREE = 0,     /* free space: Debye-Hueckel Dirichlet values on a ghost layer one h outside */
    PB_BOUNDARY_PERIODIC = 1  /* periodic box of nx*h x ny*h x nz*h: node i+nx is node i (section 2.7) */
} pb_boundary;

typedef struct {
    int32_t nx, ny, nz;     /* nodes per axis (>= 2 for pb_setup / pb_energy, >= 1 for pb_solve;
                               >= 3 with the periodic boundary) */
    int32_t boundary;       /* pb_boundary (pb_setup, pb_energy, pb_solvation_energy) */
    double h;               /* grid spacing, Angstrom (> 0) */
    double origin[3];       /* position of node (0,0,0), Angstrom */
} pb_grid;

typedef struct {
    double tol;             /* stop when ||r||/||b|| < tol (strict, recurrence residual; outer residual for REFINE64) */
    int32_t maxiter;        /* CG iteration limit (per inner solve for REFINE64); <= 0 selects 10*max(nx,ny,nz) */
    int32_t precision;      /* pb_precision */
    int32_t op;             /* pb_operator */
    int32_t warm_start;     /* nonzero: x holds the initial guess on entry; zero: start from x = 0 */
    double inner_tol;       /* REFINE64: inner tolerance relative to the current outer residual; 0 selects 1e-4 */
    int32_t max_outer;      /* REFINE64: outer step limit; 0 selects 20 */
    int32_t boundary;       /* pb_boundary of the system (PERIODIC: stencil operator only, n >= 3 per axis) */
} pb_solve_opts;

typedef struct {
    int32_t iters;          /* CG iterations (summed over inner solves for REFINE64) */
    int32_t outer_iters;    /* refinement steps (0 for plain solves) */
    int32_t status;         /* pb_status of the solve */
    int32_t kernel_launches;/* launches of the iteration kernel (fused form) or iteration loops (DIA form) */
    double relres_recur;    /* recurrence residual ||r||/||b|| at exit (outer FP64 residual for REFINE64) */
    double relres_true;     /* ||b - A x||/||b|| recomputed in FP64 with the FP64 coefficients */
    double seconds;         /* wall time of the call */
    double kernel_seconds;  /* summed duration of those launches / loops, from HIP events on `stream` */
    int32_t coded_launches; /* of kernel_launches, those whose pass read coded coefficients (see
                               pb_set_coded_coefficients); pb_solve and pb_solve_batch (not the graph
                               or the server, whose stats count them) */
    int32_t reserved;       /* zero */
} pb_info;

/* Library version string (static storage). */
const char* pb_version(void);

/* Description of the last error on the calling thread (static storage per thread). */
const char* pb_last_error(void);

/*
 * Device workspace needed by pb_setup for this grid and atom count.
 * Returns 0 for invalid arguments.
 */
size_t pb_setup_workspace_bytes(const pb_grid* grid, int64_t natoms);

/*
 * pb_setup: build the linear system of Eq. 3 from atoms (section 2.7).
 *
 *   xyz[3*natoms]       atom centres (x,y,z interleaved), Angstrom
 *   radius[natoms]      sphere radii, Angstrom
 *   charge[natoms]      partial charges, e
 *   eps_in, eps_out     solute / solvent dielectric constants (> 0)
 *   kappa_d2            Debye screening constant kappa_D^2, Angstrom^-2 (>= 0; 0 = no salt)
 * Outputs (device, written completely):
 *   eps_x[(nx+1)*ny*nz] edge dielectric; entry e + (nx+1)*(j + ny*k) is the
 *                       edge between nodes (e-1,j,k) and (e,j,k), e = 0..nx
 *                       (index -1 and nx are ghost nodes)
 *   eps_y[nx*(ny+1)*nz] entry i + nx*(e + (ny+1)*k): nodes (i,e-1,k)-(i,e,k)
 *   eps_z[nx*ny*(nz+1)] entry i + nx*(j + ny*e):     nodes (i,j,e-1)-(i,j,e)
 *   kappa2[N]           kbar^2 = eps_out*kappa_D^2 at solvent nodes, 0 inside
 *   rhs[N]              4*pi*q_node/h^3 + Debye-Hueckel Dirichlet boundary terms
 *   qgrid[N]            (nullable) the spread node charges q(i,j,k), e
 *   mask[(nx+2)*(ny+2)*(nz+2)] (nullable) 1 where the node (ghosts included,
 *                       padded index (i+1) + (nx+2)*((j+1) + (ny+2)*(k+1)))
 *                       lies strictly inside an atom sphere, else 0
 * Steps: node classification (|x-c|^2 < R^2 in FP64, no contraction), node
 * dielectric eps_in/eps_out, two-point harmonic edge means 2ab/(a+b),
 * trilinear charge spreading (g = (c-o)/h, i0 = clamp(floor g, 0, n-2)),
 * and the screened Coulomb sum sum_a q_a exp(-kappa_D d)/(eps_out d) on the
 * six ghost faces folded into rhs through the ghost-side edge dielectric.
 * Errors: PB_ERR_ARG for dims < 2, h <= 0, natoms < 0 or > 2^21-1, null
 * required pointers, eps <= 0, kappa_d2 < 0, or an atom centre outside the
 * node box (checked on the device; outputs are then undefined).
 */
pb_status pb_setup(const pb_grid* grid, int64_t natoms,
                   const double* xyz, const double* radius, const double* charge,
                   double eps_in, double eps_out, double kappa_d2,
                   double* eps_x, double* eps_y, double* eps_z,
                   double* kappa2, double* rhs, double* qgrid, uint8_t* mask,
                   void* workspace, size_t workspace_bytes, void* stream);

typedef enum {
    PB_EDGE_NODE = 0,       /* two-point harmonic mean of the endpoint node dielectrics (pb_setup) */
    PB_EDGE_FRACTION = 1    /* weighted harmonic mean 1/(f/eps_in + (1-f)/eps_out), f the fraction of
                               the edge inside the union of the spheres (section 2.7's "weighted
                               harmonic average" taken over the edge; free-space boundary) */
} pb_edge_model;

typedef struct {
    int32_t edge_model;     /* pb_edge_model */
    int32_t reserved[7];    /* zero */
} pb_setup_opts;

/* Device workspace needed by pb_setup_ex. Returns 0 for invalid arguments. */
size_t pb_setup_ex_workspace_bytes(const pb_grid* grid, int64_t natoms, const pb_setup_opts* opts);

/*
 * pb_setup_ex: pb_setup with options. With PB_EDGE_FRACTION each edge
 * dielectric is 1/(f/eps_in + (1-f)/eps_out), where f is the fraction of the
 * edge segment (between its two nodes, ghosts included) inside the union of
 * the atom spheres: each sphere covers the chord where the squared distance
 * across the edge's line is below R^2; the chords clipped to the edge are
 * merged (overlapping or touching pieces join) and their lengths summed in
 * increasing order; f = 0 gives eps_out and f = 1 eps_in exactly. Node
 * classification, the salt term, charges and the boundary are as pb_setup.
 * Errors as pb_setup, and PB_ERR_ARG for invalid options, the fractional
 * model with the periodic boundary, or more than 16 separate inside pieces
 * on one edge.
 * Status: the device path of PB_EDGE_FRACTION is switched off; this call
 * returns PB_ERR_ARG for it before launching anything (pb_last_error says
 * so). PB_EDGE_NODE is unaffected.
 */
pb_status pb_setup_ex(const pb_grid* grid, int64_t natoms,
                      const double* xyz, const double* radius, const double* charge,
                      double eps_in, double eps_out, double kappa_d2, const pb_setup_opts* opts,
                      double* eps_x, double* eps_y, double* eps_z,
                      double* kappa2, double* rhs, double* qgrid, uint8_t* mask,
                      void* workspace, size_t workspace_bytes, void* stream);

/*
 * Device workspace needed by pb_solve for this grid and option set
 * (precision and operator). Returns 0 for invalid arguments.
 */
size_t pb_solve_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, const pb_solve_opts* opts);

/*
 * pb_solve: Jacobi-preconditioned CG (section 2.2 with M = diag(A), section
 * 2.4) on the system of Eq. 3 given by the arrays pb_setup writes:
 *   eps_x, eps_y, eps_z  staggered edge dielectrics (layouts as in pb_setup), >= 0
 *   kappa2[N]            kbar^2 per node, >= 0
 *   rhs[N]               right-hand side (boundary terms already folded in)
 *   x[N]                 in: initial guess when opts->warm_start, else ignored;
 *                        out: the potential phi
 * The library applies the 1/h^2 factor. With precision PB_F32 the
 * coefficients are rounded to FP32; PB_F32_REFINE64 repeats
 * { r = b - A x in FP64; FP32 JPCG on A d = r to opts->inner_tol; x += d }
 * until the FP64 residual is below opts->tol.
 * A zero right-hand side returns x = 0 after 0 iterations.
 * info (host, nullable) receives the iteration counts and residuals.
 * Errors: PB_ERR_ARG (dims < 1, h <= 0, tol <= 0, null pointers, negative
 * or non-finite coefficients; with the stencil operator also rows wider than
 * the fused kernel's in-plane halo allows: nx > 1024 in FP32, > 512 in FP64,
 * checked before any launch), PB_ERR_NOMEM (workspace too small),
 * PB_ERR_NONFINITE (NaN/Inf in rhs or guess), PB_ERR_BREAKDOWN,
 * PB_NOT_CONVERGED, PB_ERR_TIMEOUT, PB_ERR_HIP.
 */
pb_status pb_solve(int32_t nx, int32_t ny, int32_t nz, double h,
                   const double* eps_x, const double* eps_y, const double* eps_z,
                   const double* kappa2, const double* rhs, double* x,
                   const pb_solve_opts* opts,
                   void* workspace, size_t workspace_bytes, void* stream,
                   pb_info* info);

/*
 * pb_solve_noalloc: pb_solve for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation). Same arguments, operators, precisions and results as
 * pb_solve, but no workspace: the solve runs in a scratch array the library
 * holds on each GPU for the life of the process
 * (pb_solve_noalloc_max_bytes(), 256 MiB, enough for grids up to about
 * 2.2M nodes such as 129^3), and the call makes no device allocation and
 * records no HIP events (info->kernel_seconds is 0). The scratch is shared
 * by every call on one GPU: calls that overlap on one GPU (other host
 * threads, other streams) race and must be serialised by the caller.
 * Errors: those of pb_solve, and PB_ERR_NOMEM (pb_last_error() says so)
 * when the grid needs more scratch than the library holds, before any
 * launch.
 */
pb_status pb_solve_noalloc(int32_t nx, int32_t ny, int32_t nz, double h,
                           const double* eps_x, const double* eps_y, const double* eps_z,
                           const double* kappa2, const double* rhs, double* x,
                           const pb_solve_opts* opts, void* stream, pb_info* info);
/* Bytes of the per-GPU scratch of pb_solve_noalloc. */
size_t pb_solve_noalloc_max_bytes(void);

/*
 * pb_stream_copy: copies `bytes` (a multiple of 16) from src to dst on
 * `stream` with 16-byte vector loads and stores, with the nontemporal hint
 * when `nontemporal` is nonzero: the access kinds of the fused JPCG pass's
 * streams, without arithmetic, halo or barrier. A measurement aid: timing it
 * gives the streaming ceiling the solver's bandwidth is compared with. src
 * and dst are device pointers, 16-byte aligned, not overlapping.
 * Errors: PB_ERR_ARG (null or misaligned), PB_ERR_HIP.
 */
pb_status pb_stream_copy(const void* src, void* dst, size_t bytes, int32_t nontemporal, void* stream);

/* One tiling of the fused stencil kernel, as chosen by pb_autotune. */
typedef struct {
    int32_t block;          /* threads per workgroup */
    int32_t groups;         /* 16-byte vector groups per thread per plane (segment = block*groups*vector) */
    int32_t zchunk;         /* z-planes per tile */
    int32_t grid;           /* workgroups of the persistent launch */
    double us_per_iter;     /* measured microseconds per CG iteration (pb_autotune only) */
    int32_t candidates;     /* tilings timed (pb_autotune only) */
    int32_t scheme;         /* pass form: 0 stores A.p (48 B/node/iteration in FP32),
                               1 recomputes A.p_old from p_old (40 B/node/iteration) */
    int32_t streaming;      /* 1: nontemporal loads and stores for the streams no step reads again
                               (the default once a pass's arrays exceed 1.75 times the 256 MiB
                               last-level cache); 0: cached accesses; -1 (pb_set_tuning only): the
                               shape's default */
    int32_t segments;       /* in-plane segments per plane (tiles = segments x z-chunks); 0
                               (pb_set_tuning only): any */
} pb_tuning;

/*
 * pb_autotune: time every feasible tiling of the fused stencil kernel
 * (block size, vector groups per thread, workgroups per CU and hence z-chunk)
 * for `iters_per_trial` iterations on the given system, and record the
 * fastest for this device, grid shape and precision (FP64 vs FP32/REFINE64)
 * in the library's per-process table; later pb_solve calls on that shape use
 * it. The iteration itself is the solver's own (section 2.2 with M = diag A);
 * only its launch shape is searched. Arrays and workspace as for pb_solve
 * (opts->op must be PB_OP_STENCIL; opts->tol and maxiter are ignored).
 * best (host, nullable) receives the winner. Errors: PB_ERR_ARG (also for a
 * zero right-hand side), PB_ERR_NOMEM, PB_ERR_HIP.
 */
pb_status pb_autotune(int32_t nx, int32_t ny, int32_t nz, double h,
                      const double* eps_x, const double* eps_y, const double* eps_z,
                      const double* kappa2, const double* rhs, const pb_solve_opts* opts,
                      int32_t iters_per_trial, void* workspace, size_t workspace_bytes,
                      void* stream, pb_tuning* best);

/*
 * pb_set_tuning: record a tiling (for instance one saved from an earlier
 * pb_autotune) for this grid shape and precision on the current device.
 * Fields us_per_iter/candidates are ignored. PB_ERR_ARG if the tiling is not
 * feasible for this shape and device.
 */
pb_status pb_set_tuning(int32_t nx, int32_t ny, int32_t nz, int32_t precision, const pb_tuning* tuning);

/*
 * pb_get_tuning: the tiling pb_solve will use for this grid shape and
 * precision on the current device: the one recorded by pb_autotune or
 * pb_set_tuning, else the library's default choice. us_per_iter and
 * candidates are 0. Errors: PB_ERR_ARG (bad dims or precision, null out, or
 * no feasible tiling: nx too large for the in-plane halo).
 */
pb_status pb_get_tuning(int32_t nx, int32_t ny, int32_t nz, int32_t precision, pb_tuning* out);

/*
 * Coded coefficients (FP32 stencil solves with the 40-byte pass form, free
 * boundary: pb_solve, pb_solve_batch, the batch graph and the server). The
 * operator of Eq. 3 built from the two-point dielectric model takes few
 * distinct values: three edge dielectrics over h^2 (and zero at the faces)
 * and a few dozen diagonals. When the FP32 couplings cx, cy, cz and the
 * diagonal together hold at most 256 distinct values, the library stores one
 * 4-byte word of dictionary codes per node (in workspace the 40-byte form
 * leaves unused) and the pass reads it instead of the four FP32 arrays: 28
 * bytes per node per iteration instead of 40. The decoded values are the
 * FP32 coefficients themselves, so potentials, iteration counts and
 * residuals are bitwise those of the uncoded pass. Otherwise (more values,
 * or a grid of fewer than 8,450 padded positions) the uncoded pass runs. A
 * pb_solve_batch or server launch is coded only when all its problems are;
 * a batch graph rebuilds every dictionary at each replay and its kernel
 * decides per problem on the device, so coefficients that change between
 * replays are handled. pb_info.coded_launches and
 * pb_server_stats_t.coded_launches report which ran. Building a dictionary
 * reads the operator arrays once more; the decision reads a flag back to the
 * host once per pb_solve, per batch and per admitted request (never in a
 * graph replay).
 *
 * pb_set_coded_coefficients(0) turns the coded pass off for the process;
 * 1 (the default) turns it back on. pb_get_coded_coefficients returns the
 * setting. Not synchronised with solves running on other threads.
 */
void pb_set_coded_coefficients(int32_t on);
int32_t pb_get_coded_coefficients(void);

/*
 * pb_set_periodic_pass: the pass form of fused solves with the periodic
 * boundary of section 2.7, process-wide. -1 (the default): the tiling model's
 * choice, which is the 40-byte pass wherever it applies; 0: the pass that
 * stores A p (48 bytes per node in FP32); 1: the 40-byte pass, which runs on
 * ghost-row copies of the operator and state (two copied rows below row 0
 * and above row ny-1 of every plane; grids with nx >= 5 and ny >= 4, others
 * take form 0), coded as pb_set_coded_coefficients says. The iterates of the
 * forms agree up to rounding; coded and uncoded 40-byte passes agree bit for
 * bit. Values other than -1, 0, 1 are ignored. pb_get_periodic_pass returns
 * the setting. Not synchronised with solves running on other threads.
 */
void pb_set_periodic_pass(int32_t form);
int32_t pb_get_periodic_pass(void);

/*
 * pb_tiling_candidates: the feasible tilings of the fused stencil kernel for
 * this grid shape and precision on the current device, i.e. the search space
 * of pb_autotune (the same iteration, launched in different shapes). Writes
 * min(total, max) entries into out (host array, nullable when max == 0) and
 * the total into *count (host). us_per_iter is 0; candidates holds the total.
 * Errors: PB_ERR_ARG (bad dims or precision, null count), PB_ERR_HIP.
 */
pb_status pb_tiling_candidates(int32_t nx, int32_t ny, int32_t nz, int32_t precision, pb_tuning* out,
                               int32_t max, int32_t* count);

/*
 * Batched solves (many independent systems, e.g. snapshots of a trajectory,
 * on grids of uneven size). Each problem uses the array layouts of pb_solve.
 */
typedef struct {
    int32_t nx, ny, nz;     /* nodes per axis (>= 1; nx <= 512 in FP32, <= 256 in FP64) */
    int32_t maxiter;        /* <= 0 selects 10*max(nx,ny,nz) */
    double h;               /* grid spacing, Angstrom */
    double tol;             /* stop when ||r||/||b|| < tol (recurrence residual) */
    const double* eps_x;    /* device arrays as for pb_solve */
    const double* eps_y;
    const double* eps_z;
    const double* kappa2;
    const double* rhs;
    double* x;              /* in: guess when warm_start; out: phi */
    int32_t warm_start;
    int32_t reserved;
} pb_problem;

/* Device workspace for a batch (depends on every problem's shape and the precision). 0 if invalid. */
size_t pb_batch_workspace_bytes(int32_t nprob, const pb_problem* probs, int32_t precision);

/*
 * pb_solve_batch: solve all problems (section 2.2 with M = diag(A)) in ONE
 * persistent launch. Workgroups are shared out in proportion to each
 * problem's expected work; each problem synchronises only its own
 * workgroups, and its tiling and reduction order depend on its shape and the
 * device's batch z-chunk alone, so a problem's result is bitwise identical
 * alone and in any mix.
 * precision: PB_F32 or PB_F64. infos (host, nprob entries, nullable) receive
 * per-problem iterations, status and FP64 true residuals; kernel_seconds is
 * the whole batch's device time. Returns PB_OK, PB_NOT_CONVERGED if any
 * problem did not converge, or the first error. nprob may not exceed the
 * device's co-resident workgroups of the batch kernel (PB_ERR_ARG).
 */
pb_status pb_solve_batch(int32_t nprob, const pb_problem* probs, int32_t precision,
                         void* workspace, size_t workspace_bytes, void* stream, pb_info* infos);

/*
 * Batch tiling. The batched and served kernels cut each problem into
 * z-chunks of this many planes (default 32, one setting per device). Under one
 * setting a problem's tiling, and so its result, depends on its shape alone.
 * pb_batch_set_zchunk takes 1..4096 (PB_ERR_ARG otherwise).
 *
 * pb_batch_autotune times the batch kernel on the given problems for each
 * candidate z-chunk (16, 24, 32, 48, 64). Every problem is capped at
 * iters_per_trial iterations, and the problems' x arrays are read (warm start)
 * but not written. The fastest candidate becomes the device's setting;
 * best_zchunk and best_seconds (host, nullable) receive it and its trial's
 * device time. Errors: PB_ERR_ARG (as pb_solve_batch, or iters_per_trial < 1),
 * PB_ERR_NOMEM (workspace below pb_batch_autotune_workspace_bytes), PB_ERR_HIP.
 */
pb_status pb_batch_set_zchunk(int32_t zchunk);
int32_t pb_batch_get_zchunk(void);
size_t pb_batch_autotune_workspace_bytes(int32_t nprob, const pb_problem* probs, int32_t precision);
pb_status pb_batch_autotune(int32_t nprob, const pb_problem* probs, int32_t precision, int32_t iters_per_trial,
                            void* workspace, size_t workspace_bytes, void* stream, int32_t* best_zchunk,
                            double* best_seconds);

/*
 * The same batch recorded once in a HIP graph (preparation, the persistent
 * solve and the hand-back), replayed by pb_batch_graph_launch. Array
 * pointers and shapes are fixed at creation; their contents may change
 * between launches (e.g. new snapshots written into the same buffers).
 * pb_batch_graph_results synchronises `stream` and reads per-problem infos.
 * The handle owns host-side state only; the workspace stays caller-owned and
 * must outlive the handle. Calls on one handle must not overlap.
 */
typedef struct pb_batch_graph pb_batch_graph;
pb_status pb_batch_graph_create(int32_t nprob, const pb_problem* probs, int32_t precision,
                                void* workspace, size_t workspace_bytes, void* stream,
                                pb_batch_graph** graph);
pb_status pb_batch_graph_launch(pb_batch_graph* graph, void* stream);
pb_status pb_batch_graph_results(pb_batch_graph* graph, void* stream, pb_info* infos);
/* 1 if the graph holds a cooperative launch, 0 if it fell back to a plain launch sized to co-residency. */
int32_t pb_batch_graph_is_cooperative(const pb_batch_graph* graph);
void pb_batch_graph_destroy(pb_batch_graph* graph);

/*
 * Continuous-batching server. Requests are queued by pb_server_submit; each
 * pb_server_step admits queued requests in arrival order while slots and the
 * caller's HBM arena allow (the arena size is the memory budget), advances
 * every active request by up to `chunk` CG iterations in ONE persistent
 * launch (the requests' work overlaps on the device), and retires requests
 * that converged or failed, freeing their memory for the next admissions.
 * An unfinished request's CG state stays in the arena and the next step
 * resumes it exactly: a request's result does not depend on chunking or on
 * the other requests in flight. precision PB_F32 runs FP32 Jacobi-PCG to the
 * request's tol; PB_F32_REFINE64 cycles FP64 residual / FP32 correction to a
 * relative 1e-4 / FP64 update until the FP64 residual is below tol.
 * Request arrays (pb_problem, nx <= 512) are caller-owned and must stay
 * valid until the request is reported done; its x receives phi then.
 * The server owns host-side state only; the arena stays caller-owned and
 * must outlive the server. Calls on one server must not overlap.
 */
typedef struct pb_server pb_server;

typedef struct {
    int32_t pending;        /* queued, not yet admitted */
    int32_t active;         /* admitted, not yet reported */
    size_t arena_used;      /* bytes in use (slot memory plus the launch table) */
    size_t arena_bytes;
    int64_t launches;       /* persistent launches so far */
    double device_seconds;  /* their summed device time (HIP events) */
    int64_t coded_launches; /* of those, launches that read coded coefficients (every running request's
                               operator fit its dictionary; see pb_set_coded_coefficients) */
} pb_server_stats_t;

/* Arena bytes one request occupies while admitted (0 if it cannot be served). */
size_t pb_server_request_bytes(const pb_problem* request);
/* arena: device memory, 256-byte aligned; max_slots in [1, 4096]. */
pb_status pb_server_create(void* arena, size_t arena_bytes, int32_t max_slots, pb_server** server);
/* Queue a request; *id receives its handle. PB_ERR_ARG if it can never fit. */
pb_status pb_server_submit(pb_server* server, const pb_problem* request, int32_t precision, int64_t* id);
/*
 * Queue a request given as a molecule, as the paper's user supplies it
 * (section 2.7: atom centres, radii and charges on a grid): at admission the
 * server runs the setup of pb_setup (two-point edge dielectrics, free-space
 * Debye-Hueckel boundary) inside the request's own arena memory, then solves
 * as for pb_server_submit; when the request finishes, x[N] (device, FP64,
 * layout as pb_solve's) holds the potential and *energy (host, nullable)
 * receives 1/2 sum_a q_a phi(c_a) in kcal/mol, both valid once pb_server_step
 * reports the request. xyz[3*natoms], radius[natoms], charge[natoms] are
 * device arrays that must stay valid until then. An atom outside the node
 * box finishes the request with PB_ERR_ARG. Arena bytes per request:
 * pb_server_request_bytes_atoms.
 */
pb_status pb_server_submit_atoms(pb_server* server, const pb_grid* grid, int64_t natoms, const double* xyz,
                                 const double* radius, const double* charge, double eps_in, double eps_out,
                                 double kappa_d2, double tol, int32_t maxiter, int32_t precision, double* x,
                                 double* energy, int64_t* id);
size_t pb_server_request_bytes_atoms(const pb_grid* grid, int64_t natoms);
/*
 * One admission + chunk + retirement round on `stream` (synchronises it).
 * Admissions (the setup of molecule requests, preparation) run on a stream
 * of the server's own, ordered after the work enqueued on `stream` before
 * the call and overlapping the running chunk; a request admitted by a step
 * joins the next step's launch, or this one's when no other request is
 * running. The chunk runs as a plain (not cooperative) persistent launch
 * sized to co-residency, so it must not share the device with kernels that
 * never finish.
 * Up to max_done finished requests are reported in done_ids/done_infos
 * (pb_info.seconds = submit-to-completion time); *n_done receives the count.
 * Finished requests beyond max_done are reported by later steps.
 */
pb_status pb_server_step(pb_server* server, int32_t chunk, void* stream, int32_t max_done,
                         int32_t* n_done, int64_t* done_ids, pb_info* done_infos);
pb_status pb_server_stats(const pb_server* server, pb_server_stats_t* stats);
void pb_server_destroy(pb_server* server);

/* Device workspace needed by pb_energy. Returns 0 for invalid arguments. */
size_t pb_energy_workspace_bytes(int64_t natoms);

/*
 * pb_energy: electrostatic energy 1/2 sum_a q_a phi(c_a) in kcal/mol
 * (section 3.1 reports energies), with phi(c_a) the trilinear interpolation
 * of x at the atom centre using the spreading weights of pb_setup.
 *   x[N]           the potential (device)
 *   atom_phi       (nullable, device, natoms) receives phi(c_a)
 *   energy         (host) receives the energy
 * The atom sum runs in a fixed order. Errors: PB_ERR_ARG as for pb_setup.
 */
pb_status pb_energy(const pb_grid* grid, int64_t natoms,
                    const double* xyz, const double* charge, const double* x,
                    double* atom_phi, double* energy,
                    void* workspace, size_t workspace_bytes, void* stream);

/*
 * Device workspace needed by pb_solvation_energy (the five system arrays,
 * two potentials and the larger of the setup, solve and energy workspaces).
 * Returns 0 for invalid arguments.
 */
size_t pb_solvation_workspace_bytes(const pb_grid* grid, int64_t natoms, const pb_solve_opts* opts);

/*
 * pb_solvation_energy: solvation (reaction-field) energy
 *     dG = E(solvent) - E(reference)   (kcal/mol)
 * with E = 1/2 sum_a q_a phi(c_a) as in pb_energy, from two complete
 * setups and solves on the same grid with the same charges: the solvent
 * system (eps_in inside, eps_out and kappa_d2 outside) and the reference
 * with a uniform eps_in and no salt (eps_out = eps_in, kappa_d2 = 0). The
 * grid self-energy of the charges is the same in both and cancels; this is
 * the energy the paper's accuracy comparison uses (section 3.1). For one
 * ion the continuum value is Born's -332.06 q^2/(2a) (1/eps_in - 1/eps_out).
 *   atoms, eps_in, eps_out, kappa_d2   as for pb_setup
 *   opts            solve options for both solves (opts->warm_start must be 0)
 *   phi_solv, phi_ref (device, N each, nullable) receive the two potentials
 *   dG (host) the solvation energy; e_solv, e_ref (host, nullable) the two energies
 *   info_solv, info_ref (host, nullable) the two solves' pb_info
 * Runs on `stream` and synchronises it. Returns PB_NOT_CONVERGED if either
 * solve hit its limit (dG is still written); errors as for pb_setup,
 * pb_solve and pb_energy, PB_ERR_NOMEM for a short workspace.
 */
pb_status pb_solvation_energy(const pb_grid* grid, int64_t natoms,
                              const double* xyz, const double* radius, const double* charge,
                              double eps_in, double eps_out, double kappa_d2,
                              const pb_solve_opts* opts, double* phi_solv, double* phi_ref,
                              double* dG, double* e_solv, double* e_ref,
                              pb_info* info_solv, pb_info* info_ref,
                              void* workspace, size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PBGPU_H */
