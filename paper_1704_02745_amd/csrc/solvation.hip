// Solvation (reaction-field) energy from two solves on one grid: the solvent
// system (eps_in inside, eps_out and salt outside) and the uniform eps_in
// reference without salt. Both energies carry the same grid self-energy,
// which cancels in the difference; section 3.1 compares such energies.
// Host-side composition of the library's own setup, solve and energy.
#include "pb_internal.hpp"

#include <cmath>
#include <cstring>

namespace pb {
namespace {

struct SolvLayout {
    size_t ex, ey, ez, k2, rhs, phi_s, phi_r, scratch, scratch_bytes, total;
};

bool solv_grid_ok(const pb_grid* g) {
    return g && g->nx >= 2 && g->ny >= 2 && g->nz >= 2 && std::isfinite(g->h) && g->h > 0.0;
}

// Byte offsets in the workspace: the five system arrays, two potentials, then
// one scratch region shared in turn by setup, solve and energy.
bool solv_layout(const pb_grid* g, int64_t natoms, const pb_solve_opts* opts, SolvLayout& o) {
    if (!solv_grid_ok(g) || !opts) return false;
    const size_t nx = g->nx, ny = g->ny, nz = g->nz, n = nx * ny * nz;
    const size_t sw = pb_setup_workspace_bytes(g, natoms);
    pb_solve_opts so = *opts;
    so.boundary = g->boundary;   // the solves take the grid's boundary
    const size_t vw = pb_solve_workspace_bytes(g->nx, g->ny, g->nz, &so);
    const size_t ew = pb_energy_workspace_bytes(natoms);
    if (sw == 0 || vw == 0 || ew == 0) return false;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    o.ex = take(8 * (nx + 1) * ny * nz);
    o.ey = take(8 * nx * (ny + 1) * nz);
    o.ez = take(8 * nx * ny * (nz + 1));
    o.k2 = take(8 * n);
    o.rhs = take(8 * n);
    o.phi_s = take(8 * n);
    o.phi_r = take(8 * n);
    o.scratch_bytes = std::max(sw, std::max(vw, ew));
    o.scratch = take(o.scratch_bytes);
    o.total = off;
    return true;
}

}  // namespace
}  // namespace pb

using namespace pb;

extern "C" size_t pb_solvation_workspace_bytes(const pb_grid* g, int64_t natoms, const pb_solve_opts* opts) {
    SolvLayout o;
    return solv_layout(g, natoms, opts, o) ? o.total : 0;
}

extern "C" pb_status pb_solvation_energy(const pb_grid* g, int64_t natoms, const double* xyz,
                                         const double* radius, const double* charge, double eps_in,
                                         double eps_out, double kappa_d2, const pb_solve_opts* opts,
                                         double* phi_solv, double* phi_ref, double* dG, double* e_solv,
                                         double* e_ref, pb_info* info_solv, pb_info* info_ref, void* workspace,
                                         size_t workspace_bytes, void* stream) {
    PB_ARG(solv_grid_ok(g), "pb_solvation_energy: grid needs nx,ny,nz >= 2 and h > 0");
    PB_ARG(opts && dG && workspace, "pb_solvation_energy: null opts, dG or workspace");
    PB_ARG(!opts->warm_start, "pb_solvation_energy: warm_start is not supported (both solves start at 0)");
    SolvLayout o;
    PB_ARG(solv_layout(g, natoms, opts, o), "pb_solvation_energy: invalid grid, atom count or options");
    if (workspace_bytes < o.total) {
        set_error("pb_solvation_energy: workspace of %zu bytes, %zu needed", workspace_bytes, o.total);
        return PB_ERR_NOMEM;
    }
    char* w = (char*)workspace;
    double* ex = (double*)(w + o.ex);
    double* ey = (double*)(w + o.ey);
    double* ez = (double*)(w + o.ez);
    double* k2 = (double*)(w + o.k2);
    double* rhs = (double*)(w + o.rhs);
    double* phis[2] = {phi_solv ? phi_solv : (double*)(w + o.phi_s), phi_ref ? phi_ref : (double*)(w + o.phi_r)};
    void* scratch = w + o.scratch;
    const double eo[2] = {eps_out, eps_in};
    const double kd[2] = {kappa_d2, 0.0};
    pb_info* infos[2] = {info_solv, info_ref};
    double e[2] = {0.0, 0.0};
    pb_status worst = PB_OK;
    for (int s = 0; s < 2; ++s) {
        pb_status st = pb_setup(g, natoms, xyz, radius, charge, eps_in, eo[s], kd[s], ex, ey, ez, k2, rhs, nullptr,
                                nullptr, scratch, o.scratch_bytes, stream);
        if (st != PB_OK) return st;
        pb_info info{};
        pb_solve_opts so = *opts;
        so.boundary = g->boundary;
        st = pb_solve(g->nx, g->ny, g->nz, g->h, ex, ey, ez, k2, rhs, phis[s], &so, scratch, o.scratch_bytes,
                      stream, &info);
        if (infos[s]) *infos[s] = info;
        if (st < 0) return st;
        if (st == PB_NOT_CONVERGED) worst = PB_NOT_CONVERGED;
        st = pb_energy(g, natoms, xyz, charge, phis[s], nullptr, &e[s], scratch, o.scratch_bytes, stream);
        if (st != PB_OK) return st;
    }
    *dG = e[0] - e[1];
    if (e_solv) *e_solv = e[0];
    if (e_ref) *e_ref = e[1];
    return worst;
}
