// md_langevin.hip -- md_langevin: Langevin thermostat in force form.
//
// Sec. 4 of the paper equilibrates both systems to a target temperature
// with a Langevin thermostat.  In force form each atom receives friction and
// a random kick, F += -gamma m v + sqrt(2 gamma m T / dt) xi, evaluated with
// the velocity at the time of the force evaluation.  The normals xi come
// from a counter-based generator (md_philox.hpp) so that they depend only on
// (seed, step, atom id).
#include "md_philox.hpp"

namespace md {
namespace {

struct LangevinArgs {
    const int32_t *atom_off, *unit_rep, *unit_off;
    const double *vx, *vy, *vz;
    double *fx, *fy, *fz;
    const int32_t *type, *id;
    const double *mass;
    int32_t ntypes;
    double gamma, kT_dt2;   // 2 T / dt
    uint32_t seed_lo, seed_hi;
    const uint64_t *step;
};

__global__ __launch_bounds__(kUnit) void k_langevin(LangevinArgs a)
{
    const Unit w = unit_of(blockIdx.x, a.unit_rep, a.unit_off, a.atom_off);
    const int i = w.begin + threadIdx.x;
    if (i >= w.end) return;
    double g[3];
    thermostat_normals(static_cast<uint32_t>(a.id[i]), *a.step, a.seed_lo, a.seed_hi, g);
    const double m = a.mass[a.ntypes > 1 ? a.type[i] : 0];
    const double amp = sqrt(a.gamma * m * a.kT_dt2);
    const double gm = a.gamma * m;
    a.fx[i] += -gm * a.vx[i] + amp * g[0];
    a.fy[i] += -gm * a.vy[i] + amp * g[1];
    a.fz[i] += -gm * a.vz[i] + amp * g[2];
}

__global__ void k_step_advance(uint64_t *step) { *step += 1u; }

}  // namespace
}  // namespace md

extern "C" int md_langevin(const md_batch *b, const md_atoms *atoms, const double *mass,
                           int32_t ntypes, double gamma, double temperature, double dt,
                           uint64_t seed, uint64_t *step, uint32_t *status, void *stream)
{
    using namespace md;
    (void)status;
    int e = check_batch(b);
    if (e != MD_OK) return e;
    if (!atoms || !atoms->vx || !atoms->vy || !atoms->vz || !atoms->fx || !atoms->fy ||
        !atoms->fz || !atoms->id || !mass || !step)
        return MD_EINVAL;
    if (ntypes < 1 || ntypes > MD_MAX_TYPES || (ntypes > 1 && !atoms->type)) return MD_EINVAL;
    if (!(gamma >= 0.0) || !(temperature >= 0.0) || !(dt > 0.0)) return MD_EINVAL;
    LangevinArgs a{b->atom_off, b->unit_rep, b->unit_off, atoms->vx, atoms->vy, atoms->vz,
                   atoms->fx, atoms->fy, atoms->fz, atoms->type, atoms->id, mass, ntypes,
                   gamma, 2.0 * temperature / dt, static_cast<uint32_t>(seed),
                   static_cast<uint32_t>(seed >> 32), step};
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(k_langevin, dim3(b->n_units), dim3(kUnit), 0, s, a);
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(1), 0, s, step);
    return launch_status();
}
