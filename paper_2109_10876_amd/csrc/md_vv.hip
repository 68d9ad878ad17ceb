// md_vv.hip -- md_vv_step: velocity-Verlet half steps and the rebuild test.
//
// Sec. 2.1 and Fig. 1 of the paper: Integrate1 (half kick, drift), force
// evaluation, Integrate2 (half kick); the skin sets how often atoms are
// re-binned.  The list stays valid while no atom has moved more than half
// the skin since the last build (two atoms closing in at most skin in
// total), so phase 1 flags a replica for rebuild when
//     max_i |x_i - x_build_i|^2 > (skin/2)^2.
// Positions are not wrapped here (they are wrapped at rebuild time), so the
// difference is the true displacement.
//
// One thread per atom; per-unit partials of the kinetic energy (fixed-order
// sum) and of the maximum displacement, then one workgroup per replica.
// With the thermostat (phases 2 and 3), each atom first adds md_langevin's
// force to the force it is about to use, with the velocity on entry (the one
// the forces were evaluated with) and the same Philox normals.
#include "md_philox.hpp"

namespace md {
namespace {

struct VVArgs {
    const int32_t *atom_off, *unit_rep, *unit_off;
    double *x, *y, *z, *vx, *vy, *vz;
    double *pos4;
    double *fx, *fy, *fz;
    const double *xb, *yb, *zb;
    const int32_t *type;
    const double *inv_mass;
    int32_t ntypes;
    double hdt, dt;
    double *partial;
    // thermostat (LANG variant)
    const int32_t *id;
    const double *mass;
    double gamma, kT_dt2;   // 2 T / dt
    uint32_t seed_lo, seed_hi;
    const uint64_t *step;
};

template <int PHASE, bool LANG>
__global__ __launch_bounds__(kUnit) void k_vv(VVArgs a)
{
    __shared__ double red[kWavesPerUnit];
    const int u = blockIdx.x;
    const Unit w = unit_of(u, a.unit_rep, a.unit_off, a.atom_off);
    const int i = w.begin + threadIdx.x;
    double ke = 0.0, d2 = 0.0;
    if (i < w.end) {
        const double im = a.inv_mass[a.ntypes > 1 ? a.type[i] : 0];
        double fx = a.fx[i], fy = a.fy[i], fz = a.fz[i];
        double vx = a.vx[i], vy = a.vy[i], vz = a.vz[i];
        if (LANG) {
            const double m = a.mass[a.ntypes > 1 ? a.type[i] : 0];
            double g[3];
            thermostat_normals(static_cast<uint32_t>(a.id[i]), *a.step, a.seed_lo, a.seed_hi, g);
            const double amp = sqrt(a.gamma * m * a.kT_dt2);
            const double gm = a.gamma * m;
            fx += -gm * vx + amp * g[0];
            fy += -gm * vy + amp * g[1];
            fz += -gm * vz + amp * g[2];
            a.fx[i] = fx;
            a.fy[i] = fy;
            a.fz[i] = fz;
        }
        const double k = a.hdt * im;
        if (PHASE >= 2) {   // Integrate2 (phase 2, first half of phase 3)
            vx = fma(k, fx, vx);
            vy = fma(k, fy, vy);
            vz = fma(k, fz, vz);
            ke = 0.5 * (vx * vx + vy * vy + vz * vz) / im;
        }
        if (PHASE != 2) {   // Integrate1
            vx = fma(k, fx, vx);
            vy = fma(k, fy, vy);
            vz = fma(k, fz, vz);
            const double x = fma(a.dt, vx, a.x[i]);
            const double y = fma(a.dt, vy, a.y[i]);
            const double z = fma(a.dt, vz, a.z[i]);
            a.x[i] = x;
            a.y[i] = y;
            a.z[i] = z;
            if (a.pos4) reinterpret_cast<double4 *>(a.pos4)[i] = make_double4(x, y, z, 0.0);
            const double ex = x - a.xb[i], ey = y - a.yb[i], ez = z - a.zb[i];
            d2 = norm2(ex, ey, ez);
        }
        a.vx[i] = vx;
        a.vy[i] = vy;
        a.vz[i] = vz;
    }
    if (PHASE >= 2) {
        const double s = block_sum(ke, red);
        if (threadIdx.x == 0) a.partial[size_t(u) * kPartials + 2] = s;
    }
    if (PHASE != 2) {
        const double m = block_max(d2, red);
        if (threadIdx.x == 0) a.partial[size_t(u) * kPartials + 3] = m;
    }
}

// Per replica: kinetic energy (fixed-order sum) and the rebuild gate.
__global__ __launch_bounds__(kFin) void k_vv_finalize(const int32_t *unit_off,
                                                      const double *partial, double lim2,
                                                      double *ke, uint32_t *gate,
                                                      uint64_t *step)
{
    // the thermostat's noise counter advances after every atom has read it
    if (step && blockIdx.x == 0 && threadIdx.x == 0) *step += 1u;
    __shared__ double red[kFin / kWave];
    const int r = blockIdx.x;
    const int u0 = unit_off[r], u1 = unit_off[r + 1];
    double s = 0.0, m = 0.0;
#pragma unroll 4
    for (int u = u0 + threadIdx.x; u < u1; u += kFin) {
        if (ke) s += partial[size_t(u) * kPartials + 2];
        if (gate) m = fmax(m, partial[size_t(u) * kPartials + 3]);
    }
    s = block_sum_n<kFin>(s, red);
    m = block_max_n<kFin>(m, red);
    if (threadIdx.x == 0) {
        if (ke) ke[r] = s;
        if (gate) gate[r] = m > lim2 ? 1u : 0u;
    }
}

}  // namespace
}  // namespace md

extern "C" int md_vv_step(const md_batch *b, md_atoms *atoms, int32_t phase, double dt,
                          const double *inv_mass, int32_t ntypes, double skin, uint32_t *gate,
                          double *ke, const md_thermostat *thermo, void *ws, size_t ws_bytes,
                          uint32_t *status, void *stream)
{
    using namespace md;
    (void)status;
    int e = check_batch(b);
    if (e != MD_OK) return e;
    if (phase < 1 || phase > 3 || !atoms || !inv_mass || !ws) return MD_EINVAL;
    if (ntypes < 1 || ntypes > MD_MAX_TYPES || (ntypes > 1 && !atoms->type)) return MD_EINVAL;
    if (!atoms->x || !atoms->y || !atoms->z || !atoms->vx || !atoms->vy || !atoms->vz ||
        !atoms->fx || !atoms->fy || !atoms->fz)
        return MD_EINVAL;
    if (phase != 2 && (!gate || !atoms->xb || !atoms->yb || !atoms->zb)) return MD_EINVAL;
    if (!(skin >= 0.0)) return MD_EINVAL;
    if (thermo && (phase == 1 || !thermo->step || !thermo->mass || !atoms->id ||
                   !(thermo->gamma >= 0.0) || !(thermo->temperature >= 0.0) || !(dt > 0.0)))
        return MD_EINVAL;
    const WsLayout l = ws_layout(b);
    if (ws_bytes < l.total) return MD_ENOWS;
    double *partial = ws_at<double>(ws, l.partial);
    VVArgs a{b->atom_off, b->unit_rep, b->unit_off, atoms->x, atoms->y, atoms->z, atoms->vx,
             atoms->vy, atoms->vz, atoms->pos4, atoms->fx, atoms->fy, atoms->fz, atoms->xb, atoms->yb,
             atoms->zb, atoms->type, inv_mass, ntypes, 0.5 * dt, dt, partial,
             atoms->id, thermo ? thermo->mass : nullptr, thermo ? thermo->gamma : 0.0,
             thermo ? 2.0 * thermo->temperature / dt : 0.0,
             thermo ? static_cast<uint32_t>(thermo->seed) : 0u,
             thermo ? static_cast<uint32_t>(thermo->seed >> 32) : 0u,
             thermo ? thermo->step : nullptr};
    hipStream_t s = as_stream(stream);
    const dim3 grid(b->n_units), block(kUnit);
    if (phase == 1) hipLaunchKernelGGL((k_vv<1, false>), grid, block, 0, s, a);
    else if (phase == 2 && thermo) hipLaunchKernelGGL((k_vv<2, true>), grid, block, 0, s, a);
    else if (phase == 2) hipLaunchKernelGGL((k_vv<2, false>), grid, block, 0, s, a);
    else if (thermo) hipLaunchKernelGGL((k_vv<3, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_vv<3, false>), grid, block, 0, s, a);
    double *ke_out = phase >= 2 ? ke : nullptr;
    uint32_t *gate_out = phase != 2 ? gate : nullptr;
    uint64_t *step = thermo ? thermo->step : nullptr;
    if (ke_out || gate_out || step)
        hipLaunchKernelGGL(k_vv_finalize, dim3(b->R), dim3(kFin), 0, s, b->unit_off, partial,
                           0.25 * skin * skin, ke_out, gate_out, step);
    return launch_status();
}
