// lbks_cd.hip -- concurrent dynamics: the orbitals as complex fields advanced in
// real time together with the nuclei (section "Concurrent Dynamics", eq. KSLBCD).
//
// Reading: the populations stay at equilibrium with their moment (f_jp = xi_p psi_j,
// the omega = 1 reading of the relaxation), so the two-step time-centred lattice
// equation advances the complex orbitals,
//   psi_j^{n+1} = psi_j^{n-1} - 2 i h (H - E_j) psi_j^n,  H u = K_h u + S_chi(V u),
//   K_h u = -(S_xi u - u) / (D dx^2),
// H being the operator whose steady state the relaxation reaches and E_j the
// orbital's energy at the last (re)start (the source U_jp, which holds the
// orbital's energy at E_j, read as each orbital's energy reference: a global
// phase per orbital that leaves densities and forces unchanged and keeps the
// two-step scheme's parasitic mode from growing through V; restarts re-centre
// E_j as the nuclei move).  W = 0 (the evolution keeps the orbitals orthonormal
// up to its own error).  Orbitals are
// FP64 complex, interleaved (re, im) per node: [orbital][site] of double2.  Every
// kernel gives each XCD one contiguous range of tiles, so its L2 holds the
// neighbour planes of the 19-point reads.
#include <type_traits>

#include "lbks_device.h"

namespace lbks {

namespace {

struct C2 {
    double re, im;
};

// H u at node s for every orbital (complex), from the orbitals `in` and the FP64
// potential; the 19 departure nodes are read through the caches.
template <int NO>
__device__ __forceinline__ void apply_h_node(const InstDesc &d, const double2 *__restrict__ in, int s, int x, int y,
                                             int z, const CdRef &ref, C2 (&out)[NO], C2 (&centre)[NO])
{
    const int n = orbitals<NO>(d);
    const size_t N = (size_t)d.nsite;
    const double2 *__restrict__ g = in;
    const auto *Vd = gmem((const double *)d.Vd);
    C2 su[NO], sv[NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) {
        su[j] = {0.0, 0.0};
        sv[j] = {0.0, 0.0};
        centre[j] = {0.0, 0.0};
        if (j < n) {
            const double2 c = g[(size_t)j * N + s];
            centre[j] = {c.x, c.y};
        }
    }
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const int vx = VX(p), vy = VY(p), vz = VZ(p);
        const bool ok = (unsigned)(x - vx) < (unsigned)d.nx && (unsigned)(y - vy) < (unsigned)d.ny &&
                        (unsigned)(z - vz) < (unsigned)d.nz;
        if (ok) {
            const int src = s - (vx + d.nx * (vy + d.ny * vz));
            const double vn = Vd[src];
#pragma unroll
            for (int j = 0; j < NO; ++j) {
                if (j < n) {
                    const double2 u = g[(size_t)j * N + src];
                    su[j].re += d.xi[p] * u.x;
                    su[j].im += d.xi[p] * u.y;
                    sv[j].re += d.chi[p] * vn * u.x;
                    sv[j].im += d.chi[p] * vn * u.y;
                }
            }
        }
    }
    const double kfac = -1.0 / (d.D * d.h * d.h);
#pragma unroll
    for (int j = 0; j < NO; ++j) {
        out[j].re = kfac * (su[j].re - centre[j].re) + sv[j].re - ref.e[j] * centre[j].re;
        out[j].im = kfac * (su[j].im - centre[j].im) + sv[j].im - ref.e[j] * centre[j].im;
    }
}

// Density and multipole partials of the complex orbitals w at node s (as the
// orthonormalisation kernel forms them from real orbitals).
template <int NO>
__device__ __forceinline__ void density_moments(const InstDesc &d, const C2 (&w)[NO], int s, int x, int y, int z,
                                                double (&m)[NMOM])
{
    const int n = orbitals<NO>(d);
    double rho = 0.0;
#pragma unroll
    for (int j = 0; j < NO; ++j)
        if (j < n) rho += d.occ[j] * (w[j].re * w[j].re + w[j].im * w[j].im);
    ((double *)d.rho)[s] = rho;
    const double rx = node_coord(x, d.nx, d.h), ry = node_coord(y, d.ny, d.h), rz = node_coord(z, d.nz, d.h);
    const double r2 = rx * rx + ry * ry + rz * rz;
    m[0] = rho;
    m[1] = rx * rho;
    m[2] = ry * rho;
    m[3] = rz * rho;
    m[4] = (3.0 * rx * rx - r2) * rho;
    m[5] = (3.0 * ry * ry - r2) * rho;
    m[6] = (3.0 * rz * rz - r2) * rho;
    m[7] = 3.0 * rx * ry * rho;
    m[8] = 3.0 * rx * rz * rho;
    m[9] = 3.0 * ry * rz * rho;
}

// out = (H - E_j) in.
template <int NO>
__global__ __launch_bounds__(BS) void k_cd_apply(const InstDesc *__restrict__ descs, const double2 *__restrict__ in,
                                                 double2 *__restrict__ out, CdRef ref)
{
    const InstDesc &d = descs[0];
    const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);   // each XCD walks one contiguous tile range
    const int s = tile * BS + threadIdx.x;
    if (s >= d.nsite) return;
    const int n = orbitals<NO>(d);
    const int x = s % d.nx, yz = s / d.nx, y = yz % d.ny, z = yz / d.ny;
    C2 hu[NO], c[NO];
    apply_h_node<NO>(d, in, s, x, y, z, ref, hu, c);
    const size_t N = (size_t)d.nsite;
#pragma unroll
    for (int j = 0; j < NO; ++j)
        if (j < n) out[(size_t)j * N + s] = make_double2(hu[j].re, hu[j].im);
}

// First two time levels: prev = psi_hat (real), and
// cur = prev - i h t1 - (h^2 / 2) t2 with t1 = H' prev, t2 = H' t1, H' = H - E_j; density and
// multipole partials of cur.
template <int NO>
__global__ __launch_bounds__(BS) void k_cd_taylor(const InstDesc *__restrict__ descs, const double2 *__restrict__ prev,
                                                  const double2 *__restrict__ t1, const double2 *__restrict__ t2,
                                                  double2 *__restrict__ cur, double h)
{
    const InstDesc &d = descs[0];
    const int n = orbitals<NO>(d);
    const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);   // each XCD walks one contiguous tile range
    const int s = tile * BS + threadIdx.x;
    double m[NMOM];
#pragma unroll
    for (int q = 0; q < NMOM; ++q) m[q] = 0.0;
    if (s < d.nsite) {
        const size_t N = (size_t)d.nsite;
        C2 w[NO];
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            w[j] = {0.0, 0.0};
            if (j < n) {
                const double2 a = prev[(size_t)j * N + s], b = t1[(size_t)j * N + s], c = t2[(size_t)j * N + s];
                // -i h b = h (b.im, -b.re)
                w[j].re = a.x + h * b.y - 0.5 * h * h * c.x;
                w[j].im = a.y - h * b.x - 0.5 * h * h * c.y;
                cur[(size_t)j * N + s] = make_double2(w[j].re, w[j].im);
            }
        }
        const int x = s % d.nx, yz = s / d.nx, y = yz % d.ny, z = yz / d.ny;
        density_moments<NO>(d, w, s, x, y, z, m);
    }
    block_sum_store(m, NMOM, d.m_part + tile, d.ntile);
}

// prev <- prev - 2 i h (H - E_j) cur (the new time level overwrites the oldest), with the
// density and multipole partials of the new level.
template <int NO>
__global__ __launch_bounds__(BS) void k_cd_step(const InstDesc *__restrict__ descs, const double2 *__restrict__ cur,
                                                double2 *__restrict__ prev, double h, CdRef ref)
{
    const InstDesc &d = descs[0];
    const int n = orbitals<NO>(d);
    const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);   // each XCD walks one contiguous tile range
    const int s = tile * BS + threadIdx.x;
    double m[NMOM];
#pragma unroll
    for (int q = 0; q < NMOM; ++q) m[q] = 0.0;
    if (s < d.nsite) {
        const size_t N = (size_t)d.nsite;
        const int x = s % d.nx, yz = s / d.nx, y = yz % d.ny, z = yz / d.ny;
        C2 hu[NO], c[NO], w[NO];
        apply_h_node<NO>(d, cur, s, x, y, z, ref, hu, c);
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            w[j] = {0.0, 0.0};
            if (j < n) {
                const double2 a = prev[(size_t)j * N + s];
                // -2 i h (re + i im) = 2 h (im, -re)
                w[j].re = a.x + 2.0 * h * hu[j].im;
                w[j].im = a.y - 2.0 * h * hu[j].re;
                prev[(size_t)j * N + s] = make_double2(w[j].re, w[j].im);
            }
        }
        density_moments<NO>(d, w, s, x, y, z, m);
    }
    block_sum_store(m, NMOM, d.m_part + tile, d.ntile);
}

// Per-node energy terms of the complex orbitals, laid out as k_energy_terms lays
// them out ([NO kinetic][NO potential][base terms]), so k_energy_finalize applies:
// Re <psi_j|K_h psi_j> and Re <psi_j|S_chi(V psi_j)> (= re.K re + im.K im and
// likewise), then rho V_ext, rho V_H, rho eps_x, rho eps_c, rho.
template <int NO>
__global__ __launch_bounds__(BS) void k_cd_energy_terms(const InstDesc *__restrict__ descs,
                                                        const double2 *__restrict__ cur)
{
    const InstDesc &d = descs[0];
    const int n = orbitals<NO>(d);
    const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);   // each XCD walks one contiguous tile range
    const int s = tile * BS + threadIdx.x;
    double v[2 * NO + NEBASE];
#pragma unroll
    for (int q = 0; q < 2 * NO + NEBASE; ++q) v[q] = 0.0;
    if (s < d.nsite) {
        const size_t N = (size_t)d.nsite;
        const double2 *__restrict__ g = cur;
        const auto *Vd = gmem((const double *)d.Vd);
        const int x = s % d.nx, yz = s / d.nx, y = yz % d.ny, z = yz / d.ny;
        C2 su[NO], sv[NO], u0[NO];
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            su[j] = sv[j] = u0[j] = {0.0, 0.0};
            if (j < n) {
                const double2 c = g[(size_t)j * N + s];
                u0[j] = {c.x, c.y};
            }
        }
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const int vx = VX(p), vy = VY(p), vz = VZ(p);
            const bool ok = (unsigned)(x - vx) < (unsigned)d.nx && (unsigned)(y - vy) < (unsigned)d.ny &&
                            (unsigned)(z - vz) < (unsigned)d.nz;
            if (ok) {
                const int src = s - (vx + d.nx * (vy + d.ny * vz));
                const double vn = Vd[src];
#pragma unroll
                for (int j = 0; j < NO; ++j) {
                    if (j < n) {
                        const double2 u = g[(size_t)j * N + src];
                        su[j].re += d.xi[p] * u.x;
                        su[j].im += d.xi[p] * u.y;
                        sv[j].re += d.chi[p] * vn * u.x;
                        sv[j].im += d.chi[p] * vn * u.y;
                    }
                }
            }
        }
        const double kfac = -1.0 / (d.D * d.h * d.h);
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            v[j] = u0[j].re * (kfac * (su[j].re - u0[j].re)) + u0[j].im * (kfac * (su[j].im - u0[j].im));
            v[NO + j] = u0[j].re * sv[j].re + u0[j].im * sv[j].im;
        }
        const double rho = ((const double *)d.rho)[s];
        double ex, ec, vx_, vc_;
        xc_eval(d.xc, rho, d.rho_floor, ex, ec, vx_, vc_);
        double vh = 0.0;
        if (d.hartree) vh = d.vh[((size_t)(z + 1) * (d.ny + 2) + (y + 1)) * (d.nx + 2) + (x + 1)];
        v[2 * NO + 0] = rho * d.vext[s];
        v[2 * NO + 1] = rho * vh;
        v[2 * NO + 2] = rho * ex;
        v[2 * NO + 3] = rho * ec;
        v[2 * NO + 4] = rho;
    }
    block_sum_store(v, 2 * NO + NEBASE, d.e_part + tile, d.ntile);
}

// prev = (psi_hat, 0): the real orthonormal orbitals as the first time level.
template <int NO>
__global__ __launch_bounds__(BS) void k_cd_init(const InstDesc *__restrict__ descs, double2 *__restrict__ prev)
{
    const InstDesc &d = descs[0];
    const int n = orbitals<NO>(d);
    const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);   // each XCD walks one contiguous tile range
    const int s = tile * BS + threadIdx.x;
    if (s >= d.nsite) return;
    const size_t N = (size_t)d.nsite;
    const double *ph = (const double *)d.psihat;
#pragma unroll
    for (int j = 0; j < NO; ++j)
        if (j < n) prev[(size_t)j * N + s] = make_double2(ph[(size_t)j * N + s], 0.0);
}

template <typename F>
int dispatch_no(const Plan &pl, F &&f)
{
    switch (pl.no) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 8: return f(std::integral_constant<int, 8>{});
    default: return f(std::integral_constant<int, 16>{});
    }
}

}  // namespace

int launch_cd_init(const Plan &pl, double2 *prev, hipStream_t st)
{
    return dispatch_no(pl, [&](auto no) {
        k_cd_init<decltype(no)::value><<<pl.ntile, BS, 0, st>>>(pl.d_desc, prev);
        return (int)hipGetLastError();
    });
}

int launch_cd_apply(const Plan &pl, const double2 *in, double2 *out, const CdRef &ref, hipStream_t st)
{
    return dispatch_no(pl, [&](auto no) {
        k_cd_apply<decltype(no)::value><<<pl.ntile, BS, 0, st>>>(pl.d_desc, in, out, ref);
        return (int)hipGetLastError();
    });
}

int launch_cd_taylor(const Plan &pl, const double2 *prev, const double2 *t1, const double2 *t2, double2 *cur,
                     double h, hipStream_t st)
{
    return dispatch_no(pl, [&](auto no) {
        k_cd_taylor<decltype(no)::value><<<pl.ntile, BS, 0, st>>>(pl.d_desc, prev, t1, t2, cur, h);
        return (int)hipGetLastError();
    });
}

int launch_cd_step(const Plan &pl, const double2 *cur, double2 *prev, double h, const CdRef &ref, hipStream_t st)
{
    return dispatch_no(pl, [&](auto no) {
        k_cd_step<decltype(no)::value><<<pl.ntile, BS, 0, st>>>(pl.d_desc, cur, prev, h, ref);
        return (int)hipGetLastError();
    });
}

int launch_cd_energy_terms(const Plan &pl, const double2 *cur, hipStream_t st)
{
    return dispatch_no(pl, [&](auto no) {
        k_cd_energy_terms<decltype(no)::value><<<pl.ntile, BS, 0, st>>>(pl.d_desc, cur);
        return (int)hipGetLastError();
    });
}

}  // namespace lbks
