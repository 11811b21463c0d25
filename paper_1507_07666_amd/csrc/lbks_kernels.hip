// lbks_kernels.hip -- device kernels of the lattice kinetic Kohn-Sham
// relaxation for gfx950 (CDNA4, wave64).
//
// One lattice step of a solve runs, on the device only:
//   overlap_finalize  S_jk = <psi_j|psi_k> from per-tile partials, Cholesky
//                     S = L L^T, C = L^{-T} (GS) or the paper's normalisation
//                     and Lambda_jk (W mode)               [orthogonality constraints]
//   orthonormalise    psi_hat = psi C (psi* = psi C* in W mode), rho = sum occ psi_hat^2,
//                     multipole partials of rho            [density]
//   multipole_finalize, ghost   Dirichlet data of the Hartree problem
//   sor (x 2 per sweep)         red/black over-relaxation of lap_h V_H = -4 pi rho
//   potential         V = V_ext + V_H + v_xc(rho)          [KS potential]
//   stream_collide    f_jp(r) <- (1-omega) g_jp + omega xi_p psi*_j - dt chi_p V psi_hat_j
//                     taken at r - v_p (pull), g = f C; fused moment psi_j = sum_p f_jp
//                     and overlap partials                 [LB equation per orbital]
// Every workgroup has BS = 256 threads (4 waves); each thread owns one node.
// Reductions are fixed-order (wave butterfly, then waves in order, then tiles
// in order): results do not depend on batch composition and are repeatable.
#include "lbks_device.h"

namespace lbks {

int orbital_bucket(int n)
{
    return n <= 5 ? n : (n <= 8 ? 8 : 16);
}



// -------------------------------------------------------------- init kernels

// Initial orbitals from the SplitMix64 counter-based generator (Steele, Lea,
// Flood 2014): draw k = j * sites + node of seed s is mix(s + (k+1) * gamma).
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <typename T>
__global__ __launch_bounds__(BS) void k_init_psi(const InstDesc *__restrict__ descs,
                                                 const int2 *__restrict__ tiles, int mode,
                                                 double sigma, double noise, uint64_t seed)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int s = tr.tile * BS + threadIdx.x;
    if (s >= d.nsite) return;
    const int x = s % d.nx, yz = s / d.nx, y = yz % d.ny, z = yz / d.ny;
    const double rx = node_coord(x, d.nx, d.h), ry = node_coord(y, d.ny, d.h), rz = node_coord(z, d.nz, d.h);
    const double env = exp(-(rx * rx + ry * ry + rz * rz) / (2.0 * sigma * sigma));
    T *psi = (T *)d.psi;
    for (int j = 0; j < d.n_orb; ++j) {
        const uint64_t k = (uint64_t)j * (uint64_t)d.nsite + (uint64_t)s;
        const double u = (double)(splitmix64(seed, k) >> 11) * 0x1.0p-53;
        const double v = (mode == 0) ? env + noise * (2.0 * u - 1.0) : env * (2.0 * u - 1.0);
        psi[(size_t)j * d.nsite + s] = (T)v;
    }
}

template <typename T>
__global__ __launch_bounds__(BS) void k_psi_from_stage(const InstDesc *__restrict__ descs,
                                                       const int2 *__restrict__ tiles)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int s = tr.tile * BS + threadIdx.x;
    if (s >= d.nsite) return;
    T *psi = (T *)d.psi;
    for (int j = 0; j < d.n_orb; ++j) psi[(size_t)j * d.nsite + s] = (T)d.stage[(size_t)j * d.nsite + s];
}

// Equilibrium populations f_jp = xi_p psi_j.
template <typename T>
__global__ __launch_bounds__(BS) void k_equilibrium(const InstDesc *__restrict__ descs,
                                                    const int2 *__restrict__ tiles, int parity)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int s = tr.tile * BS + threadIdx.x;
    if (s >= d.nsite) return;
    const T *psi = (const T *)d.psi;
    T *f = (T *)(parity ? d.f1 : d.f0);
    const size_t N = (size_t)d.nsite;
    for (int j = 0; j < d.n_orb; ++j) {
        const T v = psi[(size_t)j * N + s];
#pragma unroll
        for (int p = 0; p < Q; ++p) f[((size_t)j * Q + p) * N + s] = (T)d.xi[p] * v;
    }
}

// Zeroth moment psi_j = sum_p f_jp at the node and overlap partials.
template <typename T, int NO>
__global__ __launch_bounds__(BS) void k_moment(const InstDesc *__restrict__ descs,
                                               const int2 *__restrict__ tiles, int parity)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int n = orbitals<NO>(d);
    const int s = tr.tile * BS + threadIdx.x;
    const bool valid = s < d.nsite;
    const size_t N = (size_t)d.nsite;
    const T *f = (const T *)(parity ? d.f1 : d.f0);
    T *psi = (T *)d.psi;
    T acc[NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) acc[j] = (T)0;
    if (valid) {
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            if (j < n) {
#pragma unroll
                for (int p = 0; p < Q; ++p) acc[j] += f[((size_t)j * Q + p) * N + s];
                psi[(size_t)j * N + s] = acc[j];
            }
        }
    }
    overlap_partial<T, NO>(acc, n, d.s_part + tr.tile, d.ntile);
}

// Overlap partials of the orbital state itself.  With skip_brick, instances whose
// partials the brick update has already written are left alone.
template <typename T, int NO>
__global__ __launch_bounds__(BS) void k_overlap_psi(const InstDesc *__restrict__ descs,
                                                    const int2 *__restrict__ tiles, int skip_brick)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    if (skip_brick && brick_partials(d.ntile, d.ntile_brick)) return;   // uniform per workgroup
    const int n = orbitals<NO>(d);
    const int s = tr.tile * BS + threadIdx.x;
    const T *psi = (const T *)d.psi;
    T a[NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) a[j] = (s < d.nsite && j < n) ? psi[(size_t)j * d.nsite + s] : (T)0;
    overlap_partial<T, NO>(a, n, d.s_part + tr.tile, d.ntile);
}

// ---------------------------------------------------------- overlap / GS

// The coefficients of the orthonormalisation from the overlap S (packed lower,
// h^3 included), by the first wave; every thread of the workgroup calls it.  GS:
// S = L L^T, C = L^{-T} (psi_hat_j = sum_{l<=j} psi_l C_lj, classical Gram-Schmidt
// order).  W: n_j = sqrt(S_jj), C = diag(1/n), C*_lj = -Lambda_jl / n_l (l < j),
// C*_jj = 1/n_j with Lambda_jl = S_jl / (n_j n_l), i.e. psi*_j = psi_hat_j -
// sum_{l<j} Lambda_jl psi_hat_l.  Writes C[l ld + j] (GS: l <= j < n; W: the
// diagonal) and C*[l ld + j] (W: l <= j < n) and nothing else; n <= M.  Returns
// true on the lanes of the first wave that found S not positive definite.
template <int M>
__device__ bool ortho_coefficients(const double *S, int n, int ortho, double *C, double *Cs, int ld)
{
    __shared__ double L[M][M + 1];
    __shared__ double Li[M][M + 1];
    // lane i owns row i of L, lane c column c of L^{-1}
    const int lane = threadIdx.x;
    const bool w0 = threadIdx.x < 64;
    bool bad = false;
    auto Sget = [&](int i, int j) { return i >= j ? S[i * (i + 1) / 2 + j] : S[j * (j + 1) / 2 + i]; };
    if (ortho == 0) {
        // Cholesky S = L L^T by columns: L_jj = sqrt(S_jj - sum_k<j L_jk^2),
        // L_ij = (S_ij - sum_k<j L_ik L_jk) / L_jj for i > j
        for (int j = 0; j < n; ++j) {
            double sum = 0.0;
            if (w0 && lane >= j && lane < n) {
                sum = Sget(lane, j);
                for (int k = 0; k < j; ++k) sum -= L[lane][k] * L[j][k];
            }
            double djj = __shfl(sum, j, 64);
            if (!(djj > 0.0)) {
                if (w0) bad = true;
                djj = 1.0;
            }
            const double ljj = sqrt(djj);
            if (w0 && lane == j) L[j][j] = ljj;
            else if (w0 && lane > j && lane < n) L[lane][j] = sum / ljj;
            __syncthreads();
        }
        // C = L^{-T}: column c of L^{-1} by forward substitution; C[l][j] = Linv[j][l]
        if (w0 && lane < n) {
            const int c = lane;
            for (int i = c; i < n; ++i) {
                double sum = (i == c) ? 1.0 : 0.0;
                for (int k = c; k < i; ++k) sum -= L[i][k] * Li[k][c];
                Li[i][c] = sum / L[i][i];
            }
            for (int j = c; j < n; ++j) C[c * ld + j] = Li[j][c];
        }
    } else if (w0 && lane < n) {
        const int j = lane;
        const double sjj = Sget(j, j);
        if (!(sjj > 0.0)) bad = true;
        const double nj = sqrt(sjj > 0.0 ? sjj : 1.0);
        C[j * ld + j] = 1.0 / nj;
        Cs[j * ld + j] = 1.0 / nj;
        for (int l = 0; l < j; ++l) {
            const double sll = Sget(l, l);
            const double nl = sqrt(sll > 0.0 ? sll : 1.0);
            Cs[l * ld + j] = -(Sget(j, l) / (nj * nl)) / nl;
        }
    }
    return bad;
}

// S from the tile partials (fixed order), then C and C* (ortho_coefficients).
// Not launched when every instance of the plan folds the overlap.
__global__ __launch_bounds__(BS) void k_overlap_finalize(const InstDesc *__restrict__ descs,
                                                         const int *__restrict__ list)
{
    const GroupRef gr = resolve_group(list);
    const InstDesc &d = descs[gr.inst];
    const int n = d.n_orb, np = npair_of(n);
    __shared__ double S[MAXO * (MAXO + 1) / 2];
    if (!reduce_columns(d.s_part, d.ntile, np, d.g_part, (unsigned *)(d.scal + SC_CNT), gr.g, S)) return;
    const int lane = threadIdx.x;
    bool bad = false;
    if (threadIdx.x < 64)
        for (int q = lane; q < np; q += 64) {
            S[q] *= d.h3;
            d.scal[SC_S + q] = S[q];
            if (!isfinite(S[q])) bad = true;
        }
    __syncthreads();
    // entries outside the n x n block stay zero from creation
    if (ortho_coefficients<MAXO>(S, n, d.ortho, d.C, d.C + MAXO * MAXO, MAXO)) bad = true;
    bad = __any(bad);
    if (bad && lane == 0) d.scal[SC_ERR] = 1.0;   // lane 0 of the first wave: bad only ever set there
}

// psi_hat = psi C (psi* = psi C* in W mode), rho = sum_j occ_j psi_hat_j^2 and
// the multipole partials q, p_a, Q_ab of rho.  FOLD (every instance of the launch
// folds the overlap, at most five orbitals): there is no finalize kernel before
// this one; every workgroup sums S from the tile partials in that kernel's order
// (fold_columns) and forms C and C* itself, and the workgroup of tile 0 also
// stores what the finalize kernel stores (S, C, C*, the error flag) for the
// kernels after this one.  Without FOLD the kernel reads C from memory, with no
// trace of the fold in its code.
template <typename T, int NO, bool W, bool FOLD>
__global__ __launch_bounds__(BS) void k_orthonormalise(const InstDesc *__restrict__ descs,
                                                       const int2 *__restrict__ tiles)
{
    static_assert(!FOLD || NO <= 5, "the fold serves buckets of at most five orbitals");
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int n = orbitals<NO>(d);
    constexpr int NF = FOLD ? NO : 1;
    [[maybe_unused]] __shared__ double fC[2][NF * NF];   // this workgroup's C and C* ([l * NO + j]) when folded
    if constexpr (FOLD) {
        {
            __shared__ double fS[NF * (NF + 1) / 2];
            const int np = npair_of(n), t = threadIdx.x;
            if (t < 2 * NF * NF) fC[t / (NF * NF)][t % (NF * NF)] = 0.0;
            fold_columns(d.s_part, d.ntile, np, fS);
            bool bad = false;
            if (t < np) {
                fS[t] *= d.h3;
                if (!isfinite(fS[t])) bad = true;
            }
            __syncthreads();
            if (ortho_coefficients<NF>(fS, n, d.ortho, fC[0], fC[1], NF)) bad = true;
            __syncthreads();
            if (tr.tile == 0) {
                if (t < np) d.scal[SC_S + t] = fS[t];
                if (t < NF * NF) {
                    const int l = t / NF, j = t % NF;
                    if (l <= j && j < n) {
                        if (d.ortho == 0) d.C[l * MAXO + j] = fC[0][t];
                        else {
                            if (l == j) d.C[j * MAXO + j] = fC[0][t];
                            d.C[MAXO * MAXO + l * MAXO + j] = fC[1][t];
                        }
                    }
                }
                bad = __any(bad);
                if (bad && t == 0) d.scal[SC_ERR] = 1.0;   // set in the first wave only
            }
        }
    }
    const int s = tr.tile * BS + threadIdx.x;
    double m[NMOM];
#pragma unroll
    for (int q = 0; q < NMOM; ++q) m[q] = 0.0;
    if (s < d.nsite) {
        const size_t N = (size_t)d.nsite;
        const auto *psi = gmem((const T *)d.psi);
        auto *ph = gmem((T *)d.psihat);
        auto *pst = gmem((T *)d.psistar);
        double ps[NO];
#pragma unroll
        for (int l = 0; l < NO; ++l) ps[l] = (l < n) ? (double)psi[(size_t)l * N + s] : 0.0;
        // up to five orbitals, the coefficients and occupations are read before the
        // first store: the compiler cannot tell that the stores leave them alone, and
        // would otherwise reload them after every store and wait for it (for 8 and 16
        // orbitals the tables would not fit the registers)
        constexpr int NC = NO <= 5 ? NO : 1;
        double c[NC][NC], cs[NC][NC], occ[NC];
        if constexpr (NO <= 5) {
#pragma unroll
            for (int j = 0; j < NO; ++j) {
                occ[j] = (j < n) ? d.occ[j] : 0.0;
#pragma unroll
                for (int l = 0; l < NO; ++l) {
                    const bool use = l <= j && j < n;
                    if constexpr (FOLD) {
                        c[l][j] = use ? fC[0][l * NF + j] : 0.0;
                        cs[l][j] = (W && use) ? fC[1][l * NF + j] : 0.0;
                    } else {
                        c[l][j] = use ? d.C[l * MAXO + j] : 0.0;
                        cs[l][j] = (W && use) ? d.C[MAXO * MAXO + l * MAXO + j] : 0.0;
                    }
                }
            }
        }
        auto C_ = [&](int l, int j) { if constexpr (NO <= 5) return c[l][j]; else return d.C[l * MAXO + j]; };
        auto Cs_ = [&](int l, int j) {
            if constexpr (NO <= 5) return cs[l][j]; else return d.C[MAXO * MAXO + l * MAXO + j];
        };
        auto occ_ = [&](int j) { if constexpr (NO <= 5) return occ[j]; else return d.occ[j]; };
        double rho = 0.0;
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            if (j < n) {
                double hat = 0.0;
                if (W) {
                    hat = ps[j] * C_(j, j);
                    double st = 0.0;
#pragma unroll
                    for (int l = 0; l <= j; ++l) st += ps[l] * Cs_(l, j);
                    pst[(size_t)j * N + s] = (T)st;
                } else {
#pragma unroll
                    for (int l = 0; l <= j; ++l) hat += ps[l] * C_(l, j);
                }
                const T hs = (T)hat;
                ph[(size_t)j * N + s] = hs;
                const double hd = (double)hs;
                rho += occ_(j) * hd * hd;
            }
        }
        const T rs = (T)rho;
        ((T *)d.rho)[s] = rs;
        const double r = (double)rs;
        const int x = s % d.nx, yz = s / d.nx, y = yz % d.ny, z = yz / d.ny;
        const double rx = node_coord(x, d.nx, d.h), ry = node_coord(y, d.ny, d.h), rz = node_coord(z, d.nz, d.h);
        const double r2 = rx * rx + ry * ry + rz * rz;
        m[0] = r;
        m[1] = rx * r;
        m[2] = ry * r;
        m[3] = rz * r;
        m[4] = (3.0 * rx * rx - r2) * r;
        m[5] = (3.0 * ry * ry - r2) * r;
        m[6] = (3.0 * rz * rz - r2) * r;
        m[7] = 3.0 * rx * ry * r;
        m[8] = 3.0 * rx * rz * r;
        m[9] = 3.0 * ry * rz * r;
    }
    block_sum_store(m, NMOM, d.m_part + tr.tile, d.ntile);
}

// ---------------------------------------------------------------- Hartree

// Not launched when every instance of the plan folds the multipoles.
__global__ __launch_bounds__(BS) void k_multipole_finalize(const InstDesc *__restrict__ descs,
                                                           const int *__restrict__ list)
{
    const GroupRef gr = resolve_group(list);
    const InstDesc &d = descs[gr.inst];
    __shared__ double m[NMOM];
    if (!reduce_columns(d.m_part, d.ntile, NMOM, d.g_part, (unsigned *)(d.scal + SC_CNT), gr.g, m)) return;
    if ((int)threadIdx.x < NMOM) d.scal[SC_MOM + threadIdx.x] = m[threadIdx.x] * d.h3;
}

// Far field of the multipoles: q/r + p.r/r^3 + (1/2) sum_ab Q_ab r_a r_b / r^5.
__device__ __forceinline__ double multipole_potential(const double *m, double x, double y, double z)
{
#pragma clang fp contract(off)   // computed the same way in every kernel (see node_coord)
    const double r2 = x * x + y * y + z * z;
    const double r = sqrt(r2);
    const double r3 = r2 * r, r5 = r3 * r2;
    const double quad = m[4] * x * x + m[5] * y * y + m[6] * z * z
                      + 2.0 * (m[7] * x * y + m[8] * x * z + m[9] * y * z);
    return m[0] / r + (m[1] * x + m[2] * y + m[3] * z) / r3 + 0.5 * quad / r5;
}

// Ghost-face node g of 2 (ny nz + nx nz + nx ny): the two x faces (i = -1, nx),
// then the y faces, then the z faces, each in row order of its other two indices.
__device__ __forceinline__ int3 ghost_node(int g, int nx, int ny, int nz)
{
    const int fx = ny * nz, fy = nx * nz, fz = nx * ny;
    if (g < 2 * fx) {
        const int side = g / fx, r = g % fx;
        return make_int3(side ? nx : -1, r % ny, r / ny);
    }
    if ((g -= 2 * fx) < 2 * fy) {
        const int side = g / fy, r = g % fy;
        return make_int3(r % nx, side ? ny : -1, r / nx);
    }
    g -= 2 * fy;
    const int side = g / fz, r = g % fz;
    return make_int3(r % nx, r / nx, side ? nz : -1);
}

// The multipoles (h^3 included) of an instance that folds them, summed by this
// workgroup from the tile partials in the finalize kernel's order; the workgroup
// of tile 0 also stores them.  Every thread of the workgroup calls this.
__device__ __forceinline__ void fold_multipoles(const InstDesc &d, int tile, double *fm)
{
    fold_columns(d.m_part, d.ntile, NMOM, fm);
    if ((int)threadIdx.x < NMOM) {
        fm[threadIdx.x] *= d.h3;
        if (tile == 0) d.scal[SC_MOM + threadIdx.x] = fm[threadIdx.x];
    }
    __syncthreads();
}

// The far field on the six ghost faces.  fold (every instance of the launch folds
// the multipoles): there is no finalize kernel before this one; every workgroup
// sums them from the tile partials in that kernel's order (fold_columns), and the
// workgroup of tile 0 also stores them.
__global__ __launch_bounds__(BS) void k_ghost(const InstDesc *__restrict__ descs,
                                              const int2 *__restrict__ tiles, int fold)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    __shared__ double fm[NMOM];
    const double *mom = d.scal + SC_MOM;
    if (fold) {   // uniform
        fold_multipoles(d, tr.tile, fm);
        mom = fm;
    }
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int g = tr.tile * BS + threadIdx.x;
    if (g >= 2 * (ny * nz + nx * nz + nx * ny)) return;
    const int3 q = ghost_node(g, nx, ny, nz);
    const int i = q.x, j = q.y, k = q.z;
    const double v = multipole_potential(mom, node_coord(i, nx, d.h), node_coord(j, ny, d.h),
                                         node_coord(k, nz, d.h));
    d.vh[((size_t)(k + 1) * (ny + 2) + (j + 1)) * (nx + 2) + (i + 1)] = v;
}

// One colour of a red/black SOR sweep of (sum_faces V_H - 6 V_H)/h^2 = -4 pi rho;
// red = (i + j + k) even.
template <typename T>
__global__ __launch_bounds__(BS) void k_sor(const InstDesc *__restrict__ descs,
                                            const int2 *__restrict__ tiles, int color)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int hx = (nx + 1) >> 1;
    const int t = tr.tile * BS + threadIdx.x;
    if (t >= hx * ny * nz) return;
    const int xh = t % hx, yz = t / hx, y = yz % ny, z = yz / ny;
    const int x = 2 * xh + ((y + z + color) & 1);
    if (x >= nx) return;
    const size_t P = (size_t)nx + 2, PP = P * (size_t)(ny + 2);
    const size_t idx = (size_t)(z + 1) * PP + (size_t)(y + 1) * P + (size_t)(x + 1);
    auto *vh = gmem(d.vh);
    const double nb = vh[idx - 1] + vh[idx + 1] + vh[idx - P] + vh[idx + P] + vh[idx - PP] + vh[idx + PP];
    const double rho = (double)gmem((const T *)d.rho)[((size_t)z * ny + y) * nx + x];
    vh[idx] = sor_node(nb, rho, vh[idx], d.h, d.omega_sor);
}

// The first red half-sweep of a lattice step when every instance of the launch
// folds its multipoles (FOLD_M): it also does the ghost-face kernel's work, one
// launch fewer.  Every workgroup sums the multipoles (fold_multipoles); the
// workgroups write the six ghost faces between them (the values k_ghost writes,
// for the sweeps after this one); a red node next to the boundary takes its ghost
// neighbour from the same far-field expression instead of from memory, which this
// launch is writing.  The sweep is k_sor's, addition for addition.
template <typename T>
__global__ __launch_bounds__(BS) void k_sor_first(const InstDesc *__restrict__ descs,
                                                  const int2 *__restrict__ tiles)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const double h = d.h;
    const size_t P = (size_t)nx + 2, PP = P * (size_t)(ny + 2);
    auto *vh = gmem(d.vh);
    // the sweep's operands inside the grid first: they do not depend on the
    // multipoles, so their loads are in flight while those are summed
    const int hx = (nx + 1) >> 1;
    const int t = tr.tile * BS + threadIdx.x;
    const int xh = t % hx, yz = t / hx, y = yz % ny, z = yz / ny;
    const int x = 2 * xh + ((y + z) & 1);   // red
    const bool node = t < hx * ny * nz && x < nx;
    const size_t idx = (size_t)(z + 1) * PP + (size_t)(y + 1) * P + (size_t)(x + 1);
    const int nbx[6] = {x - 1, x + 1, x, x, x, x}, nby[6] = {y, y, y - 1, y + 1, y, y},
              nbz[6] = {z, z, z, z, z - 1, z + 1};
    const long long off[6] = {-1, 1, -(long long)P, (long long)P, -(long long)PP, (long long)PP};
    double v[6], rho = 0.0, old = 0.0;
    bool ghost[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        ghost[q] = nbx[q] < 0 || nbx[q] >= nx || nby[q] < 0 || nby[q] >= ny || nbz[q] < 0 || nbz[q] >= nz;
        v[q] = node && !ghost[q] ? (double)vh[(size_t)((long long)idx + off[q])] : 0.0;
    }
    if (node) {
        rho = (double)gmem((const T *)d.rho)[((size_t)z * ny + y) * nx + x];
        old = vh[idx];
    }
    __shared__ double fm[NMOM];
    fold_multipoles(d, tr.tile, fm);
    const int nghost = 2 * (ny * nz + nx * nz + nx * ny);
    for (int g = tr.tile * BS + (int)threadIdx.x; g < nghost; g += d.ntile_sor * BS) {
        const int3 c = ghost_node(g, nx, ny, nz);
        vh[(size_t)(c.z + 1) * PP + (size_t)(c.y + 1) * P + (size_t)(c.x + 1)] =
            multipole_potential(fm, node_coord(c.x, nx, h), node_coord(c.y, ny, h), node_coord(c.z, nz, h));
    }
    if (!node) return;
#pragma unroll
    for (int q = 0; q < 6; ++q)
        if (ghost[q])
            v[q] = multipole_potential(fm, node_coord(nbx[q], nx, h), node_coord(nby[q], ny, h),
                                       node_coord(nbz[q], nz, h));
    const double nb = v[0] + v[1] + v[2] + v[3] + v[4] + v[5];
    vh[idx] = sor_node(nb, rho, old, h, d.omega_sor);
}

// Residual partials: sum (lap_h V_H + 4 pi rho)^2 and sum (4 pi rho)^2.
template <typename T>
__global__ __launch_bounds__(BS) void k_residual(const InstDesc *__restrict__ descs,
                                                 const int2 *__restrict__ tiles)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int s = tr.tile * BS + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (s < d.nsite) {
        const int nx = d.nx, ny = d.ny;
        const int x = s % nx, yz = s / nx, y = yz % ny, z = yz / ny;
        const size_t P = (size_t)nx + 2, PP = P * (size_t)(ny + 2);
        const size_t idx = (size_t)(z + 1) * PP + (size_t)(y + 1) * P + (size_t)(x + 1);
        const double *vh = d.vh;
        const double nb = vh[idx - 1] + vh[idx + 1] + vh[idx - P] + vh[idx + P] + vh[idx - PP] + vh[idx + PP];
        const double b = 4.0 * 3.14159265358979323846 * (double)((const T *)d.rho)[s];
        const double r = (nb - 6.0 * vh[idx]) / (d.h * d.h) + b;
        v[0] = r * r;
        v[1] = b * b;
    }
    block_sum_store(v, 2, d.r_part + tr.tile, d.ntile);
}

__global__ __launch_bounds__(BS) void k_residual_finalize(const InstDesc *__restrict__ descs,
                                                          const int *__restrict__ list)
{
    const GroupRef gr = resolve_group(list);
    const InstDesc &d = descs[gr.inst];
    __shared__ double acc[2];
    if (!reduce_columns(d.r_part, d.ntile, 2, d.g_part, (unsigned *)(d.scal + SC_CNT), gr.g, acc)) return;
    if (threadIdx.x == 0) d.scal[SC_RES] = acc[1] > 0.0 ? sqrt(acc[0] / acc[1]) : sqrt(acc[0]);
}

// ------------------------------------------------- gradient-corrected xc

// D_a rho by central differences (rho = 0 outside the box).
template <typename T>
__device__ __forceinline__ void grad_rho(const InstDesc &d, int s, int x, int y, int z, double (&D)[3])
{
    const auto *r = gmem((const T *)d.rho);
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int sy = nx, sz = nx * ny;
    const double ih2 = 1.0 / (2.0 * d.h);
    const double xp = x + 1 < nx ? (double)r[s + 1] : 0.0, xm = x > 0 ? (double)r[s - 1] : 0.0;
    const double yp = y + 1 < ny ? (double)r[s + sy] : 0.0, ym = y > 0 ? (double)r[s - sy] : 0.0;
    const double zp = z + 1 < nz ? (double)r[s + sz] : 0.0, zm = z > 0 ? (double)r[s - sz] : 0.0;
    D[0] = (xp - xm) * ih2;
    D[1] = (yp - ym) * ih2;
    D[2] = (zp - zm) * ih2;
}

// Per node: df/drho and 2 (df/dsigma) D_a rho of the gradient-corrected
// functional, sigma = |D rho|^2, for the potential
//   v_xc = df/drho - sum_a D_a [2 (df/dsigma) D_a rho],
// the exact derivative of the discrete energy h^3 sum_r f(rho_r, sigma_r).
template <typename T>
__global__ __launch_bounds__(BS) void k_gga(const InstDesc *__restrict__ descs, const int2 *__restrict__ tiles)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int s = tr.tile * BS + threadIdx.x;
    if (s >= d.nsite) return;
    const int x = s % d.nx, yz = s / d.nx, y = yz % d.ny, z = yz / d.ny;
    double D[3];
    grad_rho<T>(d, s, x, y, z, D);
    double fx, fc, fr, fs;
    gga_eval((double)((const T *)d.rho)[s], D[0] * D[0] + D[1] * D[1] + D[2] * D[2], d.rho_floor,
             d.xc == XC_GGA_POLARISED, fx, fc, fr, fs);
    const size_t N = (size_t)d.nsite;
    d.gga[s] = fr;
    d.gga[N + s] = 2.0 * fs * D[0];
    d.gga[2 * N + s] = 2.0 * fs * D[1];
    d.gga[3 * N + s] = 2.0 * fs * D[2];
}

// v_xc of the gradient-corrected functional at node s from the k_gga fields.
__device__ __forceinline__ double gga_potential(const InstDesc &d, int s, int x, int y, int z)
{
    const size_t N = (size_t)d.nsite;
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int sy = nx, sz = nx * ny;
    const auto *g = gmem((const double *)d.gga);
    const auto *gx = g + N, *gy = g + 2 * N, *gz = g + 3 * N;
    const double ih2 = 1.0 / (2.0 * d.h);
    double div = ((x + 1 < nx ? gx[s + 1] : 0.0) - (x > 0 ? gx[s - 1] : 0.0)) * ih2;
    div += ((y + 1 < ny ? gy[s + sy] : 0.0) - (y > 0 ? gy[s - sy] : 0.0)) * ih2;
    div += ((z + 1 < nz ? gz[s + sz] : 0.0) - (z > 0 ? gz[s - sz] : 0.0)) * ih2;
    return g[s] - div;
}

// ------------------------------------------------------------- potential

// V = V_ext + V_H + v_x + v_c at node s = (x, y, z), summed in that order in FP64,
// with the node's Hartree value vh given.
template <typename T>
__device__ __forceinline__ double potential_with(const InstDesc &d, int s, int x, int y, int z, double vh)
{
    double V = gmem(d.vext)[s];
    if (d.hartree) V += vh;
    if (d.xc >= XC_GGA) {
        V += gga_potential(d, s, x, y, z);
    } else if (d.xc) {
        double ex, ec, vx, vc;
        xc_eval(d.xc, (double)gmem((const T *)d.rho)[s], d.rho_floor, ex, ec, vx, vc);
        V += vx;
        V += vc;
    }
    return V;
}

template <typename T>
__device__ __forceinline__ double potential_at(const InstDesc &d, int s, int x, int y, int z)
{
    const double vh = d.hartree ? gmem(d.vh)[((size_t)(z + 1) * (d.ny + 2) + (y + 1)) * (d.nx + 2) + (x + 1)] : 0.0;
    return potential_with<T>(d, s, x, y, z, vh);
}

// The KS potential at every node (stored in the bulk precision for the collide,
// or in FP64 for the energies).
template <typename T>
__global__ __launch_bounds__(BS) void k_potential(const InstDesc *__restrict__ descs,
                                                  const int2 *__restrict__ tiles, int to_fp64)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int s = tr.tile * BS + threadIdx.x;
    if (s >= d.nsite) return;
    const int x = s % d.nx, yz = s / d.nx, y = yz % d.ny, z = yz / d.ny;
    const double V = potential_at<T>(d, s, x, y, z);
    if (to_fp64) d.Vd[s] = V;
    else ((T *)d.V)[s] = (T)V;
}

// Last half-sweep of a step fused with the potential: each thread owns one x-pair
// (one red and one black node), relaxes the black node, and then writes V at both
// nodes (the red one is final since the preceding red half-sweep).  Every load
// comes before the first store (the new black value is passed on in a register),
// so no load waits for a store.
template <typename T>
__global__ __launch_bounds__(BS) void k_sor_black_potential(const InstDesc *__restrict__ descs,
                                                            const int2 *__restrict__ tiles)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int hx = (nx + 1) >> 1;
    const int t = tr.tile * BS + threadIdx.x;
    if (t >= hx * ny * nz) return;
    const int xh = t % hx, yz = t / hx, y = yz % ny, z = yz / ny;
    const int xb = 2 * xh + ((y + z + 1) & 1);
    const int xr = 2 * xh + ((y + z) & 1);
    const size_t P = (size_t)nx + 2, PP = P * (size_t)(ny + 2);
    const size_t idx = (size_t)(z + 1) * PP + (size_t)(y + 1) * P + (size_t)(xb + 1);
    const int sb = (z * ny + y) * nx + xb, sr = (z * ny + y) * nx + xr;
    auto *vh = gmem(d.vh);
    double vb = 0.0, Vb = 0.0, Vr = 0.0;
    if (xb < nx) {
        const double nb = vh[idx - 1] + vh[idx + 1] + vh[idx - P] + vh[idx + P] + vh[idx - PP] + vh[idx + PP];
        const double rho = (double)gmem((const T *)d.rho)[((size_t)z * ny + y) * nx + xb];
        vb = sor_node(nb, rho, vh[idx], d.h, d.omega_sor);
        Vb = potential_with<T>(d, sb, xb, y, z, vb);
    }
    if (xr < nx) Vr = potential_at<T>(d, sr, xr, y, z);   // red V_H is not written here
    auto *Vo = gmem((T *)d.V);
    if (xb < nx) {
        vh[idx] = vb;
        Vo[sb] = (T)Vb;
    }
    if (xr < nx) Vo[sr] = (T)Vr;
}

// V_ext(r) = -sum_I Z_I / sqrt(|r - R_I|^2 + a^2); ZR = [Z, x, y, z] per nucleus, then a^2.
template <typename T>
__global__ __launch_bounds__(BS) void k_vext(const InstDesc *__restrict__ descs,
                                             const int2 *__restrict__ tiles, int nnuc,
                                             const double *__restrict__ ZR)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int s = tr.tile * BS + threadIdx.x;
    if (s >= d.nsite) return;
    const int x = s % d.nx, yz = s / d.nx, y = yz % d.ny, z = yz / d.ny;
    const double rx = node_coord(x, d.nx, d.h), ry = node_coord(y, d.ny, d.h), rz = node_coord(z, d.nz, d.h);
    double v = 0.0;
    for (int I = 0; I < nnuc; ++I) {
        const double dx = rx - ZR[4 * I + 1], dy = ry - ZR[4 * I + 2], dz = rz - ZR[4 * I + 3];
        v -= ZR[4 * I] / sqrt(dx * dx + dy * dy + dz * dz + ZR[4 * nnuc]);
    }
    d.vext[s] = v;
}


// ---------------------------------------------------------------- energies

// Per-node energy terms: psi_hat_j K_h psi_hat_j with K_h u = -(S_xi u - u)/(D h^2),
// psi_hat_j S_chi(V psi_hat_j), and rho V_ext, rho V_H, rho eps_x, rho eps_c, rho.
template <typename T, int NO>
__global__ __launch_bounds__(BS) void k_energy_terms(const InstDesc *__restrict__ descs,
                                                     const int2 *__restrict__ tiles)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int n = orbitals<NO>(d);
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int s = tr.tile * BS + threadIdx.x;
    double v[2 * NO + NEBASE];
#pragma unroll
    for (int q = 0; q < 2 * NO + NEBASE; ++q) v[q] = 0.0;
    if (s < d.nsite) {
        const size_t N = (size_t)d.nsite;
        const T *ph = (const T *)d.psihat;
        const double *Vd = d.Vd;
        const int x = s % nx, yz = s / nx, y = yz % ny, z = yz / ny;
        double su[NO], sv[NO], u0[NO];
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            su[j] = 0.0;
            sv[j] = 0.0;
            u0[j] = (j < n) ? (double)ph[(size_t)j * N + s] : 0.0;
        }
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const int vx = VX(p), vy = VY(p), vz = VZ(p);
            const bool ok = (unsigned)(x - vx) < (unsigned)nx && (unsigned)(y - vy) < (unsigned)ny &&
                            (unsigned)(z - vz) < (unsigned)nz;
            if (ok) {
                const int src = s - (vx + nx * (vy + ny * vz));
                const double vn = Vd[src];
#pragma unroll
                for (int j = 0; j < NO; ++j) {
                    if (j < n) {
                        const double u = (double)ph[(size_t)j * N + src];
                        su[j] += d.xi[p] * u;
                        sv[j] += d.chi[p] * vn * u;
                    }
                }
            }
        }
        const double kfac = -1.0 / (d.D * d.h * d.h);
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            v[j] = u0[j] * (kfac * (su[j] - u0[j]));
            v[NO + j] = u0[j] * sv[j];
        }
        const double rho = (double)((const T *)d.rho)[s];
        double ex, ec, vx_, vc_;
        if (d.xc >= XC_GGA) {
            // energies per volume; divided back by rho so that rho * e below is f
            double D[3], fx, fc, fr, fs;
            grad_rho<T>(d, s, x, y, z, D);
            gga_eval(rho, D[0] * D[0] + D[1] * D[1] + D[2] * D[2], d.rho_floor, d.xc == XC_GGA_POLARISED, fx, fc,
                     fr, fs);
            ex = rho > 0.0 ? fx / rho : 0.0;
            ec = rho > 0.0 ? fc / rho : 0.0;
        } else {
            xc_eval(d.xc, rho, d.rho_floor, ex, ec, vx_, vc_);
        }
        double vh = 0.0;
        if (d.hartree) vh = d.vh[((size_t)(z + 1) * (ny + 2) + (y + 1)) * (nx + 2) + (x + 1)];
        v[2 * NO + 0] = rho * d.vext[s];
        v[2 * NO + 1] = rho * vh;
        v[2 * NO + 2] = rho * ex;
        v[2 * NO + 3] = rho * ec;
        v[2 * NO + 4] = rho;
    }
    // layout [NO kinetic][NO potential][NEBASE base terms], NO = orbital bucket
    block_sum_store(v, 2 * NO + NEBASE, d.e_part + tr.tile, d.ntile);
}

__global__ __launch_bounds__(BS) void k_energy_finalize(const InstDesc *__restrict__ descs,
                                                        const int *__restrict__ list)
{
    const GroupRef gr = resolve_group(list);
    const InstDesc &d = descs[gr.inst];
    const int n = d.n_orb, no = d.n_orb <= 5 ? d.n_orb : (d.n_orb <= 8 ? 8 : 16);
    const int nv = 2 * no + NEBASE;
    __shared__ double tot[2 * MAXO + NEBASE];
    if (!reduce_columns(d.e_part, d.ntile, nv, d.g_part, (unsigned *)(d.scal + SC_CNT), gr.g, tot)) return;
    if (threadIdx.x == 0)
        for (int q = 0; q < nv; ++q) tot[q] *= d.h3;
    __syncthreads();
    if (threadIdx.x != 0) return;
    double *E = d.scal + SC_ENER;
    double ekin = 0.0;
    for (int j = 0; j < MAXO; ++j) E[9 + j] = 0.0;
    for (int j = 0; j < n; ++j) {
        E[9 + j] = tot[j] + tot[no + j];
        ekin += d.occ[j] * tot[j];
    }
    const double eext = tot[2 * no + 0];
    const double eh = d.hartree ? 0.5 * tot[2 * no + 1] : 0.0;
    const double ex = d.xc ? tot[2 * no + 2] : 0.0;
    const double ec = d.xc ? tot[2 * no + 3] : 0.0;
    E[0] = ekin + eext + eh + ex + ec + d.e_nn;
    E[1] = ekin;
    E[2] = eext;
    E[3] = eh;
    E[4] = ex;
    E[5] = ec;
    E[6] = d.e_nn;
    E[7] = tot[2 * no + 4];
    E[8] = d.scal[SC_RES];
}

// ---------------------------------------------------- projected operator

// Rows of the relaxation operator projected on the orthonormalised orbitals,
// H_jk = <psi_hat_j | K_h psi_hat_k + S_chi(V psi_hat_k)>: its diagonal is eps_j,
// its eigenvalues are the Ritz values on the orbitals' span (they do not depend
// on rotations inside the span, so nearly degenerate levels are told apart
// before the orbitals have stopped mixing).  One launch takes rows j0 ..
// j0 + ham_rows(NO) - 1 into the energy partial array (column r NO + k = row
// j0 + r, column k).
template <int NO>
__host__ __device__ constexpr int ham_rows()
{
    return NO < padded_cols(2 * NO + NEBASE) / NO ? NO : padded_cols(2 * NO + NEBASE) / NO;
}

template <typename T, int NO>
__global__ __launch_bounds__(BS) void k_ham_terms(const InstDesc *__restrict__ descs, const int2 *__restrict__ tiles,
                                                  int j0)
{
    constexpr int RB = ham_rows<NO>();
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int n = orbitals<NO>(d);
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int s = tr.tile * BS + threadIdx.x;
    double v[RB * NO];
#pragma unroll
    for (int q = 0; q < RB * NO; ++q) v[q] = 0.0;
    if (s < d.nsite) {
        const size_t N = (size_t)d.nsite;
        const T *ph = (const T *)d.psihat;
        const double *Vd = d.Vd;
        const int x = s % nx, yz = s / nx, y = yz % ny, z = yz / ny;
        double su[NO], sv[NO], u0[NO];
#pragma unroll
        for (int k = 0; k < NO; ++k) {
            su[k] = 0.0;
            sv[k] = 0.0;
            u0[k] = (k < n) ? (double)ph[(size_t)k * N + s] : 0.0;
        }
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const int vx = VX(p), vy = VY(p), vz = VZ(p);
            const bool ok = (unsigned)(x - vx) < (unsigned)nx && (unsigned)(y - vy) < (unsigned)ny &&
                            (unsigned)(z - vz) < (unsigned)nz;
            if (ok) {
                const int src = s - (vx + nx * (vy + ny * vz));
                const double vn = Vd[src];
#pragma unroll
                for (int k = 0; k < NO; ++k) {
                    if (k < n) {
                        const double u = (double)ph[(size_t)k * N + src];
                        su[k] += d.xi[p] * u;
                        sv[k] += d.chi[p] * vn * u;
                    }
                }
            }
        }
        const double kfac = -1.0 / (d.D * d.h * d.h);
        double w[NO];
#pragma unroll
        for (int k = 0; k < NO; ++k) w[k] = kfac * (su[k] - u0[k]) + sv[k];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int j = j0 + r;
            double uj = 0.0;
#pragma unroll
            for (int jj = 0; jj < NO; ++jj)
                if (jj == j) uj = u0[jj];
#pragma unroll
            for (int k = 0; k < NO; ++k) v[r * NO + k] = uj * w[k];
        }
    }
    block_sum_store(v, RB * NO, d.e_part + tr.tile, d.ntile);
}

// Totals of the rows taken by k_ham_terms, times h^3, into the staging area:
// stage[j n + k] = H_jk for j0 <= j < j0 + rb, k < n.
__global__ __launch_bounds__(BS) void k_ham_finalize(const InstDesc *__restrict__ descs, const int *__restrict__ list,
                                                     int j0, int no, int rb)
{
    const GroupRef gr = resolve_group(list);
    const InstDesc &d = descs[gr.inst];
    const int n = d.n_orb;
    __shared__ double tot[2 * MAXO + NEBASE + RCH];
    if (!reduce_columns(d.e_part, d.ntile, rb * no, d.g_part, (unsigned *)(d.scal + SC_CNT), gr.g, tot)) return;
    __syncthreads();
    for (int q = threadIdx.x; q < rb * no; q += BS) {
        const int j = j0 + q / no, k = q % no;
        if (j < n && k < n) d.stage[(size_t)j * n + k] = tot[q] * d.h3;
    }
}

// ----------------------------------------------------------------- forces

// Per-node Hellmann-Feynman terms of the Born-Oppenheimer forces: for nuclei
// I = i0 .. i0 + NUCG - 1, rho (r - R_I) / (|r - R_I|^2 + a^2)^(3/2) (three
// columns per nucleus).
template <typename T>
__global__ __launch_bounds__(BS) void k_force_terms(const InstDesc *__restrict__ descs,
                                                    const int2 *__restrict__ tiles, int i0)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int s = tr.tile * BS + threadIdx.x;
    const int nn = d.nnuc;
    const int m = nn - i0 < NUCG ? nn - i0 : NUCG;
    double v[3 * NUCG];
#pragma unroll
    for (int q = 0; q < 3 * NUCG; ++q) v[q] = 0.0;
    if (s < d.nsite) {
        const double r = (double)((const T *)d.rho)[s];
        const int x = s % d.nx, yz = s / d.nx, y = yz % d.ny, z = yz / d.ny;
        const double rx = node_coord(x, d.nx, d.h), ry = node_coord(y, d.ny, d.h), rz = node_coord(z, d.nz, d.h);
        const double *zr = d.zr + 4 * i0;
        const double a2 = d.zr[4 * nn];
#pragma unroll
        for (int I = 0; I < NUCG; ++I) {
            if (I < m) {
                const double dx = rx - zr[4 * I + 1], dy = ry - zr[4 * I + 2], dz = rz - zr[4 * I + 3];
                const double d2 = dx * dx + dy * dy + dz * dz + a2;
                const double w = r / (d2 * sqrt(d2));
                v[3 * I] = w * dx;
                v[3 * I + 1] = w * dy;
                v[3 * I + 2] = w * dz;
            }
        }
    }
    block_sum_store(v, 3 * m, d.f_part + tr.tile, d.ntile);
}

// F_I = Z_I h^3 sum_r (the terms above) + sum_{J != I} Z_I Z_J (R_I - R_J) / |R_I - R_J|^3
// for the same nuclei, into the scalar block.
__global__ __launch_bounds__(BS) void k_force_finalize(const InstDesc *__restrict__ descs,
                                                       const int *__restrict__ list, int i0)
{
    const GroupRef gr = resolve_group(list);
    const InstDesc &d = descs[gr.inst];
    const int nn = d.nnuc;
    const int m = nn - i0 < NUCG ? nn - i0 : NUCG;
    __shared__ double tot[3 * NUCG];
    if (!reduce_columns(d.f_part, d.ntile, 3 * m, d.g_part, (unsigned *)(d.scal + SC_CNT), gr.g, tot)) return;
    const int q = threadIdx.x;
    if (q < 3 * m) {
        const int I = i0 + q / 3, c = q % 3;
        const double *zr = d.zr;
        double f = (zr[4 * I] * d.h3) * tot[q];
        for (int J = 0; J < nn; ++J) {
            if (J == I) continue;
            const double dx = zr[4 * I + 1] - zr[4 * J + 1], dy = zr[4 * I + 2] - zr[4 * J + 2],
                         dz = zr[4 * I + 3] - zr[4 * J + 3];
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            const double cc = zr[4 * I] * zr[4 * J] / (r * r * r);
            f += cc * (c == 0 ? dx : (c == 1 ? dy : dz));
        }
        d.scal[SC_FORCE + 3 * i0 + q] = f;
    }
}

// Orbitals and density to the FP64 staging buffer.
template <typename T>
__global__ __launch_bounds__(BS) void k_stage_orbitals(const InstDesc *__restrict__ descs,
                                                       const int2 *__restrict__ tiles)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int s = tr.tile * BS + threadIdx.x;
    if (s >= d.nsite) return;
    const size_t N = (size_t)d.nsite;
    for (int j = 0; j < d.n_orb; ++j) d.stage[(size_t)j * N + s] = (double)((const T *)d.psihat)[(size_t)j * N + s];
    d.stage[(size_t)d.n_orb * N + s] = (double)((const T *)d.rho)[s];
}

// Plain copy, 16 bytes per lane, one element per lane over an exact grid, with
// non-temporal loads and stores like the populations of the update kernel: the
// bandwidth reference and the HBM-counter calibration.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void k_copy16(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src, size_t n16)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// Energies and error flags of many instances into one buffer (one read-back).
__global__ void k_gather(const double *const *__restrict__ scal, int count, int width, double *__restrict__ dst)
{
    const int i = blockIdx.x;
    const int k = threadIdx.x;
    if (i >= count) return;
    if (k < 25) dst[(size_t)i * width + k] = scal[i][SC_ENER + k];
    else if (k == 25) dst[(size_t)i * width + k] = scal[i][SC_ERR];
}

// ---------------------------------------------------------------- launchers

int launch_init_psi(const Plan &pl, int mode, double sigma, double noise, uint64_t seed, hipStream_t st)
{
    return dispatch_tt(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_init_psi<typename TG::T><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site, mode, sigma, noise, seed);
        LAUNCH_CHECK();
    });
}

int launch_psi_from_stage(const Plan &pl, hipStream_t st)
{
    return dispatch_tt(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_psi_from_stage<typename TG::T><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site);
        LAUNCH_CHECK();
    });
}

int launch_equilibrium(const Plan &pl, int parity, hipStream_t st)
{
    return dispatch_tt(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_equilibrium<typename TG::T><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site, parity);
        LAUNCH_CHECK();
    });
}

int launch_moment(const Plan &pl, int parity, hipStream_t st)
{
    return dispatch_tn(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_moment<typename TG::T, TG::NO><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site, parity);
        LAUNCH_CHECK();
    });
}

int launch_overlap_psi(const Plan &pl, hipStream_t st, bool skip_brick)
{
    return dispatch_tn(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_overlap_psi<typename TG::T, TG::NO><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site, skip_brick ? 1 : 0);
        LAUNCH_CHECK();
    });
}

int launch_overlap_finalize(const Plan &pl, hipStream_t st)
{
    if (pl.fold_s) return 0;   // every instance's orthonormalisation sums S itself
    k_overlap_finalize<<<grid_group(pl), BS, 0, st>>>(pl.d_desc, pl.tt.inst);
    LAUNCH_CHECK();
}

int launch_orthonormalise(const Plan &pl, hipStream_t st)
{
    return dispatch_tnw(pl, [&](auto tg) {
        using TG = decltype(tg);
        if constexpr (TG::NO <= 5) {
            if (pl.fold_s) {
                k_orthonormalise<typename TG::T, TG::NO, TG::W, true><<<grid_site(pl), BS, 0, st>>>(pl.d_desc,
                                                                                                    pl.tt.site);
                LAUNCH_CHECK();
            }
        }
        k_orthonormalise<typename TG::T, TG::NO, TG::W, false><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site);
        LAUNCH_CHECK();
    });
}

int launch_multipole_finalize(const Plan &pl, hipStream_t st)
{
    if (pl.fold_m) return 0;   // every instance's ghost-face kernel sums the multipoles itself
    k_multipole_finalize<<<grid_group(pl), BS, 0, st>>>(pl.d_desc, pl.tt.inst);
    LAUNCH_CHECK();
}

int launch_ghost(const Plan &pl, hipStream_t st)
{
    k_ghost<<<grid_ghost(pl), BS, 0, st>>>(pl.d_desc, pl.tt.ghost, pl.fold_m ? 1 : 0);
    LAUNCH_CHECK();
}

int launch_sor(const Plan &pl, int color, hipStream_t st)
{
    return dispatch_tt(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_sor<typename TG::T><<<grid_sor(pl), BS, 0, st>>>(pl.d_desc, pl.tt.sor, color);
        LAUNCH_CHECK();
    });
}

int launch_sor_first(const Plan &pl, hipStream_t st)
{
    return dispatch_tt(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_sor_first<typename TG::T><<<grid_sor(pl), BS, 0, st>>>(pl.d_desc, pl.tt.sor);
        LAUNCH_CHECK();
    });
}

int launch_sor_black_potential(const Plan &pl, hipStream_t st)
{
    return dispatch_tt(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_sor_black_potential<typename TG::T><<<grid_sor(pl), BS, 0, st>>>(pl.d_desc, pl.tt.sor);
        LAUNCH_CHECK();
    });
}

int launch_residual(const Plan &pl, hipStream_t st)
{
    return dispatch_tt(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_residual<typename TG::T><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site);
        LAUNCH_CHECK();
    });
}

int launch_residual_finalize(const Plan &pl, hipStream_t st)
{
    k_residual_finalize<<<grid_group(pl), BS, 0, st>>>(pl.d_desc, pl.tt.inst);
    LAUNCH_CHECK();
}

int launch_potential(const Plan &pl, int to_fp64, hipStream_t st)
{
    return dispatch_tt(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_potential<typename TG::T><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site, to_fp64);
        LAUNCH_CHECK();
    });
}

int launch_vext(const Plan &pl, int nnuc, const double *dZR, hipStream_t st)
{
    return dispatch_tt(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_vext<typename TG::T><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site, nnuc, dZR);
        LAUNCH_CHECK();
    });
}



int launch_gga(const Plan &pl, hipStream_t st)
{
    return dispatch_tt(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_gga<typename TG::T><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site);
        LAUNCH_CHECK();
    });
}

int launch_force_terms(const Plan &pl, int i0, hipStream_t st)
{
    return dispatch_tt(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_force_terms<typename TG::T><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site, i0);
        LAUNCH_CHECK();
    });
}

int launch_force_finalize(const Plan &pl, int i0, hipStream_t st)
{
    k_force_finalize<<<grid_group(pl), BS, 0, st>>>(pl.d_desc, pl.tt.inst, i0);
    LAUNCH_CHECK();
}

int launch_energy_terms(const Plan &pl, hipStream_t st)
{
    return dispatch_tn(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_energy_terms<typename TG::T, TG::NO><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site);
        LAUNCH_CHECK();
    });
}

int launch_ham_rows(const Plan &pl, int j0, int *rows_done, hipStream_t st)
{
    return dispatch_tn(pl, [&](auto tg) {
        using TG = decltype(tg);
        constexpr int RB = ham_rows<TG::NO>();
        k_ham_terms<typename TG::T, TG::NO><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site, j0);
        int e = (int)hipGetLastError();
        if (e) return e;
        k_ham_finalize<<<grid_group(pl), BS, 0, st>>>(pl.d_desc, pl.tt.inst, j0, TG::NO, RB);
        *rows_done = RB;
        return (int)hipGetLastError();
    });
}

int launch_energy_finalize(const Plan &pl, hipStream_t st)
{
    k_energy_finalize<<<grid_group(pl), BS, 0, st>>>(pl.d_desc, pl.tt.inst);
    LAUNCH_CHECK();
}

int launch_stage_orbitals(const Plan &pl, hipStream_t st)
{
    return dispatch_tt(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_stage_orbitals<typename TG::T><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site);
        LAUNCH_CHECK();
    });
}

int launch_gather(const double *const *scal, int count, int width, double *dst, hipStream_t st)
{
    if (count <= 0) return 0;
    if (!scal || !dst) return (int)hipErrorInvalidValue;   // no table built for these members
    k_gather<<<count, 32, 0, st>>>(scal, count, width, dst);
    LAUNCH_CHECK();
}

int launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    const size_t n16 = bytes / 16;
    const size_t blocks = (n16 + 255) / 256;
    if (blocks == 0) return 0;
    if (blocks > 0x7fffffff) return (int)hipErrorInvalidValue;
    k_copy16<<<(unsigned)blocks, 256, 0, st>>>((u32x4 *)dst, (const u32x4 *)src, n16);
    LAUNCH_CHECK();
}

}  // namespace lbks
