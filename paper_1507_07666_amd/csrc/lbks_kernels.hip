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
#include "lbks_kernels.h"

#include <hip/hip_runtime.h>
#include <math.h>

namespace lbks {

// ------------------------------------------------------------------ lattice

// D3Q19 velocities: 0 rest; 1..6 faces (+x -x +y -y +z -z); 7..10 xy edges
// (++ -+ +- --); 11..14 xz edges (++ -+ +- --); 15..18 yz edges (++ -+ +- --).
__host__ __device__ constexpr int VX(int p)
{
    return (p == 1 || p == 7 || p == 9 || p == 11 || p == 13) ? 1
         : (p == 2 || p == 8 || p == 10 || p == 12 || p == 14) ? -1 : 0;
}
__host__ __device__ constexpr int VY(int p)
{
    return (p == 3 || p == 7 || p == 8 || p == 15 || p == 17) ? 1
         : (p == 4 || p == 9 || p == 10 || p == 16 || p == 18) ? -1 : 0;
}
__host__ __device__ constexpr int VZ(int p)
{
    return (p == 5 || p == 11 || p == 12 || p == 15 || p == 16) ? 1
         : (p == 6 || p == 13 || p == 14 || p == 17 || p == 18) ? -1 : 0;
}

// ---------------------------------------------------------------- helpers

// Workgroups are dealt round-robin to the 8 XCDs; remap so that each XCD
// works on one contiguous range of tiles (neighbour planes stay in its L2).
__device__ __forceinline__ int xcd_remap(int b, int nblk)
{
    const int X = 8;
    const int xcd = b % X, idx = b / X, q = nblk / X, r = nblk % X;
    return (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

struct TileRef {
    int inst, tile;
};

__device__ __forceinline__ TileRef resolve(const int2 *table)
{
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    if (table) {
        const int2 t = table[b];
        return {t.x, t.y};
    }
    return {0, b};
}

__device__ __forceinline__ int resolve_inst(const int *list)
{
    return list ? list[blockIdx.x] : (int)blockIdx.x;
}

__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Sum v[0..nv) over the workgroup; thread q < nv writes its total to out[q * stride].
template <int NV>
__device__ __forceinline__ void block_sum_store(double (&v)[NV], int nv, double *out, int stride)
{
    __shared__ double red[BS / 64][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        if (q < nv) {
            const double x = wave_sum(v[q]);
            if (lane == 0) red[wave][q] = x;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nv) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < BS / 64; ++w) s += red[w][threadIdx.x];
        out[(size_t)threadIdx.x * stride] = s;
    }
}

constexpr int FB = 1024;   // threads of the per-instance finalize kernels

// Column sums out[q] = sum_t part[q * ntile + t] for q < nq, in a fixed order
// (each thread strides the tiles, then the waves are summed in order).  The
// partial arrays hold whole chunks of RCH columns (unused ones stay zero), so
// every load is unconditional and all of a thread's loads are in flight at once.
// `out` is LDS; every thread of the FB-wide workgroup must call this.
__device__ void reduce_columns(const double *__restrict__ part, int ntile, int nq, double *out)
{
    constexpr int U = 4;   // tiles per thread per round
    __shared__ double red[FB / 64][RCH];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q0 = 0; q0 < nq; q0 += RCH) {
        const double *col = part + (size_t)q0 * ntile;
        double acc[RCH];
#pragma unroll
        for (int c = 0; c < RCH; ++c) acc[c] = 0.0;
        for (int t0 = 0; t0 < ntile; t0 += U * FB) {
            double v[U][RCH];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int t = t0 + k * FB + (int)threadIdx.x;
                const int tc = t < ntile ? t : ntile - 1;
#pragma unroll
                for (int c = 0; c < RCH; ++c) v[k][c] = col[(size_t)c * ntile + tc];
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const double w = (t0 + k * FB + (int)threadIdx.x) < ntile ? 1.0 : 0.0;
#pragma unroll
                for (int c = 0; c < RCH; ++c) acc[c] += w * v[k][c];
            }
        }
#pragma unroll
        for (int c = 0; c < RCH; ++c) {
            const double x = wave_sum(acc[c]);
            if (lane == 0) red[wave][c] = x;
        }
        __syncthreads();
        if ((int)threadIdx.x < RCH && q0 + (int)threadIdx.x < nq) {
            double sum = 0.0;
            for (int w = 0; w < FB / 64; ++w) sum += red[w][threadIdx.x];
            out[q0 + threadIdx.x] = sum;
        }
        __syncthreads();
    }
}

__device__ __forceinline__ double node_coord(int i, int n, double h)
{
    return ((double)i - 0.5 * (double)(n - 1)) * h;
}

__device__ __forceinline__ int npair_of(int n) { return n * (n + 1) / 2; }

// Local exchange-correlation per electron (e*) and potential (v* = d(rho e*)/d rho):
// Slater exchange; correlation of Lee-Yang-Parr at zero gradient,
// e_c = -a (1 + b C_F exp(-c u)) / (1 + d u), u = rho^(-1/3); or Perdew-Zunger 1981.
__device__ void xc_eval(int kind, double rho, double floor, double &ex, double &ec, double &vx,
                        double &vc)
{
    ex = ec = vx = vc = 0.0;
    if (kind == 0 || !(rho >= floor) || !(rho > 0.0)) return;
    const double PI = 3.14159265358979323846;
    vx = -cbrt(3.0 * rho / PI);
    ex = 0.75 * vx;
    if (kind == 2) {
        const double a = 0.04918, b = 0.132, c = 0.2533, d = 0.349;
        const double CF = 2.8712340001881915;   // (3/10)(3 pi^2)^(2/3)
        const double u = 1.0 / cbrt(rho);
        const double e = exp(-c * u);
        const double num = 1.0 + b * CF * e, den = 1.0 + d * u;
        const double g = num / den;
        const double gp = (-b * CF * c * e * den - d * num) / (den * den);
        ec = -a * g;
        vc = -a * (g - (u / 3.0) * gp);
    } else if (kind == 3) {
        const double rs = cbrt(3.0 / (4.0 * PI * rho));
        if (rs >= 1.0) {
            const double gam = -0.1423, b1 = 1.0529, b2 = 0.3334;
            const double sq = sqrt(rs);
            const double den = 1.0 + b1 * sq + b2 * rs;
            ec = gam / den;
            vc = ec * (1.0 + (7.0 / 6.0) * b1 * sq + (4.0 / 3.0) * b2 * rs) / den;
        } else {
            const double A = 0.0311, B = -0.048, Cc = 0.0020, Dd = -0.0116;
            const double lr = log(rs);
            ec = A * lr + B + Cc * rs * lr + Dd * rs;
            vc = A * lr + (B - A / 3.0) + (2.0 / 3.0) * Cc * rs * lr + (2.0 * Dd - Cc) * rs / 3.0;
        }
    }
}

// --------------------------------------------------------------- dispatch

template <typename TT, int NOO, bool WW>
struct Tag {
    using T = TT;
    static constexpr int NO = NOO;
    static constexpr bool W = WW;
};

template <int NO, bool W, typename F>
int dispatch_t(const Plan &pl, F &f)
{
    if (pl.precision) return f(Tag<float, NO, W>{});
    return f(Tag<double, NO, W>{});
}
template <int NO, typename F>
int dispatch_w(const Plan &pl, F &f)
{
    if (pl.wmode) return dispatch_t<NO, true>(pl, f);
    return dispatch_t<NO, false>(pl, f);
}
template <typename F>
int dispatch_tnw(const Plan &pl, F &&f)
{
    switch (pl.no) {
    case 1: return dispatch_w<1>(pl, f);
    case 2: return dispatch_w<2>(pl, f);
    case 3: return dispatch_w<3>(pl, f);
    case 4: return dispatch_w<4>(pl, f);
    case 5: return dispatch_w<5>(pl, f);
    case 8: return dispatch_w<8>(pl, f);
    default: return dispatch_w<16>(pl, f);
    }
}
template <typename F>
int dispatch_tn(const Plan &pl, F &&f)
{
    switch (pl.no) {
    case 1: return dispatch_t<1, false>(pl, f);
    case 2: return dispatch_t<2, false>(pl, f);
    case 3: return dispatch_t<3, false>(pl, f);
    case 4: return dispatch_t<4, false>(pl, f);
    case 5: return dispatch_t<5, false>(pl, f);
    case 8: return dispatch_t<8, false>(pl, f);
    default: return dispatch_t<16, false>(pl, f);
    }
}
template <typename F>
int dispatch_tt(const Plan &pl, F &&f)
{
    return dispatch_t<1, false>(pl, f);
}

int orbital_bucket(int n)
{
    return n <= 5 ? n : (n <= 8 ? 8 : 16);
}

static inline int grid_site(const Plan &pl) { return pl.tt.site ? pl.tt.n_site : pl.ntile; }
static inline int grid_ghost(const Plan &pl) { return pl.tt.ghost ? pl.tt.n_ghost : pl.ntile_ghost; }
static inline int grid_sor(const Plan &pl) { return pl.tt.sor ? pl.tt.n_sor : pl.ntile_sor; }
static inline int grid_inst(const Plan &pl) { return pl.tt.inst ? pl.tt.n_inst : 1; }

#define LAUNCH_CHECK() return (int)hipGetLastError()

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
    const int n = d.n_orb;
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
    double prod[NO * (NO + 1) / 2];
    int q = 0;
#pragma unroll
    for (int j = 0; j < NO; ++j)
#pragma unroll
        for (int k = 0; k <= j; ++k) prod[q++] = (double)acc[j] * (double)acc[k];
    block_sum_store(prod, npair_of(n), d.s_part + tr.tile, d.ntile);
}

// Overlap partials of the orbital state itself (collapsed scheme).
template <typename T, int NO>
__global__ __launch_bounds__(BS) void k_overlap_psi(const InstDesc *__restrict__ descs,
                                                    const int2 *__restrict__ tiles)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int n = d.n_orb;
    const int s = tr.tile * BS + threadIdx.x;
    const T *psi = (const T *)d.psi;
    double a[NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) a[j] = (s < d.nsite && j < n) ? (double)psi[(size_t)j * d.nsite + s] : 0.0;
    double prod[NO * (NO + 1) / 2];
    int q = 0;
#pragma unroll
    for (int j = 0; j < NO; ++j)
#pragma unroll
        for (int k = 0; k <= j; ++k) prod[q++] = a[j] * a[k];
    block_sum_store(prod, npair_of(n), d.s_part + tr.tile, d.ntile);
}

// ---------------------------------------------------------- overlap / GS

// S from the tile partials (fixed order), then C.  GS: S = L L^T, C = L^{-T}
// (psi_hat_j = sum_{l<=j} psi_l C_lj, classical Gram-Schmidt order).  W:
// n_j = sqrt(S_jj), C = diag(1/n), C*_lj = -Lambda_jl / n_l (l < j), C*_jj = 1/n_j
// with Lambda_jl = S_jl / (n_j n_l), i.e. psi*_j = psi_hat_j - sum_{l<j} Lambda_jl psi_hat_l.
__global__ __launch_bounds__(FB) void k_overlap_finalize(const InstDesc *__restrict__ descs,
                                                         const int *__restrict__ list)
{
    const InstDesc &d = descs[resolve_inst(list)];
    const int n = d.n_orb, np = npair_of(n);
    __shared__ double S[MAXO * (MAXO + 1) / 2];
    __shared__ double L[MAXO][MAXO + 1];
    __shared__ double Li[MAXO][MAXO + 1];
    reduce_columns(d.s_part, d.ntile, np, S);
    if (threadIdx.x != 0) return;
    double *C = d.C;
    double *Cs = d.C + MAXO * MAXO;
    bool bad = false;
    for (int q = 0; q < np; ++q) {
        S[q] *= d.h3;
        d.scal[SC_S + q] = S[q];
        if (!isfinite(S[q])) bad = true;
    }
    auto Sget = [&](int i, int j) { return i >= j ? S[i * (i + 1) / 2 + j] : S[j * (j + 1) / 2 + i]; };
    // entries outside the n x n block stay zero from creation
    if (d.ortho == 0) {
        for (int i = 0; i < n; ++i)
            for (int j = 0; j <= i; ++j) {
                double sum = Sget(i, j);
                for (int k = 0; k < j; ++k) sum -= L[i][k] * L[j][k];
                if (i == j) {
                    if (!(sum > 0.0)) {
                        bad = true;
                        sum = 1.0;
                    }
                    L[i][i] = sqrt(sum);
                } else {
                    L[i][j] = sum / L[j][j];
                }
            }
        // C = L^{-T}: column c of L^{-1} by forward substitution; C[l][j] = Linv[j][l]
        for (int c = 0; c < n; ++c)
            for (int i = c; i < n; ++i) {
                double sum = (i == c) ? 1.0 : 0.0;
                for (int k = c; k < i; ++k) sum -= L[i][k] * Li[k][c];
                Li[i][c] = sum / L[i][i];
            }
        for (int l = 0; l < n; ++l)
            for (int j = l; j < n; ++j) C[l * MAXO + j] = Li[j][l];
    } else {
        double nrm[MAXO];
        for (int j = 0; j < n; ++j) {
            const double sjj = Sget(j, j);
            if (!(sjj > 0.0)) bad = true;
            nrm[j] = sqrt(sjj > 0.0 ? sjj : 1.0);
        }
        for (int j = 0; j < n; ++j) {
            C[j * MAXO + j] = 1.0 / nrm[j];
            Cs[j * MAXO + j] = 1.0 / nrm[j];
            for (int l = 0; l < j; ++l) Cs[l * MAXO + j] = -(Sget(j, l) / (nrm[j] * nrm[l])) / nrm[l];
        }
    }
    if (bad) d.scal[SC_ERR] = 1.0;
}

// psi_hat = psi C (psi* = psi C* in W mode), rho = sum_j occ_j psi_hat_j^2 and
// the multipole partials q, p_a, Q_ab of rho.
template <typename T, int NO, bool W>
__global__ __launch_bounds__(BS) void k_orthonormalise(const InstDesc *__restrict__ descs,
                                                       const int2 *__restrict__ tiles)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int n = d.n_orb;
    const int s = tr.tile * BS + threadIdx.x;
    double m[NMOM];
#pragma unroll
    for (int q = 0; q < NMOM; ++q) m[q] = 0.0;
    if (s < d.nsite) {
        const size_t N = (size_t)d.nsite;
        const T *psi = (const T *)d.psi;
        T *ph = (T *)d.psihat;
        T *pst = (T *)d.psistar;
        double ps[NO];
#pragma unroll
        for (int l = 0; l < NO; ++l) ps[l] = (l < n) ? (double)psi[(size_t)l * N + s] : 0.0;
        double rho = 0.0;
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            if (j < n) {
                double hat = 0.0;
                if (W) {
                    hat = ps[j] * d.C[j * MAXO + j];
                    double st = 0.0;
#pragma unroll
                    for (int l = 0; l <= j; ++l) st += ps[l] * d.C[MAXO * MAXO + l * MAXO + j];
                    pst[(size_t)j * N + s] = (T)st;
                } else {
#pragma unroll
                    for (int l = 0; l <= j; ++l) hat += ps[l] * d.C[l * MAXO + j];
                }
                const T hs = (T)hat;
                ph[(size_t)j * N + s] = hs;
                const double hd = (double)hs;
                rho += d.occ[j] * hd * hd;
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

__global__ __launch_bounds__(FB) void k_multipole_finalize(const InstDesc *__restrict__ descs,
                                                           const int *__restrict__ list)
{
    const InstDesc &d = descs[resolve_inst(list)];
    __shared__ double m[NMOM];
    reduce_columns(d.m_part, d.ntile, NMOM, m);
    if ((int)threadIdx.x < NMOM) d.scal[SC_MOM + threadIdx.x] = m[threadIdx.x] * d.h3;
}

// Far field of the multipoles: q/r + p.r/r^3 + (1/2) sum_ab Q_ab r_a r_b / r^5.
__device__ __forceinline__ double multipole_potential(const double *m, double x, double y, double z)
{
    const double r2 = x * x + y * y + z * z;
    const double r = sqrt(r2);
    const double r3 = r2 * r, r5 = r3 * r2;
    const double quad = m[4] * x * x + m[5] * y * y + m[6] * z * z
                      + 2.0 * (m[7] * x * y + m[8] * x * z + m[9] * y * z);
    return m[0] / r + (m[1] * x + m[2] * y + m[3] * z) / r3 + 0.5 * quad / r5;
}

__global__ __launch_bounds__(BS) void k_ghost(const InstDesc *__restrict__ descs,
                                              const int2 *__restrict__ tiles)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    int g = tr.tile * BS + threadIdx.x;
    const int fx = ny * nz, fy = nx * nz, fz = nx * ny;
    if (g >= 2 * (fx + fy + fz)) return;
    int i, j, k;
    if (g < 2 * fx) {
        const int side = g / fx, r = g % fx;
        j = r % ny;
        k = r / ny;
        i = side ? nx : -1;
    } else if ((g -= 2 * fx) < 2 * fy) {
        const int side = g / fy, r = g % fy;
        i = r % nx;
        k = r / nx;
        j = side ? ny : -1;
    } else {
        g -= 2 * fy;
        const int side = g / fz, r = g % fz;
        i = r % nx;
        j = r / nx;
        k = side ? nz : -1;
    }
    const double v = multipole_potential(d.scal + SC_MOM, node_coord(i, nx, d.h), node_coord(j, ny, d.h),
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
    double *vh = d.vh;
    const double nb = vh[idx - 1] + vh[idx + 1] + vh[idx - P] + vh[idx + P] + vh[idx - PP] + vh[idx + PP];
    const double four_pi_h2 = 4.0 * 3.14159265358979323846 * d.h * d.h;
    const double rho = (double)((const T *)d.rho)[((size_t)z * ny + y) * nx + x];
    const double gs = (nb + four_pi_h2 * rho) / 6.0;
    vh[idx] = (1.0 - d.omega_sor) * vh[idx] + d.omega_sor * gs;
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

__global__ __launch_bounds__(FB) void k_residual_finalize(const InstDesc *__restrict__ descs,
                                                          const int *__restrict__ list)
{
    const InstDesc &d = descs[resolve_inst(list)];
    __shared__ double acc[2];
    reduce_columns(d.r_part, d.ntile, 2, acc);
    if (threadIdx.x == 0) d.scal[SC_RES] = acc[1] > 0.0 ? sqrt(acc[0] / acc[1]) : sqrt(acc[0]);
}

// ------------------------------------------------------------- potential

// V = V_ext + V_H + v_x + v_c at every node (FP64 arithmetic; stored in the bulk
// precision for the collide, or in FP64 for the energies).
template <typename T>
__global__ __launch_bounds__(BS) void k_potential(const InstDesc *__restrict__ descs,
                                                  const int2 *__restrict__ tiles, int to_fp64)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int s = tr.tile * BS + threadIdx.x;
    if (s >= d.nsite) return;
    double V = d.vext[s];
    if (d.hartree) {
        const int nx = d.nx, ny = d.ny;
        const int x = s % nx, yz = s / nx, y = yz % ny, z = yz / ny;
        V += d.vh[((size_t)(z + 1) * (ny + 2) + (y + 1)) * (nx + 2) + (x + 1)];
    }
    if (d.xc) {
        double ex, ec, vx, vc;
        xc_eval(d.xc, (double)((const T *)d.rho)[s], d.rho_floor, ex, ec, vx, vc);
        V += vx;
        V += vc;
    }
    if (to_fp64) d.Vd[s] = V;
    else ((T *)d.V)[s] = (T)V;
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

// --------------------------------------------------------- stream-collide

// Pull form of the lattice Boltzmann equation with the orthogonalisation and
// potential sources: the population entering node r along v_p is the
// post-collision population of r - v_p,
//   f_jp(r; t+1) = (1 - omega) g_jp + omega xi_p psi*_j - dt chi_p V psi_hat_j  at r - v_p,
// g_jp = sum_{l<=j} f_lp C_lj, and zero when r - v_p is outside the box.  The new
// moment psi_j = sum_p f_jp and the overlap partials psi_j psi_k are fused.
template <typename T, int NO, bool W>
__global__ __launch_bounds__(BS) void k_stream_collide(const InstDesc *__restrict__ descs,
                                                       const int2 *__restrict__ tiles, int parity)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int n = d.n_orb;
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int s = tr.tile * BS + threadIdx.x;
    const bool valid = s < d.nsite;
    T acc[NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) acc[j] = (T)0;
    if (valid) {
        const size_t N = (size_t)d.nsite;
        const T *__restrict__ fs = (const T *)(parity ? d.f1 : d.f0);
        T *__restrict__ fd = (T *)(parity ? d.f0 : d.f1);
        const T *__restrict__ ph = (const T *)d.psihat;
        const T *__restrict__ pst = (const T *)d.psistar;
        const T *__restrict__ Vp = (const T *)d.V;
        const T a = (T)(1.0 - d.omega);
        const T om = (T)d.omega;
        const T dt = (T)d.dt;
        T c[NO][NO];
#pragma unroll
        for (int l = 0; l < NO; ++l)
#pragma unroll
            for (int j = 0; j < NO; ++j) c[l][j] = (T)d.C[l * MAXO + j];
        const int x = s % nx, yz = s / nx, y = yz % ny, z = yz / ny;
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const int vx = VX(p), vy = VY(p), vz = VZ(p);
            const bool ok = (unsigned)(x - vx) < (unsigned)nx && (unsigned)(y - vy) < (unsigned)ny &&
                            (unsigned)(z - vz) < (unsigned)nz;
            T out[NO];
            if (ok) {
                const int src = s - (vx + nx * (vy + ny * vz));
                T fl[NO];
#pragma unroll
                for (int l = 0; l < NO; ++l)
                    fl[l] = (l < n) ? __builtin_nontemporal_load(fs + ((size_t)l * Q + p) * N + src) : (T)0;
                const T vn = Vp[src];
                const T cp = om * (T)d.xi[p];
                const T dp = dt * (T)d.chi[p] * vn;
#pragma unroll
                for (int j = 0; j < NO; ++j) {
                    if (j < n) {
                        T g;
                        if (W) {
                            g = c[j][j] * fl[j];
                            out[j] = a * g + cp * pst[(size_t)j * N + src] - dp * ph[(size_t)j * N + src];
                        } else {
                            g = (T)0;
#pragma unroll
                            for (int l = 0; l <= j; ++l) g += c[l][j] * fl[l];
                            out[j] = a * g + (cp - dp) * ph[(size_t)j * N + src];
                        }
                    } else {
                        out[j] = (T)0;
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < NO; ++j) out[j] = (T)0;
            }
#pragma unroll
            for (int j = 0; j < NO; ++j) {
                if (j < n) {
                    // populations are read once per step: stream them past the caches
                    __builtin_nontemporal_store(out[j], fd + ((size_t)j * Q + p) * N + s);
                    acc[j] += out[j];
                }
            }
        }
        T *psi = (T *)d.psi;
#pragma unroll
        for (int j = 0; j < NO; ++j)
            if (j < n) psi[(size_t)j * N + s] = acc[j];
    }
    double prod[NO * (NO + 1) / 2];
    int q = 0;
#pragma unroll
    for (int j = 0; j < NO; ++j)
#pragma unroll
        for (int k = 0; k <= j; ++k) prod[q++] = (double)acc[j] * (double)acc[k];
    block_sum_store(prod, npair_of(n), d.s_part + tr.tile, d.ntile);
}

// omega = 1 without populations: psi_j(r) <- sum_p [xi_p psi*_j - dt chi_p V psi_hat_j](r - v_p),
// exactly the moment of the population update at omega = 1.
template <typename T, int NO, bool W>
__global__ __launch_bounds__(BS) void k_collapsed(const InstDesc *__restrict__ descs,
                                                  const int2 *__restrict__ tiles)
{
    const TileRef tr = resolve(tiles);
    const InstDesc &d = descs[tr.inst];
    const int n = d.n_orb;
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int s = tr.tile * BS + threadIdx.x;
    const bool valid = s < d.nsite;
    T acc[NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) acc[j] = (T)0;
    if (valid) {
        const size_t N = (size_t)d.nsite;
        const T *__restrict__ ph = (const T *)d.psihat;
        const T *__restrict__ pst = (const T *)d.psistar;
        const T *__restrict__ Vp = (const T *)d.V;
        const T dt = (T)d.dt;
        const int x = s % nx, yz = s / nx, y = yz % ny, z = yz / ny;
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const int vx = VX(p), vy = VY(p), vz = VZ(p);
            const bool ok = (unsigned)(x - vx) < (unsigned)nx && (unsigned)(y - vy) < (unsigned)ny &&
                            (unsigned)(z - vz) < (unsigned)nz;
            if (ok) {
                const int src = s - (vx + nx * (vy + ny * vz));
                const T cp = (T)d.xi[p];
                const T dp = dt * (T)d.chi[p] * Vp[src];
#pragma unroll
                for (int j = 0; j < NO; ++j) {
                    if (j < n) {
                        if (W) acc[j] += cp * pst[(size_t)j * N + src] - dp * ph[(size_t)j * N + src];
                        else acc[j] += (cp - dp) * ph[(size_t)j * N + src];
                    }
                }
            }
        }
        T *psi = (T *)d.psi;
#pragma unroll
        for (int j = 0; j < NO; ++j)
            if (j < n) psi[(size_t)j * N + s] = acc[j];
    }
    double prod[NO * (NO + 1) / 2];
    int q = 0;
#pragma unroll
    for (int j = 0; j < NO; ++j)
#pragma unroll
        for (int k = 0; k <= j; ++k) prod[q++] = (double)acc[j] * (double)acc[k];
    block_sum_store(prod, npair_of(n), d.s_part + tr.tile, d.ntile);
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
    const int n = d.n_orb;
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
        xc_eval(d.xc, rho, d.rho_floor, ex, ec, vx_, vc_);
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

__global__ __launch_bounds__(FB) void k_energy_finalize(const InstDesc *__restrict__ descs,
                                                        const int *__restrict__ list)
{
    const InstDesc &d = descs[resolve_inst(list)];
    const int n = d.n_orb, no = d.n_orb <= 5 ? d.n_orb : (d.n_orb <= 8 ? 8 : 16);
    const int nv = 2 * no + NEBASE;
    __shared__ double tot[2 * MAXO + NEBASE];
    reduce_columns(d.e_part, d.ntile, nv, tot);
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

__global__ void k_copy16(uint4 *__restrict__ dst, const uint4 *__restrict__ src, size_t n16)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
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

int launch_overlap_psi(const Plan &pl, hipStream_t st)
{
    return dispatch_tn(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_overlap_psi<typename TG::T, TG::NO><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site);
        LAUNCH_CHECK();
    });
}

int launch_overlap_finalize(const Plan &pl, hipStream_t st)
{
    k_overlap_finalize<<<grid_inst(pl), FB, 0, st>>>(pl.d_desc, pl.tt.inst);
    LAUNCH_CHECK();
}

int launch_orthonormalise(const Plan &pl, hipStream_t st)
{
    return dispatch_tnw(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_orthonormalise<typename TG::T, TG::NO, TG::W><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site);
        LAUNCH_CHECK();
    });
}

int launch_multipole_finalize(const Plan &pl, hipStream_t st)
{
    k_multipole_finalize<<<grid_inst(pl), FB, 0, st>>>(pl.d_desc, pl.tt.inst);
    LAUNCH_CHECK();
}

int launch_ghost(const Plan &pl, hipStream_t st)
{
    k_ghost<<<grid_ghost(pl), BS, 0, st>>>(pl.d_desc, pl.tt.ghost);
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
    k_residual_finalize<<<grid_inst(pl), FB, 0, st>>>(pl.d_desc, pl.tt.inst);
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

int launch_stream_collide(const Plan &pl, int parity, hipStream_t st)
{
    return dispatch_tnw(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_stream_collide<typename TG::T, TG::NO, TG::W><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site, parity);
        LAUNCH_CHECK();
    });
}

int launch_collapsed_update(const Plan &pl, hipStream_t st)
{
    return dispatch_tnw(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_collapsed<typename TG::T, TG::NO, TG::W><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site);
        LAUNCH_CHECK();
    });
}

int launch_energy_terms(const Plan &pl, hipStream_t st)
{
    return dispatch_tn(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_energy_terms<typename TG::T, TG::NO><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site);
        LAUNCH_CHECK();
    });
}

int launch_energy_finalize(const Plan &pl, hipStream_t st)
{
    k_energy_finalize<<<grid_inst(pl), FB, 0, st>>>(pl.d_desc, pl.tt.inst);
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
    k_gather<<<count, 32, 0, st>>>(scal, count, width, dst);
    LAUNCH_CHECK();
}

int launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    const size_t n16 = bytes / 16;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;
    if (blocks == 0) return 0;
    k_copy16<<<(unsigned)blocks, 256, 0, st>>>((uint4 *)dst, (const uint4 *)src, n16);
    LAUNCH_CHECK();
}

}  // namespace lbks
