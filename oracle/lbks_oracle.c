/*
 * lbks_oracle.c -- plain FP64 CPU oracle of the lattice kinetic Kohn-Sham
 * relaxation (Mendoza, Herrmann, Succi, "Lattice Boltzmann Model for
 * Electronic Structure Simulations").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file: only the test suite, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code with the GPU library.
 *
 * Every function does one step of the method, in the paper's order and
 * notation, with plain loops and no fusion.  Reductions are serial loops in
 * site order, so results do not depend on the thread count.  OpenMP only
 * splits element-wise loops over z-planes.
 *
 * Readings of passages the paper leaves garbled or silent (D3Q19 lattice,
 * xi_p and chi_p with the weights w_p, sign of the potential source,
 * Delta t = 2 (1/omega - 1/2) D h^2, Dirichlet-zero inflow, local Slater +
 * uniform-limit LYP exchange-correlation, multipole-bounded red/black SOR
 * Hartree solve) are listed with the functions that use them.
 *
 * Layouts: a scalar field is [nz][ny][nx], x fastest; orbital fields are
 * [n_orb][nz][ny][nx]; populations are [n_orb][19][nz][ny][nx]; the Hartree
 * potential carries one ghost layer on every side, [nz+2][ny+2][nx+2].
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Threads of the element-wise loops (n >= 1); results do not depend on it. */
void orc_set_threads(int n) { omp_set_num_threads(n < 1 ? 1 : n); }
int orc_max_threads(void) { return omp_get_max_threads(); }

#define ORC_Q 19

typedef long long i64;

/* ------------------------------------------------------------------ lattice */

/*
 * Velocity set, weights, xi_p and chi_p (section "The kinetic approach",
 * equilibrium f^e_p = xi_p psi and source V_p = chi_p V psi).
 * Reading: D3Q19, i.e. all v in {-1,0,1}^3 with |v|^2 <= 2, weights 1/3, 1/18,
 * 1/36 by |v|^2 = 0, 1, 2 and c_s^2 = 1/3.  The printed xi_p lacks the weight
 * that the sentence around it names, so xi_p = w_p (1 + (D - c_s^2) q_p) with
 * q_p = (|v_p|^2 - 3 c_s^2) / (2 c_s^4); chi_p = w_p (1 - (|v_p|^2 - 3 c_s^2) / (2 c_s^2))
 * with the stray parenthesis dropped.
 */
int orc_lattice(double D, int *v, double *w, double *xi, double *chi, double *cs2_out)
{
    const double cs2 = 1.0 / 3.0;
    int p = 0;
    for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
            for (int c = -1; c <= 1; ++c) {
                int v2 = a * a + b * b + c * c;
                if (v2 > 2) continue;
                v[3 * p + 0] = c;   /* x component */
                v[3 * p + 1] = b;   /* y component */
                v[3 * p + 2] = a;   /* z component */
                double wp = (v2 == 0) ? 1.0 / 3.0 : (v2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
                double qp = ((double)v2 - 3.0 * cs2) / (2.0 * cs2 * cs2);
                w[p] = wp;
                xi[p] = wp * (1.0 + (D - cs2) * qp);
                chi[p] = wp * (1.0 - ((double)v2 - 3.0 * cs2) / (2.0 * cs2));
                ++p;
            }
    if (cs2_out) *cs2_out = cs2;
    return p;
}

/* ---------------------------------------------------------------- reductions */

/* <a|b> without the volume element: plain serial sum in site order. */
double orc_dot(i64 n, const double *a, const double *b)
{
    double s = 0.0;
    for (i64 i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

double orc_sum(i64 n, const double *a)
{
    double s = 0.0;
    for (i64 i = 0; i < n; ++i) s += a[i];
    return s;
}

/* ------------------------------------------------------------------- moments */

/* psi_j(r) = sum_p f_jp(r): zeroth moment of the populations (kinetic
 * representation of the wave function). */
void orc_moment(int n_orb, i64 nsite, const double *f, double *psi)
{
#pragma omp parallel for schedule(static)
    for (i64 s = 0; s < nsite; ++s)
        for (int j = 0; j < n_orb; ++j) {
            double acc = 0.0;
            for (int p = 0; p < ORC_Q; ++p) acc += f[((i64)j * ORC_Q + p) * nsite + s];
            psi[(i64)j * nsite + s] = acc;
        }
}

/* S_jk = <psi_j|psi_k> = h^3 sum_r psi_j psi_k (orthogonality constraints). */
void orc_overlap(int n_orb, i64 nsite, double h, const double *psi, double *S)
{
    const double h3 = h * h * h;
    for (int j = 0; j < n_orb; ++j)
        for (int k = 0; k <= j; ++k) {
            double s = h3 * orc_dot(nsite, psi + (i64)j * nsite, psi + (i64)k * nsite);
            S[j * n_orb + k] = s;
            S[k * n_orb + j] = s;
        }
}

/*
 * Gram-Schmidt through the Cholesky factor: S = L L^T, C = L^{-T} (upper
 * triangular), so that psi_hat_j = sum_{l<=j} psi_l C_lj is the classical
 * Gram-Schmidt sequence of the psi_j (orbital j is orthogonalised against all
 * l < j, as in the orthogonalisation potential W_jp).  Returns -1 if S is not
 * positive definite.
 */
int orc_cholesky_inverse(int n, const double *S, double *C)
{
    double L[16 * 16];
    double Li[16 * 16];
    if (n < 1 || n > 16) return -2;
    memset(L, 0, sizeof L);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = S[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * 16 + k] * L[j * 16 + k];
            if (i == j) {
                if (!(s > 0.0)) return -1;
                L[i * 16 + i] = sqrt(s);
            } else {
                L[i * 16 + j] = s / L[j * 16 + j];
            }
        }
    /* Li = L^{-1} by forward substitution, column by column. */
    memset(Li, 0, sizeof Li);
    for (int c = 0; c < n; ++c)
        for (int i = c; i < n; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) s -= L[i * 16 + k] * Li[k * 16 + c];
            Li[i * 16 + c] = s / L[i * 16 + i];
        }
    for (int l = 0; l < n; ++l)
        for (int j = 0; j < n; ++j) C[l * n + j] = Li[j * 16 + l];   /* C = Li^T */
    return 0;
}

/* dst_j = sum_l src_l C_lj for blocks of `len` values per orbital. */
void orc_combine(int n_orb, i64 len, const double *C, const double *src, double *dst)
{
#pragma omp parallel for schedule(static)
    for (i64 s = 0; s < len; ++s)
        for (int j = 0; j < n_orb; ++j) {
            double acc = 0.0;
            for (int l = 0; l < n_orb; ++l) acc += src[(i64)l * len + s] * C[l * n_orb + j];
            dst[(i64)j * len + s] = acc;
        }
}

/*
 * Paper-literal orthogonalisation (equations for W_jp and psi*_j): each
 * orbital is normalised, n_j = sqrt(S_jj), psi_hat_j = psi_j / n_j,
 * g_jp = f_jp / n_j, and the equilibrium uses
 * psi*_j = psi_hat_j - sum_{l<j} Lambda_jl psi_hat_l with
 * Lambda_jl = <psi_hat_j|psi_hat_l> / <psi_hat_l|psi_hat_l> = S_jl / (n_j n_l).
 */
void orc_w_fields(int n_orb, i64 nsite, const double *S, const double *psi, const double *f,
                  double *psihat, double *psistar, double *g)
{
    double n[16], lam[16 * 16];
    for (int j = 0; j < n_orb; ++j) n[j] = sqrt(S[j * n_orb + j]);
    for (int j = 0; j < n_orb; ++j)
        for (int l = 0; l < n_orb; ++l) lam[j * 16 + l] = S[j * n_orb + l] / (n[j] * n[l]);
#pragma omp parallel for schedule(static)
    for (i64 s = 0; s < nsite; ++s) {
        for (int j = 0; j < n_orb; ++j) psihat[(i64)j * nsite + s] = psi[(i64)j * nsite + s] / n[j];
        for (int j = 0; j < n_orb; ++j) {
            double acc = psihat[(i64)j * nsite + s];
            for (int l = 0; l < j; ++l) acc -= lam[j * 16 + l] * psihat[(i64)l * nsite + s];
            psistar[(i64)j * nsite + s] = acc;
        }
        for (int j = 0; j < n_orb; ++j)
            for (int p = 0; p < ORC_Q; ++p)
                g[((i64)j * ORC_Q + p) * nsite + s] = f[((i64)j * ORC_Q + p) * nsite + s] / n[j];
    }
}

/* rho(r) = sum_j occ_j |psi_hat_j(r)|^2 (closed-shell occupations). */
void orc_density(int n_orb, i64 nsite, const double *occ, const double *psihat, double *rho)
{
#pragma omp parallel for schedule(static)
    for (i64 s = 0; s < nsite; ++s) {
        double acc = 0.0;
        for (int j = 0; j < n_orb; ++j) {
            double v = psihat[(i64)j * nsite + s];
            acc += occ[j] * v * v;
        }
        rho[s] = acc;
    }
}

/* ------------------------------------------------------------------- Hartree */

static double coord(int i, int n, double h) { return ((double)i - 0.5 * (double)(n - 1)) * h; }

/*
 * Multipoles of rho about the origin (reading of the Hartree boundary):
 * m = {q, p_x, p_y, p_z, Q_xx, Q_yy, Q_zz, Q_xy, Q_xz, Q_yz} with
 * q = <1|rho>, p_a = <r_a|rho>, Q_ab = <3 r_a r_b - r^2 delta_ab|rho>.
 */
void orc_multipoles(int nx, int ny, int nz, double h, const double *rho, double *m)
{
    const double h3 = h * h * h;
    double acc[10] = {0};
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double x = coord(i, nx, h), y = coord(j, ny, h), z = coord(k, nz, h);
                double r2 = x * x + y * y + z * z;
                double d = rho[((i64)k * ny + j) * nx + i];
                acc[0] += d;
                acc[1] += x * d;
                acc[2] += y * d;
                acc[3] += z * d;
                acc[4] += (3.0 * x * x - r2) * d;
                acc[5] += (3.0 * y * y - r2) * d;
                acc[6] += (3.0 * z * z - r2) * d;
                acc[7] += 3.0 * x * y * d;
                acc[8] += 3.0 * x * z * d;
                acc[9] += 3.0 * y * z * d;
            }
    for (int t = 0; t < 10; ++t) m[t] = h3 * acc[t];
}

/* Far-field Hartree potential of the multipoles: q/r + p.r/r^3 + (1/2) sum Q_ab r_a r_b / r^5. */
double orc_multipole_value(const double *m, double x, double y, double z)
{
    double r2 = x * x + y * y + z * z;
    double r = sqrt(r2);
    double r3 = r2 * r, r5 = r3 * r2;
    double quad = m[4] * x * x + m[5] * y * y + m[6] * z * z
                + 2.0 * (m[7] * x * y + m[8] * x * z + m[9] * y * z);
    return m[0] / r + (m[1] * x + m[2] * y + m[3] * z) / r3 + 0.5 * quad / r5;
}

#define VH(i, j, k) vh[(((i64)(k) + 1) * (ny + 2) + ((j) + 1)) * (nx + 2) + ((i) + 1)]

/* Dirichlet data on the six ghost faces (edges and corners are never read). */
void orc_boundary(int nx, int ny, int nz, double h, const double *m, double *vh)
{
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
            VH(-1, j, k) = orc_multipole_value(m, coord(-1, nx, h), coord(j, ny, h), coord(k, nz, h));
            VH(nx, j, k) = orc_multipole_value(m, coord(nx, nx, h), coord(j, ny, h), coord(k, nz, h));
        }
    for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nx; ++i) {
            VH(i, -1, k) = orc_multipole_value(m, coord(i, nx, h), coord(-1, ny, h), coord(k, nz, h));
            VH(i, ny, k) = orc_multipole_value(m, coord(i, nx, h), coord(ny, ny, h), coord(k, nz, h));
        }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            VH(i, j, -1) = orc_multipole_value(m, coord(i, nx, h), coord(j, ny, h), coord(-1, nz, h));
            VH(i, j, nz) = orc_multipole_value(m, coord(i, nx, h), coord(j, ny, h), coord(nz, nz, h));
        }
}

/* Over-relaxation factor for red/black SOR on the 7-point Laplacian:
 * Jacobi radius mu = (cos(pi/(nx+1)) + cos(pi/(ny+1)) + cos(pi/(nz+1))) / 3,
 * omega = 2 / (1 + sqrt(1 - mu^2)) (= 2 / (1 + sin(pi/(n+1))) on a cube). */
double orc_sor_omega(int nx, int ny, int nz)
{
    const double pi = 3.14159265358979323846;
    double mu = (cos(pi / (nx + 1)) + cos(pi / (ny + 1)) + cos(pi / (nz + 1))) / 3.0;
    return 2.0 / (1.0 + sqrt(1.0 - mu * mu));
}

/*
 * One SOR sweep of the discrete Poisson equation
 * (sum of the 6 face neighbours - 6 V_H) / h^2 = -4 pi rho:
 * first every red node ((i+j+k) even), then every black node.
 */
void orc_sor_sweep(int nx, int ny, int nz, double h, double omega, const double *rho, double *vh)
{
    const double four_pi_h2 = 4.0 * 3.14159265358979323846 * h * h;
    for (int color = 0; color < 2; ++color) {
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    if (((i + j + k) & 1) != color) continue;
                    double nb = VH(i - 1, j, k) + VH(i + 1, j, k) + VH(i, j - 1, k)
                              + VH(i, j + 1, k) + VH(i, j, k - 1) + VH(i, j, k + 1);
                    double gs = (nb + four_pi_h2 * rho[((i64)k * ny + j) * nx + i]) / 6.0;
                    VH(i, j, k) = (1.0 - omega) * VH(i, j, k) + omega * gs;
                }
    }
}

/* Relative residual ||lap_h V_H + 4 pi rho||_2 / ||4 pi rho||_2 over the nodes. */
double orc_poisson_residual(int nx, int ny, int nz, double h, const double *rho, const double *vh)
{
    const double fp = 4.0 * 3.14159265358979323846;
    double rr = 0.0, bb = 0.0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double nb = VH(i - 1, j, k) + VH(i + 1, j, k) + VH(i, j - 1, k)
                          + VH(i, j + 1, k) + VH(i, j, k - 1) + VH(i, j, k + 1);
                double b = fp * rho[((i64)k * ny + j) * nx + i];
                double r = (nb - 6.0 * VH(i, j, k)) / (h * h) + b;
                rr += r * r;
                bb += b * b;
            }
    return bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
}

/* Copy the node values of the padded Hartree potential into a plain field. */
void orc_vh_interior(int nx, int ny, int nz, const double *vh, double *out)
{
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) out[((i64)k * ny + j) * nx + i] = VH(i, j, k);
}
#undef VH

/* --------------------------------------------------------- nuclei, xc, V */

/* Nuclear attraction, read as V_ext(r) = -sum_I Z_I / sqrt(|r - R_I|^2 + a^2)
 * (softened Coulomb; positions relative to the grid centre). */
void orc_vext(int nx, int ny, int nz, double h, int nnuc, const double *Z, const double *R,
              double a, double *vext)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double x = coord(i, nx, h), y = coord(j, ny, h), z = coord(k, nz, h);
                double v = 0.0;
                for (int I = 0; I < nnuc; ++I) {
                    double dx = x - R[3 * I], dy = y - R[3 * I + 1], dz = z - R[3 * I + 2];
                    v -= Z[I] / sqrt(dx * dx + dy * dy + dz * dz + a * a);
                }
                vext[((i64)k * ny + j) * nx + i] = v;
            }
}

/* Ion-ion repulsion sum_{I<J} Z_I Z_J / |R_I - R_J| (bare Coulomb). */
double orc_enn(int nnuc, const double *Z, const double *R)
{
    double e = 0.0;
    for (int I = 0; I < nnuc; ++I)
        for (int J = I + 1; J < nnuc; ++J) {
            double dx = R[3 * I] - R[3 * J], dy = R[3 * I + 1] - R[3 * J + 1], dz = R[3 * I + 2] - R[3 * J + 2];
            e += Z[I] * Z[J] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    return e;
}

/*
 * Forces on the nuclei in the Born-Oppenheimer scenario (section "Concurrent
 * Dynamics": the ions move on the surface defined by the electronic ground
 * state).  Hellmann-Feynman: with the density held fixed, the electronic force
 * is minus the derivative of <V_ext|rho> with respect to R_I,
 *   F_I^el = Z_I h^3 sum_r rho(r) (r - R_I) / (|r - R_I|^2 + a^2)^(3/2),
 * and the ion-ion force is minus the gradient of E_NN,
 *   F_I^NN = sum_{J != I} Z_I Z_J (R_I - R_J) / |R_I - R_J|^3.
 * F is [nnuc][3], electronic plus ion-ion, in hartree per bohr.  Sums run over
 * the nodes in site order.
 */
void orc_forces(int nx, int ny, int nz, double h, int nnuc, const double *Z, const double *R,
                double a, const double *rho, double *F)
{
    for (int I = 0; I < nnuc; ++I) {
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    double dx = coord(i, nx, h) - R[3 * I];
                    double dy = coord(j, ny, h) - R[3 * I + 1];
                    double dz = coord(k, nz, h) - R[3 * I + 2];
                    double d2 = dx * dx + dy * dy + dz * dz + a * a;
                    double w = rho[((i64)k * ny + j) * nx + i] / (d2 * sqrt(d2));
                    fx += w * dx;
                    fy += w * dy;
                    fz += w * dz;
                }
        double hz = Z[I] * h * h * h;
        F[3 * I] = hz * fx;
        F[3 * I + 1] = hz * fy;
        F[3 * I + 2] = hz * fz;
        for (int J = 0; J < nnuc; ++J) {
            if (J == I) continue;
            double dx = R[3 * I] - R[3 * J], dy = R[3 * I + 1] - R[3 * J + 1], dz = R[3 * I + 2] - R[3 * J + 2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double c = Z[I] * Z[J] / (r * r * r);
            F[3 * I] += c * dx;
            F[3 * I + 1] += c * dy;
            F[3 * I + 2] += c * dz;
        }
    }
}

enum { ORC_XC_NONE = 0, ORC_XC_X = 1, ORC_XC_X_LYPLOCAL = 2, ORC_XC_X_PZ81 = 3, ORC_XC_B88_LYP = 4,
       ORC_XC_B88_LYP_POLARISED = 5 };

/*
 * Local exchange-correlation per unit charge (eps) and potential (v = d(rho eps)/drho)
 * at density rho (the paper leaves V_xc unspecified).  Reading:
 *  - Slater exchange: eps_x = -(3/4)(3/pi)^(1/3) rho^(1/3), v_x = -(3 rho/pi)^(1/3);
 *  - correlation of Lee, Yang and Parr (1988) at zero density gradient,
 *    eps_c = -a g(u), g(u) = (1 + b C_F e^{-c u}) / (1 + d u), u = rho^(-1/3),
 *    C_F = (3/10)(3 pi^2)^(2/3), (a, b, c, d) = (0.04918, 0.132, 0.2533, 0.349);
 *    v_c = -a (g - (u/3) g'(u));
 *  - alternatively Perdew-Zunger 1981 unpolarised correlation.
 * Below `floor` everything is zero.
 */
void orc_xc_point(int kind, double rho, double floor, double *ex, double *ec, double *vx, double *vc)
{
    const double pi = 3.14159265358979323846;
    *ex = *ec = *vx = *vc = 0.0;
    if (kind == ORC_XC_NONE || !(rho >= floor) || rho <= 0.0) return;
    double c13 = cbrt(rho);
    *vx = -cbrt(3.0 * rho / pi);
    *ex = 0.75 * (*vx);
    if (kind == ORC_XC_X_LYPLOCAL) {
        const double a = 0.04918, b = 0.132, c = 0.2533, d = 0.349;
        const double CF = 0.3 * pow(3.0 * pi * pi, 2.0 / 3.0);
        double u = 1.0 / c13;
        double e = exp(-c * u);
        double num = 1.0 + b * CF * e;
        double den = 1.0 + d * u;
        double g = num / den;
        double gp = (-b * CF * c * e * den - d * num) / (den * den);
        *ec = -a * g;
        *vc = -a * (g - (u / 3.0) * gp);
    } else if (kind == ORC_XC_X_PZ81) {
        double rs = cbrt(3.0 / (4.0 * pi * rho));
        if (rs >= 1.0) {
            const double gam = -0.1423, b1 = 1.0529, b2 = 0.3334;
            double sq = sqrt(rs);
            double den = 1.0 + b1 * sq + b2 * rs;
            *ec = gam / den;
            *vc = (*ec) * (1.0 + (7.0 / 6.0) * b1 * sq + (4.0 / 3.0) * b2 * rs) / den;
        } else {
            const double A = 0.0311, B = -0.048, C = 0.0020, Dd = -0.0116;
            double lr = log(rs);
            *ec = A * lr + B + C * rs * lr + Dd * rs;
            *vc = A * lr + (B - A / 3.0) + (2.0 / 3.0) * C * rs * lr + (2.0 * Dd - C) * rs / 3.0;
        }
    }
}

void orc_xc(int kind, i64 nsite, const double *rho, double floor, double *ex, double *ec,
            double *vx, double *vc)
{
#pragma omp parallel for schedule(static)
    for (i64 s = 0; s < nsite; ++s) orc_xc_point(kind, rho[s], floor, ex + s, ec + s, vx + s, vc + s);
}

/*
 * Gradient-corrected exchange-correlation (the functionals the paper's Table 1
 * compares with: Becke 1988 exchange and Lee-Yang-Parr 1988 correlation),
 * spin-unpolarised, as energy densities per volume f(rho, sigma), sigma = |grad rho|^2.
 *
 * Becke 1988, per spin density n = rho/2 with gradient g = |grad rho|/2:
 *   e_s = -C n^(4/3) - beta n^(4/3) H(x),  x = g / n^(4/3),
 *   H(x) = x^2 / (1 + 6 beta x asinh x),  C = (3/4)(6/pi)^(1/3),  beta = 0.0042;
 * the total is 2 e_s, which at sigma = 0 is Slater exchange.
 *
 * Lee-Yang-Parr 1988, closed shell, u = rho^(-1/3):
 *   E_c = -a int [rho + b rho^(-2/3) (C_F rho^(5/3) - 2 t_W + (t_W + lap rho / 2) / 9)
 *                 e^(-c u)] / (1 + d u),   t_W = sigma / (8 rho) - lap rho / 8.
 * Reading: the Laplacian terms are integrated by parts (the density vanishes at
 * the box walls), which leaves f_c = f0(rho) + f1(rho) sigma with
 *   f0 = -a rho (1 + b C_F e^(-c u)) / (1 + d u)            (the local form above),
 *   f1 = a b rho^(-5/3) e^(-c u) / (1 + d u) (3 + 7 delta) / 72,
 *   delta = c u + d u / (1 + d u).
 * Below `floor` everything is zero.  Outputs: energy densities and their partial
 * derivatives with respect to rho and sigma, exchange and correlation apart.
 */
void orc_gga_point(double rho, double sigma, double floor, double *fx, double *fc, double *fx_r, double *fc_r,
                   double *fx_s, double *fc_s)
{
    const double pi = 3.14159265358979323846;
    *fx = *fc = *fx_r = *fc_r = *fx_s = *fc_s = 0.0;
    if (!(rho >= floor) || rho <= 0.0) return;
    /* Becke 1988 */
    {
        const double beta = 0.0042, C = 0.75 * cbrt(6.0 / pi);
        double n = 0.5 * rho, n13 = cbrt(n), n43 = n * n13;
        double x = 0.5 * sqrt(sigma) / n43;
        double as = asinh(x);
        double q = 1.0 + 6.0 * beta * x * as;
        double H = x * x / q;
        /* H'(x) / x, finite at x = 0 */
        double Hpx = (2.0 * q - 6.0 * beta * x * (as + x / sqrt(1.0 + x * x))) / (q * q);
        double es = -C * n43 - beta * n43 * H;
        *fx = 2.0 * es;
        /* d(2 e_s)/d rho = d e_s/dn at fixed g; d/dn = -(4/3) C n^(1/3) - (4/3) beta n^(1/3) (H - x H') */
        *fx_r = -(4.0 / 3.0) * C * n13 - (4.0 / 3.0) * beta * n13 * (H - x * x * Hpx);
        /* d(2 e_s)/d sigma = -beta H'(x) / (2 sqrt(sigma)) = -beta (H'/x) / (4 n^(4/3)) */
        *fx_s = -beta * Hpx / (4.0 * n43);
    }
    /* Lee-Yang-Parr 1988 */
    {
        const double a = 0.04918, b = 0.132, c = 0.2533, d = 0.349;
        const double CF = 0.3 * pow(3.0 * pi * pi, 2.0 / 3.0);
        double u = 1.0 / cbrt(rho);
        double e = exp(-c * u);
        double den = 1.0 + d * u;
        /* f0 and its derivative: the local form, f0 = rho eps_c, f0' = v_c */
        double num = 1.0 + b * CF * e;
        double g = num / den;
        double gp = (-b * CF * c * e * den - d * num) / (den * den);
        double f0 = -a * rho * g;
        double f0p = -a * (g - (u / 3.0) * gp);
        double delta = c * u + d * u / den;
        double A = pow(rho, -5.0 / 3.0) * e / den;   /* rho^(-5/3) e^(-cu) / (1 + du) */
        double f1 = a * b * A * (3.0 + 7.0 * delta) / 72.0;
        /* f1' = a b A / (216 rho) [(delta - 5)(3 + 7 delta) - 7 u (c + d / (1 + du)^2)] */
        double f1p = a * b * A / (216.0 * rho) * ((delta - 5.0) * (3.0 + 7.0 * delta) - 7.0 * u * (c + d / (den * den)));
        *fc = f0 + f1 * sigma;
        *fc_r = f0p + f1p * sigma;
        *fc_s = f1;
    }
}

/*
 * The same functionals for a fully spin-polarised density (every electron in one
 * spin channel: rho_up = rho, rho_down = 0, as for the hydrogen atom of Table 1).
 * Becke's exchange is a sum over spin channels, here the one channel with spin
 * density n = rho and gradient g = sqrt(sigma):
 *   f_x = -C n^(4/3) - beta n^(4/3) x^2 / (1 + 6 beta x asinh x),  x = g / n^(4/3).
 * Lee-Yang-Parr correlation in its spin-resolved form has every term either
 * proportional to rho_up rho_down or cancelling when rho_down = 0, so f_c = 0.
 */
void orc_gga_point_polarised(double rho, double sigma, double floor, double *fx, double *fc, double *fx_r,
                             double *fc_r, double *fx_s, double *fc_s)
{
    const double pi = 3.14159265358979323846;
    *fx = *fc = *fx_r = *fc_r = *fx_s = *fc_s = 0.0;
    if (!(rho >= floor) || rho <= 0.0) return;
    const double beta = 0.0042, C = 0.75 * cbrt(6.0 / pi);
    double n13 = cbrt(rho), n43 = rho * n13;
    double x = sqrt(sigma) / n43;
    double as = asinh(x);
    double q = 1.0 + 6.0 * beta * x * as;
    double H = x * x / q;
    double Hpx = (2.0 * q - 6.0 * beta * x * (as + x / sqrt(1.0 + x * x))) / (q * q);   /* H'(x) / x */
    *fx = -C * n43 - beta * n43 * H;
    /* d/dn at fixed g: -(4/3) C n^(1/3) - (4/3) beta n^(1/3) (H - x H'), as for one channel above */
    *fx_r = -(4.0 / 3.0) * C * n13 - (4.0 / 3.0) * beta * n13 * (H - x * x * Hpx);
    /* d/d sigma = -beta n^(4/3) H'(x) x / (2 sigma) = -beta (H'/x) / (2 n^(4/3)) */
    *fx_s = -beta * Hpx / (2.0 * n43);
}

/*
 * Gradient-corrected exchange-correlation on the grid.  sigma = |D rho|^2 with
 * central differences D_a rho = (rho(r + e_a) - rho(r - e_a)) / 2h and rho = 0
 * outside the box; the potential is the exact derivative of the discrete energy
 * h^3 sum_r f(rho_r, sigma_r) with respect to rho_s, divided by h^3:
 *   v = df/drho - sum_a D_a [2 (df/dsigma) D_a rho]   (same central differences).
 * ex, ec: energy per particle (f / rho, zero where rho = 0) so that E = h^3 <rho|e>;
 * vx, vc: the exchange and correlation parts of v.  polarised: the fully
 * spin-polarised functionals (orc_gga_point_polarised), else spin-unpolarised.
 */
void orc_gga(int nx, int ny, int nz, double h, const double *rho, double floor, int polarised, double *ex,
             double *ec, double *vx, double *vc)
{
    const i64 N = (i64)nx * ny * nz;
    double *gx = (double *)calloc((size_t)N * 6, sizeof(double));   /* 2 f_s D_a rho, exchange then correlation */
    const i64 sx = 1, sy = nx, sz = (i64)nx * ny;
    const double ih2 = 1.0 / (2.0 * h);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                i64 s = ((i64)k * ny + j) * nx + i;
                double xp = i + 1 < nx ? rho[s + sx] : 0.0, xm = i > 0 ? rho[s - sx] : 0.0;
                double yp = j + 1 < ny ? rho[s + sy] : 0.0, ym = j > 0 ? rho[s - sy] : 0.0;
                double zp = k + 1 < nz ? rho[s + sz] : 0.0, zm = k > 0 ? rho[s - sz] : 0.0;
                double D[3] = {(xp - xm) * ih2, (yp - ym) * ih2, (zp - zm) * ih2};
                double sigma = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
                double fx, fc, fxr, fcr, fxs, fcs;
                if (polarised)
                    orc_gga_point_polarised(rho[s], sigma, floor, &fx, &fc, &fxr, &fcr, &fxs, &fcs);
                else
                    orc_gga_point(rho[s], sigma, floor, &fx, &fc, &fxr, &fcr, &fxs, &fcs);
                ex[s] = rho[s] > 0.0 ? fx / rho[s] : 0.0;
                ec[s] = rho[s] > 0.0 ? fc / rho[s] : 0.0;
                vx[s] = fxr;
                vc[s] = fcr;
                for (int a = 0; a < 3; ++a) {
                    gx[(i64)a * N + s] = 2.0 * fxs * D[a];
                    gx[(i64)(3 + a) * N + s] = 2.0 * fcs * D[a];
                }
            }
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                i64 s = ((i64)k * ny + j) * nx + i;
                for (int part = 0; part < 2; ++part) {
                    const double *G = gx + (i64)3 * part * N;
                    double div = 0.0;
                    div += ((i + 1 < nx ? G[s + sx] : 0.0) - (i > 0 ? G[s - sx] : 0.0)) * ih2;
                    div += ((j + 1 < ny ? G[N + s + sy] : 0.0) - (j > 0 ? G[N + s - sy] : 0.0)) * ih2;
                    div += ((k + 1 < nz ? G[2 * N + s + sz] : 0.0) - (k > 0 ? G[2 * N + s - sz] : 0.0)) * ih2;
                    if (part == 0) vx[s] -= div;
                    else vc[s] -= div;
                }
            }
    free(gx);
}

/* ---------------------------------------------------- collide and stream */

/*
 * BGK collision with the equilibrium and potential sources (lattice Boltzmann
 * equation for orbital j):
 *   f^post_jp = g_jp - omega (g_jp - xi_p psi*_j) - Delta t chi_p V psi_hat_j
 *             = (1 - omega) g_jp + omega xi_p psi*_j - Delta t chi_p V psi_hat_j,
 * where g is the normalised (or orthonormalised) population.  Reading of the
 * source: the imaginary-time equation needs -V psi, so the source enters with
 * a minus sign, scaled by the physical time step Delta t of one lattice step.
 */
void orc_collide(int n_orb, i64 nsite, double omega, double dt, const double *xi, const double *chi,
                 const double *g, const double *psistar, const double *psihat, const double *V,
                 double *fpost)
{
#pragma omp parallel for schedule(static)
    for (i64 s = 0; s < nsite; ++s)
        for (int j = 0; j < n_orb; ++j)
            for (int p = 0; p < ORC_Q; ++p) {
                i64 idx = ((i64)j * ORC_Q + p) * nsite + s;
                fpost[idx] = (1.0 - omega) * g[idx] + omega * xi[p] * psistar[(i64)j * nsite + s]
                           - dt * chi[p] * V[s] * psihat[(i64)j * nsite + s];
            }
}

/*
 * Streaming f_jp(r + v_p; t+1) = f^post_jp(r; t).  Populations that would
 * enter from outside the box are zero; populations leaving the box are
 * discarded (Dirichlet-zero reading of the boundary).
 */
void orc_stream(int n_orb, int nx, int ny, int nz, const int *v, const double *fpost, double *f)
{
    const i64 nsite = (i64)nx * ny * nz;
    for (int j = 0; j < n_orb; ++j)
        for (int p = 0; p < ORC_Q; ++p) {
            const double *src = fpost + ((i64)j * ORC_Q + p) * nsite;
            double *dst = f + ((i64)j * ORC_Q + p) * nsite;
            int vx = v[3 * p], vy = v[3 * p + 1], vz = v[3 * p + 2];
#pragma omp parallel for schedule(static)
            for (int k = 0; k < nz; ++k)
                for (int jj = 0; jj < ny; ++jj)
                    for (int i = 0; i < nx; ++i) {
                        int si = i - vx, sj = jj - vy, sk = k - vz;
                        double val = 0.0;
                        if (si >= 0 && si < nx && sj >= 0 && sj < ny && sk >= 0 && sk < nz)
                            val = src[((i64)sk * ny + sj) * nx + si];
                        dst[((i64)k * ny + jj) * nx + i] = val;
                    }
        }
}

/* Initial populations at equilibrium, f_jp = xi_p psi_j. */
void orc_equilibrium(int n_orb, i64 nsite, const double *xi, const double *psi, double *f)
{
#pragma omp parallel for schedule(static)
    for (i64 s = 0; s < nsite; ++s)
        for (int j = 0; j < n_orb; ++j)
            for (int p = 0; p < ORC_Q; ++p)
                f[((i64)j * ORC_Q + p) * nsite + s] = xi[p] * psi[(i64)j * nsite + s];
}

/* (S_w u)(r) = sum_p wts_p u(r - v_p), zero outside the box. */
void orc_apply_sw(int nx, int ny, int nz, const int *v, const double *wts, const double *u, double *out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double acc = 0.0;
                for (int p = 0; p < ORC_Q; ++p) {
                    int si = i - v[3 * p], sj = j - v[3 * p + 1], sk = k - v[3 * p + 2];
                    if (si >= 0 && si < nx && sj >= 0 && sj < ny && sk >= 0 && sk < nz)
                        acc += wts[p] * u[((i64)sk * ny + sj) * nx + si];
                }
                out[((i64)k * ny + j) * nx + i] = acc;
            }
}
