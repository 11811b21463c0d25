/*
 * lbks.h -- C ABI of the lattice kinetic Kohn-Sham relaxation library for
 * AMD Instinct MI355X (gfx950).
 *
 * The library finds the lowest n_orb Kohn-Sham orbitals, the density, the
 * total energy and the orbital energies of a set of nuclei (Kohn-Sham
 * equations with the orthogonality constraints, section "Kohn-Sham
 * formulation") as the steady state of one lattice Boltzmann imaginary-time
 * relaxation per orbital, coupled through the self-consistent potential and
 * the orthogonalisation source (section "The kinetic approach to Kohn-Sham
 * theory", lattice Boltzmann equation per orbital and its Gram-Schmidt form).
 *
 * Units are atomic units (hartree, bohr).  Grids are cubic-celled boxes of
 * N[0] x N[1] x N[2] nodes with spacing h; node (i, j, k) sits at
 * ((i - (N[0]-1)/2) h, (j - (N[1]-1)/2) h, (k - (N[2]-1)/2) h), so the origin
 * is the box centre.  Scalar fields are laid out [k][j][i] (x fastest) and
 * orbital fields [orbital][k][j][i].
 *
 * Conventions for every call:
 *  - return value 0 (LBKS_OK) on success, a negative LBKS_E_* code on error;
 *    lbks_last_error() then holds a message.  No C++ exception crosses the ABI.
 *  - pointer arguments documented as "host" are ordinary CPU memory owned by
 *    the caller and only read or written during the call.
 *  - a context is not thread-safe; distinct contexts are independent.
 *  - all GPU work is enqueued on the stream given at creation; calls that
 *    return results to the host synchronise that stream.
 */
#ifndef LBKS_H
#define LBKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBKS_MAX_ORB 16
#define LBKS_MAX_NUC 64

/* status codes */
#define LBKS_OK 0
#define LBKS_NOT_CONVERGED 1
#define LBKS_E_INVAL (-1)
#define LBKS_E_NOMEM (-2)
#define LBKS_E_HIP (-3)
#define LBKS_E_NUMERIC (-4)
#define LBKS_E_STATE (-5)

/* orthogonalisation: exact Cholesky Gram-Schmidt each step, or the paper's
 * orthogonalisation source (normalised orbitals, lagged projection
 * psi*_j = psi_j - sum_{k<j} Lambda_jk psi_k in the equilibrium). */
#define LBKS_ORTHO_GS 0
#define LBKS_ORTHO_W 1

/* exchange-correlation (the paper leaves V_xc open): none, Slater exchange,
 * Slater + Lee-Yang-Parr correlation at zero density gradient, Slater +
 * Perdew-Zunger 1981, or the gradient-corrected functionals the paper's Table 1
 * compares with: Becke 1988 exchange + Lee-Yang-Parr 1988 correlation
 * (spin-unpolarised; the gradient is taken by central differences and the
 * potential is the exact derivative of the discrete energy; 32 more bytes of
 * device memory per node), or the same for a fully spin-polarised density
 * (every electron in one spin channel, as for the hydrogen atom of Table 1:
 * Becke exchange of that channel, no Lee-Yang-Parr correlation). */
#define LBKS_XC_NONE 0
#define LBKS_XC_X 1
#define LBKS_XC_X_LYPLOCAL 2
#define LBKS_XC_X_PZ81 3
#define LBKS_XC_B88_LYP 4
#define LBKS_XC_B88_LYP_POLARISED 5

/* precision: everything in FP64, or populations, orbitals, density and
 * potential stored and streamed in FP32 while the overlap, Cholesky factor,
 * Hartree potential, Poisson residual and all energy sums stay FP64. */
#define LBKS_FP64 0
#define LBKS_FP32_BULK 1

/* initial orbitals: exp(-r^2/2s^2) + noise (2u-1); exp(-r^2/2s^2)(2u-1);
 * or supplied later with lbks_set_orbitals.  u is the SplitMix64 draw
 * k = ((j N[2] + z) N[1] + y) N[0] + x under `seed`, mapped to [0,1) by its
 * 53 high bits. */
#define LBKS_INIT_GAUSS_NOISE 0
#define LBKS_INIT_RANDOM_GAUSS 1
#define LBKS_INIT_USER 2

/* relaxation scheme: populations f_jp stored and streamed (the lattice
 * Boltzmann equation as written, any omega), or, at omega = 1 only, the
 * equivalent update of the orbital fields alone
 * psi_j <- S_xi psi*_j - dt S_chi (V psi_hat_j), which needs no populations. */
#define LBKS_SCHEME_POPULATIONS 0
#define LBKS_SCHEME_COLLAPSED 1

typedef struct lbks_params {
    int32_t N[3];            /* nodes per axis, each in [4, 1024]; N0 N1 N2 < 2^29 */
    double h;                /* node spacing (bohr) */
    int32_t n_orb;           /* orbitals, 1..LBKS_MAX_ORB */
    int32_t n_elec;          /* electrons; occupations 2,2,...,n_elec-2(n_orb-1), or 1 each
                                with LBKS_XC_B88_LYP_POLARISED (n_elec = n_orb) */
    double omega;            /* BGK relaxation frequency (default 1) */
    double D;                /* second moment of the equilibrium weights xi_p (default 1/3) */
    int32_t ortho;           /* LBKS_ORTHO_* */
    int32_t xc;              /* LBKS_XC_* */
    int32_t hartree;         /* 1: include the Hartree potential */
    int32_t poisson_sweeps;  /* red/black SOR sweeps per lattice step (default 2) */
    int32_t precision;       /* LBKS_FP64 or LBKS_FP32_BULK */
    double softening;        /* a in -Z / sqrt(|r-R|^2 + a^2) (bohr) */
    int32_t init;            /* LBKS_INIT_* */
    double init_sigma;       /* s of the initial Gaussian envelope (bohr) */
    double init_noise;       /* noise amplitude for LBKS_INIT_GAUSS_NOISE */
    uint64_t seed;           /* SplitMix64 seed of the initial orbitals */
    double rho_floor;        /* exchange-correlation is zero below this density */
    int32_t scheme;          /* LBKS_SCHEME_* */
    int32_t stop_checks;     /* stopping rule of lbks_relax: consecutive passing checks needed (0, 1: one) */
    double deps_tol;         /* > 0: a check also needs |change of sum_j eps_j| < deps_tol */
    int32_t hermite;         /* order of the Hermite expansion of the equilibrium and source
                                weights: 2 (0 means 2) or 4 (see LBKS_HERMITE_4) */
    int32_t fold;            /* 0 (default): on grids of at most 65536 nodes (256 tiles of 256) the
                                overlap totals (at most five orbitals) and the multipole totals are
                                summed by every workgroup of the kernel that uses them, in the order
                                of the separate reduction kernel, and the first red Poisson
                                half-sweep of a step also writes the ghost faces: three launches
                                fewer per lattice step, the same results bit for bit.  A batch
                                launch folds when all its members allow it.  -1: always the
                                separate kernels */
    int32_t reserved[2];     /* must be zero */
} lbks_params;

/* Fourth-order Hermite weights (params.hermite = 4; the paper uses fourth order
 * in its He run, section Results): on the D3Q19 velocities the equilibrium
 * weights also match the mixed fourth moment of a Gaussian of variance D,
 *   sum_p xi_p = 1, sum xi_p v_a v_b = D delta_ab, sum xi_p v_x^2 v_y^2 = D^2,
 *   i.e. xi = 1 - 3D + 3D^2 (rest), D/2 - D^2 (faces), D^2/4 (edges),
 * equal to the second-order weights at D = c_s^2 = 1/3, and the potential
 * source has no second or mixed fourth moment,
 *   sum chi_p = 1, sum chi_p v_a v_b = 0, sum chi_p v_x^2 v_y^2 = 0,
 * which on D3Q19 leaves chi = 1 on the rest velocity: the potential acts at the
 * node, so the relaxation operator is symmetric and the fixed point variational.
 * Stable for D in (0, 1/2] (the symbol of S_xi stays non-negative). */
#define LBKS_HERMITE_4 4

/* Device binding.  `stream` is a hipStream_t (NULL: the library creates one).
 * `alloc`/`free` (both or neither) route every device allocation of the
 * context through the caller's allocator, e.g. the PyTorch caching allocator;
 * NULL means hipMalloc/hipFree.  `device` is the HIP device ordinal. */
typedef struct lbks_device {
    void *stream;
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
    int32_t device;
    int32_t reserved[3];
} lbks_device;

/* Energies of the current state (hartree).  e_total = e_kin + e_ext +
 * e_hartree + e_x + e_c + e_nn.  eps[j] = <psi_hat_j|K_h psi_hat_j> +
 * <psi_hat_j|S_chi (V psi_hat_j)> for j < n_orb (unused entries zero). */
typedef struct lbks_energies {
    double e_total, e_kin, e_ext, e_hartree, e_x, e_c, e_nn;
    double n_electrons;       /* <1|rho> */
    double poisson_residual;  /* ||lap_h V_H + 4 pi rho|| / ||4 pi rho|| */
    double eps[LBKS_MAX_ORB];
    int64_t steps;            /* lattice steps taken since creation */
} lbks_energies;

typedef struct lbks_ctx lbks_ctx;

/* Fill `p` with the defaults: omega 1, D 1/3, GS, Slater + LYP-local, Hartree
 * on, 2 SOR sweeps, FP64, softening 0.05, random-Gaussian start of width 1,
 * seed 0, density floor 1e-14, population scheme.  Grid, h, n_orb and n_elec
 * are zeroed and must be set. */
int lbks_params_default(lbks_params *p);

/* Create a solve context and initialise psi^0 and the populations at
 * equilibrium, f_jp = xi_p psi^0_j (lattice Boltzmann equilibrium).
 * Rejects (LBKS_E_INVAL) parameters outside the stable region: omega in
 * (0, 2), D in (0, 7/18] (the relaxation stencil keeps a non-negative symbol),
 * n_elec outside (2 (n_orb - 1), 2 n_orb] (or != n_orb for the fully
 * spin-polarised functional), hermite not 0, 2 or 4 (D up to 1/2 with 4), a
 * nonzero reserved field, or the collapsed scheme at
 * omega != 1.  LBKS_E_NOMEM if the device memory cannot be allocated.
 * The context owns its device memory until lbks_destroy. */
int lbks_create(const lbks_params *p, const lbks_device *dev, lbks_ctx **out);

/* Set the nuclei (host arrays: Z[n], xyz[3n] in bohr relative to the box
 * centre): rebuilds V_ext(r) = -sum_I Z_I / sqrt(|r - R_I|^2 + a^2) on the
 * device and the ion-ion energy sum_{I<J} Z_I Z_J / |R_I - R_J| (the nuclear
 * term of the KS Hamiltonian).  Orbitals and the Hartree potential are kept,
 * so a geometry scan warm-starts from the previous point.  LBKS_E_INVAL if
 * n is outside [1, LBKS_MAX_NUC], a charge is not positive, or a nucleus lies
 * outside the box. */
int lbks_set_nuclei(lbks_ctx *ctx, int32_t n, const double *Z, const double *xyz);

/* Run lattice steps (lattice Boltzmann equation per orbital with the
 * orthogonalisation source, then the self-consistent potential).  Steps run
 * in chunks of `check_every`; if dE_tol > 0 the energies (with the current
 * Hartree potential) are evaluated after each chunk.  A check passes when the
 * total energy changed by less than dE_tol since the previous check and, if
 * params.deps_tol > 0, the sum of the orbital energies by less than deps_tol
 * (an eigenvalue-based test in the spirit of the paper's rule on the change of
 * the eigenvalues); the call returns LBKS_OK after params.stop_checks
 * consecutive passing checks (at least one).  The previous check and the count
 * persist across calls (so splitting a run into calls whose max_steps are
 * multiples of check_every changes nothing) and are forgotten when
 * set_nuclei, set_potential, set_orbitals or lbks_energy change the state.  With dE_tol <= 0 exactly max_steps steps run.  Returns
 * LBKS_NOT_CONVERGED when max_steps is reached, LBKS_E_NUMERIC if the overlap
 * matrix stops being finite and positive definite, LBKS_E_STATE if no
 * potential was set.  *steps_done (may be NULL) receives the steps run. */
int lbks_relax(lbks_ctx *ctx, int64_t max_steps, double dE_tol, int32_t check_every,
               int64_t *steps_done);

/* Energies of the current state (host struct `out`, owned by the caller), the
 * quantities of the Kohn-Sham functional (section "Kohn-Sham formulation": the
 * kinetic, external, Hartree and exchange-correlation terms of the KS
 * Hamiltonian and the density) and the eigenvalues of the KS equation (eq. KSE)
 * that the results section reports for atoms (Table 1, Fig. 1).  The orbitals
 * are those of the current populations, orthonormalised; eps_j is the Rayleigh
 * quotient <psi_hat_j|K_h psi_hat_j> + <psi_hat_j|S_chi(V psi_hat_j)> of the
 * lattice operator whose steady state the relaxation reaches, with
 * K_h u = -(S_xi u - u)/(D h^2); e_total = sum_j occ_j <psi_hat_j|K_h psi_hat_j>
 * + <V_ext|rho> + 1/2 <V_H|rho> + <rho|eps_x + eps_c> + E_NN.  First relaxes the
 * Hartree potential for the current density to a relative residual <= 1e-12,
 * or to the roundoff floor of a fine grid (the residual <= 1e-9 and no more than
 * 10 % below its value 50 sweeps earlier); this state change is kept.
 * LBKS_E_INVAL if out is NULL, LBKS_E_STATE without nuclei or potential,
 * LBKS_E_NUMERIC if the overlap is not positive definite or the Hartree
 * relaxation does not converge. */
int lbks_energy(lbks_ctx *ctx, lbks_energies *out);

/* The relaxation operator projected on the current orthonormalised orbitals
 * (host, FP64, row-major n_orb x n_orb, n_H >= n_orb^2, owned by the caller):
 *   H_jk = <psi_hat_j | K_h psi_hat_k + S_chi(V psi_hat_k)>,
 * with V built from their density as in lbks_energy (same Hartree relaxation,
 * kept).  Its diagonal holds the eps_j of lbks_energy; its eigenvalues are the
 * Ritz values of the operator on the span of the orbitals.  The KS equation
 * (eq. KSE) determines the occupied levels, not the orbitals inside a set of
 * nearly equal levels, which the relaxation (eq. KSLB-2) separates only
 * slowly; the Ritz values do not depend on such rotations.  LBKS_E_INVAL if H
 * is NULL or too small, LBKS_E_STATE without nuclei or potential,
 * LBKS_E_NUMERIC if the overlap or an entry is not finite. */
int lbks_hamiltonian(lbks_ctx *ctx, double *H, size_t n_H);

/* Forces on the nuclei (host, FP64, F[3 I + c] for nucleus I and axis c, in
 * hartree per bohr, n_F >= 3 * nuclei) for the current state, as used by
 * Born-Oppenheimer dynamics (section "Concurrent Dynamics": the ions move on the
 * surface of the electronic ground state).  Hellmann-Feynman form: with the
 * density rho of the orthonormalised current orbitals held fixed,
 *   F_I = Z_I h^3 sum_r rho(r) (r - R_I) / (|r - R_I|^2 + a^2)^(3/2)
 *         + sum_{J != I} Z_I Z_J (R_I - R_J) / |R_I - R_J|^3,
 * i.e. minus the gradient of <V_ext|rho> + E_NN.  At a converged state this is
 * minus the gradient of the total energy up to the lattice's smoothing of the
 * potential source.  The state is not changed.  LBKS_E_STATE if the potential
 * came from lbks_set_potential (no nuclei), LBKS_E_INVAL if F is NULL or too
 * small, LBKS_E_NUMERIC if the overlap or a force is not finite. */
int lbks_forces(lbks_ctx *ctx, double *F, size_t n_F);

/* Copy the current orthonormal orbitals (host, FP64, [n_orb][z][y][x],
 * n_psi >= n_orb * sites) and optionally the density (host, n_rho >= sites;
 * rho may be NULL), the solution of the KS equations with their orthogonality
 * constraints (section "Kohn-Sham formulation": the orbitals phi_j, eq. ORTOG,
 * and the density rho = sum_j occ_j |phi_j|^2).  The orbitals are the moments
 * psi_j = sum_p f_jp of the current populations (kinetic representation,
 * section "The kinetic approach to Kohn-Sham theory") after Gram-Schmidt:
 * <psi_hat_j|psi_hat_k> = delta_jk; each orbital's sign is arbitrary and
 * degenerate orbitals may mix.  The caller owns both buffers.  LBKS_E_INVAL if
 * psi is NULL or a buffer is too small; the state is not changed. */
int lbks_orbitals(lbks_ctx *ctx, double *psi, size_t n_psi, double *rho, size_t n_rho);

/* Release the context and all its device memory. */
void lbks_destroy(lbks_ctx *ctx);

/* Message of the last error on `ctx` (or, when ctx is NULL, of the last failed
 * lbks_create or batch relaxation on this thread).  Valid until the next call on
 * the same context. */
const char *lbks_last_error(const lbks_ctx *ctx);

/* ---- extensions ---- */

/* The sequential order of the time-dependent Gram-Schmidt procedure (the
 * closing remark on eq. KSLB-2, section "The kinetic approach to Kohn-Sham
 * theory": evolve psi_0 to its ground state, then psi_1, and so on), on the
 * omega = 1 field update (params.scheme = LBKS_SCHEME_COLLAPSED, Gram-Schmidt):
 * in stage k only orbital k takes lattice steps, the others keep their fields;
 * every orbital is orthonormalised in order each step (so orbital k is projected
 * against the converged lower ones) and the density is that of all orbitals in
 * their current state.  Stage k ends when eps_k changed by less than deps_tol
 * over check_every steps; a sweep runs the stages k = 0 .. n_orb - 1, and sweeps
 * repeat until the total energy changed by less than dE_tol from the previous
 * sweep (the later orbitals' density drives V in the earlier stages, so one
 * sweep is not self-consistent).  Returns LBKS_OK, LBKS_NOT_CONVERGED (max_steps
 * or max_sweeps reached), or an error; *steps_done and *sweeps_done (may be
 * NULL) receive the counts.  LBKS_E_INVAL for another scheme or orthogonalisation
 * or non-positive tolerances; LBKS_E_STATE without a potential, for a batch
 * member or during concurrent dynamics. */
int lbks_relax_sequential(lbks_ctx *ctx, int64_t max_steps, double dE_tol, double deps_tol, int32_t check_every,
                          int32_t max_sweeps, int64_t *steps_done, int32_t *sweeps_done);

/* ---- concurrent dynamics: electrons and nuclei moved together in real time
 * (section "Concurrent Dynamics", eq. KSLBCD) ----
 *
 * The orbitals become complex fields advanced by the two-step time-centred
 * lattice scheme, in this reading of eq. KSLBCD: the populations are at
 * equilibrium with their moment (f_jp = xi_p psi_j, the omega = 1 relaxation),
 * so the scheme advances the orbitals themselves,
 *   psi_j^{n+1} = psi_j^{n-1} - 2 i h (H - E_j) psi_j^n,  H u = K_h u + S_chi(V u),
 * with K_h u = -(S_xi u - u) / (D dx^2) and V = V_ext + V_H + v_xc of the
 * density sum_j occ_j |psi_j^n|^2, rebuilt before every step (multipole
 * boundary and params.poisson_sweeps warm-started red/black sweeps).  H is the
 * operator whose steady state lbks_relax reaches, so a relaxed ground state is
 * stationary.  The paper's U_jp = kappa w_p q_p E_j phi_j, which keeps the
 * energy at E_j, is read as each orbital's energy reference E_j (its eps_j at
 * the start): a global phase per orbital, which leaves densities, energies and
 * forces unchanged and stops the two-step scheme's parasitic mode from growing
 * through the density-dependent V.  Once the nuclei move, the orbitals' energies
 * drift away from E_j and that mode grows again; restarts remove it: every
 * restart_every-th step re-centres E_j on h^3 Re<psi_j^n|H psi_j^n> (that step's
 * V) and is the one-step start from psi^n instead of the two-step update.
 * W_jp is 0 (the evolution keeps the orbitals orthonormal up to the scheme's own
 * error).  The nuclei are moved by the caller (lbks_set_nuclei between steps;
 * lbks_forces gives the Hellmann-Feynman forces of the current density).
 * Times in atomic units (1 fs = 41.341 a.u.).  FP64 contexts with a local
 * functional, omega = 1 and Gram-Schmidt only; not for batch members.  While
 * the dynamics runs, lbks_relax, lbks_energy, lbks_hamiltonian, lbks_orbitals
 * and lbks_set_orbitals return LBKS_E_STATE. */

/* Start from the current orbitals (orthonormalised; normally a relaxed ground
 * state): psi^0 = psi_hat, V_H converged for its density, E_j = eps_j of that
 * state, and psi^1 = psi^0 - i h H' psi^0 - (h^2 / 2) H' H' psi^0, H' = H - E_j.  Allocates the complex
 * orbitals (4 n_orb sites double2: two time levels and two work levels) through
 * the context's allocator on the first start.  LBKS_E_INVAL for a context that
 * is not FP64, local-functional, omega = 1, Gram-Schmidt, or for h outside
 * (0, 0.95 / bound) with bound = max((1 - min symbol of S_xi) / (D dx^2), depth
 * of V_ext at the nodes nearest the nuclei), or restart_every < 0;
 * LBKS_E_STATE without a potential or for a batch member; LBKS_E_NOMEM.
 * restart_every: steps restart_every, 2 restart_every, ... (counted from this
 * start) are restarts; 0 = never (a few hundred steps suit moving nuclei). */
int lbks_cd_start(lbks_ctx *ctx, double h, int64_t restart_every);

/* Advance `steps` time steps with the current nuclei.  A restart step reads the
 * orbital energies back to the host (one synchronisation). */
int lbks_cd_step(lbks_ctx *ctx, int64_t steps);

/* Energies of psi^n (host struct): the terms of lbks_energy with
 * Re <psi_j|K_h psi_j> and Re <psi_j|S_chi(V psi_j)> (eps_j is the latter's sum),
 * after converging V_H for the current density (kept); steps = time steps since
 * the start.  LBKS_E_NUMERIC if a value is not finite (an unstable step). */
int lbks_cd_energy(lbks_ctx *ctx, lbks_energies *out);

/* Copy psi^n: real and imaginary parts (host, FP64, [n_orb][z][y][x] each,
 * n >= n_orb * sites). */
int lbks_cd_orbitals(lbks_ctx *ctx, double *re, double *im, size_t n);

/* Leave the dynamics and free the complex orbitals; the relaxation state
 * (populations) is the one from before lbks_cd_start. */
int lbks_cd_stop(lbks_ctx *ctx);

/* Replace V_ext by an arbitrary potential (host, FP64, one value per node);
 * the ion-ion energy becomes zero.  Used for model wells (harmonic
 * oscillator, empty box). */
int lbks_set_potential(lbks_ctx *ctx, const double *v_ext);

/* Replace the orbitals (host, FP64, [n_orb][z][y][x]) and reset the
 * populations to equilibrium f_jp = xi_p psi_j; the Hartree potential is
 * kept, except after an LBKS_E_NUMERIC failure, when it restarts from zero.
 * Used for warm starts, checkpoint/resume and recovery. */
int lbks_set_orbitals(lbks_ctx *ctx, const double *psi);

/* Grid nodes and orbital count of a context. */
int lbks_shape(const lbks_ctx *ctx, int32_t N[3], int32_t *n_orb);

/* Device bytes the context holds. */
size_t lbks_device_bytes(const lbks_ctx *ctx);

/* Device bytes lbks_create would allocate for these parameters (0 if they are
 * invalid). */
size_t lbks_estimate_bytes(const lbks_params *p);

/* Kernel timing: when enabled, every launch of the update kernel (the population
 * stream-collide or the omega = 1 field update) and of the concurrent-dynamics
 * step is bracketed by HIP events on the context's stream.  lbks_kernel_time
 * returns the summed duration (ms) and the launch count since the last reset,
 * and synchronises the stream.  kernel: 0 = update kernel, 1 = concurrent-
 * dynamics step (lbks_cd_step; a restart step counts as one launch). */
int lbks_set_timing(lbks_ctx *ctx, int32_t enable);
int lbks_kernel_time(lbks_ctx *ctx, int32_t kernel, double *total_ms, int64_t *launches);

/* Update-kernel variants 0..15: bit 0 computes the per-workgroup overlap partial
 * S = Phi^T Phi on the matrix cores (V_MFMA_F64_16X16X4F64) instead of a wave
 * butterfly, bit 1 compiles the kernel for 8 waves per SIMD, bit 2 runs the
 * workgroups in dispatch order instead of giving each XCD one contiguous range
 * of tiles, bit 3 gives each lane of the population update 16 bytes of
 * x-consecutive nodes (2 in FP64, 4 in FP32) read and written with one access
 * per plane (orbital buckets of at most five; bit 0 then rolls its loop over the
 * 19 directions, which trades overlap between directions for four times the
 * waves, bit 1 is unused, and larger buckets ignore bit 3).  Every variant
 * computes the same per-node arithmetic; the overlap's summation order differs
 * with bits 0 and 3, and the compiler may contract a product into a fused
 * multiply-add differently in the wide form (last-bit differences); bit 2
 * changes nothing in the results.  The LDS-staged omega = 1 update
 * (Gram-Schmidt, at most five orbitals) reads bits 0 and 1 as its brick depth in
 * z (8, 12, 16, 24 nodes) and bit 2 as its workgroup order; the collapsed
 * node-per-lane update ignores bit 3.
 * Defaults before autotuning: 13 for the population update of at most five
 * orbitals on grids of more than 65536 nodes (0 (FP64) or 1 (FP32) on smaller
 * ones), 0 (FP64) or 1 (FP32) for the brick update, otherwise 4 (FP64) or 3
 * (FP32).  lbks_set_variant: LBKS_E_INVAL outside 0..15. */
int lbks_set_variant(lbks_ctx *ctx, int32_t variant);
int lbks_get_variant(const lbks_ctx *ctx);

/* Which totals this context's kernels sum themselves (params.fold): bit 0 the
 * overlap, bit 1 the multipoles; 0 when neither is folded or params.fold = -1;
 * LBKS_E_INVAL for a NULL context. */
int lbks_get_fold(const lbks_ctx *ctx);

/* Time every distinct update-kernel variant `reps` times on the context's
 * current state and keep the fastest (state unchanged).  Choices are cached per
 * (precision, orbital bucket, orthogonalisation, scheme, node count) for the
 * process; with force = 0 a cached choice is reused without timing.  chosen
 * (may be NULL) receives the variant, avg_ms (NULL, or 16 doubles) the
 * per-launch times, -1 for a variant not timed (the same kernel as a lower one)
 * and for all when the cache answered.  LBKS_E_STATE if no potential is set. */
int lbks_autotune(lbks_ctx *ctx, int32_t reps, int32_t force, int32_t *chosen, double *avg_ms);

/* Plain device-to-device copy of `bytes` (a multiple of 16) on `stream` with
 * the library's own copy kernel (device pointers, 16-byte aligned; one 16-byte
 * element per lane, non-temporal loads and stores): the bandwidth reference and
 * the calibration of memory counters against a kernel of known traffic.
 * LBKS_E_INVAL on a bad size or alignment. */
int lbks_copy_kernel(void *dst, const void *src, size_t bytes, void *stream);

/* ---- batches: many solves advanced together, one launch per kernel ---- */

typedef struct lbks_batch lbks_batch;

/* A batch shares one stream and launches each step kernel once for all of its
 * active contexts (uneven grids and orbital counts), captured into HIP graphs
 * that are rebuilt when the membership changes.  The contexts stay ordinary
 * lbks_ctx handles for set_nuclei, energy and orbitals; they must have been
 * created on the batch's stream and device. */
int lbks_batch_create(const lbks_device *dev, lbks_batch **out);
int lbks_batch_attach(lbks_batch *b, lbks_ctx *ctx);
int lbks_batch_detach(lbks_batch *b, lbks_ctx *ctx);

/* Advance every attached context in lockstep chunks of `check_every` steps.
 * After each chunk the energy of each context still running is checked as
 * in lbks_relax; a converged context stops taking steps (status[i] = LBKS_OK),
 * one that reaches max_steps gets LBKS_NOT_CONVERGED, one whose overlap fails
 * LBKS_E_NUMERIC.  status and steps (may be NULL) are host arrays indexed in
 * attach order.  Returns the number of contexts attached. */
int lbks_batch_relax(lbks_batch *b, int64_t max_steps, double dE_tol, int32_t check_every,
                     int32_t *status, int64_t *steps);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): lbks_batch_relax with
 * the same arguments, results and statuses, whose descriptor, tile and gather
 * tables go to a fixed device workspace of LBKS_STATIC_WORKSPACE_BYTES inside
 * the library (one per GPU, held until the process ends) instead of memory the
 * batch allocates, and whose steps are launched one by one instead of from HIP
 * graphs.  It calls no device allocation routine; the members' own buffers were
 * allocated at lbks_create.  The tables are rebuilt in the workspace on every
 * call.  Every call on one GPU shares that GPU's workspace: calls that overlap
 * in time on one GPU (other threads, other streams) race and must not be made.
 * LBKS_E_INVAL (message from lbks_last_error(NULL)) when the tables of the
 * current members need more than LBKS_STATIC_WORKSPACE_BYTES; LBKS_E_HIP if
 * the workspace's address cannot be obtained. */
#define LBKS_STATIC_WORKSPACE_BYTES (2u << 20)
int lbks_batch_relax_static(lbks_batch *b, int64_t max_steps, double dE_tol, int32_t check_every,
                            int32_t *status, int64_t *steps);
int lbks_batch_size(const lbks_batch *b);

/* The hipStream_t the batch launches on (members must be created on it). */
void *lbks_batch_stream(const lbks_batch *b);
void lbks_batch_destroy(lbks_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* LBKS_H */
