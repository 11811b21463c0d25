// lbks_kernels.h -- per-solve device descriptor and the launchers of the
// relaxation kernels (internal to liblbks.so).
//
// One solve ("instance") is a descriptor of its grid, parameters and device
// buffers.  Every kernel takes an array of descriptors plus an optional tile
// table mapping each workgroup to (instance, tile), so one launch serves a
// single solve or a whole batch of uneven solves.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbks {

constexpr int Q = 19;          // D3Q19 velocities
constexpr int BS = 256;        // threads per workgroup in every site kernel
constexpr int MAXO = 16;       // orbital capacity of the descriptor
constexpr int NMOM = 10;       // q, p_xyz, Q_xx Q_yy Q_zz Q_xy Q_xz Q_yz
constexpr int NEBASE = 5;      // rho V_ext, rho V_H, rho eps_x, rho eps_c, rho
constexpr int RCH = 8;         // partial arrays hold whole chunks of RCH columns
constexpr int BX = 32, BY = 8, BZ = 8;   // brick of the LDS-staged omega = 1 update (BX * BY = BS);
                                         // BZ is the shallowest of its depths

__host__ __device__ constexpr int bricks_of(int nx, int ny, int nz, int bz = BZ)
{
    return ((nx + BX - 1) / BX) * ((ny + BY - 1) / BY) * ((nz + bz - 1) / bz);
}
// Depth in z of the bricks for an update-kernel variant (bits 0 and 1): 8, 12, 16, 24.
__host__ __device__ constexpr int brick_depth(int variant) { return BZ + 4 * (variant & 3) + 4 * ((variant & 3) == 3); }
// The brick update writes the overlap partials itself (brick b into tile slot b,
// the slots past the last brick zero) when an instance has no more bricks of the
// shallowest depth than node tiles, so for every depth; otherwise a separate pass
// over the node tiles writes them.
__host__ __device__ constexpr bool brick_partials(int ntile, int nbrick) { return nbrick <= ntile; }
constexpr int NUCG = 16;       // nuclei per force-kernel pass
constexpr int MAXNUC = 64;     // nuclei per solve (LBKS_MAX_NUC)
constexpr int XC_GGA = 4;      // LBKS_XC_B88_LYP (kinds from here on are gradient-corrected)
constexpr int XC_GGA_POLARISED = 5;   // LBKS_XC_B88_LYP_POLARISED

constexpr int RG = 16;         // first-level workgroups per instance of the finalize kernels (8: 9.9, 16: 9.4,
                               // 32: 10.2, 64: 12.4 us for the overlap finalize at 96^3)

// Columns of a partial array padded to a whole number of chunks.
__host__ __device__ constexpr int padded_cols(int nq) { return (nq + RCH - 1) / RCH * RCH; }

// Small instances skip the two finalize kernels whose totals one kernel needs
// next: every workgroup of that kernel sums the tile partials itself, in the
// finalize kernel's order of additions, so the results are the same bit for bit.
// The overlap S goes to the orthonormalisation (up to five orbitals), the
// multipoles to the ghost-face kernel or the step's first red sweep, for
// instances of at most RG * FOLD_GROUP tiles (measured on MI355X: 48.5 -> 39.2 us
// per step at 32^3; with 432 or 1024 tiles the multipole fold alone no longer
// pays).  InstDesc::fold holds the bits an instance allows; a launch folds when
// every instance in it allows (Plan::fold_s, fold_m), so a mixed batch takes the
// finalize kernels for all its members, which gives the same bits.
constexpr int FOLD_S = 1, FOLD_M = 2;
constexpr int FOLD_GROUP = 16;   // tiles per first-level group, at most
inline int fold_bits(int ntile, int n_orb, bool enabled)
{
    if (!enabled || ntile > RG * FOLD_GROUP) return 0;
    return (n_orb <= 5 ? FOLD_S : 0) | FOLD_M;
}

// Offsets into the per-instance FP64 scalar block.
constexpr int SC_MOM = 0;                  // 10 multipoles
constexpr int SC_S = 16;                   // packed lower overlap, 136 values
constexpr int SC_ENER = 160;               // lbks_energies prefix: 9 + 16 doubles
constexpr int SC_RES = 192;                // Poisson relative residual
constexpr int SC_ERR = 193;                // nonzero: overlap not finite / not SPD
constexpr int SC_CNT = 194;                // finalize-kernel counter (an unsigned in this slot)
constexpr int SC_FORCE = 200;              // forces on the nuclei, [MAXNUC][3]
constexpr int SC_SIZE = 400;

struct InstDesc {
    int nx, ny, nz, n_orb;
    int nsite;                 // nx*ny*nz (< 2^31)
    int ntile;                 // site tiles of BS nodes
    int ntile_ghost;           // tiles over the six ghost faces
    int ntile_sor;             // tiles over one colour of the SOR sweep
    int ntile_brick;           // BX x BY x BZ bricks (the shallowest depth) of the omega = 1 field update
    int ortho, xc, hartree, precision;
    int scheme;
    int nnuc;                  // nuclei set by lbks_set_nuclei (0 after lbks_set_potential)
    unsigned active;           // orbitals that take the omega = 1 field update (bit j); the others keep
                               // their fields (the sequential Gram-Schmidt order); all ones otherwise
    int fold;                  // FOLD_S / FOLD_M: the overlap / multipole totals may be summed by their consumer
    double h, h3, omega, dt, D, omega_sor, rho_floor, e_nn;
    double occ[MAXO];
    double xi[Q], chi[Q];
    // buffers (bulk precision unless noted)
    void *f0, *f1;             // populations [n_orb][Q][site]
    void *psi;                 // sum_p f, or the orbital state of the collapsed scheme
    void *psihat;              // orthonormalised orbitals
    void *psistar;             // equilibrium orbitals of the W mode
    void *rho;                 // density
    void *V;                   // KS potential used by the collide
    double *Vd;                // FP64 potential for energies (== V in FP64 mode)
    double *vext;              // FP64 external potential
    double *vh;                // FP64 Hartree potential with one ghost layer
    double *s_part;            // [padded_cols(npair)][ntile]
    double *m_part;            // [padded_cols(NMOM)][ntile]
    double *e_part;            // [padded_cols(2*bucket(n_orb) + NEBASE)][ntile]
    double *r_part;            // [padded_cols(2)][ntile]
    double *f_part;            // [padded_cols(3 NUCG)][ntile]
    double *g_part;            // [padded_cols(widest partial)][RG] first-level column sums
    double *gga;               // gradient-corrected xc: df/drho, then 2 df/dsigma D_a rho (a = x, y, z); [4][site] FP64
    const double *zr;          // nuclei: Z, x, y, z per nucleus, then the softening squared
    double *C;                 // [MAXO*MAXO] C, then [MAXO*MAXO] C* (W mode)
    double *scal;              // [SC_SIZE]
    double *stage;             // FP64 staging, (n_orb + 1) * nsite
};

// Tile tables for batched launches: entry b of a table is (instance, tile).
struct TileTables {
    const int2 *site = nullptr;   int n_site = 0;
    const int2 *ghost = nullptr;  int n_ghost = 0;
    const int2 *sor = nullptr;    int n_sor = 0;
    const int *inst = nullptr;    int n_inst = 0;   // instance list for per-instance kernels
    const int2 *brick = nullptr;  int n_brick = 0;
    const int2 *site_w = nullptr; int n_site_w = 0;   // tiles of the wide update: BS * (16 / element size) nodes
};

// Launch plan of one kernel family: descriptor array on the device, tile
// tables (null tables: a single instance, descriptor 0), and the template
// buckets that apply to every instance in the plan.
struct Plan {
    const InstDesc *d_desc = nullptr;
    TileTables tt;
    int precision = 0;    // 0 FP64, 1 FP32 bulk
    int no = 1;           // orbital bucket: 1,2,3,4,5,8,16
    bool wmode = false;
    bool gga = false;     // gradient-corrected exchange-correlation (needs the k_gga pass)
    int ntile = 0, ntile_ghost = 0, ntile_sor = 0, ntile_brick = 0;   // single-instance counts
    int nbrick[4] = {0, 0, 0, 0};   // single-instance bricks of each depth (brick_depth of variant bits 0, 1)
    int n_inst = 1;
    int variant = 0;      // update-kernel variant (autotuned): bit 0 matrix-core overlap, bit 1 8-wave
                          // occupancy, bit 2 workgroups in dispatch order, bit 3 16 bytes of nodes per lane
                          // in the population update (buckets up to five orbitals; bit 0 then rolls its loop
                          // over the directions, bit 1 is unused);
                          // the brick update reads bits 0 and 1 as its depth and bit 2 as its order
    bool brick_partials = true;   // every instance gets its overlap partials from the brick update
    bool fold_s = false, fold_m = false;   // every instance folds the overlap / multipole finalize
};

// Default update-kernel variant per precision (measured on MI355X): FP64 keeps the
// wave-butterfly overlap at the compiler's occupancy with workgroups in dispatch
// order, FP32 takes the matrix-core overlap at 8 waves per SIMD with the XCD remap.
inline int default_variant(int precision) { return precision ? 3 : 4; }
constexpr int N_VARIANTS = 16;
// nodes per lane of the wide population update for an element size
constexpr int wide_nodes(int elem_bytes) { return 16 / elem_bytes; }
// variants the autotuner times: the eight node-per-lane forms, and the wide form in
// both workgroup orders when it applies (its bits 0 and 1 change nothing)
inline bool variant_distinct(int v, int no, bool populations)
{
    return v < 8 || (populations && no <= 5 && (v & 2) == 0);
}

int orbital_bucket(int n_orb);

// Launchers (enqueue on `st`; return hipError_t as int).
int launch_init_psi(const Plan &pl, int mode, double sigma, double noise, uint64_t seed, hipStream_t st);
int launch_psi_from_stage(const Plan &pl, hipStream_t st);
int launch_equilibrium(const Plan &pl, int parity, hipStream_t st);
int launch_moment(const Plan &pl, int parity, hipStream_t st);
int launch_overlap_psi(const Plan &pl, hipStream_t st, bool skip_brick = false);
int launch_overlap_finalize(const Plan &pl, hipStream_t st);
int launch_orthonormalise(const Plan &pl, hipStream_t st);
int launch_multipole_finalize(const Plan &pl, hipStream_t st);
int launch_ghost(const Plan &pl, hipStream_t st);
int launch_sor(const Plan &pl, int color, hipStream_t st);
int launch_sor_first(const Plan &pl, hipStream_t st);   // red, with the ghost faces (every instance FOLD_M)
int launch_sor_black_potential(const Plan &pl, hipStream_t st);   // last black half-sweep + V
int launch_potential(const Plan &pl, int to_fp64, hipStream_t st);
int launch_stream_collide(const Plan &pl, int parity, hipStream_t st);
int launch_collapsed_update(const Plan &pl, hipStream_t st);
int launch_energy_terms(const Plan &pl, hipStream_t st);
int launch_energy_finalize(const Plan &pl, hipStream_t st);
// rows j0 .. j0 + *rows_done - 1 of the projected operator into the staging area
int launch_ham_rows(const Plan &pl, int j0, int *rows_done, hipStream_t st);
int launch_residual(const Plan &pl, hipStream_t st);
int launch_residual_finalize(const Plan &pl, hipStream_t st);
int launch_vext(const Plan &pl, int nnuc, const double *dZR, hipStream_t st);
int launch_stage_orbitals(const Plan &pl, hipStream_t st);
int launch_gga(const Plan &pl, hipStream_t st);
int launch_force_terms(const Plan &pl, int i0, hipStream_t st);     // nuclei i0 .. i0 + NUCG - 1
int launch_force_finalize(const Plan &pl, int i0, hipStream_t st);
int launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st);
// concurrent dynamics (complex FP64 orbitals [orbital][site] of double2, single instance);
// orbital j is advanced with H - eref[j]
struct CdRef {
    double e[MAXO];
};
int launch_cd_init(const Plan &pl, double2 *prev, hipStream_t st);
int launch_cd_apply(const Plan &pl, const double2 *in, double2 *out, const CdRef &ref, hipStream_t st);
int launch_cd_taylor(const Plan &pl, const double2 *prev, const double2 *t1, const double2 *t2, double2 *cur,
                     double h, hipStream_t st);
int launch_cd_step(const Plan &pl, const double2 *cur, double2 *prev, double h, const CdRef &ref, hipStream_t st);
int launch_cd_energy_terms(const Plan &pl, const double2 *cur, hipStream_t st);
// dst[i * width + k] = scal_i[SC_ENER + k] (k < 25), dst[i * width + 25] = scal_i[SC_ERR]
int launch_gather(const double *const *scal, int count, int width, double *dst, hipStream_t st);

}  // namespace lbks
