// lbks_capi.hip -- host runtime and C ABI of liblbks.so.
//
// A context owns one solve: its descriptor (grid, parameters, buffer
// pointers), a device copy of it, and one device allocation carved into the
// buffers.  Each lattice step is a fixed sequence of kernel launches on the
// context's stream; the host only enqueues and, at chunk boundaries, reads
// back a few hundred bytes (energies and the error flag).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/lbks.h"
#include "lbks_kernels.h"

using namespace lbks;

namespace {

thread_local std::string g_create_error;

struct Buf {
    size_t off = 0, bytes = 0;
};

}  // namespace

struct lbks_ctx {
    lbks_params p{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void *(*ualloc)(size_t, void *) = nullptr;
    void (*ufree)(void *, void *) = nullptr;
    void *user = nullptr;
    void *base = nullptr;       // the single device allocation
    size_t bytes = 0;
    InstDesc h{};               // host copy of the descriptor
    InstDesc *d_desc = nullptr; // device copy (inside base)
    Plan plan{};
    int parity = 0;             // populations live in f0 (0) or f1 (1)
    int64_t steps = 0;
    bool has_potential = false;
    bool have_prev = false;     // stopping rule: energies of the previous chunk check
    double e_prev = 0.0;
    double tr_prev = 0.0;       // sum of the orbital energies at that check
    int passes = 0;             // consecutive passing checks
    double *d_zr = nullptr;     // nuclei table [4 * LBKS_MAX_NUC + 1]
    std::string err;
    // timing of the update kernel (kind 0) and of the concurrent-dynamics step (kind 1)
    bool timing = false;
    std::vector<hipEvent_t> ev;  // pairs (start, stop)
    std::vector<int> ev_kind;    // the kind of each pair
    size_t ev_used = 0;
    double timed_ms[2] = {0.0, 0.0};
    int64_t timed_launches[2] = {0, 0};
    lbks_batch *batch = nullptr;
    // concurrent dynamics (lbks_cd_*): complex orbitals at two time levels plus two
    // work levels, [4][n_orb][site] of double2
    bool cd = false;
    double cd_h = 0.0;
    double2 *cd_buf = nullptr;
    int cd_cur = 1;             // level holding psi^n (the other of levels 0, 1 holds psi^{n-1})
    int64_t cd_steps = 0;
    CdRef cd_ref{};             // energy reference E_j of each orbital (its energy at the last (re)start)
    int64_t cd_restart = 0;     // period of the restarts (0: none)
    std::vector<double> nuc;    // nuclei of the last lbks_set_nuclei: Z, x, y, z per nucleus
    double vext_depth = 0.0;    // max |v| of a potential from lbks_set_potential
};

// One launch group of a batch: members sharing every template and sequence choice.
struct BatchGroup {
    int precision = 0, no = 1, scheme = 0, hartree = 1, sweeps = 2, variant = 0;
    bool wmode = false, gga = false;
    std::vector<int> members;   // indices into lbks_batch::members
    Plan plan{};
};

struct lbks_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void *(*ualloc)(size_t, void *) = nullptr;
    void (*ufree)(void *, void *) = nullptr;
    void *user = nullptr;
    std::vector<lbks_ctx *> members;
    std::vector<char> running;          // members that take steps in this relax
    std::vector<BatchGroup> groups;
    void *mem = nullptr;                // descriptors, tile tables, gather buffer
    size_t mem_bytes = 0;
    double *d_gather = nullptr;         // [members][GATHER_W]
    const double **d_scal = nullptr;    // members' scalar blocks
    uint64_t member_epoch = 0;          // bumped by every attach and detach
    uint64_t table_epoch = ~0ull;       // member_epoch the device tables were built for
    bool tables_static = false;         // the tables sit in the static workspace (lbks_batch_relax_static)
    bool dirty = true;
    int bparity = 0;                    // population buffer parity within the current plan
    int64_t epoch_steps = 0;            // steps since the plan was built
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    bool use_graph = true;
    std::string err;
};

namespace {

int fail(lbks_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    else g_create_error = msg;
    return code;
}

int hip_fail(lbks_ctx *c, hipError_t e, const char *where)
{
    return fail(c, LBKS_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(c, expr)                                        \
    do {                                                       \
        hipError_t _e = (expr);                                \
        if (_e != hipSuccess) return hip_fail((c), _e, #expr); \
    } while (0)

#define KCHK(c, expr)                                                        \
    do {                                                                     \
        int _e = (expr);                                                     \
        if (_e != 0) return hip_fail((c), (hipError_t)_e, #expr);            \
    } while (0)

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// D3Q19 weights in the velocity order of the kernels (rest, 6 faces, 12 edges).
// Second order: equilibrium xi_p = w_p (1 + (D - c_s^2) q_p) and potential source
// chi_p = w_p (1 - c_s^2 q_p), q_p = (|v_p|^2 - 3 c_s^2) / (2 c_s^4), c_s^2 = 1/3.
// Fourth order: xi also matches the mixed fourth moment D^2 of a Gaussian of
// variance D (rest 1 - 3D + 3D^2, faces D/2 - D^2, edges D^2/4), and chi has no
// second or mixed fourth moment (all of it on the rest velocity).
void lattice_constants(double D, int hermite, double *xi, double *chi)
{
    const double cs2 = 1.0 / 3.0;
    for (int p = 0; p < Q; ++p) {
        const int v2 = p == 0 ? 0 : (p <= 6 ? 1 : 2);
        if (hermite == 4) {
            xi[p] = v2 == 0 ? 1.0 - 3.0 * D + 3.0 * D * D : (v2 == 1 ? 0.5 * D - D * D : 0.25 * D * D);
            chi[p] = v2 == 0 ? 1.0 : 0.0;
            continue;
        }
        const double w = v2 == 0 ? 1.0 / 3.0 : (v2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        const double q = ((double)v2 - 3.0 * cs2) / (2.0 * cs2 * cs2);
        xi[p] = w * (1.0 + (D - cs2) * q);
        chi[p] = w * (1.0 - cs2 * q);
    }
}

struct Layout {
    Buf desc, f0, f1, psi, psihat, psistar, rho, V, Vd, vext, vh, s_part, m_part, e_part, r_part, f_part, gga, g_part, C,
        scal, stage, zr;
    size_t total = 0;
};

int validate(const lbks_params *p, std::string &why)
{
    if (!p) { why = "params is NULL"; return LBKS_E_INVAL; }
    for (int a = 0; a < 3; ++a)
        if (p->N[a] < 4 || p->N[a] > 1024) { why = "grid size out of [4, 1024]"; return LBKS_E_INVAL; }
    if ((double)p->N[0] * p->N[1] * p->N[2] * 8.0 >= 4294967296.0) {
        why = "grid too large: nodes x 8 bytes must stay below 2^32";
        return LBKS_E_INVAL;
    }
    if (!(p->h > 0.0) || !isfinite(p->h)) { why = "h must be positive"; return LBKS_E_INVAL; }
    if (p->n_orb < 1 || p->n_orb > LBKS_MAX_ORB) { why = "n_orb out of [1, 16]"; return LBKS_E_INVAL; }
    if (p->xc == LBKS_XC_B88_LYP_POLARISED) {
        if (p->n_elec != p->n_orb) {
            why = "a fully spin-polarised density holds one electron per orbital: n_elec must equal n_orb";
            return LBKS_E_INVAL;
        }
    } else if (p->n_elec < 1 || p->n_elec > 2 * p->n_orb || p->n_elec <= 2 * (p->n_orb - 1)) {
        why = "n_elec must satisfy 2(n_orb-1) < n_elec <= 2 n_orb";
        return LBKS_E_INVAL;
    }
    if (!(p->omega > 0.0 && p->omega < 2.0)) { why = "omega must lie in (0, 2)"; return LBKS_E_INVAL; }
    if (p->hermite != 0 && p->hermite != 2 && p->hermite != 4) { why = "hermite must be 0, 2 or 4"; return LBKS_E_INVAL; }
    if (p->hermite == 4) {
        if (!(p->D > 0.0 && p->D <= 0.5 + 1e-15)) {
            why = "D must lie in (0, 1/2] with fourth-order weights: larger D makes the relaxation stencil's symbol negative";
            return LBKS_E_INVAL;
        }
    } else if (!(p->D > 0.0 && p->D <= 7.0 / 18.0 + 1e-15)) {
        why = "D must lie in (0, 7/18]: larger D makes the relaxation stencil's symbol negative";
        return LBKS_E_INVAL;
    }
    if (p->ortho != LBKS_ORTHO_GS && p->ortho != LBKS_ORTHO_W) { why = "bad ortho"; return LBKS_E_INVAL; }
    if (p->xc < LBKS_XC_NONE || p->xc > LBKS_XC_B88_LYP_POLARISED) { why = "bad xc"; return LBKS_E_INVAL; }
    if (p->poisson_sweeps < 0 || p->poisson_sweeps > 64) { why = "poisson_sweeps out of [0, 64]"; return LBKS_E_INVAL; }
    if (p->precision != LBKS_FP64 && p->precision != LBKS_FP32_BULK) { why = "bad precision"; return LBKS_E_INVAL; }
    if (!(p->softening >= 0.0)) { why = "softening must be >= 0"; return LBKS_E_INVAL; }
    if (p->init < LBKS_INIT_GAUSS_NOISE || p->init > LBKS_INIT_USER) { why = "bad init"; return LBKS_E_INVAL; }
    if (p->init != LBKS_INIT_USER && !(p->init_sigma > 0.0)) { why = "init_sigma must be positive"; return LBKS_E_INVAL; }
    if (p->scheme != LBKS_SCHEME_POPULATIONS && p->scheme != LBKS_SCHEME_COLLAPSED) { why = "bad scheme"; return LBKS_E_INVAL; }
    if (p->scheme == LBKS_SCHEME_COLLAPSED && p->omega != 1.0) {
        why = "the collapsed scheme exists only at omega = 1";
        return LBKS_E_INVAL;
    }
    if (p->stop_checks < 0 || p->stop_checks > 1000) { why = "stop_checks must be in [0, 1000]"; return LBKS_E_INVAL; }
    if (!(p->deps_tol >= 0.0) || !isfinite(p->deps_tol)) { why = "deps_tol must be finite and >= 0"; return LBKS_E_INVAL; }
    if (p->fold != 0 && p->fold != -1) { why = "fold must be 0 or -1"; return LBKS_E_INVAL; }
    for (int i = 0; i < 2; ++i)
        if (p->reserved[i]) { why = "reserved fields must be zero"; return LBKS_E_INVAL; }
    return 0;
}

Layout plan_layout(const lbks_params *p)
{
    Layout L;
    const size_t N = (size_t)p->N[0] * p->N[1] * p->N[2];
    const size_t s = p->precision == LBKS_FP32_BULK ? 4 : 8;
    const size_t n = (size_t)p->n_orb;
    const size_t ntile = (N + BS - 1) / BS;
    const int no = orbital_bucket(p->n_orb);
    const size_t padded = (size_t)(p->N[0] + 2) * (p->N[1] + 2) * (p->N[2] + 2);
    size_t off = 0;
    auto take = [&](Buf &b, size_t bytes) {
        b.off = off;
        b.bytes = bytes;
        off += align_up(bytes);
    };
    take(L.desc, sizeof(InstDesc));
    const bool pops = p->scheme == LBKS_SCHEME_POPULATIONS;
    take(L.f0, pops ? n * Q * N * s : 0);
    take(L.f1, pops ? n * Q * N * s : 0);
    take(L.psi, n * N * s);
    take(L.psihat, n * N * s);
    take(L.psistar, p->ortho == LBKS_ORTHO_W ? n * N * s : 0);
    take(L.rho, N * s);
    take(L.V, N * s);
    take(L.Vd, s == 8 ? 0 : N * 8);
    take(L.vext, N * 8);
    take(L.vh, padded * 8);
    take(L.s_part, (size_t)padded_cols(no * (no + 1) / 2) * ntile * 8);
    take(L.m_part, (size_t)padded_cols(NMOM) * ntile * 8);
    take(L.e_part, (size_t)padded_cols(2 * no + NEBASE) * ntile * 8);
    take(L.r_part, (size_t)padded_cols(2) * ntile * 8);
    take(L.f_part, (size_t)padded_cols(3 * NUCG) * ntile * 8);
    take(L.gga, p->xc >= LBKS_XC_B88_LYP ? 4 * N * 8 : 0);
    {
        const int widest = std::max(std::max(no * (no + 1) / 2, NMOM), std::max(2 * no + NEBASE, 3 * NUCG));
        take(L.g_part, (size_t)padded_cols(widest) * RG * 8);
    }
    take(L.C, 2 * MAXO * MAXO * 8);
    take(L.scal, SC_SIZE * 8);
    take(L.stage, (n + 1) * N * 8);
    take(L.zr, (4 * LBKS_MAX_NUC + 1) * 8);
    L.total = off;
    return L;
}

void *dev_alloc(lbks_ctx *c, size_t bytes)
{
    if (c->ualloc) return c->ualloc(bytes, c->user);
    void *ptr = nullptr;
    if (hipMalloc(&ptr, bytes) != hipSuccess) return nullptr;
    return ptr;
}

void dev_free(lbks_ctx *c, void *ptr)
{
    if (!ptr) return;
    if (c->ufree) c->ufree(ptr, c->user);
    else (void)hipFree(ptr);
}

void mark_batch_dirty(lbks_ctx *c);

// The state changed: the stopping rule starts over.
void reset_rule(lbks_ctx *c)
{
    c->have_prev = false;
    c->passes = 0;
}

// One check of the stopping rule (see lbks_relax): true once params.stop_checks
// consecutive checks (at least one) had |dE| < dE_tol and, if deps_tol > 0,
// |d sum_j eps_j| < deps_tol against the previous check.
bool rule_check(lbks_ctx *c, double etot, const double *eps, double dE_tol)
{
    double tr = 0.0;
    for (int j = 0; j < c->p.n_orb; ++j) tr += eps[j];
    const bool pass = c->have_prev && fabs(etot - c->e_prev) < dE_tol &&
                      (!(c->p.deps_tol > 0.0) || fabs(tr - c->tr_prev) < c->p.deps_tol);
    c->passes = pass ? c->passes + 1 : 0;
    c->e_prev = etot;
    c->tr_prev = tr;
    c->have_prev = true;
    return c->passes >= std::max(1, (int)c->p.stop_checks);
}

int upload_desc(lbks_ctx *c)
{
    mark_batch_dirty(c);
    reset_rule(c);
    HIPCHK(c, hipMemcpyAsync(c->d_desc, &c->h, sizeof(InstDesc), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return 0;
}

// ---------------------------------------------------------- step sequences

// Kernel sequences on a plan (one solve or one batch group); return hipError_t.
#define PCHK(expr)                  \
    do {                            \
        int _e = (expr);            \
        if (_e != 0) return _e;     \
    } while (0)

int plan_orthonormalise(const Plan &pl, hipStream_t st)
{
    PCHK(launch_overlap_finalize(pl, st));
    PCHK(launch_orthonormalise(pl, st));
    return 0;
}

// V of the current density: the multipole boundary, `sweeps` red/black SOR
// sweeps warm-started from the last V_H, the potential.  When every instance
// folds its multipoles the first red half-sweep also writes the ghost faces.
int plan_hartree_potential(const Plan &pl, int hartree, int sweeps, hipStream_t st)
{
    if (hartree) {
        PCHK(launch_multipole_finalize(pl, st));   // launches nothing when every instance folds
        const bool first = pl.fold_m && sweeps > 0;
        if (!first) PCHK(launch_ghost(pl, st));
        for (int k = 0; k < sweeps; ++k) {
            PCHK(k == 0 && first ? launch_sor_first(pl, st) : launch_sor(pl, 0, st));
            if (k + 1 < sweeps) PCHK(launch_sor(pl, 1, st));
        }
        // the last black half-sweep also evaluates the potential
        if (sweeps > 0) return launch_sor_black_potential(pl, st);
    }
    PCHK(launch_potential(pl, 0, st));
    return 0;
}

// Everything of one lattice step before the lattice Boltzmann update.
int plan_pre_update(const Plan &pl, int hartree, int sweeps, hipStream_t st)
{
    PCHK(plan_orthonormalise(pl, st));
    if (pl.gga) PCHK(launch_gga(pl, st));
    return plan_hartree_potential(pl, hartree, sweeps, st);
}

int plan_update(const Plan &pl, int scheme, int parity, hipStream_t st)
{
    if (scheme == LBKS_SCHEME_POPULATIONS) return launch_stream_collide(pl, parity, st);
    return launch_collapsed_update(pl, st);
}

int plan_energy(const Plan &pl, hipStream_t st)
{
    PCHK(plan_orthonormalise(pl, st));
    if (pl.gga) PCHK(launch_gga(pl, st));
    PCHK(launch_potential(pl, 1, st));
    PCHK(launch_energy_terms(pl, st));
    PCHK(launch_energy_finalize(pl, st));
    return 0;
}

int enqueue_orthonormalise(lbks_ctx *c)
{
    KCHK(c, launch_overlap_finalize(c->plan, c->stream));
    KCHK(c, launch_orthonormalise(c->plan, c->stream));
    return 0;
}

int enqueue_hartree_boundary(lbks_ctx *c)
{
    KCHK(c, launch_multipole_finalize(c->plan, c->stream));
    KCHK(c, launch_ghost(c->plan, c->stream));
    return 0;
}

int enqueue_sweeps(lbks_ctx *c, int sweeps)
{
    for (int k = 0; k < sweeps; ++k) {
        KCHK(c, launch_sor(c->plan, 0, c->stream));
        KCHK(c, launch_sor(c->plan, 1, c->stream));
    }
    return 0;
}

hipEvent_t next_event(lbks_ctx *c)
{
    if (c->ev_used == c->ev.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev.push_back(e);
    }
    return c->ev[c->ev_used++];
}

int flush_timing(lbks_ctx *c)
{
    if (c->ev_used == 0) return 0;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
        const int k = c->ev_kind[i / 2];
        c->timed_ms[k] += ms;
        c->timed_launches[k] += 1;
    }
    c->ev_used = 0;
    c->ev_kind.clear();
    return 0;
}

// One lattice step: orthonormalise, density, Hartree sweeps, potential, then the
// lattice Boltzmann update of every orbital (populations or collapsed form).
// Start a timed launch of `kind`: records the start event on the context's stream
// and returns the stop event to record after the launch.
int timing_begin(lbks_ctx *c, int kind, hipEvent_t *stop)
{
    int rc;
    if (c->ev_used + 2 > 4096 && (rc = flush_timing(c))) return rc;
    hipEvent_t e0 = next_event(c), e1 = next_event(c);
    if (!e0 || !e1) return fail(c, LBKS_E_HIP, "hipEventCreate failed");
    c->ev_kind.push_back(kind);
    HIPCHK(c, hipEventRecord(e0, c->stream));
    *stop = e1;
    return 0;
}

int enqueue_step(lbks_ctx *c)
{
    int rc;
    KCHK(c, plan_pre_update(c->plan, c->p.hartree, c->p.poisson_sweeps, c->stream));
    hipEvent_t e1 = nullptr;
    if (c->timing && (rc = timing_begin(c, 0, &e1))) return rc;
    KCHK(c, plan_update(c->plan, c->p.scheme, c->parity, c->stream));
    if (c->p.scheme == LBKS_SCHEME_POPULATIONS) c->parity ^= 1;
    if (c->timing) HIPCHK(c, hipEventRecord(e1, c->stream));
    c->steps += 1;
    return 0;
}

// Energies of the current state into the scalar block (device).
int enqueue_energy(lbks_ctx *c)
{
    KCHK(c, plan_energy(c->plan, c->stream));
    return 0;
}

int read_energies(lbks_ctx *c, lbks_energies *out, double *errflag)
{
    double buf[SC_SIZE];
    HIPCHK(c, hipMemcpyAsync(buf, c->h.scal, sizeof(buf), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (out) {
        memset(out, 0, sizeof(*out));
        out->e_total = buf[SC_ENER + 0];
        out->e_kin = buf[SC_ENER + 1];
        out->e_ext = buf[SC_ENER + 2];
        out->e_hartree = buf[SC_ENER + 3];
        out->e_x = buf[SC_ENER + 4];
        out->e_c = buf[SC_ENER + 5];
        out->e_nn = buf[SC_ENER + 6];
        out->n_electrons = buf[SC_ENER + 7];
        out->poisson_residual = buf[SC_ENER + 8];
        for (int j = 0; j < LBKS_MAX_ORB; ++j) out->eps[j] = buf[SC_ENER + 9 + j];
        out->steps = c->steps;
    }
    if (errflag) *errflag = buf[SC_ERR];
    return 0;
}

// Update-kernel variant before any autotuning (measured on MI355X at the 96^3-128^3
// workloads): the population update of at most five orbitals takes the rolled wide
// form in dispatch order, the brick update depth 8 (FP64) or 12 (FP32) with the
// XCD remap, the node-per-lane kernels their per-precision default.
// Default update-kernel variant (measured on MI355X).  The rolled wide population
// update walks the 19 directions one after another and needs many waves in
// flight to hide that; on small grids (at most RG * FOLD_GROUP = 256 tiles, the
// grids that also fold their reductions) it has too few, and the node-per-lane
// form with the XCD remap is faster: He 32^3 FP64 28.8 against 39.4 us per step.
int initial_variant(int precision, bool populations, int no, bool wmode, int ntile)
{
    if (no <= 5 && populations) return ntile <= RG * FOLD_GROUP ? (precision ? 1 : 0) : 13;
    if (no <= 5 && !wmode) return precision ? 1 : 0;
    return default_variant(precision);
}

int read_scalar(lbks_ctx *c, int idx, double *v)
{
    HIPCHK(c, hipMemcpyAsync(v, c->h.scal + idx, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return 0;
}

}  // namespace

// ============================================================== public ABI

extern "C" int lbks_params_default(lbks_params *p)
{
    if (!p) return LBKS_E_INVAL;
    memset(p, 0, sizeof(*p));
    p->omega = 1.0;
    p->D = 1.0 / 3.0;
    p->ortho = LBKS_ORTHO_GS;
    p->xc = LBKS_XC_X_LYPLOCAL;
    p->hartree = 1;
    p->poisson_sweeps = 2;
    p->precision = LBKS_FP64;
    p->softening = 0.05;
    p->init = LBKS_INIT_RANDOM_GAUSS;
    p->init_sigma = 1.0;
    p->init_noise = 0.0;
    p->seed = 0;
    p->rho_floor = 1e-14;
    p->scheme = LBKS_SCHEME_POPULATIONS;
    return 0;
}

extern "C" size_t lbks_estimate_bytes(const lbks_params *p)
{
    std::string why;
    if (validate(p, why)) return 0;
    return plan_layout(p).total;
}

extern "C" int lbks_create(const lbks_params *p, const lbks_device *dev, lbks_ctx **out)
{
    g_create_error.clear();
    if (!out) return fail(nullptr, LBKS_E_INVAL, "out is NULL");
    *out = nullptr;
    std::string why;
    if (int rc = validate(p, why)) return fail(nullptr, rc, why);
    if (dev && ((dev->alloc == nullptr) != (dev->free == nullptr)))
        return fail(nullptr, LBKS_E_INVAL, "alloc and free must both be set or both be NULL");
    lbks_ctx *c = new lbks_ctx();
    c->p = *p;
    c->device = dev ? dev->device : 0;
    if (hipSetDevice(c->device) != hipSuccess) {
        delete c;
        return fail(nullptr, LBKS_E_HIP, "hipSetDevice failed");
    }
    if (dev && dev->stream) {
        c->stream = (hipStream_t)dev->stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return fail(nullptr, LBKS_E_HIP, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    if (dev) {
        c->ualloc = dev->alloc;
        c->ufree = dev->free;
        c->user = dev->user;
    }
    Layout L = plan_layout(p);
    c->base = dev_alloc(c, L.total);
    if (!c->base) {
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return fail(nullptr, LBKS_E_NOMEM, "device allocation failed");
    }
    c->bytes = L.total;
    char *b = (char *)c->base;
    auto at = [&](const Buf &x) -> void * { return x.bytes ? (void *)(b + x.off) : nullptr; };
    InstDesc &h = c->h;
    memset(&h, 0, sizeof(h));
    h.nx = p->N[0];
    h.ny = p->N[1];
    h.nz = p->N[2];
    h.n_orb = p->n_orb;
    h.nsite = h.nx * h.ny * h.nz;
    h.ntile = (h.nsite + BS - 1) / BS;
    h.ntile_ghost = (2 * (h.ny * h.nz + h.nx * h.nz + h.nx * h.ny) + BS - 1) / BS;
    h.ntile_sor = (((h.nx + 1) / 2) * h.ny * h.nz + BS - 1) / BS;
    h.ntile_brick = bricks_of(h.nx, h.ny, h.nz);
    h.ortho = p->ortho;
    h.xc = p->xc;
    h.hartree = p->hartree;
    h.precision = p->precision;
    h.scheme = p->scheme;
    h.h = p->h;
    h.h3 = p->h * p->h * p->h;
    h.omega = p->omega;
    h.D = p->D;
    // one lattice step is dt = 2 (1/omega - 1/2) D h^2 of imaginary time (hbar = m = 1)
    h.dt = 2.0 * (1.0 / p->omega - 0.5) * p->D * p->h * p->h;
    {
        const double PI = 3.14159265358979323846;
        const double mu = (cos(PI / (h.nx + 1)) + cos(PI / (h.ny + 1)) + cos(PI / (h.nz + 1))) / 3.0;
        h.omega_sor = 2.0 / (1.0 + sqrt(1.0 - mu * mu));
    }
    h.rho_floor = p->rho_floor;
    h.active = ~0u;
    h.fold = fold_bits(h.ntile, h.n_orb, p->fold == 0);
    h.e_nn = 0.0;
    for (int j = 0; j < MAXO; ++j) h.occ[j] = 0.0;
    if (p->xc == LBKS_XC_B88_LYP_POLARISED) {
        for (int j = 0; j < p->n_orb; ++j) h.occ[j] = 1.0;   // one spin: one electron per orbital
    } else {
        for (int j = 0; j < p->n_orb; ++j) h.occ[j] = 2.0;
        h.occ[p->n_orb - 1] = (double)p->n_elec - 2.0 * (p->n_orb - 1);
    }
    lattice_constants(p->D, p->hermite, h.xi, h.chi);
    h.f0 = at(L.f0);
    h.f1 = at(L.f1);
    h.psi = at(L.psi);
    h.psihat = at(L.psihat);
    h.psistar = at(L.psistar);
    h.rho = at(L.rho);
    h.V = at(L.V);
    h.Vd = p->precision == LBKS_FP64 ? (double *)h.V : (double *)at(L.Vd);
    h.vext = (double *)at(L.vext);
    h.vh = (double *)at(L.vh);
    h.s_part = (double *)at(L.s_part);
    h.m_part = (double *)at(L.m_part);
    h.e_part = (double *)at(L.e_part);
    h.r_part = (double *)at(L.r_part);
    h.f_part = (double *)at(L.f_part);
    h.gga = (double *)at(L.gga);
    h.g_part = (double *)at(L.g_part);
    h.C = (double *)at(L.C);
    h.scal = (double *)at(L.scal);
    h.stage = (double *)at(L.stage);
    c->d_zr = (double *)at(L.zr);
    h.zr = c->d_zr;
    h.nnuc = 0;
    c->d_desc = (InstDesc *)at(L.desc);
    Plan &pl = c->plan;
    pl.d_desc = c->d_desc;
    pl.precision = p->precision == LBKS_FP32_BULK ? 1 : 0;
    pl.no = orbital_bucket(p->n_orb);
    pl.wmode = p->ortho == LBKS_ORTHO_W;
    pl.gga = p->xc >= LBKS_XC_B88_LYP;
    pl.ntile = h.ntile;
    pl.ntile_ghost = h.ntile_ghost;
    pl.ntile_sor = h.ntile_sor;
    pl.ntile_brick = h.ntile_brick;
    for (int k = 0; k < 4; ++k) pl.nbrick[k] = bricks_of(h.nx, h.ny, h.nz, brick_depth(k));
    pl.brick_partials = brick_partials(h.ntile, h.ntile_brick);
    pl.fold_s = (h.fold & FOLD_S) != 0;
    pl.fold_m = (h.fold & FOLD_M) != 0;
    pl.n_inst = 1;
    pl.variant = initial_variant(pl.precision, p->scheme == LBKS_SCHEME_POPULATIONS, pl.no, pl.wmode, h.ntile);

    int rc = 0;
    auto bail = [&](int code) {
        std::string m = c->err;
        lbks_destroy(c);
        return fail(nullptr, code, m);
    };
    // zero everything once (fields, Hartree potential incl. ghosts, scalars)
    if (hipMemsetAsync(c->base, 0, L.total, c->stream) != hipSuccess) {
        c->err = "hipMemsetAsync failed";
        return bail(LBKS_E_HIP);
    }
    if ((rc = upload_desc(c))) return bail(rc);
    if (p->init != LBKS_INIT_USER) {
        if (launch_init_psi(pl, p->init == LBKS_INIT_GAUSS_NOISE ? 0 : 1, p->init_sigma, p->init_noise, p->seed,
                            c->stream)) {
            c->err = "init kernel failed";
            return bail(LBKS_E_HIP);
        }
        if (p->scheme == LBKS_SCHEME_POPULATIONS) {
            if (launch_equilibrium(pl, 0, c->stream) || launch_moment(pl, 0, c->stream)) {
                c->err = "init kernel failed";
                return bail(LBKS_E_HIP);
            }
        } else {
            if (launch_overlap_psi(pl, c->stream)) {
                c->err = "init kernel failed";
                return bail(LBKS_E_HIP);
            }
        }
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) {
        c->err = "initialisation failed on the device";
        return bail(LBKS_E_HIP);
    }
    *out = c;
    return LBKS_OK;
}

extern "C" void lbks_destroy(lbks_ctx *c)
{
    if (!c) return;
    if (c->batch) lbks_batch_detach(c->batch, c);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    dev_free(c, c->cd_buf);
    dev_free(c, c->base);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

extern "C" const char *lbks_last_error(const lbks_ctx *c)
{
    return c ? c->err.c_str() : g_create_error.c_str();
}

extern "C" int lbks_shape(const lbks_ctx *c, int32_t N[3], int32_t *n_orb)
{
    if (!c) return LBKS_E_INVAL;
    if (N) {
        N[0] = c->p.N[0];
        N[1] = c->p.N[1];
        N[2] = c->p.N[2];
    }
    if (n_orb) *n_orb = c->p.n_orb;
    return 0;
}

extern "C" size_t lbks_device_bytes(const lbks_ctx *c) { return c ? c->bytes : 0; }

extern "C" int lbks_set_nuclei(lbks_ctx *c, int32_t n, const double *Z, const double *xyz)
{
    if (!c) return LBKS_E_INVAL;
    if (n < 1 || n > LBKS_MAX_NUC || !Z || !xyz) return fail(c, LBKS_E_INVAL, "bad nuclei count or NULL array");
    double zr[4 * LBKS_MAX_NUC + 1];
    const double hx = 0.5 * (c->p.N[0] - 1) * c->p.h, hy = 0.5 * (c->p.N[1] - 1) * c->p.h,
                 hz = 0.5 * (c->p.N[2] - 1) * c->p.h;
    for (int I = 0; I < n; ++I) {
        if (!(Z[I] > 0.0) || !isfinite(Z[I])) return fail(c, LBKS_E_INVAL, "nuclear charges must be positive");
        const double x = xyz[3 * I], y = xyz[3 * I + 1], z = xyz[3 * I + 2];
        if (!(fabs(x) <= hx && fabs(y) <= hy && fabs(z) <= hz)) return fail(c, LBKS_E_INVAL, "nucleus outside the box");
        zr[4 * I] = Z[I];
        zr[4 * I + 1] = x;
        zr[4 * I + 2] = y;
        zr[4 * I + 3] = z;
    }
    zr[4 * n] = c->p.softening * c->p.softening;
    // ion-ion repulsion (bare Coulomb)
    double enn = 0.0;
    for (int I = 0; I < n; ++I)
        for (int J = I + 1; J < n; ++J) {
            const double dx = xyz[3 * I] - xyz[3 * J], dy = xyz[3 * I + 1] - xyz[3 * J + 1],
                         dz = xyz[3 * I + 2] - xyz[3 * J + 2];
            enn += Z[I] * Z[J] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    HIPCHK(c, hipMemcpyAsync(c->d_zr, zr, sizeof(double) * (4 * n + 1), hipMemcpyHostToDevice, c->stream));
    KCHK(c, launch_vext(c->plan, n, c->d_zr, c->stream));
    c->nuc.assign(zr, zr + 4 * n);
    c->h.e_nn = enn;
    c->h.nnuc = n;
    int rc = upload_desc(c);
    if (rc) return rc;
    c->has_potential = true;
    return 0;
}

extern "C" int lbks_set_potential(lbks_ctx *c, const double *v)
{
    if (!c || !v) return LBKS_E_INVAL;
    HIPCHK(c, hipMemcpyAsync(c->h.vext, v, sizeof(double) * (size_t)c->h.nsite, hipMemcpyHostToDevice, c->stream));
    c->h.e_nn = 0.0;
    c->h.nnuc = 0;
    c->nuc.clear();
    c->vext_depth = 0.0;
    for (int i = 0; i < c->h.nsite; ++i) c->vext_depth = std::max(c->vext_depth, fabs(v[i]));
    int rc = upload_desc(c);
    if (rc) return rc;
    c->has_potential = true;
    return 0;
}

extern "C" int lbks_set_orbitals(lbks_ctx *c, const double *psi)
{
    if (c && c->cd) return fail(c, LBKS_E_STATE, "concurrent dynamics is running (lbks_cd_stop first)");
    if (!c || !psi) return LBKS_E_INVAL;
    const size_t n = (size_t)c->p.n_orb * c->h.nsite;
    reset_rule(c);
    // new orbitals are a recovery point: after a numeric failure the Hartree
    // potential may hold non-finite values too, so it restarts from zero
    double errf = 0.0;
    int rc0 = read_scalar(c, SC_ERR, &errf);
    if (rc0) return rc0;
    if (errf != 0.0) {
        const size_t padded = (size_t)(c->h.nx + 2) * (c->h.ny + 2) * (c->h.nz + 2);
        HIPCHK(c, hipMemsetAsync(c->h.vh, 0, padded * sizeof(double), c->stream));
        HIPCHK(c, hipMemsetAsync(c->h.scal + SC_ERR, 0, sizeof(double), c->stream));
    }
    HIPCHK(c, hipMemcpyAsync(c->h.stage, psi, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
    KCHK(c, launch_psi_from_stage(c->plan, c->stream));
    if (c->p.scheme == LBKS_SCHEME_POPULATIONS) {
        KCHK(c, launch_equilibrium(c->plan, c->parity, c->stream));
        KCHK(c, launch_moment(c->plan, c->parity, c->stream));
    } else {
        KCHK(c, launch_overlap_psi(c->plan, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return 0;
}

extern "C" int lbks_relax(lbks_ctx *c, int64_t max_steps, double dE_tol, int32_t check_every, int64_t *steps_done)
{
    if (!c) return LBKS_E_INVAL;
    if (c && c->cd) return fail(c, LBKS_E_STATE, "concurrent dynamics is running (lbks_cd_stop first)");
    if (steps_done) *steps_done = 0;
    if (!c->has_potential) return fail(c, LBKS_E_STATE, "no nuclei or potential set");
    if (max_steps < 0) return fail(c, LBKS_E_INVAL, "max_steps < 0");
    if (check_every < 1) check_every = 1;
    int64_t done = 0;
    int rc;
    while (done < max_steps) {
        const int64_t n = std::min<int64_t>(check_every, max_steps - done);
        for (int64_t k = 0; k < n; ++k)
            if ((rc = enqueue_step(c))) return rc;
        done += n;
        if (steps_done) *steps_done = done;
        if (dE_tol > 0.0) {
            if ((rc = enqueue_energy(c))) return rc;
            lbks_energies e;
            double errf = 0.0;
            if ((rc = read_energies(c, &e, &errf))) return rc;
            if (errf != 0.0 || !isfinite(e.e_total))
                return fail(c, LBKS_E_NUMERIC, "overlap matrix not finite or not positive definite");
            if (rule_check(c, e.e_total, e.eps, dE_tol)) return LBKS_OK;
        }
    }
    double errf = 0.0;
    if ((rc = read_scalar(c, SC_ERR, &errf))) return rc;
    if (errf != 0.0) return fail(c, LBKS_E_NUMERIC, "overlap matrix not finite or not positive definite");
    if (c->timing && (rc = flush_timing(c))) return rc;
    return LBKS_NOT_CONVERGED;
}

namespace {

// Orthonormalise the current orbitals and, with Hartree on, converge V_H for
// their density (the state lbks_energy and lbks_hamiltonian evaluate).
int converge_vh(lbks_ctx *c);

int converge_hartree(lbks_ctx *c)
{
    int rc;
    reset_rule(c);   // the Hartree relaxation below changes the state
    if ((rc = enqueue_orthonormalise(c))) return rc;
    return converge_vh(c);
}

// Converge V_H for the density in place (multipole partials of that density in
// m_part).
int converge_vh(lbks_ctx *c)
{
    int rc;
    if (c->p.hartree) {
        if ((rc = enqueue_hartree_boundary(c))) return rc;
        // converge V_H for the current density: blocks of 10 sweeps until the
        // relative residual is <= 1e-12, or until it has reached the roundoff
        // floor of a fine grid (<= 1e-9 and no more than 10 % below its value
        // five blocks earlier)
        const double tol = 1e-12;
        std::vector<double> hist;
        for (int it = 0;; ++it) {
            KCHK(c, launch_residual(c->plan, c->stream));
            KCHK(c, launch_residual_finalize(c->plan, c->stream));
            double res = 0.0;
            if ((rc = read_scalar(c, SC_RES, &res))) return rc;
            hist.push_back(res);
            if (!(res > tol)) break;
            if (it >= 5 && res <= 1e-9 && res >= 0.9 * hist[it - 5]) break;
            if (!isfinite(res) || it > 20000) {
                char msg[128];
                snprintf(msg, sizeof msg, "Poisson relaxation did not converge (relative residual %.3e after %d sweeps)",
                         res, 10 * it);
                return fail(c, LBKS_E_NUMERIC, msg);
            }
            if ((rc = enqueue_sweeps(c, 10))) return rc;
        }
    }
    return 0;
}

}  // namespace

extern "C" int lbks_energy(lbks_ctx *c, lbks_energies *out)
{
    if (!c || !out) return LBKS_E_INVAL;
    if (c && c->cd) return fail(c, LBKS_E_STATE, "concurrent dynamics is running (lbks_cd_stop first)");
    if (!c->has_potential) return fail(c, LBKS_E_STATE, "no nuclei or potential set");
    int rc;
    if ((rc = converge_hartree(c))) return rc;
    if ((rc = enqueue_energy(c))) return rc;
    double errf = 0.0;
    if ((rc = read_energies(c, out, &errf))) return rc;
    if (errf != 0.0) return fail(c, LBKS_E_NUMERIC, "overlap matrix not finite or not positive definite");
    if (!c->p.hartree) out->poisson_residual = 0.0;
    return 0;
}

extern "C" int lbks_hamiltonian(lbks_ctx *c, double *H, size_t n_H)
{
    if (!c || !H) return LBKS_E_INVAL;
    if (c && c->cd) return fail(c, LBKS_E_STATE, "concurrent dynamics is running (lbks_cd_stop first)");
    if (!c->has_potential) return fail(c, LBKS_E_STATE, "no nuclei or potential set");
    const size_t n = (size_t)c->p.n_orb;
    if (n_H < n * n) return fail(c, LBKS_E_INVAL, "H buffer too small");
    if (n * n > (n + 1) * (size_t)c->h.nsite) return fail(c, LBKS_E_INVAL, "grid too small to stage H");
    int rc;
    if ((rc = converge_hartree(c))) return rc;
    if (c->plan.gga) KCHK(c, launch_gga(c->plan, c->stream));
    KCHK(c, launch_potential(c->plan, 1, c->stream));
    for (int j0 = 0; j0 < (int)n;) {
        int rows = 0;
        KCHK(c, launch_ham_rows(c->plan, j0, &rows, c->stream));
        j0 += rows;
    }
    std::vector<double> buf(n * n + 1);
    HIPCHK(c, hipMemcpyAsync(buf.data(), c->h.stage, n * n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(buf.data() + n * n, c->h.scal + SC_ERR, sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (buf[n * n] != 0.0) return fail(c, LBKS_E_NUMERIC, "overlap matrix not finite or not positive definite");
    for (size_t q = 0; q < n * n; ++q) {
        if (!isfinite(buf[q])) return fail(c, LBKS_E_NUMERIC, "projected operator not finite");
        H[q] = buf[q];
    }
    return 0;
}

extern "C" int lbks_relax_sequential(lbks_ctx *c, int64_t max_steps, double dE_tol, double deps_tol,
                                     int32_t check_every, int32_t max_sweeps, int64_t *steps_done,
                                     int32_t *sweeps_done)
{
    if (!c) return LBKS_E_INVAL;
    if (steps_done) *steps_done = 0;
    if (sweeps_done) *sweeps_done = 0;
    if (c->cd) return fail(c, LBKS_E_STATE, "concurrent dynamics is running (lbks_cd_stop first)");
    if (!c->has_potential) return fail(c, LBKS_E_STATE, "no nuclei or potential set");
    if (c->batch) return fail(c, LBKS_E_STATE, "a batch member relaxes with the batch");
    if (c->p.scheme != LBKS_SCHEME_COLLAPSED || c->p.ortho != LBKS_ORTHO_GS)
        return fail(c, LBKS_E_INVAL, "the sequential order runs on the omega = 1 field update with Gram-Schmidt");
    if (!(dE_tol > 0.0) || !(deps_tol > 0.0) || max_steps < 0 || max_sweeps < 1)
        return fail(c, LBKS_E_INVAL, "dE_tol and deps_tol must be positive, max_sweeps >= 1");
    if (check_every < 1) check_every = 1;
    const int n = c->p.n_orb;
    int64_t steps = 0;
    int rc = LBKS_NOT_CONVERGED, sweep = 0;
    double e_prev = 0.0;
    bool have_prev = false;
    auto set_active = [&](unsigned mask) -> int {
        c->h.active = mask;
        return upload_desc(c);
    };
    auto energies = [&](lbks_energies *e) -> int {
        int r;
        if ((r = enqueue_energy(c))) return r;
        double errf = 0.0;
        if ((r = read_energies(c, e, &errf))) return r;
        if (errf != 0.0 || !isfinite(e->e_total))
            return fail(c, LBKS_E_NUMERIC, "overlap matrix not finite or not positive definite");
        return 0;
    };
    int err = 0;
    for (sweep = 1; sweep <= max_sweeps && !err; ++sweep) {
        for (int k = 0; k < n && !err; ++k) {
            if ((err = set_active(1u << k))) break;
            bool have = false;
            double eps_prev = 0.0;
            while (steps < max_steps) {
                const int64_t m = std::min<int64_t>(check_every, max_steps - steps);
                for (int64_t i = 0; i < m && !err; ++i) err = enqueue_step(c);
                if (err) break;
                steps += m;
                lbks_energies e;
                if ((err = energies(&e))) break;
                if (have && fabs(e.eps[k] - eps_prev) < deps_tol) break;
                eps_prev = e.eps[k];
                have = true;
            }
        }
        if (err) break;
        lbks_energies e;
        if ((err = energies(&e))) break;
        if (steps >= max_steps) break;
        if (have_prev && fabs(e.e_total - e_prev) < dE_tol) {
            rc = LBKS_OK;
            break;
        }
        e_prev = e.e_total;
        have_prev = true;
    }
    const int e2 = set_active(~0u);
    if (steps_done) *steps_done = steps;
    if (sweeps_done) *sweeps_done = std::min(sweep, max_sweeps);
    if (err) return err;
    if (e2) return e2;
    reset_rule(c);
    return rc;
}

// ================================================ concurrent dynamics

namespace {

double2 *cd_level(lbks_ctx *c, int k) { return c->cd_buf + (size_t)k * c->p.n_orb * c->h.nsite; }

// V of the density in place: multipole boundary, K_P red/black sweeps, potential.
int cd_potential(lbks_ctx *c)
{
    KCHK(c, plan_hartree_potential(c->plan, c->p.hartree, c->p.poisson_sweeps, c->stream));
    return 0;
}

// Bound of the kinetic part of H for the stability of the time-centred step:
// (1 - min symbol of S_xi) / (D dx^2) over a grid of wave vectors.
void cd_bounds(const lbks_ctx *c, double *kin, double *vdepth)
{
    double smin = 1.0;
    const int K = 16;
    for (int a = 0; a <= K; ++a)
        for (int b = 0; b <= K; ++b)
            for (int e = 0; e <= K; ++e) {
                const double kx = M_PI * a / K, ky = M_PI * b / K, kz = M_PI * e / K;
                double sym = 0.0;
                for (int p = 0; p < Q; ++p) {
                    const int vx = (p == 1 || p == 7 || p == 9 || p == 11 || p == 13) ? 1
                                 : (p == 2 || p == 8 || p == 10 || p == 12 || p == 14) ? -1 : 0;
                    const int vy = (p == 3 || p == 7 || p == 8 || p == 15 || p == 17) ? 1
                                 : (p == 4 || p == 9 || p == 10 || p == 16 || p == 18) ? -1 : 0;
                    const int vz = (p == 5 || p == 11 || p == 12 || p == 15 || p == 16) ? 1
                                 : (p == 6 || p == 13 || p == 14 || p == 17 || p == 18) ? -1 : 0;
                    sym += c->h.xi[p] * cos(kx * vx + ky * vy + kz * vz);
                }
                smin = std::min(smin, sym);
            }
    *kin = (1.0 - smin) / (c->p.D * c->p.h * c->p.h);
    *vdepth = 0.0;
}

}  // namespace

extern "C" int lbks_cd_start(lbks_ctx *c, double h, int64_t restart_every)
{
    if (!c) return LBKS_E_INVAL;
    if (restart_every < 0) return fail(c, LBKS_E_INVAL, "restart_every < 0");
    if (!c->has_potential) return fail(c, LBKS_E_STATE, "no nuclei or potential set");
    if (c->batch) return fail(c, LBKS_E_STATE, "a batch member cannot run concurrent dynamics (detach it)");
    if (c->p.precision != LBKS_FP64 || c->p.xc >= LBKS_XC_B88_LYP || c->p.omega != 1.0 ||
        c->p.ortho != LBKS_ORTHO_GS)
        return fail(c, LBKS_E_INVAL, "concurrent dynamics needs FP64, a local functional, omega = 1 and Gram-Schmidt");
    if (!(h > 0.0) || !isfinite(h)) return fail(c, LBKS_E_INVAL, "time step must be positive");
    double kin = 0.0, vdepth = 0.0;
    cd_bounds(c, &kin, &vdepth);
    // depth of V_ext at the node nearest each nucleus (what the grid resolves), or
    // the largest |v| of a potential set directly
    if (c->nuc.empty()) vdepth = c->vext_depth;
    for (size_t I = 0; 4 * I + 3 < c->nuc.size(); ++I) {
        double d2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double half = 0.5 * (c->p.N[a] - 1) * c->p.h;
            const double t = (c->nuc[4 * I + 1 + a] + half) / c->p.h;
            const double dn = (t - floor(t + 0.5)) * c->p.h;
            d2 += dn * dn;
        }
        vdepth += c->nuc[4 * I] / sqrt(d2 + c->p.softening * c->p.softening);
    }
    const double lam = std::max(kin, vdepth);
    if (h * lam >= 0.95) {
        char msg[200];
        snprintf(msg, sizeof msg, "time step %.4g exceeds the stable bound 0.95 / %.4g = %.4g of the time-centred step", h,
                 lam, 0.95 / lam);
        return fail(c, LBKS_E_INVAL, msg);
    }
    const size_t lvl = (size_t)c->p.n_orb * c->h.nsite;
    if (!c->cd_buf) {
        c->cd_buf = (double2 *)dev_alloc(c, 4 * lvl * sizeof(double2));
        if (!c->cd_buf) return fail(c, LBKS_E_NOMEM, "device allocation of the complex orbitals failed");
    }
    int rc;
    c->cd = false;
    if ((rc = converge_hartree(c))) return rc;     // psi_hat, rho and V_H of the current orbitals
    // energy references: the orbitals' energies eps_j at the start
    if ((rc = enqueue_energy(c))) return rc;
    {
        lbks_energies e0;
        double errf = 0.0;
        if ((rc = read_energies(c, &e0, &errf))) return rc;
        if (errf != 0.0) return fail(c, LBKS_E_NUMERIC, "overlap matrix not finite or not positive definite");
        for (int j = 0; j < MAXO; ++j) c->cd_ref.e[j] = j < c->p.n_orb ? e0.eps[j] : 0.0;
    }
    KCHK(c, launch_potential(c->plan, 0, c->stream));
    KCHK(c, launch_cd_init(c->plan, cd_level(c, 0), c->stream));
    KCHK(c, launch_cd_apply(c->plan, cd_level(c, 0), cd_level(c, 2), c->cd_ref, c->stream));
    KCHK(c, launch_cd_apply(c->plan, cd_level(c, 2), cd_level(c, 3), c->cd_ref, c->stream));
    KCHK(c, launch_cd_taylor(c->plan, cd_level(c, 0), cd_level(c, 2), cd_level(c, 3), cd_level(c, 1), h, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->cd = true;
    c->cd_h = h;
    c->cd_cur = 1;
    c->cd_steps = 0;
    c->cd_restart = restart_every;
    return 0;
}

namespace {

// Restart step (V of psi^n in place): E_j <- h^3 Re<psi_j^n|H psi_j^n>, then the
// new level is the one-step start from psi^n, psi^n - i h H' psi^n - (h^2 / 2) H' H' psi^n.
int cd_restart_step(lbks_ctx *c)
{
    const Plan &pl = c->plan;
    double2 *cur = cd_level(c, c->cd_cur);
    KCHK(c, launch_cd_energy_terms(pl, cur, c->stream));
    KCHK(c, launch_energy_finalize(pl, c->stream));
    lbks_energies e;
    int rc;
    if ((rc = read_energies(c, &e, nullptr))) return rc;
    for (int j = 0; j < c->p.n_orb; ++j)
        if (!isfinite(e.eps[j])) return fail(c, LBKS_E_NUMERIC, "orbital energy not finite at a restart");
    for (int j = 0; j < MAXO; ++j) c->cd_ref.e[j] = j < c->p.n_orb ? e.eps[j] : 0.0;
    KCHK(c, launch_cd_apply(pl, cur, cd_level(c, 2), c->cd_ref, c->stream));
    KCHK(c, launch_cd_apply(pl, cd_level(c, 2), cd_level(c, 3), c->cd_ref, c->stream));
    KCHK(c, launch_cd_taylor(pl, cur, cd_level(c, 2), cd_level(c, 3), cd_level(c, 1 - c->cd_cur), c->cd_h,
                             c->stream));
    return 0;
}

}  // namespace

extern "C" int lbks_cd_step(lbks_ctx *c, int64_t steps)
{
    if (!c) return LBKS_E_INVAL;
    if (!c->cd) return fail(c, LBKS_E_STATE, "concurrent dynamics not started (lbks_cd_start)");
    if (steps < 0) return fail(c, LBKS_E_INVAL, "steps < 0");
    int rc;
    for (int64_t k = 0; k < steps; ++k) {
        if ((rc = cd_potential(c))) return rc;
        hipEvent_t stop = nullptr;
        if (c->timing && (rc = timing_begin(c, 1, &stop))) return rc;
        if (c->cd_restart > 0 && (c->cd_steps + 1) % c->cd_restart == 0) {
            if ((rc = cd_restart_step(c))) return rc;
        } else {
            KCHK(c, launch_cd_step(c->plan, cd_level(c, c->cd_cur), cd_level(c, 1 - c->cd_cur), c->cd_h, c->cd_ref,
                                   c->stream));
        }
        if (stop) HIPCHK(c, hipEventRecord(stop, c->stream));
        c->cd_cur = 1 - c->cd_cur;
        c->cd_steps += 1;
    }
    return 0;
}

extern "C" int lbks_cd_energy(lbks_ctx *c, lbks_energies *out)
{
    if (!c || !out) return LBKS_E_INVAL;
    if (!c->cd) return fail(c, LBKS_E_STATE, "concurrent dynamics not started (lbks_cd_start)");
    int rc;
    if ((rc = converge_vh(c))) return rc;
    KCHK(c, launch_potential(c->plan, 1, c->stream));
    KCHK(c, launch_cd_energy_terms(c->plan, cd_level(c, c->cd_cur), c->stream));
    KCHK(c, launch_energy_finalize(c->plan, c->stream));
    if ((rc = read_energies(c, out, nullptr))) return rc;
    if (!c->p.hartree) out->poisson_residual = 0.0;
    out->steps = c->cd_steps;
    for (int j = 0; j < LBKS_MAX_ORB; ++j)
        if (!isfinite(out->eps[j])) return fail(c, LBKS_E_NUMERIC, "orbital energy not finite");
    if (!isfinite(out->e_total)) return fail(c, LBKS_E_NUMERIC, "total energy not finite");
    return 0;
}

extern "C" int lbks_cd_orbitals(lbks_ctx *c, double *re, double *im, size_t n)
{
    if (!c || !re || !im) return LBKS_E_INVAL;
    if (!c->cd) return fail(c, LBKS_E_STATE, "concurrent dynamics not started (lbks_cd_start)");
    const size_t lvl = (size_t)c->p.n_orb * c->h.nsite;
    if (n < lvl) return fail(c, LBKS_E_INVAL, "orbital buffers too small");
    std::vector<double2> host(lvl);
    HIPCHK(c, hipMemcpyAsync(host.data(), cd_level(c, c->cd_cur), lvl * sizeof(double2), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i < lvl; ++i) {
        re[i] = host[i].x;
        im[i] = host[i].y;
    }
    return 0;
}

extern "C" int lbks_cd_stop(lbks_ctx *c)
{
    if (!c) return LBKS_E_INVAL;
    if (c->stream) HIPCHK(c, hipStreamSynchronize(c->stream));
    dev_free(c, c->cd_buf);
    c->cd_buf = nullptr;
    c->cd = false;
    return 0;
}

static_assert(MAXNUC == LBKS_MAX_NUC, "nuclei capacity of the kernels and of the C ABI differ");

extern "C" int lbks_forces(lbks_ctx *c, double *F, size_t n_F)
{
    if (!c || !F) return LBKS_E_INVAL;
    const int nn = c->h.nnuc;
    if (nn < 1) return fail(c, LBKS_E_STATE, "no nuclei set (forces need lbks_set_nuclei)");
    if (n_F < (size_t)(3 * nn)) return fail(c, LBKS_E_INVAL, "force buffer too small");
    int rc;
    // during concurrent dynamics the density of the current complex orbitals is in place
    if (!c->cd && (rc = enqueue_orthonormalise(c))) return rc;
    for (int i0 = 0; i0 < nn; i0 += NUCG) {
        KCHK(c, launch_force_terms(c->plan, i0, c->stream));
        KCHK(c, launch_force_finalize(c->plan, i0, c->stream));
    }
    double buf[3 * MAXNUC + 1];
    HIPCHK(c, hipMemcpyAsync(buf, c->h.scal + SC_FORCE, sizeof(double) * 3 * nn, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(buf + 3 * nn, c->h.scal + SC_ERR, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (buf[3 * nn] != 0.0) return fail(c, LBKS_E_NUMERIC, "overlap matrix not finite or not positive definite");
    for (int q = 0; q < 3 * nn; ++q) {
        if (!isfinite(buf[q])) return fail(c, LBKS_E_NUMERIC, "force not finite");
        F[q] = buf[q];
    }
    return 0;
}

extern "C" int lbks_orbitals(lbks_ctx *c, double *psi, size_t n_psi, double *rho, size_t n_rho)
{
    if (!c || !psi) return LBKS_E_INVAL;
    if (c && c->cd) return fail(c, LBKS_E_STATE, "concurrent dynamics is running (lbks_cd_stop first)");
    const size_t N = (size_t)c->h.nsite, n = (size_t)c->p.n_orb;
    if (n_psi < n * N) return fail(c, LBKS_E_INVAL, "psi buffer too small");
    if (rho && n_rho < N) return fail(c, LBKS_E_INVAL, "rho buffer too small");
    int rc;
    if ((rc = enqueue_orthonormalise(c))) return rc;
    KCHK(c, launch_stage_orbitals(c->plan, c->stream));
    HIPCHK(c, hipMemcpyAsync(psi, c->h.stage, n * N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (rho) HIPCHK(c, hipMemcpyAsync(rho, c->h.stage + n * N, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return 0;
}

extern "C" int lbks_set_timing(lbks_ctx *c, int32_t enable)
{
    if (!c) return LBKS_E_INVAL;
    int rc = flush_timing(c);
    if (rc) return rc;
    c->timing = enable != 0;
    for (int k = 0; k < 2; ++k) {
        c->timed_ms[k] = 0.0;
        c->timed_launches[k] = 0;
    }
    return 0;
}

extern "C" int lbks_kernel_time(lbks_ctx *c, int32_t kernel, double *total_ms, int64_t *launches)
{
    if (!c || kernel < 0 || kernel > 1) return LBKS_E_INVAL;
    int rc = flush_timing(c);
    if (rc) return rc;
    if (total_ms) *total_ms = c->timed_ms[kernel];
    if (launches) *launches = c->timed_launches[kernel];
    return 0;
}

extern "C" int lbks_copy_kernel(void *dst, const void *src, size_t bytes, void *stream)
{
    if (!dst || !src || (bytes % 16) || (((uintptr_t)dst | (uintptr_t)src) & 15)) return LBKS_E_INVAL;
    int e = launch_copy(dst, src, bytes, (hipStream_t)stream);
    return e ? LBKS_E_HIP : 0;
}

extern "C" int lbks_set_variant(lbks_ctx *c, int32_t variant)
{
    if (!c || variant < 0 || variant >= N_VARIANTS) return LBKS_E_INVAL;
    c->plan.variant = variant;
    mark_batch_dirty(c);
    return 0;
}

extern "C" int lbks_get_variant(const lbks_ctx *c)
{
    return c ? c->plan.variant : LBKS_E_INVAL;
}

extern "C" int lbks_get_fold(const lbks_ctx *c)
{
    return c ? c->h.fold : LBKS_E_INVAL;
}

namespace {

struct TuneKey {
    int precision, no, wmode, scheme, nsite;
    bool operator<(const TuneKey &o) const
    {
        return std::tie(precision, no, wmode, scheme, nsite) < std::tie(o.precision, o.no, o.wmode, o.scheme, o.nsite);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tuned;

}  // namespace

extern "C" int lbks_autotune(lbks_ctx *c, int32_t reps, int32_t force, int32_t *chosen, double *avg_ms)
{
    if (!c) return LBKS_E_INVAL;
    if (!c->has_potential) return fail(c, LBKS_E_STATE, "no nuclei or potential set");
    if (reps < 1) reps = 1;
    const TuneKey key{c->plan.precision, c->plan.no, c->plan.wmode ? 1 : 0, c->p.scheme, c->h.nsite};
    if (!force) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            c->plan.variant = it->second;
            mark_batch_dirty(c);
            if (chosen) *chosen = it->second;
            if (avg_ms)
                for (int v = 0; v < N_VARIANTS; ++v) avg_ms[v] = -1.0;
            return 0;
        }
    }
    const bool pops = c->p.scheme == LBKS_SCHEME_POPULATIONS;
    const size_t state_bytes = (size_t)c->p.n_orb * c->h.nsite * (c->plan.precision ? 4 : 8);
    // derived fields of the current state (the Hartree potential is not touched)
    KCHK(c, plan_orthonormalise(c->plan, c->stream));
    KCHK(c, launch_potential(c->plan, 0, c->stream));
    if (!pops) HIPCHK(c, hipMemcpyAsync(c->h.stage, c->h.psi, state_bytes, hipMemcpyDeviceToDevice, c->stream));
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    const int saved = c->plan.variant;
    int best = saved;
    double best_ms = 1e300;
    double ms_v[N_VARIANTS];
    int rc = 0;
    for (int v = 0; v < N_VARIANTS && !rc; ++v) {
        ms_v[v] = -1.0;
        if (!variant_distinct(v, c->plan.no, pops)) continue;   // same kernel as a variant already timed
        c->plan.variant = v;
        // one untimed launch, then `reps` timed ones; each launch recomputes the same
        // output from the same inputs
        if (plan_update(c->plan, c->p.scheme, c->parity, c->stream)) rc = LBKS_E_HIP;
        if (!rc && hipEventRecord(e0, c->stream) != hipSuccess) rc = LBKS_E_HIP;
        for (int k = 0; k < reps && !rc; ++k)
            if (plan_update(c->plan, c->p.scheme, c->parity, c->stream)) rc = LBKS_E_HIP;
        if (!rc && hipEventRecord(e1, c->stream) != hipSuccess) rc = LBKS_E_HIP;
        float ms = 0.f;
        if (!rc && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = LBKS_E_HIP;
        ms_v[v] = ms / reps;
        if (!rc && ms_v[v] < best_ms) {
            best_ms = ms_v[v];
            best = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->plan.variant = rc ? saved : best;
    // restore what the timed launches overwrote: the moment and overlap partials of
    // the current populations, or the orbital state of the collapsed scheme
    if (pops) {
        KCHK(c, launch_moment(c->plan, c->parity, c->stream));
    } else {
        HIPCHK(c, hipMemcpyAsync(c->h.psi, c->h.stage, state_bytes, hipMemcpyDeviceToDevice, c->stream));
        KCHK(c, launch_overlap_psi(c->plan, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (rc) return fail(c, rc, "autotune launch failed");
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[key] = best;
    }
    mark_batch_dirty(c);
    if (chosen) *chosen = best;
    if (avg_ms)
        for (int v = 0; v < N_VARIANTS; ++v) avg_ms[v] = ms_v[v];
    return 0;
}

// ================================================================ batches

namespace {

constexpr int GATHER_W = 32;   // per member: the 25 energy values, then the error flag
constexpr int GATHER_ERR = 25;

void mark_batch_dirty(lbks_ctx *c)
{
    if (c && c->batch) c->batch->dirty = true;
}

void batch_destroy_graphs(lbks_batch *b)
{
    for (int k = 0; k < 2; ++k) {
        if (b->exec[k]) (void)hipGraphExecDestroy(b->exec[k]);
        if (b->graph[k]) (void)hipGraphDestroy(b->graph[k]);
        b->exec[k] = nullptr;
        b->graph[k] = nullptr;
    }
}

void batch_free_mem(lbks_batch *b)
{
    if (!b->mem) return;
    if (b->ufree) b->ufree(b->mem, b->user);
    else (void)hipFree(b->mem);
    b->mem = nullptr;
    b->mem_bytes = 0;
}

// Fold the steps taken under the current plan into the members' own state.
void batch_commit(lbks_batch *b)
{
    for (const BatchGroup &g : b->groups)
        for (int i : g.members) {
            lbks_ctx *c = b->members[i];
            if (c->p.scheme == LBKS_SCHEME_POPULATIONS && (b->epoch_steps & 1)) c->parity ^= 1;
            c->steps += b->epoch_steps;
        }
    b->epoch_steps = 0;
    b->bparity = 0;
}

int batch_fail(lbks_batch *b, int code, const std::string &m)
{
    b->err = m;
    return code;
}

// Enqueue one lattice step of every running member at batch parity bp.
int batch_enqueue_step(lbks_batch *b, int bp)
{
    for (const BatchGroup &g : b->groups) {
        int e = plan_pre_update(g.plan, g.hartree, g.sweeps, b->stream);
        if (!e) e = plan_update(g.plan, g.scheme, bp, b->stream);
        if (e) return e;
    }
    return 0;
}

// Group the running members, upload their descriptors and tile tables, and
// capture one step per parity into HIP graphs.  With `fixed` the tables go to that
// device memory of `fixed_cap` bytes instead of the batch's own allocation, and no
// graph is captured (the steps are launched one by one): nothing is allocated.
int batch_build(lbks_batch *b, void *fixed = nullptr, size_t fixed_cap = 0)
{
    batch_commit(b);
    batch_destroy_graphs(b);
    b->groups.clear();
    const int m = (int)b->members.size();
    for (int i = 0; i < m; ++i) {
        if (!b->running[i]) continue;
        const lbks_ctx *c = b->members[i];
        BatchGroup key;
        key.precision = c->plan.precision;
        key.no = c->plan.no;
        key.wmode = c->plan.wmode;
        key.scheme = c->p.scheme;
        key.hartree = c->p.hartree;
        key.sweeps = c->p.poisson_sweeps;
        key.variant = c->plan.variant;
        key.gga = c->plan.gga;
        BatchGroup *g = nullptr;
        for (BatchGroup &x : b->groups)
            if (x.precision == key.precision && x.no == key.no && x.wmode == key.wmode && x.scheme == key.scheme &&
                x.hartree == key.hartree && x.sweeps == key.sweeps && x.variant == key.variant && x.gga == key.gga)
                g = &x;
        if (!g) {
            b->groups.push_back(key);
            g = &b->groups.back();
        }
        g->members.push_back(i);
    }
    // sizes
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    };
    struct Off {
        size_t desc, site, ghost, sor, inst, brick, site_w;
        int n_site, n_ghost, n_sor, n_brick, n_site_w;
    };
    std::vector<Off> go(b->groups.size());
    for (size_t k = 0; k < b->groups.size(); ++k) {
        const BatchGroup &g = b->groups[k];
        Off &o = go[k];
        o.n_site = o.n_ghost = o.n_sor = o.n_brick = o.n_site_w = 0;
        const int kw = wide_nodes(g.precision ? 4 : 8);
        for (int i : g.members) {
            const InstDesc &h = b->members[i]->h;
            o.n_site += h.ntile;
            o.n_ghost += h.ntile_ghost;
            o.n_sor += h.ntile_sor;
            o.n_brick += bricks_of(h.nx, h.ny, h.nz, brick_depth(g.variant));
            o.n_site_w += (h.ntile + kw - 1) / kw;
        }
        o.desc = take(sizeof(InstDesc) * g.members.size());
        o.site = take(sizeof(int2) * o.n_site);
        o.ghost = take(sizeof(int2) * o.n_ghost);
        o.sor = take(sizeof(int2) * o.n_sor);
        o.inst = take(sizeof(int) * g.members.size());
        o.brick = take(sizeof(int2) * o.n_brick);
        o.site_w = take(sizeof(int2) * o.n_site_w);
    }
    const size_t gather_off = take(sizeof(double) * GATHER_W * std::max(m, 1));
    const size_t scal_off = take(sizeof(double *) * std::max(m, 1));
    if (fixed && off > fixed_cap) {
        char msg[192];
        snprintf(msg, sizeof msg, "the batch tables need %zu bytes, more than the %zu-byte static workspace "
                 "(lbks_batch_relax allocates instead)", off, fixed_cap);
        return batch_fail(b, LBKS_E_INVAL, msg);
    }
    if (!fixed && off > b->mem_bytes) {
        batch_free_mem(b);
        void *p = nullptr;
        if (b->ualloc) p = b->ualloc(off, b->user);
        else if (hipMalloc(&p, off) != hipSuccess) p = nullptr;
        if (!p) return batch_fail(b, LBKS_E_NOMEM, "batch table allocation failed");
        b->mem = p;
        b->mem_bytes = off;
    }
    std::vector<char> host(off, 0);
    char *base = fixed ? (char *)fixed : (char *)b->mem;
    for (size_t k = 0; k < b->groups.size(); ++k) {
        BatchGroup &g = b->groups[k];
        const Off &o = go[k];
        InstDesc *hd = (InstDesc *)(host.data() + o.desc);
        int2 *ts = (int2 *)(host.data() + o.site);
        int2 *tg = (int2 *)(host.data() + o.ghost);
        int2 *tr = (int2 *)(host.data() + o.sor);
        int *ti = (int *)(host.data() + o.inst);
        int2 *tb = (int2 *)(host.data() + o.brick);
        int2 *tw = (int2 *)(host.data() + o.site_w);
        const int kw = wide_nodes(g.precision ? 4 : 8);
        int ns = 0, ng = 0, nr = 0, nb = 0, nw = 0;
        bool all_brick = true, all_fold_s = true, all_fold_m = true;
        for (size_t q = 0; q < g.members.size(); ++q) {
            const lbks_ctx *c = b->members[g.members[q]];
            InstDesc d = c->h;
            if (c->parity) std::swap(d.f0, d.f1);   // batch parity 0 = the member's current populations
            hd[q] = d;
            for (int t = 0; t < d.ntile; ++t) ts[ns++] = make_int2((int)q, t);
            for (int t = 0; t < d.ntile_ghost; ++t) tg[ng++] = make_int2((int)q, t);
            for (int t = 0; t < d.ntile_sor; ++t) tr[nr++] = make_int2((int)q, t);
            for (int t = 0; t < bricks_of(d.nx, d.ny, d.nz, brick_depth(g.variant)); ++t) tb[nb++] = make_int2((int)q, t);
            for (int t = 0; t < (d.ntile + kw - 1) / kw; ++t) tw[nw++] = make_int2((int)q, t);
            all_brick = all_brick && brick_partials(d.ntile, d.ntile_brick);
            all_fold_s = all_fold_s && (d.fold & FOLD_S);
            all_fold_m = all_fold_m && (d.fold & FOLD_M);
            ti[q] = (int)q;
        }
        Plan &pl = g.plan;
        pl = Plan{};
        pl.d_desc = (const InstDesc *)(base + o.desc);
        pl.tt.site = (const int2 *)(base + o.site);
        pl.tt.n_site = o.n_site;
        pl.tt.ghost = (const int2 *)(base + o.ghost);
        pl.tt.n_ghost = o.n_ghost;
        pl.tt.sor = (const int2 *)(base + o.sor);
        pl.tt.n_sor = o.n_sor;
        pl.tt.inst = (const int *)(base + o.inst);
        pl.tt.n_inst = (int)g.members.size();
        pl.tt.brick = (const int2 *)(base + o.brick);
        pl.tt.n_brick = o.n_brick;
        pl.tt.site_w = (const int2 *)(base + o.site_w);
        pl.tt.n_site_w = o.n_site_w;
        pl.brick_partials = all_brick;
        pl.fold_s = all_fold_s;
        pl.fold_m = all_fold_m;
        pl.precision = g.precision;
        pl.no = g.no;
        pl.wmode = g.wmode;
        pl.gga = g.gga;
        pl.n_inst = (int)g.members.size();
        pl.variant = g.variant;
    }
    const double **hs = (const double **)(host.data() + scal_off);
    for (int i = 0; i < m; ++i) hs[i] = b->members[i]->h.scal;
    b->d_gather = (double *)(base + gather_off);
    b->d_scal = (const double **)(base + scal_off);
    b->table_epoch = b->member_epoch;
    b->tables_static = fixed != nullptr;
    if (hipMemcpyAsync(base, host.data(), off, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return batch_fail(b, LBKS_E_HIP, "batch table upload failed");
    if (!fixed && b->use_graph && !b->groups.empty()) {
        for (int bp = 0; bp < 2; ++bp) {
            if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return batch_fail(b, LBKS_E_HIP, "hipStreamBeginCapture failed");
            const int e = batch_enqueue_step(b, bp);
            const hipError_t ee = hipStreamEndCapture(b->stream, &b->graph[bp]);
            if (e || ee != hipSuccess) return batch_fail(b, LBKS_E_HIP, "graph capture of the batched step failed");
            if (hipGraphInstantiate(&b->exec[bp], b->graph[bp], nullptr, nullptr, 0) != hipSuccess)
                return batch_fail(b, LBKS_E_HIP, "hipGraphInstantiate failed");
        }
    }
    b->dirty = false;
    return 0;
}

}  // namespace

extern "C" int lbks_batch_create(const lbks_device *dev, lbks_batch **out)
{
    if (!out) return LBKS_E_INVAL;
    *out = nullptr;
    if (dev && ((dev->alloc == nullptr) != (dev->free == nullptr))) return LBKS_E_INVAL;
    lbks_batch *b = new lbks_batch();
    b->device = dev ? dev->device : 0;
    if (hipSetDevice(b->device) != hipSuccess) {
        delete b;
        return LBKS_E_HIP;
    }
    if (dev && dev->stream) {
        b->stream = (hipStream_t)dev->stream;
    } else {
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
            delete b;
            return LBKS_E_HIP;
        }
        b->own_stream = true;
    }
    if (dev) {
        b->ualloc = dev->alloc;
        b->ufree = dev->free;
        b->user = dev->user;
    }
    *out = b;
    return 0;
}

extern "C" void *lbks_batch_stream(const lbks_batch *b) { return b ? (void *)b->stream : nullptr; }

extern "C" int lbks_batch_attach(lbks_batch *b, lbks_ctx *c)
{
    if (!b || !c || c->batch) return LBKS_E_INVAL;
    if (c->stream != b->stream || c->device != b->device)
        return fail(c, LBKS_E_INVAL, "context must share the batch's stream and device");
    if (c->timing) return fail(c, LBKS_E_INVAL, "disable kernel timing before attaching to a batch");
    batch_commit(b);
    b->members.push_back(c);
    b->running.assign(b->members.size(), 1);
    c->batch = b;
    b->member_epoch += 1;
    b->dirty = true;
    return 0;
}

extern "C" int lbks_batch_detach(lbks_batch *b, lbks_ctx *c)
{
    if (!b || !c || c->batch != b) return LBKS_E_INVAL;
    (void)hipStreamSynchronize(b->stream);
    batch_commit(b);
    b->members.erase(std::remove(b->members.begin(), b->members.end(), c), b->members.end());
    b->running.assign(b->members.size(), 1);
    b->groups.clear();
    c->batch = nullptr;
    b->member_epoch += 1;
    b->dirty = true;
    return 0;
}

extern "C" int lbks_batch_size(const lbks_batch *b) { return b ? (int)b->members.size() : 0; }

namespace {

// The relaxation of lbks_batch_relax; with `fixed` every table build of this call
// goes to that workspace (lbks_batch_relax_static).
int batch_relax_impl(lbks_batch *b, int64_t max_steps, double dE_tol, int32_t check_every, int32_t *status,
                     int64_t *steps, void *fixed, size_t fixed_cap)
{
    const int m = (int)b->members.size();
    bool built = false;                 // tables built during this call
    auto build = [&]() -> int {
        const int e = batch_build(b, fixed, fixed_cap);
        if (!e) built = true;
        return e;
    };
    std::vector<int> st(m, LBKS_NOT_CONVERGED);
    std::vector<int64_t> done(m, 0);
    batch_commit(b);
    b->running.assign(m, 1);
    for (int i = 0; i < m; ++i)
        if (!b->members[i]->has_potential) {
            st[i] = LBKS_E_STATE;
            b->running[i] = 0;
        }
    b->dirty = true;
    if (check_every < 1) check_every = 1;
    std::vector<double> gat((size_t)GATHER_W * std::max(m, 1));
    // The gather reads the members' scalar blocks through the pointer table of the
    // last build; a relax that stepped nothing (max_steps == 0, no member with a
    // potential) or follows an attach or detach builds the table first.
    auto gather = [&]() -> int {
        // the static workspace is shared by every call on the device: its tables
        // are trusted only when built in this call
        if (!b->d_scal || b->table_epoch != b->member_epoch || b->tables_static != (fixed != nullptr) ||
            (fixed && !built)) {
            const int e = build();
            if (e) return e;
        }
        if (launch_gather(b->d_scal, m, GATHER_W, b->d_gather, b->stream)) return LBKS_E_HIP;
        if (hipMemcpyAsync(gat.data(), b->d_gather, sizeof(double) * GATHER_W * m, hipMemcpyDeviceToHost,
                           b->stream) != hipSuccess ||
            hipStreamSynchronize(b->stream) != hipSuccess)
            return LBKS_E_HIP;
        return 0;
    };
    int64_t t = 0;
    int rc = 0;
    while (t < max_steps) {
        bool any = false;
        for (int i = 0; i < m; ++i) any |= b->running[i] != 0;
        if (!any) break;
        if (b->dirty && (rc = build())) break;
        const int64_t n = std::min<int64_t>(check_every, max_steps - t);
        for (int64_t k = 0; k < n; ++k) {
            if (b->exec[b->bparity]) {
                if (hipGraphLaunch(b->exec[b->bparity], b->stream) != hipSuccess) {
                    rc = batch_fail(b, LBKS_E_HIP, "hipGraphLaunch failed");
                    break;
                }
            } else if (batch_enqueue_step(b, b->bparity)) {
                rc = batch_fail(b, LBKS_E_HIP, "batched step launch failed");
                break;
            }
            b->bparity ^= 1;
            b->epoch_steps += 1;
        }
        if (rc) break;
        t += n;
        for (int i = 0; i < m; ++i)
            if (b->running[i]) done[i] += n;
        if (dE_tol > 0.0) {
            for (const BatchGroup &g : b->groups)
                if (plan_energy(g.plan, b->stream)) rc = batch_fail(b, LBKS_E_HIP, "batched energy failed");
            if (rc || (rc = gather())) break;
            for (int i = 0; i < m; ++i) {
                if (!b->running[i]) continue;
                const double *e = &gat[(size_t)GATHER_W * i];
                const double etot = e[0], errf = e[GATHER_ERR];
                if (errf != 0.0 || !isfinite(etot)) {
                    st[i] = LBKS_E_NUMERIC;
                    b->running[i] = 0;
                    b->dirty = true;
                } else {
                    lbks_ctx *c = b->members[i];
                    if (rule_check(c, etot, e + 9, dE_tol)) {
                        st[i] = LBKS_OK;
                        b->running[i] = 0;
                        b->dirty = true;
                    }
                }
            }
        }
    }
    if (!rc && dE_tol <= 0.0 && m > 0 && !(rc = gather())) {
        for (int i = 0; i < m; ++i)
            if (b->running[i] && gat[(size_t)GATHER_W * i + GATHER_ERR] != 0.0) st[i] = LBKS_E_NUMERIC;
    }
    batch_commit(b);
    b->dirty = true;
    for (int i = 0; i < m; ++i) {
        if (status) status[i] = st[i];
        if (steps) steps[i] = done[i];
    }
    if (rc) g_create_error = b->err;    // lbks_last_error(NULL) reports a failed batch call
    return rc ? rc : m;
}

// Fixed device workspace of lbks_batch_relax_static.  Each GPU the library runs on
// holds its own copy until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[LBKS_STATIC_WORKSPACE_BYTES];
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;    // device -> address of that device's copy of `scratch`

// Address of `scratch` on device `dev`, which must be the current device (looked
// up once per device).
int scratch_address(int dev, void **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return 0;
    }
    void *ptr = nullptr;
    if (hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LBKS_E_HIP;
    g_scratch_ptr[dev] = ptr;
    *out = ptr;
    return 0;
}

}  // namespace

extern "C" int lbks_batch_relax(lbks_batch *b, int64_t max_steps, double dE_tol, int32_t check_every,
                                int32_t *status, int64_t *steps)
{
    if (!b) return LBKS_E_INVAL;
    return batch_relax_impl(b, max_steps, dE_tol, check_every, status, steps, nullptr, 0);
}

extern "C" int lbks_batch_relax_static(lbks_batch *b, int64_t max_steps, double dE_tol, int32_t check_every,
                                       int32_t *status, int64_t *steps)
{
    if (!b) return LBKS_E_INVAL;
    if (hipSetDevice(b->device) != hipSuccess) return LBKS_E_HIP;
    void *ws = nullptr;
    if (scratch_address(b->device, &ws)) {
        g_create_error = "hipGetSymbolAddress of the static workspace failed";
        return LBKS_E_HIP;
    }
    return batch_relax_impl(b, max_steps, dE_tol, check_every, status, steps, ws, LBKS_STATIC_WORKSPACE_BYTES);
}

extern "C" void lbks_batch_destroy(lbks_batch *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    batch_commit(b);
    for (lbks_ctx *c : b->members) c->batch = nullptr;
    batch_destroy_graphs(b);
    batch_free_mem(b);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}
