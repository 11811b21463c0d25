// lbks_collide.hip -- the lattice Boltzmann update kernels (stream-collide of
// the populations, and the equivalent omega = 1 update of the orbital fields),
// each compiled in four variants for the autotuner: overlap partial by wave
// butterfly or on the matrix cores, and compiler-chosen or 8-wave occupancy.
#include "lbks_device.h"

namespace lbks {

// --------------------------------------------------------- stream-collide

// Pull form of the lattice Boltzmann equation with the orthogonalisation and
// potential sources: the population entering node r along v_p is the
// post-collision population of r - v_p,
//   f_jp(r; t+1) = (1 - omega) g_jp + omega xi_p psi*_j - dt chi_p V psi_hat_j  at r - v_p,
// g_jp = sum_{l<=j} f_lp C_lj, and zero when r - v_p is outside the box.  The new
// moment psi_j = sum_p f_jp and the overlap partials psi_j psi_k are fused.
// Variant bits: 1 = overlap partial on the matrix cores (else wave butterfly),
// 2 = ask the compiler for 8 waves per SIMD (else its own register budget),
// 4 = workgroups in dispatch order (else the XCD remap); bit 4 is a kernel argument.
template <int V>
__device__ __forceinline__ constexpr int waves_hint() { return (V & 2) ? 8 : 1; }

template <typename T, int NO, int V>
__device__ __forceinline__ void overlap_partial_v(const T (&acc)[NO], int n, double *out, int stride)
{
    if constexpr (V & 1) {
        overlap_partial<T, NO>(acc, n, out, stride);
    } else {
        double prod[NO * (NO + 1) / 2];
        int q = 0;
#pragma unroll
        for (int j = 0; j < NO; ++j)
#pragma unroll
            for (int k = 0; k <= j; ++k) prod[q++] = (double)acc[j] * (double)acc[k];
        block_sum_store(prod, npair_of(n), out, stride);
    }
}

template <typename T, int NO, bool W, int V>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(waves_hint<V>(), 8))) void k_stream_collide(const InstDesc *__restrict__ descs,
                                                       const int2 *__restrict__ tiles, int parity, int linear)
{
    const TileRef tr = resolve(tiles, linear);
    const InstDesc &d = descs[tr.inst];
    const int n = orbitals<NO>(d);
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const long long N = d.nsite;
    const unsigned plane = (unsigned)N * (unsigned)sizeof(T);
    const int s = tr.tile * BS + threadIdx.x;
    const bool valid = s < d.nsite;
    const void *fs = parity ? d.f1 : d.f0;
    void *fd = parity ? d.f0 : d.f1;
    const T a = (T)(1.0 - d.omega);
    const T om = (T)d.omega;
    const T dt = (T)d.dt;
    T c[NO][NO];
#pragma unroll
    for (int l = 0; l < NO; ++l)
#pragma unroll
        for (int j = 0; j < NO; ++j) c[l][j] = (T)d.C[l * MAXO + j];
    const int x = s % nx, yz = s / nx, y = yz % ny, z = yz / ny;
    const unsigned off = (unsigned)s * (unsigned)sizeof(T);
    T acc[NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) acc[j] = (T)0;
#pragma unroll
    for (int p = 0; p < Q; ++p) {
        const int vx = VX(p), vy = VY(p), vz = VZ(p);
        const bool ok = valid && (unsigned)(x - vx) < (unsigned)nx && (unsigned)(y - vy) < (unsigned)ny &&
                        (unsigned)(z - vz) < (unsigned)nz;
        // byte offset of the source node r - v_p; when it falls outside the box the
        // loads are discarded by `ok` (and read 0 if beyond the plane)
        const unsigned src = off - (unsigned)((vx + nx * (vy + ny * vz)) * (int)sizeof(T));
        // every load of this direction is issued before its first store: the
        // compiler cannot reorder buffer loads above buffer stores, and a wait
        // for a load issued after a store also waits for the store
        T fl[NO], hat[NO], star[NO];
#pragma unroll
        for (int l = 0; l < NO; ++l)
            fl[l] = (l < n) ? bload<T, BUF_NT>(plane_rsrc(fs, ((long long)l * Q + p) * N, sizeof(T), plane), src)
                            : (T)0;
        const T vn = bload<T, 0>(plane_rsrc(d.V, 0, sizeof(T), plane), src);
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            hat[j] = (j < n) ? bload<T, 0>(plane_rsrc(d.psihat, (long long)j * N, sizeof(T), plane), src) : (T)0;
            star[j] = (W && j < n) ? bload<T, 0>(plane_rsrc(d.psistar, (long long)j * N, sizeof(T), plane), src)
                                   : (T)0;
        }
        const T cp = om * (T)d.xi[p];
        const T dp = dt * (T)d.chi[p] * vn;
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            if (j < n) {
                T o;
                if (W) {
                    o = a * (c[j][j] * fl[j]) + cp * star[j] - dp * hat[j];
                } else {
                    T g = (T)0;
#pragma unroll
                    for (int l = 0; l <= j; ++l) g += c[l][j] * fl[l];
                    o = a * g + (cp - dp) * hat[j];
                }
                o = ok ? o : (T)0;
                // populations are read once per step: stream them past the caches
                bstore<T, BUF_NT>(o, plane_rsrc(fd, ((long long)j * Q + p) * N, sizeof(T), plane), off);
                acc[j] += o;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NO; ++j)
        if (j < n) bstore<T, 0>(acc[j], plane_rsrc(d.psi, (long long)j * N, sizeof(T), plane), off);
    overlap_partial_v<T, NO, V>(acc, n, d.s_part + tr.tile, d.ntile);
}

// The same update with K = 16 / sizeof(T) x-consecutive nodes per lane (2 in FP64, 4
// in FP32): for a run of consecutive flat nodes the pull sources along v_p are the
// same run shifted by the uniform flat offset d_p = v_px + nx (v_py + ny v_pz), so one
// 16-byte access per plane serves the lane (at any element offset; planes are read
// through guarded resources).  Workgroup w covers K node tiles; its overlap partial
// goes to tile slot K w and the other K - 1 slots are zeroed.  The arithmetic per
// node is that of k_stream_collide.  Variant bit 2 (dispatch order) applies, bit 0
// rolls the loop over the directions; the overlap partial is always the
// wave-halving form.
template <typename T, int NO, bool W, bool ROLL>
__global__ __launch_bounds__(BS) void k_stream_collide_wide(const InstDesc *__restrict__ descs,
                                                            const int2 *__restrict__ tiles, int parity, int linear)
{
    constexpr int K = 16 / (int)sizeof(T);
    const TileRef tr = resolve(tiles, linear);
    const InstDesc &d = descs[tr.inst];
    const int n = orbitals<NO>(d);
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const long long N = d.nsite;
    const unsigned plane = (unsigned)N * (unsigned)sizeof(T);
    const int s0 = (tr.tile * BS + (int)threadIdx.x) * K;
    const bool whole = s0 + K <= d.nsite;           // all K nodes inside the grid
    const void *fs = parity ? d.f1 : d.f0;
    void *fd = parity ? d.f0 : d.f1;
    const T a = (T)(1.0 - d.omega);
    const T om = (T)d.omega;
    const T dt = (T)d.dt;
    T c[NO][NO];
#pragma unroll
    for (int l = 0; l < NO; ++l)
#pragma unroll
        for (int j = 0; j < NO; ++j) c[l][j] = (T)d.C[l * MAXO + j];
    int xs[K], ys[K], zs[K];
    bool valid[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const int s = s0 + i;
        valid[i] = s < d.nsite;
        xs[i] = s % nx;
        const int yz = s / nx;
        ys[i] = yz % ny;
        zs[i] = yz / ny;
    }
    const unsigned off = (unsigned)s0 * (unsigned)sizeof(T);
    T acc[NO][K];
#pragma unroll
    for (int j = 0; j < NO; ++j)
#pragma unroll
        for (int i = 0; i < K; ++i) acc[j][i] = (T)0;
    auto direction = [&](int p) {
        const int vx = VX(p), vy = VY(p), vz = VZ(p);
        bool ok[K];
#pragma unroll
        for (int i = 0; i < K; ++i)
            ok[i] = valid[i] && (unsigned)(xs[i] - vx) < (unsigned)nx && (unsigned)(ys[i] - vy) < (unsigned)ny &&
                    (unsigned)(zs[i] - vz) < (unsigned)nz;
        // guarded byte offset of the source run r - v_p (modulo 2^32: a run wholly
        // before the plane wraps far out of range and reads zeros, discarded by ok)
        const unsigned src = off + PLANE_GUARD - (unsigned)((vx + nx * (vy + ny * vz)) * (int)sizeof(T));
        T fl[NO][K], hat[NO][K], star[NO][K], vn[K];
#pragma unroll
        for (int l = 0; l < NO; ++l) {
            if (l < n) bload16<T, K, BUF_NT>(fl[l], plane_rsrc_guarded(fs, ((long long)l * Q + p) * N, sizeof(T), plane), src);
            else
#pragma unroll
                for (int i = 0; i < K; ++i) fl[l][i] = (T)0;
        }
        bload16<T, K, 0>(vn, plane_rsrc_guarded(d.V, 0, sizeof(T), plane), src);
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            if (j < n) bload16<T, K, 0>(hat[j], plane_rsrc_guarded(d.psihat, (long long)j * N, sizeof(T), plane), src);
            if (W && j < n) bload16<T, K, 0>(star[j], plane_rsrc_guarded(d.psistar, (long long)j * N, sizeof(T), plane), src);
        }
        const T cp = om * (T)d.xi[p];
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            if (j < n) {
                T o[K];
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    const T dp = dt * (T)d.chi[p] * vn[i];
                    T v;
                    if (W) {
                        v = a * (c[j][j] * fl[j][i]) + cp * star[j][i] - dp * hat[j][i];
                    } else {
                        T g = (T)0;
#pragma unroll
                        for (int l = 0; l <= j; ++l) g += c[l][j] * fl[l][i];
                        v = a * g + (cp - dp) * hat[j][i];
                    }
                    o[i] = ok[i] ? v : (T)0;
                    acc[j][i] += o[i];
                }
                const auto rd = plane_rsrc(fd, ((long long)j * Q + p) * N, sizeof(T), plane);
                if (whole) {
                    bstore16<T, K, BUF_NT>(o, rd, off);
                } else {
#pragma unroll
                    for (int i = 0; i < K; ++i)
                        if (valid[i]) bstore<T, BUF_NT>(o[i], rd, off + (unsigned)(i * (int)sizeof(T)));
                }
            }
        }
    };
    // unrolled, the compiler overlaps the directions but keeps a whole workgroup's
    // worth of registers per wave (one wave per SIMD); rolled, four waves per SIMD
    // keep more loads in flight
    if constexpr (ROLL) {
#pragma unroll 1
        for (int p = 0; p < Q; ++p) direction(p);
    } else {
#pragma unroll
        for (int p = 0; p < Q; ++p) direction(p);
    }
#pragma unroll
    for (int j = 0; j < NO; ++j) {
        if (j < n) {
            const auto rp = plane_rsrc(d.psi, (long long)j * N, sizeof(T), plane);
            if (whole) {
                bstore16<T, K, 0>(acc[j], rp, off);
            } else {
#pragma unroll
                for (int i = 0; i < K; ++i)
                    if (valid[i]) bstore<T, 0>(acc[j][i], rp, off + (unsigned)(i * (int)sizeof(T)));
            }
        }
    }
    double prod[NO * (NO + 1) / 2];
    {
        int q = 0;
#pragma unroll
        for (int j = 0; j < NO; ++j)
#pragma unroll
            for (int k = 0; k <= j; ++k) {
                double sum = 0.0;
#pragma unroll
                for (int i = 0; i < K; ++i) sum += (double)acc[j][i] * (double)acc[k][i];
                prod[q++] = sum;
            }
    }
    const int slot = tr.tile * K;
    block_sum_store(prod, npair_of(n), d.s_part + slot, d.ntile);
    if ((int)threadIdx.x < npair_of(n))
        for (int t = slot + 1; t < slot + K && t < d.ntile; ++t) d.s_part[(size_t)threadIdx.x * d.ntile + t] = 0.0;
}

// omega = 1 without populations: psi_j(r) <- sum_p [xi_p psi*_j - dt chi_p V psi_hat_j](r - v_p),
// exactly the moment of the population update at omega = 1.
template <typename T, int NO, bool W, int V>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(waves_hint<V>(), 8))) void k_collapsed(const InstDesc *__restrict__ descs,
                                                  const int2 *__restrict__ tiles, int linear)
{
    const TileRef tr = resolve(tiles, linear);
    const InstDesc &d = descs[tr.inst];
    const int n = orbitals<NO>(d);
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
        if (d.active != ~0u) {                      // sequential order: frozen orbitals keep their fields
#pragma unroll
            for (int j = 0; j < NO; ++j)
                if (j < n && !((d.active >> j) & 1u)) acc[j] = psi[(size_t)j * N + s];
        }
#pragma unroll
        for (int j = 0; j < NO; ++j)
            if (j < n) psi[(size_t)j * N + s] = acc[j];
    }
    overlap_partial_v<T, NO, V>(acc, n, d.s_part + tr.tile, d.ntile);
}

// The same omega = 1 update (Gram-Schmidt mode, psi* = psi_hat) with the fields
// staged in LDS: a workgroup owns a brick of BX x BY nodes in x, y and marches
// over DZ planes in z (DZ = 8, 12, 16 or 24, the brick variant).  Each plane of
// psi_hat_j and V, with a one-node halo, goes through one of two LDS slots (the
// plane after it is fetched into registers meanwhile), and each thread reads the
// 3 x 3 neighbourhood of its column in that plane once: the in-plane terms go to
// the output node in the same plane, the terms with v_z = +-1 (the five offsets
// of the plus shape) to the nodes above and below, held in a register queue of
// three output planes.  An output plane is complete, and written, once the plane
// above it has been read: 9 x (NO + 1) LDS reads per plane instead of 19 per
// field and node.  Terms from outside the box are exact zeros in LDS.  The
// overlap partial of the brick (psi_j psi_k summed over its nodes in FP64, the
// planes in order) goes to tile slot b when the instance has no more bricks of
// the shallowest depth than node tiles (the slots from the brick count on are zeroed by the
// bricks in turn); otherwise k_overlap_psi writes the partials.
template <typename T, int NO, int DZ>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_collapsed_brick(const InstDesc *__restrict__ descs,
                                                        const int2 *__restrict__ bricks, int linear)
{
    constexpr int PX = BX + 2, PY = BY + 2, PL = PX * PY;
    constexpr int NL = (PL + BS - 1) / BS;         // plane positions per thread
    __shared__ T lds[2][NO + 1][PL];              // psi_hat_0 .. psi_hat_{NO-1}, V; two plane slots
    const TileRef tr = resolve(bricks, linear);
    const InstDesc &d = descs[tr.inst];
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    const int gx = (nx + BX - 1) / BX, gy = (ny + BY - 1) / BY;
    const int nb = bricks_of(nx, ny, nz, DZ);
    const int b = tr.tile;
    if (b >= nb) return;                           // uniform per workgroup, before any barrier
    const int x0 = (b % gx) * BX, y0 = ((b / gx) % gy) * BY, z0 = (b / (gx * gy)) * DZ;
    const int zlast = min(z0 + DZ, nz) - 1;        // last output plane of the brick
    const int tx = threadIdx.x % BX, ty = threadIdx.x / BX;
    const int x = x0 + tx, y = y0 + ty;
    const bool mine = x < nx && y < ny;
    const size_t N = (size_t)d.nsite;
    const auto *__restrict__ ph = gmem((const T *)d.psihat);
    const auto *__restrict__ Vp = gmem((const T *)d.V);
    auto *psi = gmem((T *)d.psi);
    // the weights by speed class (|v_p|^2 = 0, 1, 2: velocities 0, 1, 7), and dt chi
    // formed as the node kernel forms it
    T cxi[3], cdc[3];
    {
        const T dt = (T)d.dt;
        const int rep[3] = {0, 1, 7};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cxi[c] = (T)d.xi[rep[c]];
            cdc[c] = dt * (T)d.chi[rep[c]];
        }
    }
    // one plane (zero outside the box) into registers, then into an LDS slot
    T pre[NL][NO + 1];
    auto fetch = [&](int z) {
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int i = (int)threadIdx.x + q * BS;
            const int lx = x0 - 1 + i % PX, ly = y0 - 1 + i / PX;
            const bool in = i < PL && z >= 0 && z < nz && lx >= 0 && lx < nx && ly >= 0 && ly < ny;
            const size_t g = in ? ((size_t)z * ny + ly) * nx + lx : 0;
#pragma unroll
            for (int j = 0; j < NO; ++j) pre[q][j] = in ? ph[(size_t)j * N + g] : (T)0;
            pre[q][NO] = in ? Vp[g] : (T)0;
        }
    };
    auto store = [&](int slot) {
#pragma unroll
        for (int q = 0; q < NL; ++q) {
            const int i = (int)threadIdx.x + q * BS;
            if (i < PL)
#pragma unroll
                for (int j = 0; j <= NO; ++j) lds[slot][j][i] = pre[q][j];
        }
    };
    // register queue: lo = output plane zp - 1 (complete after plane zp), mid = zp, hi = zp + 1
    T lo[NO], mid[NO], hi[NO];
#pragma unroll
    for (int j = 0; j < NO; ++j) lo[j] = mid[j] = hi[j] = (T)0;
    double prod[NO * (NO + 1) / 2];
#pragma unroll
    for (int q = 0; q < NO * (NO + 1) / 2; ++q) prod[q] = 0.0;
    fetch(z0 - 1);
    for (int zp = z0 - 1; zp <= zlast + 1; ++zp) {
        const int slot = (zp - z0 + 1) & 1;
        store(slot);                                // this slot was last read two planes ago
        if (zp <= zlast) fetch(zp + 1);             // in flight while this plane is read
        __syncthreads();
        if (mine) {
#pragma unroll
            for (int oy = -1; oy <= 1; ++oy) {
                // one row of three offsets at a time: no LDS read moves across rows (register
                // pressure), and no inner loop whose registers would be shuffled around the
                // plane in flight (which would wait for it)
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int ox = -1; ox <= 1; ++ox) {
                    // the departure node (x + ox, y + oy) of the velocities (-ox, -oy, v_z)
                    const int li = (ty + 1 + oy) * PX + (tx + 1 + ox);
                    const T vn = lds[slot][NO][li];
                    const int c = ox * ox + oy * oy;
                    const T w0 = cxi[c] - cdc[c] * vn;           // v_z = 0: the node in this plane
                    if (c <= 1) {
                        const T w1 = cxi[c + 1] - cdc[c + 1] * vn;   // v_z = +1 above, v_z = -1 below
#pragma unroll
                        for (int j = 0; j < NO; ++j) {
                            const T u = lds[slot][j][li];
                            mid[j] += w0 * u;
                            hi[j] += w1 * u;
                            lo[j] += w1 * u;
                        }
                    } else {
#pragma unroll
                        for (int j = 0; j < NO; ++j) mid[j] += w0 * lds[slot][j][li];
                    }
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            const int z = zp - 1;
            if (z >= z0) {                          // output plane z is complete
                const size_t s = ((size_t)z * ny + y) * nx + x;
                if (d.active != ~0u) {              // sequential order: frozen orbitals keep their fields
#pragma unroll
                    for (int j = 0; j < NO; ++j)
                        if (!((d.active >> j) & 1u)) lo[j] = psi[(size_t)j * N + s];
                }
#pragma unroll
                for (int j = 0; j < NO; ++j) psi[(size_t)j * N + s] = lo[j];
                int q = 0;
#pragma unroll
                for (int j = 0; j < NO; ++j)
#pragma unroll
                    for (int kk = 0; kk <= j; ++kk) prod[q++] += (double)lo[j] * (double)lo[kk];
            }
#pragma unroll
            for (int j = 0; j < NO; ++j) {
                lo[j] = mid[j];
                mid[j] = hi[j];
                hi[j] = (T)0;
            }
        }
    }
    if (brick_partials(d.ntile, d.ntile_brick)) {   // uniform per workgroup
        const int np = NO * (NO + 1) / 2;
        block_sum_store(prod, np, d.s_part + b, d.ntile);
        if ((int)threadIdx.x < np)
            for (int t = nb + b; t < d.ntile; t += nb) d.s_part[(size_t)threadIdx.x * d.ntile + t] = 0.0;
    }
}

template <int V>
static int launch_stream_collide_v(const Plan &pl, int parity, hipStream_t st)
{
    return dispatch_tnw(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_stream_collide<typename TG::T, TG::NO, TG::W, V><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site, parity,
                                                                                       (pl.variant >> 2) & 1);
        LAUNCH_CHECK();
    });
}

template <int V>
static int launch_collapsed_v(const Plan &pl, hipStream_t st)
{
    return dispatch_tnw(pl, [&](auto tg) {
        using TG = decltype(tg);
        k_collapsed<typename TG::T, TG::NO, TG::W, V><<<grid_site(pl), BS, 0, st>>>(pl.d_desc, pl.tt.site, (pl.variant >> 2) & 1);
        LAUNCH_CHECK();
    });
}

// Wide form (variant bit 3) for buckets of at most five orbitals; larger buckets
// take the node-per-lane kernel of the other bits.
static int launch_stream_collide_wide(const Plan &pl, int parity, hipStream_t st)
{
    return dispatch_tnw(pl, [&](auto tg) {
        using TG = decltype(tg);
        if constexpr (TG::NO <= 5) {
            constexpr int K = 16 / (int)sizeof(typename TG::T);
            const int grid = pl.tt.site_w ? pl.tt.n_site_w : (pl.ntile + K - 1) / K;
            const int linear = (pl.variant >> 2) & 1;
            if (pl.variant & 1)
                k_stream_collide_wide<typename TG::T, TG::NO, TG::W, true><<<grid, BS, 0, st>>>(pl.d_desc, pl.tt.site_w,
                                                                                               parity, linear);
            else
                k_stream_collide_wide<typename TG::T, TG::NO, TG::W, false><<<grid, BS, 0, st>>>(pl.d_desc, pl.tt.site_w,
                                                                                                parity, linear);
            return (int)hipGetLastError();
        } else {
            return (int)hipErrorInvalidValue;
        }
    });
}

bool stream_collide_is_wide(const Plan &pl) { return (pl.variant & 8) && pl.no <= 5; }

int launch_stream_collide(const Plan &pl, int parity, hipStream_t st)
{
    if (stream_collide_is_wide(pl)) return launch_stream_collide_wide(pl, parity, st);
    switch (pl.variant & 3) {
    case 0: return launch_stream_collide_v<0>(pl, parity, st);
    case 1: return launch_stream_collide_v<1>(pl, parity, st);
    case 2: return launch_stream_collide_v<2>(pl, parity, st);
    default: return launch_stream_collide_v<3>(pl, parity, st);
    }
}

// Gram-Schmidt mode with at most five orbitals: the LDS-staged brick update (with
// the overlap partials, or followed by them), its depth (variant bits 0 and 1) and
// workgroup order (bit 2) autotuned; otherwise the node-per-thread update with the
// fused overlap partials, in the autotuned variant.
bool collapsed_uses_bricks(const Plan &pl) { return !pl.wmode && pl.no <= 5; }

int launch_collapsed_update(const Plan &pl, hipStream_t st)
{
    if (collapsed_uses_bricks(pl)) {
        const int linear = (pl.variant >> 2) & 1;
        const int e = dispatch_tn(pl, [&](auto tg) {
            using TG = decltype(tg);
            if constexpr (TG::NO <= 5) {
                using T = typename TG::T;
                const int g = grid_brick(pl);
                switch (brick_depth(pl.variant)) {
                case 8: k_collapsed_brick<T, TG::NO, 8><<<g, BS, 0, st>>>(pl.d_desc, pl.tt.brick, linear); break;
                case 12: k_collapsed_brick<T, TG::NO, 12><<<g, BS, 0, st>>>(pl.d_desc, pl.tt.brick, linear); break;
                case 16: k_collapsed_brick<T, TG::NO, 16><<<g, BS, 0, st>>>(pl.d_desc, pl.tt.brick, linear); break;
                default: k_collapsed_brick<T, TG::NO, 24><<<g, BS, 0, st>>>(pl.d_desc, pl.tt.brick, linear); break;
                }
                return (int)hipGetLastError();
            } else {
                return (int)hipErrorInvalidValue;
            }
        });
        if (e) return e;
        return pl.brick_partials ? 0 : launch_overlap_psi(pl, st, true);
    }
    switch (pl.variant & 3) {
    case 0: return launch_collapsed_v<0>(pl, st);
    case 1: return launch_collapsed_v<1>(pl, st);
    case 2: return launch_collapsed_v<2>(pl, st);
    default: return launch_collapsed_v<3>(pl, st);
    }
}

}  // namespace lbks
