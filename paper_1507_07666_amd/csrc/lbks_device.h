// lbks_device.h -- device helpers shared by the kernel translation units of
// liblbks.so: the D3Q19 velocity set, workgroup-to-tile mapping, fixed-order
// reductions (wave butterfly, column sums, the matrix-core overlap partial),
// buffer and global-address-space access, local exchange-correlation, and the
// template dispatch on (precision, orbital bucket, orthogonalisation mode).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "lbks_kernels.h"

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

// linear = 1 keeps the dispatch order instead of the remap (update-kernel variant
// bit 2): the workgroups in flight then cover one window of tiles, so the many
// population streams each touch one region at a time; the neighbour-plane field
// reads are then split over the XCDs' L2s.  Which order is faster depends on the
// grid, so the autotuner decides.
__device__ __forceinline__ TileRef resolve(const int2 *table, int linear = 0)
{
    const int b = linear ? (int)blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
    if (table) {
        const int2 t = table[b];
        return {t.x, t.y};
    }
    return {0, b};
}

__host__ __device__ constexpr int pow2_ceil(int n) { return n <= 1 ? 1 : 2 * pow2_ceil((n + 1) / 2); }
__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

// One halving step of wave_reduce_scatter: lanes whose bit M is set keep the
// upper half of their W remaining elements, the others the lower half, and each
// adds the partner's (lane ^ M) copy of the half it keeps.
template <int W, int M, int P>
__device__ __forceinline__ void halve_step(double (&v)[P], int lane)
{
    if constexpr (W > 1) {
        const bool hi = (lane & M) != 0;
#pragma unroll
        for (int k = 0; k < W / 2; ++k) {
            const double keep = hi ? v[k + W / 2] : v[k];
            const double give = hi ? v[k] : v[k + W / 2];
            v[k] = keep + __shfl_xor(give, M, 64);
        }
        halve_step<W / 2, M / 2, P>(v, lane);
    }
}

// Element-wise sum of v[0..P) over the 64 lanes of a wave (P a power of two, at
// most 64) by recursive halving: log2 P exchange steps leave each lane one element
// summed over 64 / P lanes, which a butterfly over the remaining lane bits
// completes.  P - 1 + log2(64 / P) shuffles in all, against 6 P for a butterfly
// per element.  Lane l returns the total of element (l >> (6 - log2 P)) & (P - 1);
// the order of the additions is fixed.  v is overwritten.
template <int P>
__device__ __forceinline__ double wave_reduce_scatter(double (&v)[P])
{
    static_assert(P >= 1 && P <= 64 && (P & (P - 1)) == 0, "P must be a power of two <= 64");
    const int lane = threadIdx.x & 63;
    halve_step<P, 32, P>(v, lane);
    double x = v[0];
#pragma unroll
    for (int m = 32 / P; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    return x;
}

// Sum v[0..nv) over the workgroup; thread q < nv writes its total to out[q * stride].
// The wave sums go by chunks of up to 16 elements through wave_reduce_scatter,
// then the waves are added in order.
template <int NV>
__device__ __forceinline__ void block_sum_store(const double (&v)[NV], int nv, double *out, int stride)
{
    constexpr int C = pow2_ceil(NV < 16 ? NV : 16);   // elements per reduce-scatter
    constexpr int NCH = (NV + C - 1) / C;
    constexpr int SH = 6 - ilog2(C);                   // lane l holds element l >> SH of its chunk
    __shared__ double red[BS / 64][NCH * C];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        if (c * C < nv) {
            double t[C];
#pragma unroll
            for (int e = 0; e < C; ++e) t[e] = (c * C + e < NV) ? v[c * C + e] : 0.0;
            const double x = wave_reduce_scatter<C>(t);
            if ((lane & ((1 << SH) - 1)) == 0) red[wave][c * C + (lane >> SH)] = x;
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

// Grid of a finalize kernel: RG workgroups per instance.  Workgroup b serves
// instance list[b / RG] and takes group g of its tiles; g runs over the XCD of b
// in contiguous blocks, as the site kernels' tiles do.
struct GroupRef {
    int inst, g;
};

__device__ __forceinline__ GroupRef resolve_group(const int *list)
{
    const int b = (int)blockIdx.x;
    return {list ? list[b / RG] : b / RG, xcd_remap(b % RG, RG)};
}

// A global-memory view of a device pointer (loads become global_load, not flat).
// A flat load may be served by LDS or by memory, so before using its value the
// compiler waits for every outstanding load; global loads are counted in order,
// and several stay in flight.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gmem(const T *p)
{
    return (const __attribute__((address_space(1))) T *)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gmem(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}

// acc[c] += col[c * ntile + t] for c < NC and t = t0 + tid, t0 + tid + BS, ... < t1;
// the NC loads of a round are unconditional and in flight together.
template <int NC>
__device__ __forceinline__ void sum_tiles(const double *col, int ntile, int t0, int t1, double (&acc)[2 * RCH])
{
    const auto *g = gmem(col);
    for (int t = t0 + (int)threadIdx.x; t < t1; t += BS) {
        double v[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) v[c] = g[(size_t)c * ntile + t];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += v[c];
    }
}

// Column totals out[q] = sum_t part[q * ntile + t] (q < nq) of one instance's tile
// partials, in two levels within one launch of RG workgroups per instance.
// Workgroup g adds tiles [g ntile / RG, (g + 1) ntile / RG) of every column and
// stores the sums at g_part[q * RG + g]; the workgroup that finishes last (a
// device-scope counter, reset by that workgroup) adds the RG sums of each column
// in the order g = 0, 1, ..., leaves the totals in `out` (LDS) and returns true;
// the others return false.  Every addition is in a fixed order, so the totals do
// not depend on which workgroup finishes last.  No workgroup waits for another.
// The partial arrays hold whole chunks of RCH columns (unused ones stay zero).
// Every thread of the BS-wide workgroup must call this.
static __device__ bool reduce_columns(const double *__restrict__ part, int ntile, int nq, double *g_part,
                                      unsigned *count, int g, double *out)
{
    __shared__ double red[BS / 64][2 * RCH];
    __shared__ int last;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t0 = (int)((long long)ntile * g / RG), t1 = (int)((long long)ntile * (g + 1) / RG);
    const int ncol = padded_cols(nq);
    for (int q0 = 0; q0 < ncol; q0 += 2 * RCH) {
        const int nc = ncol - q0 < 2 * RCH ? ncol - q0 : 2 * RCH;   // RCH or 2 RCH
        const double *col = part + (size_t)q0 * ntile;
        double acc[2 * RCH];
#pragma unroll
        for (int c = 0; c < 2 * RCH; ++c) acc[c] = 0.0;
        if (nc == 2 * RCH) sum_tiles<2 * RCH>(col, ntile, t0, t1, acc);
        else sum_tiles<RCH>(col, ntile, t0, t1, acc);
        const double x = wave_reduce_scatter<2 * RCH>(acc);
        if ((lane & 3) == 0) red[wave][lane >> 2] = x;
        __syncthreads();
        if ((int)threadIdx.x < nc) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < BS / 64; ++w) s += red[w][threadIdx.x];
            g_part[(size_t)(q0 + threadIdx.x) * RG + g] = s;
        }
        __syncthreads();
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(count, 1u) == (unsigned)(RG - 1);
    __syncthreads();
    if (!last) return false;
    __threadfence();
    if ((int)threadIdx.x < nq) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < RG; ++k) s += g_part[(size_t)threadIdx.x * RG + k];
        out[threadIdx.x] = s;
    }
    if (threadIdx.x == 0) atomicExch(count, 0u);
    __syncthreads();
    return true;
}

// The totals of reduce_columns, bit for bit, summed by one workgroup alone, for
// an instance whose first-level groups hold at most L tiles (L <= 64, ntile <= RG
// L) and nq RG <= BS.  In reduce_columns a group then sits in the first wave
// alone: lane l holds 0 + part[t0 + l] (zero past the group), the wave adds its
// lanes pairwise over lane bit 5, then 4, ..., 0 (wave_reduce_scatter), and the
// zero sums of the other waves leave the group sum unchanged (x + 0 = x for every
// x but -0, which 0 + part never is).  Here thread (c, g) forms group g of column c
// by the same pairwise tree (pairs past lane L - 1 add zeros and are skipped),
// then thread c adds the RG group sums in the order g = 0, 1, ..., as the last
// workgroup of reduce_columns does.  Totals land in `out` (LDS; grp is LDS
// scratch of RG nq doubles); every thread of the workgroup must call this.
template <int L>
__device__ void fold_columns_l(const double *__restrict__ part, int ntile, int nq, double *grp, double *out)
{
    static_assert(L >= 1 && L <= 64 && (L & (L - 1)) == 0, "L must be a power of two <= 64");
    const int t = threadIdx.x;
    if (t < nq * RG) {
        const int c = t / RG, g = t % RG;
        const int t0 = (int)((long long)ntile * g / RG), t1 = (int)((long long)ntile * (g + 1) / RG);
        const auto *col = gmem(part) + (size_t)c * ntile + t0;
        double a[L];
#pragma unroll
        for (int l = 0; l < L; ++l) a[l] = t0 + l < t1 ? 0.0 + col[l] : 0.0;
#pragma unroll
        for (int b = L / 2; b >= 1; b >>= 1)
#pragma unroll
            for (int m = 0; m < b; ++m) a[m] += a[m + b];
        grp[c * RG + g] = 0.0 + a[0];
    }
    __syncthreads();
    if (t < nq) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < RG; ++k) s += grp[t * RG + k];
        out[t] = s;
    }
    __syncthreads();
}

// fold_columns_l with the smaller tree (8 or 16 tiles) that holds the longest
// group, ceil(ntile / RG) <= 16 tiles: a larger tree only adds zeros, so either
// gives the same totals, and the smaller one issues fewer loads.
__device__ __forceinline__ void fold_columns(const double *__restrict__ part, int ntile, int nq, double *out)
{
    __shared__ double grp[RG * RG];     // [column][group]: nq RG <= BS gives nq <= BS / RG = RG
    if ((ntile + RG - 1) / RG <= 8) fold_columns_l<8>(part, ntile, nq, grp, out);
    else fold_columns_l<16>(part, ntile, nq, grp, out);
}

// Coordinate of node i of n (the grid centred on the origin).  Here, in
// multipole_potential and in sor_node no multiply is fused into an add: each
// is inlined into several kernels, and the fusions the compiler finds depend on
// the code around it, so a value two kernels must agree on bit for bit (a ghost
// face written by one and recomputed by another) has to be computed the same way
// everywhere.
__device__ __forceinline__ double node_coord(int i, int n, double h)
{
#pragma clang fp contract(off)
    return ((double)i - 0.5 * (double)(n - 1)) * h;
}

// One successive over-relaxation update of V_H at a node from the sum of its six
// neighbours: V <- (1 - w) V + w (nb + 4 pi h^2 rho) / 6.
__device__ __forceinline__ double sor_node(double nb, double rho, double old, double h, double omega)
{
#pragma clang fp contract(off)
    const double four_pi_h2 = 4.0 * 3.14159265358979323846 * h * h;
    const double gs = (nb + four_pi_h2 * rho) / 6.0;
    return (1.0 - omega) * old + omega * gs;
}

__device__ __forceinline__ int npair_of(int n) { return n * (n + 1) / 2; }

// Orbital count inside a kernel instantiated for bucket NO: buckets 1..5 hold
// exactly NO orbitals, so the count is a compile-time constant there and every
// per-orbital guard folds away; buckets 8 and 16 read it from the descriptor.
template <int NO>
__device__ __forceinline__ int orbitals(const InstDesc &d)
{
    return NO <= 5 ? NO : d.n_orb;
}

// Global-memory views of descriptor pointers.  Buffers reached through the
// descriptor are generic pointers to the compiler, which would address every load
// with a 64-bit per-lane flat address; in the global address space a load is a
// scalar (uniform) plane base plus one 32-bit per-lane byte offset.
#define GAS __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ const GAS T *gplane(const void *base, long long elems)
{
    return (const GAS T *)base + elems;
}
template <typename T>
__device__ __forceinline__ GAS T *gplane_w(void *base, long long elems)
{
    return (GAS T *)base + elems;
}
template <typename T>
__device__ __forceinline__ const GAS T *at_bytes(const GAS T *plane, unsigned off_bytes)
{
    return (const GAS T *)((const GAS char *)plane + off_bytes);
}
template <typename T>
__device__ __forceinline__ GAS T *at_bytes_w(GAS T *plane, unsigned off_bytes)
{
    return (GAS T *)((GAS char *)plane + off_bytes);
}

// Buffer access: a plane is a scalar resource (base, byte range) and a node a
// 32-bit per-lane byte offset, so no per-load 64-bit address is formed.  An offset
// outside the plane's range reads 0 and drops stores (hardware range check).
constexpr int BUF_WORD3 = 0x00020000;   // gfx9-family raw buffer format word
constexpr int BUF_NT = 2;               // non-temporal (streaming) cache policy

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *base, long long elems, int elem_bytes,
                                                             unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((char *)base + elems * elem_bytes, 0, (int)bytes, BUF_WORD3);
}

template <typename T, int AUX>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, unsigned off)
{
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, AUX));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, AUX));
}

template <typename T, int AUX>
__device__ __forceinline__ void bstore(T v, __amdgpu_buffer_rsrc_t r, unsigned off)
{
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)), v), r, (int)off, 0, AUX);
    else
        __builtin_amdgcn_raw_buffer_store_b32(
            __builtin_bit_cast(decltype(__builtin_amdgcn_raw_buffer_load_b32(r, 0, 0, 0)), v), r, (int)off, 0, AUX);
}

// 16 bytes per lane: K = 16 / sizeof(T) x-consecutive nodes in one buffer access.
template <typename T, int K, int AUX>
__device__ __forceinline__ void bload16(T (&out)[K], __amdgpu_buffer_rsrc_t r, unsigned off)
{
    static_assert(K * sizeof(T) == 16, "16 bytes per lane");
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, AUX);
    __builtin_memcpy(out, &v, 16);
}
template <typename T, int K, int AUX>
__device__ __forceinline__ void bstore16(const T (&in)[K], __amdgpu_buffer_rsrc_t r, unsigned off)
{
    static_assert(K * sizeof(T) == 16, "16 bytes per lane");
    decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0)) v;
    __builtin_memcpy(&v, in, 16);
    __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)off, 0, AUX);
}

// A plane resource widened by PLANE_GUARD bytes on each side, for 16-byte loads
// at any element offset: a vector with at least one element inside the plane
// is then wholly in range (a hardware range check may drop a partly-outside
// access).  The guard bytes lie inside the context's one allocation (the planes
// that are read this way are neither its first nor its last buffer).
constexpr unsigned PLANE_GUARD = 256;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc_guarded(const void *base, long long elems, int elem_bytes,
                                                                     unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((char *)base + elems * elem_bytes - PLANE_GUARD, 0,
                                             (int)(bytes + 2 * PLANE_GUARD), BUF_WORD3);
}

typedef double v4d __attribute__((ext_vector_type(4)));

// Overlap partial of one workgroup, S_jk = sum over its nodes of psi_j psi_k
// (k <= j < n), as Phi^T Phi on the matrix cores: per wave the 64 nodes form 16
// blocks of 4, each one V_MFMA_F64_16X16X4F64 with Phi^T (16 orbitals x 4 nodes)
// as A and Phi as B; lane l, register r of the result holds S(l % 16, 4r + l / 16).
// The four waves are then summed in order; thread q < npair writes out[q * stride]
// in the packed order q = j (j + 1) / 2 + k.  Every thread must call this.
template <typename T, int NO>
__device__ void overlap_partial(const T (&acc)[NO], int n, double *out, int stride)
{
    __shared__ double phi[BS / 64][64][NO + 1];
    __shared__ double red[BS / 64][NO][NO];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 0; o < NO; ++o) phi[wave][lane][o] = (double)acc[o];
    __syncthreads();
    v4d S = {0.0, 0.0, 0.0, 0.0};
    const int o = lane & 15, k = lane >> 4;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const double a = o < NO ? phi[wave][4 * m + k][o] : 0.0;
        S = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, S, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int col = 4 * r + k;
        if (o < NO && col < NO) red[wave][o][col] = S[r];
    }
    __syncthreads();
    const int q = threadIdx.x;
    if (q < npair_of(n)) {
        int j = 0;
        while ((j + 1) * (j + 2) / 2 <= q) ++j;
        const int kk = q - j * (j + 1) / 2;
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < BS / 64; ++w) sum += red[w][j][kk];
        out[(size_t)q * stride] = sum;
    }
}

// Gradient-corrected exchange-correlation, spin-unpolarised, per volume, as a
// function of rho and sigma = |grad rho|^2: Becke 1988 exchange, per spin
// density n = rho/2 with x = |grad n| / n^(4/3),
//   e_s = -C n^(4/3) - beta n^(4/3) x^2 / (1 + 6 beta x asinh x),  total 2 e_s,
// and Lee-Yang-Parr 1988 correlation with its Laplacian terms integrated by
// parts, f_c = f0(rho) + f1(rho) sigma,
//   f0 = -a rho (1 + b C_F e^(-c u)) / (1 + d u),
//   f1 = a b rho^(-5/3) e^(-c u) / (1 + d u) (3 + 7 delta) / 72,
//   u = rho^(-1/3), delta = c u + d u / (1 + d u).
// Returns fx, fc and the derivatives of fx + fc with respect to rho (fr) and
// sigma (fs); all zero below the density floor.  polarised: every electron in one
// spin channel (n = rho, |grad n|^2 = sigma, a single e_s), where the
// Lee-Yang-Parr correlation vanishes.
static __device__ void gga_eval(double rho, double sigma, double floor, bool polarised, double &fx, double &fc,
                                double &fr, double &fs)
{
    fx = fc = fr = fs = 0.0;
    if (!(rho >= floor) || !(rho > 0.0)) return;
    const double PI = 3.14159265358979323846;
    if (polarised) {
        const double beta = 0.0042, C = 0.75 * cbrt(6.0 / PI);
        const double n13 = cbrt(rho), n43 = rho * n13;
        const double x = sqrt(sigma) / n43;
        const double as = asinh(x);
        const double q = 1.0 + 6.0 * beta * x * as;
        const double H = x * x / q;
        const double Hx = (2.0 * q - 6.0 * beta * x * (as + x / sqrt(1.0 + x * x))) / (q * q);   // H'(x) / x
        fx = -C * n43 - beta * n43 * H;
        fr = -(4.0 / 3.0) * n13 * (C + beta * (H - x * x * Hx));
        fs = -beta * Hx / (2.0 * n43);
        return;
    }
    // exchange
    const double beta = 0.0042, C = 0.75 * cbrt(6.0 / PI);
    const double n = 0.5 * rho, n13 = cbrt(n), n43 = n * n13;
    const double x = 0.5 * sqrt(sigma) / n43;
    const double as = asinh(x);
    const double q = 1.0 + 6.0 * beta * x * as;
    const double H = x * x / q;
    const double Hx = (2.0 * q - 6.0 * beta * x * (as + x / sqrt(1.0 + x * x))) / (q * q);   // H'(x) / x
    fx = 2.0 * (-C * n43 - beta * n43 * H);
    const double fx_r = -(4.0 / 3.0) * n13 * (C + beta * (H - x * x * Hx));
    const double fx_s = -beta * Hx / (4.0 * n43);
    // correlation
    const double a = 0.04918, b = 0.132, c = 0.2533, d = 0.349;
    const double CF = 0.3 * cbrt(9.0 * PI * PI * PI * PI);   // (3/10)(3 pi^2)^(2/3)
    const double u = 1.0 / cbrt(rho);
    const double ecu = exp(-c * u);
    const double den = 1.0 + d * u;
    const double num = 1.0 + b * CF * ecu;
    const double g = num / den;
    const double gp = (-b * CF * c * ecu * den - d * num) / (den * den);
    const double dl = c * u + d * u / den;
    const double A = u * u * u * u * u * ecu / den;                   // rho^(-5/3) e^(-cu) / (1 + du)
    const double f1 = a * b * A * (3.0 + 7.0 * dl) / 72.0;
    const double f1p = a * b * A / (216.0 * rho) * ((dl - 5.0) * (3.0 + 7.0 * dl) - 7.0 * u * (c + d / (den * den)));
    fc = -a * rho * g + f1 * sigma;
    const double fc_r = -a * (g - (u / 3.0) * gp) + f1p * sigma;
    fr = fx_r + fc_r;
    fs = fx_s + f1;
}

// Local exchange-correlation per electron (e*) and potential (v* = d(rho e*)/d rho):
// Slater exchange; correlation of Lee-Yang-Parr at zero gradient,
// e_c = -a (1 + b C_F exp(-c u)) / (1 + d u), u = rho^(-1/3); or Perdew-Zunger 1981.
static __device__ void xc_eval(int kind, double rho, double floor, double &ex, double &ec, double &vx,
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


static inline int grid_site(const Plan &pl) { return pl.tt.site ? pl.tt.n_site : pl.ntile; }
static inline int grid_ghost(const Plan &pl) { return pl.tt.ghost ? pl.tt.n_ghost : pl.ntile_ghost; }
static inline int grid_sor(const Plan &pl) { return pl.tt.sor ? pl.tt.n_sor : pl.ntile_sor; }
static inline int grid_brick(const Plan &pl) { return pl.tt.brick ? pl.tt.n_brick : pl.nbrick[pl.variant & 3]; }
static inline int grid_inst(const Plan &pl) { return pl.tt.inst ? pl.tt.n_inst : 1; }
static inline int grid_group(const Plan &pl) { return RG * grid_inst(pl); }

#define LAUNCH_CHECK() return (int)hipGetLastError()

}  // namespace lbks
