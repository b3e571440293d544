// gfx950 ray-march library for the DART-Ray V2 radiative-transfer method
// (Natale et al. 2017, arXiv:1709.03802): host API and kernels.
//
// Data layout on the device:
//  * leaves: one 64-byte record per leaf (int4 box: lower corner in
//    finest-level cell units and span; rho; 1/(V c); six face-neighbour
//    codes); positions along rays are in finest-level cell units so that cell
//    faces and source-cell centres are exact, and ray geometry is FP64;
//  * locator: one code per root cell and 8 codes per internal octree node;
//    code >= 0 is an internal node, code < 0 is leaf -code-1;
//  * energy-density accumulators: FP64, [cell][wavelength];
//  * S arrays: one block per wavelength, [cell][HEALPix nested pixel].
//
// Fixed-Nside passes bin the energy-density deposits by ray direction
// (ubar[r][c][l], wavelength fastest); because every ray of direction r
// shares the phase-function row w(.|r), the scattered source function follows
// exactly from S[l][c][p] = albedo c alpha V * sum_r ubar[r][c][l] w_l(p|r),
// computed by a flush kernel after each batch of directions.  One row of
// accumulates per crossing replaces the N_pix accumulates per wavelength of a
// direct deposit.  Adaptive rays have no fixed direction set: their passes
// that scatter light log (cell, direction, deposit) tuples, sort them by cell
// and expand each cell's tuples over the pixels in registers.

#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "dr_internal.h"

#define DR_VERSION "dartray-gfx950 0.1"

namespace dr {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg)
{
    set_error(msg);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return DARTRAY_E_DEVICE;
}

#define DR_HIP(call)                                        \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(e_, #call);   \
    } while (0)

#define DR_LAUNCH_CHECK(what)                               \
    do {                                                    \
        hipError_t e_ = hipGetLastError();                  \
        if (e_ != hipSuccess) return hip_fail(e_, what);    \
    } while (0)

// ---------------------------------------------------------------------------
// Small utility kernels
// ---------------------------------------------------------------------------

template <typename T>
__global__ void k_fill(T *p, size_t n, T v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
static int fill(Grid &g, T *p, size_t n, T v)
{
    if (n == 0) return DARTRAY_OK;
    unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks), dim3(256), 0, g.stream, p, n, v);
    DR_LAUNCH_CHECK("fill");
    return DARTRAY_OK;
}

__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline uint64_t wave_sum_u64(uint64_t v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// block-wide FP64 sum (blockDim.x multiple of 64, <= 1024); result valid in thread 0
__device__ inline double block_sum(double v, double *sh)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
    __syncthreads();
    return r;
}

__device__ inline void atomic_add_f32(float *p, float v)
{
    unsafeAtomicAdd(p, v);
}

__device__ inline void atomic_add_f64(double *p, double v)
{
    unsafeAtomicAdd(p, v);
}

// ---------------------------------------------------------------------------
// Direction and phase tables (FP64 on the device, rounded to FP32)
// ---------------------------------------------------------------------------

struct Frame {
    double R[9];
};

// Nside of table entry e (entry 4 (N^2 - 1) + pix): the largest N with 4 (N^2 - 1) <= e
__host__ __device__ inline int64_t entry_nside(int64_t e)
{
    int64_t N = 1;
    while (4 * (4 * N * N - 1) <= e) N *= 2;
    return N;
}

__host__ __device__ inline int64_t entry_of(int64_t nside, int64_t pix) { return 4 * (nside * nside - 1) + pix; }

__global__ void k_dir_all(float4 *dirs, double4 *dirs64, int64_t total, Frame f)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int64_t N = entry_nside(e);
    double v[3];
    dr_pix_vec(N, e - entry_of(N, 0), f.R, v);
    dirs[e] = make_float4((float)v[0], (float)v[1], (float)v[2], 0.f);
    dirs64[e] = make_double4(v[0], v[1], v[2], 0.0);
}

__global__ void k_sca64(double *out, Frame f)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kScaDirs) return;
    const int64_t N = entry_nside(e);
    dr_pix_vec(N, e - entry_of(N, 0), f.R, out + 3 * e);
}

__device__ inline double hg_phase(double g, double mu)
{
    const double den = 1.0 + g * g - 2.0 * g * mu;
    return (1.0 - g * g) / (4.0 * kPi * den * sqrt(den));
}

// w_l(p | n_r) = Phi_l(n_p . n_r) / sum_q Phi_l(n_q . n_r), one thread per (r, l)
__global__ void k_wtab(float *wtab, const LambdaTable *lt, const double *sca64, int nside_ray, int64_t nray,
                       int w_row, Frame f)
{
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int nl = lt->n_lambda;
    if (idx >= nray * nl) return;
    const int64_t r = idx / nl;
    const int l = (int)(idx - r * nl);
    double n[3];
    dr_pix_vec(nside_ray, r, f.R, n);
    const int ns = lt->nside_sca[l];
    const int npix = lt->npix[l];
    const double g = lt->g[l];
    const double *v = sca64 + 3 * entry_of(ns, 0);
    double sum = 0.0;
    for (int p = 0; p < npix; ++p) sum += hg_phase(g, v[3 * p] * n[0] + v[3 * p + 1] * n[1] + v[3 * p + 2] * n[2]);
    float *row = wtab + r * (int64_t)w_row + lt->w_off[l];
    for (int p = 0; p < npix; ++p)
        row[p] = (float)(hg_phase(g, v[3 * p] * n[0] + v[3 * p + 1] * n[1] + v[3 * p + 2] * n[2]) / sum);
}

// 1 / sum_p Phi_l(n_p . n_e) for every table entry e from e0 on, in FP64
__global__ void k_invz(float *invz, const LambdaTable *lt, const double *sca64, int64_t e0, int64_t total, Frame f)
{
    const int64_t e = e0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int64_t N = entry_nside(e);
    double n[3];
    dr_pix_vec(N, e - entry_of(N, 0), f.R, n);
    const int nl = lt->n_lambda;
    for (int l = 0; l < nl; ++l) {
        const double *v = sca64 + 3 * entry_of(lt->nside_sca[l], 0);
        const double g = lt->g[l];
        double sum = 0.0;
        for (int p = 0; p < lt->npix[l]; ++p)
            sum += hg_phase(g, v[3 * p] * n[0] + v[3 * p + 1] * n[1] + v[3 * p + 2] * n[2]);
        invz[e * nl + l] = (float)(1.0 / sum);
    }
}

// ---------------------------------------------------------------------------
// Source selection: flags in Morton order, emitted luminosity (FP64), and a
// stable compaction into src_list.
// ---------------------------------------------------------------------------

// Direct pass: flag the sources (cells in Morton order, then the point
// sources n .. n + n_point - 1) that emit at some wavelength and are allowed
// by the mask; sum the launched luminosity per wavelength; count every
// emitting source, mask or not (N_s of Eq. 11).
__global__ void k_source_flags(int32_t *flags, const int32_t *morton, int64_t n, int32_t n_point,
                               const LambdaTable *lt, const float *emis_lum, const float *ps_lum,
                               const uint8_t *mask, double *tally, int32_t *n_all)
{
    __shared__ double sh[16];
    const int nl = lt->n_lambda;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t c = i < n + n_point ? morton[i] : -1;
    bool emits = false;
    const bool allowed = c >= 0 && (mask == nullptr || mask[c] != 0);
    for (int l = 0; l < nl; ++l) {
        const double e = c < 0 ? 0.0
                               : c < n ? (double)emis_lum[(int64_t)l * n + c]
                                       : (double)ps_lum[(int64_t)l * n_point + (c - n)];
        emits |= e > 0.0;
        const double b = block_sum(allowed ? e : 0.0, sh);
        if (threadIdx.x == 0 && b != 0.0) atomic_add_f64(&tally[l * DARTRAY_N_TALLY + DARTRAY_T_EMITTED], b);
    }
    if (i < n + n_point) flags[i] = (emits && allowed) ? 1 : 0;
    const uint64_t em = __ballot(emits);
    if ((threadIdx.x & 63) == 0 && em) atomicAdd(n_all, (int32_t)__popcll(em));
}

// Scattering pass, step 1: a coalesced sweep of wavelength blockIdx.y's block
// of the pending scattered luminosity flags every cell with a positive entry
// (cell_flag indexed by cell) and sums the block over the cells the mask
// allows in FP64.  S is never negative, so a positive entry is the same as a
// positive row sum.
__global__ void k_sflag_sweep(const float *S, const LambdaTable *lt, const uint8_t *mask, uint8_t *cell_flag,
                              double *tally)
{
    __shared__ double sh[16];
    const int l = blockIdx.y;
    const int64_t lo = lt->s_off[l], hi = lt->s_off[l + 1];
    const uint32_t npix = (uint32_t)lt->npix[l];
    const bool small = hi - lo < ((int64_t)1 << 32);
    double acc = 0.0;
    for (int64_t i = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < hi; i += (int64_t)gridDim.x * blockDim.x) {
        const float v = S[i];
        if (v > 0.f) {
            const int64_t cell = small ? (int64_t)((uint32_t)(i - lo) / npix) : (i - lo) / (int64_t)npix;
            cell_flag[cell] = 1;
            if (mask == nullptr || mask[cell] != 0) acc += (double)v;
        }
    }
    const double b = block_sum(acc, sh);
    if (threadIdx.x == 0 && b != 0.0) atomic_add_f64(&tally[l * DARTRAY_N_TALLY + DARTRAY_T_EMITTED], b);
}

// Scattering pass, step 2: flags in Morton order for the compaction (cells
// holding scattered light that the mask allows), and the count of every cell
// holding scattered light (N_s of Eq. 11).
__global__ void k_sflag_gather(int32_t *flags, const int32_t *morton, const uint8_t *cell_flag, const uint8_t *mask,
                               int64_t n, int32_t *n_all)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = morton[i];
        const bool has = cell_flag[c] != 0;
        flags[i] = (has && (mask == nullptr || mask[c] != 0)) ? 1 : 0;
        const uint64_t hm = __ballot(has);
        if ((threadIdx.x & 63) == 0 && hm) atomicAdd(n_all, (int32_t)__popcll(hm));
    }
}

constexpr int kScanBlock = 1024;

__global__ void k_scan_count(const int32_t *flags, int64_t n, int32_t *block_counts)
{
    __shared__ int32_t sh[kScanBlock / 64];
    const int64_t i = blockIdx.x * (int64_t)kScanBlock + threadIdx.x;
    int v = i < n ? flags[i] : 0;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < kScanBlock / 64; ++w) s += sh[w];
        block_counts[blockIdx.x] = s;
    }
}

// exclusive scan of block counts (single block, sequential over chunks)
__global__ void k_scan_blocks(int32_t *block_counts, int64_t nblocks, int32_t *total)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int32_t run = 0;
    for (int64_t b = 0; b < nblocks; ++b) {
        const int32_t v = block_counts[b];
        block_counts[b] = run;
        run += v;
    }
    *total = run;
}

__global__ void k_scan_scatter(const int32_t *flags, const int32_t *morton, int64_t n, const int32_t *block_offs,
                               int32_t *src_list)
{
    __shared__ int32_t sh[kScanBlock / 64];
    const int64_t i = blockIdx.x * (int64_t)kScanBlock + threadIdx.x;
    const int f = i < n ? flags[i] : 0;
    const int lane = threadIdx.x & 63;
    const uint64_t ballot = __ballot(f);
    const int before = __popcll(ballot & ((1ull << lane) - 1ull));
    if (lane == 0) sh[threadIdx.x >> 6] = __popcll(ballot);
    __syncthreads();
    int wave_off = 0;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) wave_off += sh[w];
    if (f) src_list[block_offs[blockIdx.x] + wave_off + before] = morton[i];
}

// ---------------------------------------------------------------------------
// Traversal
// ---------------------------------------------------------------------------

struct Geo {
    const LeafRec *rec;
    const int32_t *root_tab;
    const int32_t *nodes;
    int32_t fine[3];
    int32_t nroot[3];
    int32_t max_level;
};

__device__ inline int32_t locate_fine(const Geo &g, int fx, int fy, int fz)
{
    if ((unsigned)fx >= (unsigned)g.fine[0] || (unsigned)fy >= (unsigned)g.fine[1] ||
        (unsigned)fz >= (unsigned)g.fine[2])
        return -1;
    const int L = g.max_level;
    int32_t v = g.root_tab[((fz >> L) * g.nroot[1] + (fy >> L)) * g.nroot[0] + (fx >> L)];
    int bit = L - 1;
    while (v >= 0) {
        const int oct = ((fx >> bit) & 1) | (((fy >> bit) & 1) << 1) | (((fz >> bit) & 1) << 2);
        v = g.nodes[v * 8 + oct];
        --bit;
    }
    return -v - 1;
}

// The transmitted fraction e^{-tau} is 1 + em1 (em1 = e^{-tau} - 1) in thin
// cells, where it keeps extinguished + transmitted equal to the input to the
// last bit, and e^{-tau} itself in thick cells, where 1 + em1 would cancel.
//
// em1 = e^{-tau} - 1 for tau >= 0 at a few FP32 operations: below 0.5 the
// Taylor series of expm1 through the x^8 / 8! term (truncation under 1.5e-8
// relative), above it one hardware base-2 exponential minus 1 (no
// cancellation there, e^{-tau} <= 0.61; relative error about tau * 6e-8 from
// rounding tau log2(e)).  Sets thick when the second branch was taken, in
// which case tr holds e^{-tau}.
__device__ inline float fast_em1(float tau, bool &thick, float &tr)
{
    thick = tau >= 0.5f;
    if (!thick) {
        const float x = -tau;
        float p = 1.f / 40320.f;
        p = fmaf(p, x, 1.f / 5040.f);
        p = fmaf(p, x, 1.f / 720.f);
        p = fmaf(p, x, 1.f / 120.f);
        p = fmaf(p, x, 1.f / 24.f);
        p = fmaf(p, x, 1.f / 6.f);
        p = fmaf(p, x, 0.5f);
        p = fmaf(p, x, 1.f);
        tr = 0.f;
        return p * x;
    }
    tr = __builtin_amdgcn_exp2f(-tau * 1.44269504088896341f);
    return tr - 1.f;
}

// g = (1 - e^{-tau}) / tau for tau >= 0: below 0.5 the Taylor series
// sum_k (-tau)^k / (k + 1)! through k = 7 (truncation under 1.4e-8
// relative), above it (1 - e^{-tau}) / tau from one hardware base-2
// exponential.  Sets thick when the second branch was taken, in which case
// tr holds e^{-tau} (the transmitted fraction, where 1 - tau g would cancel).
__device__ inline float g_series(float tau)
{
    const float x = -tau;
    float p = 1.f / 40320.f;
    p = fmaf(p, x, 1.f / 5040.f);
    p = fmaf(p, x, 1.f / 720.f);
    p = fmaf(p, x, 1.f / 120.f);
    p = fmaf(p, x, 1.f / 24.f);
    p = fmaf(p, x, 1.f / 6.f);
    p = fmaf(p, x, 0.5f);
    return fmaf(p, x, 1.f);
}

// g = (1 - e^{-tau}) / tau in FP64 for 0 <= tau < 0.5: the Taylor series
// sum_k (-tau)^k / (k + 1)! through k = 13 (truncation under 5e-17 relative)
__device__ inline double g_series64(double tau)
{
    const double x = -tau;
    double p = 1.0 / 87178291200.0;           // 1 / 14!
    p = fma(p, x, 1.0 / 6227020800.0);
    p = fma(p, x, 1.0 / 479001600.0);
    p = fma(p, x, 1.0 / 39916800.0);
    p = fma(p, x, 1.0 / 3628800.0);
    p = fma(p, x, 1.0 / 362880.0);
    p = fma(p, x, 1.0 / 40320.0);
    p = fma(p, x, 1.0 / 5040.0);
    p = fma(p, x, 1.0 / 720.0);
    p = fma(p, x, 1.0 / 120.0);
    p = fma(p, x, 1.0 / 24.0);
    p = fma(p, x, 1.0 / 6.0);
    p = fma(p, x, 0.5);
    return fma(p, x, 1.0);
}

__device__ inline float fast_g(float tau, bool &thick, float &tr)
{
    thick = tau >= 0.5f;
    if (!thick) {
        tr = 0.f;
        return g_series(tau);
    }
    tr = __builtin_amdgcn_exp2f(-tau * 1.44269504088896341f);
    return (1.f - tr) * __builtin_amdgcn_rcpf(tau);
}

// fine-level cell coordinate of position p along an axis with direction
// component d and F fine cells: on a face, the side d points to; a ray lying
// in the face plane (d == 0) takes the side away from the block's central
// plane, so that mirror-image rays visit mirror-image cells (the upper side
// on the central plane itself)
template <typename T>
__device__ inline int fine_coord(T p, T d, int F)
{
    const T fl = floor(p);
    int i = (int)fl;
    if (p == fl && (d < T(0) || (d == T(0) && T(2) * fl < T(F)))) i -= 1;
    return i;
}

// A segment [t, te] of a ray whose length is zero up to the rounding of its
// two end distances -- at most 2^-46 of the exit distance, a few tens of ulps
// of an FP64 distance -- is a ray through an edge or corner of the cell
// (zero length in exact arithmetic).  It deposits nothing, takes no decision
// and does not advance the ray's distance, so the residue folds into the next
// crossing.  Every march and the adjoint use this one rule.
__host__ __device__ inline bool is_graze(double len, double te) { return !(len > 0x1p-46 * te); }

// A ray in finest-level cell units.  The marches keep their geometry in FP64:
// distances along a ray reach hundreds of cells, and the adaptive march takes
// its split, block and step-1 extent decisions on these values.  The
// debugging traversal runs the same FP64 instance.
template <typename T>
struct RayT {
    T o[3];       // origin (source-cell centre), fine units
    T n[3];       // unit direction
    T inv[3];     // 1/n (unused for zero components)
};

// exit distance from the leaf with box b along ray R, and the exit axis
// (exact ties resolved x before y before z)
template <typename T>
__device__ inline T exit_t(const RayT<T> &R, const int4 b, int &axis)
{
    const T INF = T(__builtin_huge_valf());
    const int lo[3] = {b.x, b.y, b.z};
    T best = INF;
    axis = 0;
    // selects rather than branches: the face the direction points to, no
    // exit across an axis the ray runs parallel to
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int face = R.n[a] > T(0) ? lo[a] + b.w : lo[a];
        const T ta = ((T)face - R.o[a]) * R.inv[a];
        const T t = R.n[a] != T(0) ? ta : INF;
        axis = t < best ? a : axis;
        best = t < best ? t : best;
    }
    return best;
}

// the leaf across the exit face that contains the exit point: one load of the
// face-neighbour code, plus a descent when the region across is subdivided
template <typename T>
__device__ inline int32_t next_leaf(const Geo &g, const RayT<T> &R, const int4 b, const int32_t *nb, int axis, T te)
{
    // no runtime index into the ray or the neighbour array: those would be
    // kept in scratch memory; the sign comes from an unrolled compare and
    // the code from a register vector
    bool pos = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) pos = a == axis ? R.n[a] > T(0) : pos;
    typedef int32_t nb8 __attribute__((ext_vector_type(8)));
    const nb8 nv = {nb[0], nb[1], nb[2], nb[3], nb[4], nb[5], -1, -1};
    const int32_t code = nv[2 * axis + (pos ? 1 : 0)];
    if (code >= -1) return code;            // a leaf, or outside the root block
    const int lo[3] = {b.x, b.y, b.z};
    int f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (a == axis) {
            f[a] = pos ? lo[a] + b.w : lo[a] - 1;
        } else {
            int q = fine_coord<T>(fma(te, R.n[a], R.o[a]), R.n[a], g.fine[a]);
            q = q < lo[a] ? lo[a] : q;
            q = q > lo[a] + b.w - 1 ? lo[a] + b.w - 1 : q;
            f[a] = q;
        }
    }
    int32_t v = -code - 2;                  // internal node at this leaf's level
    int bit = 30 - __clz(b.w);              // log2(span) - 1
    while (v >= 0) {
        const int oct = ((f[0] >> bit) & 1) | (((f[1] >> bit) & 1) << 1) | (((f[2] >> bit) & 1) << 2);
        v = g.nodes[v * 8 + oct];
        --bit;
    }
    return -v - 1;
}

// The traversal of the marches (FP64 exit distances, face-neighbour steps)
// for given rays: every segment, zero-length ones included.
__global__ void k_debug_cells(Geo g, int nrays, const double *origin, const double *dir, int max_cross,
                              int64_t *cells, double *lengths, int32_t *counts)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrays) return;
    RayT<double> R;
    for (int a = 0; a < 3; ++a) {
        R.o[a] = origin[3 * i + a];
        R.n[a] = dir[3 * i + a];
        R.inv[a] = 1.0 / R.n[a];
    }
    int32_t c = locate_fine(g, fine_coord<double>(R.o[0], R.n[0], g.fine[0]), fine_coord<double>(R.o[1], R.n[1], g.fine[1]),
                            fine_coord<double>(R.o[2], R.n[2], g.fine[2]));
    double t = 0.0;
    int m = 0;
    while (c >= 0 && m < max_cross) {
        const LeafRec &rc = g.rec[c];
        const int4 b = rc.box;
        int32_t nbc[6];
        for (int q = 0; q < 6; ++q) nbc[q] = rc.nb[q];
        int axis;
        const double te = exit_t<double>(R, b, axis);
        cells[(int64_t)i * max_cross + m] = c;
        lengths[(int64_t)i * max_cross + m] = te > t ? te - t : 0.0;
        ++m;
        if (te > t) t = te;
        c = next_leaf<double>(g, R, b, nbc, axis, te);
    }
    counts[i] = m;
}

// ---------------------------------------------------------------------------
// Fixed-Nside march: lanes are 64 Morton-consecutive sources, one direction
// per wave.  Deposits go to the direction bins ubar[r - r0][c][l].
// ---------------------------------------------------------------------------

struct FixedArgs {
    Geo geo;
    const int32_t *src_list;
    const int32_t *n_src;
    const double4 *dirs;         // FP64 directions of this Nside
    const float *emis_lum;       // direct pass
    const double4 *ps_pos;       // point sources (index n + k): position, fine units
    const int32_t *ps_cell;      // the leaf holding each point
    const float *ps_lum;         // [n_lambda][n_point] luminosity
    int32_t n_point;
    const float *S_pending;      // scatter pass
    const LambdaTable *lt;
    float *ubar;                 // [nb][n][n_lambda] direction-binned energy density
    double *tally;
    uint64_t *counters;          // null: this launch does not count
    double *esc_dir;             // [n_lambda][nray] escape by direction, or null
    int64_t n;
    int32_t scatter;
    int32_t r0;
    int32_t nb;
    int32_t l0;                  // wavelengths l0 .. l0 + nlc - 1 ride on this launch
    int32_t nlc;
    int32_t order;               // 0: a wave's next item is the next direction, 1: the next source tile
    int32_t nside_ray;
    int32_t log2_nside_ray;
    float inv_nray;
    double h_fine;
    int64_t max_steps;           // caller's per-ray limit (0 = none)
    int64_t hard_cap;            // bound no straight ray can exceed; ends any loop
    int32_t linear;              // uniform grid, leaf i at root position i (x fastest)
};

// Launch luminosity of source s along ray r at wavelength l: the direct pass
// spreads 4 pi j V evenly over the rays; a scattering pass takes the pending
// scattered luminosity of the nested pixel that contains r (scaled by
// N_pix / N_ray), or sums the pixels inside r when rays are coarser.
__device__ inline float fixed_launch(const FixedArgs &A, const LambdaTable *lt, int l, int32_t s, int r)
{
    if (s >= A.n) return A.scatter ? 0.f : A.ps_lum[(int64_t)l * A.n_point + (s - A.n)] * A.inv_nray;
    if (!A.scatter) return A.emis_lum[(int64_t)l * A.n + s] * A.inv_nray;
    const int npix = lt->npix[l];
    const float *row = A.S_pending + lt->s_off[l] + (int64_t)s * npix;
    const int ls = 31 - __clz(lt->nside_sca[l]);
    if (A.log2_nside_ray >= ls) return row[r >> (2 * (A.log2_nside_ray - ls))] * ((float)npix * A.inv_nray);
    float v = 0.f;
    const int sh = 2 * (ls - A.log2_nside_ray);
    for (int q = r << sh; q < ((r + 1) << sh); ++q) v += row[q];
    return v;
}

// v of lane (k + R) & 3 of this lane's quad (k its place in the quad)
template <int R>
__device__ inline int quad_rot(int v)
{
    constexpr int ctrl = ((0 + R) & 3) | (((1 + R) & 3) << 2) | (((2 + R) & 3) << 4) | (((3 + R) & 3) << 6);
    return __builtin_amdgcn_update_dpp(0, v, ctrl, 0xF, 0xF, false);
}

template <int R>
__device__ inline float quad_rot_f(float v)
{
    return __int_as_float(quad_rot<R>(__float_as_int(v)));
}

// per-lane counters
template <int NL>
struct FixedAcc {
    uint32_t ncross, nrays, nmax, nrows;
    __device__ void clear() { ncross = nrays = nmax = nrows = 0; }
};

// LDS of the march (256-thread workgroups at most): each wave's deposit
// staging, its wavelengths' opacities and its FP64 escaped-luminosity sums
template <int NL>
struct alignas(16) FixedStage {
    float du[NL][256];           // each lane's deposit row of the step
    alignas(16) int32_t cell[256];    // each lane's deposit cell of the step (-1 none)
    alignas(16) int32_t hcell[256];   // the cell of each lane's open row (-1 none)
    float ed[NL][256];           // rows going out, at compacted slots
    int32_t ecell[256];
    uint8_t list[256];
    float kap[4][NL];
    double esc[4][NL];
    double edir[4][NL];          // this item's escape (one direction per item)
};

__device__ inline void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One work item (64 sources of source tile `tile`, direction r0 + rl): the
// wave's lanes walk their rays in lock step, one cell per iteration, and the
// iteration's deposits go out wave-cooperatively: the wavelength values of a
// crossing are one contiguous row of the bin array, and one atomic
// instruction carries 64 / NL crossings.  A tile of a dense source list is a
// 4 x 4 x 4 block of cells (Morton order); each quad of lanes takes four of
// them on a line along the direction's dominant axis, so the quad's parallel
// rays, less than a cell apart sideways near that axis, cross many cells a
// step or two apart.  Groups of eight lanes pair two such quads, side by side
// along the axis of the next-largest direction component.  Rows of one cell
// in one step are summed by the group's lowest lane depositing there, and a
// row stays open while the group keeps depositing into its cell (it moves to
// that lowest lane); it goes out at the first step in which no lane of the
// group deposits into that cell.
//
// LIN (a linearly numbered uniform grid): a cell's box and the cell across its
// exit face follow from the cell's integer position, so the walk needs no
// record load to find the next cell, and the next cell's density is loaded
// one step ahead; the exit distances are those of the same exit_t, so the
// cells and segments are those of the record walk.
template <int NL, bool LIN>
__device__ void fixed_item(const FixedArgs &A, int64_t tile, int rl, int nsrc, FixedStage<NL> &st, FixedAcc<NL> &acc)
{
    const LambdaTable *lt = A.lt;
    const int nl = lt->n_lambda;
    const int nlc = A.nlc, l0 = A.l0;
    const int lane = threadIdx.x & 63;
    const int wbase = threadIdx.x & ~63;
    const int w = threadIdx.x >> 6;
    const int r = A.r0 + rl;
    const double4 nd = A.dirs[r];
    // lane -> source m of the tile (x, y, z are Morton bits 0-2 and 3-5):
    // lane bits 0-1 take the two bits of the dominant axis, lane bit 2 the
    // low bit of the axis of the next-largest direction component, lane bits
    // 3-5 the other three
    const double a0 = fabs(nd.x), a1 = fabs(nd.y), a2 = fabs(nd.z);
    const int ax = a1 > a0 ? (a2 > a1 ? 2 : 1) : (a2 > a0 ? 2 : 0);
    const int o1 = ax == 0 ? 1 : 0, o2 = ax == 2 ? 1 : 2;
    const int mid = (o2 == 1 ? a1 : a2) > (o1 == 0 ? a0 : a1) ? o2 : o1;
    const int go = lane & 7, gq = lane >> 3;
    int m = ((go & 1) << ax) | (((go >> 1) & 1) << (ax + 3)) | (((go >> 2) & 1) << mid);
    for (int b = 0, j = 0; b < 6; ++b) {
        if (b == ax || b == ax + 3 || b == mid) continue;
        m |= ((gq >> j) & 1) << b;
        ++j;
    }
    const int64_t si = tile * 64 + m;
    bool active = si < nsrc;
    int32_t c = 0;
    // FP64 geometry: distances along a ray reach hundreds of cells, where FP32
    // would leave segments near the graze limit with percent-level errors
    RayT<double> R;
    float L[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) L[l] = 0.f;
    if (lane < NL) st.kap[w][lane] = lane < nlc ? lt->kappa[l0 + lane] : 0.f;
    wave_sync_lds();
    if (active) {
        const int32_t s = A.src_list[si];
        R.n[0] = nd.x;
        R.n[1] = nd.y;
        R.n[2] = nd.z;
        if (s < A.n) {
            // an emitting cell: rays start at its centre
            const int4 b = A.geo.rec[s].box;
            const double half = 0.5 * (double)b.w;
            R.o[0] = (double)b.x + half;
            R.o[1] = (double)b.y + half;
            R.o[2] = (double)b.z + half;
        } else {
            const double4 p = A.ps_pos[s - A.n];
            R.o[0] = p.x;
            R.o[1] = p.y;
            R.o[2] = p.z;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) R.inv[a] = 1.0 / R.n[a];
        float lsum = 0.f;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            if (l < nlc) {
                L[l] = fixed_launch(A, lt, l0 + l, s, r);
                lsum += L[l];
            }
        }
        // the counting launch traces a ray when any wavelength carries light
        if (!(lsum > 0.f) && A.counters)
            for (int l = 0; l < nl; ++l)
                if (l < l0 || l >= l0 + nlc) lsum += fixed_launch(A, lt, l, s, r);
        active = lsum > 0.f;
        c = s < A.n ? s : A.ps_cell[s - A.n];
        if (active) ++acc.nrays;
    }
    // LIN: the cell's position, and its density and 1/(V c)
    int32_t cx = 0, cy = 0, cz = 0;
    float rho_c = 0.f, ivc_c = 0.f;
    if (LIN && active) {
        const LeafRec &r0c = A.geo.rec[c];
        cx = r0c.box.x;
        cy = r0c.box.y;
        cz = r0c.box.z;
        rho_c = r0c.rho;
        ivc_c = r0c.ivc;
    }
    double t = 0.0;
    int64_t steps = 0;
    float *ubase = A.ubar + (size_t)rl * (size_t)A.n * nl + l0;
    // the row this lane holds: cell (-1 none), values
    int32_t h_cell = -1;
    float h_du[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) h_du[l] = 0.f;
    // staging of the held rows in the wave's 64 slots of st.ed: the rows that
    // go out compacted from the bottom, the rows that stay open compacted from
    // the top; then the outgoing rows as atomic instructions over 64 / NL rows
    // each
    auto stage_rows = [&](bool out, bool keep) {
        const uint64_t om = __ballot(out), km = __ballot(keep);
        if (out || keep) {
            const uint64_t below = (1ull << lane) - 1ull;
            const int slot = out ? wbase + __popcll(om & below) : wbase + 63 - __popcll(km & below);
            st.ecell[slot] = h_cell;
#pragma unroll
            for (int l = 0; l < NL; ++l) st.ed[l][slot] = h_du[l];
        }
        acc.nrows += out ? 1u : 0u;
        wave_sync_lds();
        const int cnt = __popcll(om);
        constexpr int PER = 64 / NL;
        for (int k0 = 0; k0 < cnt; k0 += PER) {
            const int q = k0 + lane / NL;
            const int l = lane % NL;
            if (q < cnt && l < nlc) atomic_add_f32(ubase + (size_t)st.ecell[wbase + q] * nl + l, st.ed[l][wbase + q]);
        }
        return km;
    };
    while (__ballot(active)) {
        bool dep = false;
        int32_t dcell = -1;
        if (active) {
            int4 b;
            float rho, ivc;
            int32_t nbc[6];
            if (LIN) {
                b = make_int4(cx, cy, cz, 1);
                rho = rho_c;
                ivc = ivc_c;
            } else {
                const LeafRec &rc = A.geo.rec[c];
                b = rc.box;
                rho = rc.rho;
                ivc = rc.ivc;
#pragma unroll
                for (int q = 0; q < 6; ++q) nbc[q] = rc.nb[q];
            }
            int axis;
            const double te = exit_t(R, b, axis);
            const double len = te - t;
            if (!is_graze(len, te)) {
                const float lp = (float)(len * A.h_fine);
#pragma unroll
                for (int l = 0; l < NL; ++l) {
                    if (l < nlc) {
                        const float alpha = st.kap[w][l] * rho;
                        const float tau = alpha * lp;
                        bool thick;
                        float tr;
                        const float em1 = fast_em1(tau, thick, tr);   // exp(-tau) - 1
                        const float ext = -L[l] * em1;
                        st.du[l][threadIdx.x] =
                            alpha > 0.f ? ext * ivc * __builtin_amdgcn_rcpf(alpha) : L[l] * lp * ivc;
                        L[l] = thick ? L[l] * tr : fmaf(L[l], em1, L[l]);   // transmission, fused
                    }
                }
                dcell = c;
                dep = true;
                ++acc.ncross;
                ++steps;   // the per-ray limit counts crossings of positive length
                t = te;
            }
            int32_t nx;
            if (LIN) {
                // one cell along the exit axis, in the direction of travel
                bool pos = false;
#pragma unroll
                for (int a = 0; a < 3; ++a) pos = a == axis ? R.n[a] > 0.0 : pos;
                const int d = pos ? 1 : -1;
                cx += axis == 0 ? d : 0;
                cy += axis == 1 ? d : 0;
                cz += axis == 2 ? d : 0;
                const bool inside = (unsigned)cx < (unsigned)A.geo.nroot[0] &&
                                    (unsigned)cy < (unsigned)A.geo.nroot[1] &&
                                    (unsigned)cz < (unsigned)A.geo.nroot[2];
                const int32_t stride = axis == 0 ? 1 : axis == 1 ? A.geo.nroot[0] : A.geo.nroot[0] * A.geo.nroot[1];
                nx = inside ? c + d * stride : -1;
                if (nx >= 0) rho_c = A.geo.rec[nx].rho;    // for the next step
            } else {
                nx = next_leaf<double>(A.geo, R, b, nbc, axis, te);
            }
            bool escaped = false;
            if (nx < 0) {
                active = false;
                escaped = true;
            } else if ((A.max_steps > 0 && steps >= A.max_steps) || steps >= A.hard_cap) {
                // stopped before its next cell: its light is not escaped light
                ++acc.nmax;
                active = false;
            } else {
                c = nx;
            }
            if (escaped) {
#pragma unroll
                for (int l = 0; l < NL; ++l)
                    if (l < nlc && L[l] != 0.f) {
                        atomicAdd(&st.esc[w][l], (double)L[l]);
                        if (A.esc_dir) atomicAdd(&st.edir[w][l], (double)L[l]);
                    }
            }
        }
        // ---- rows: a held row stays open while its group keeps depositing
        // into its cell and moves to the lowest lane depositing there; the
        // lowest lane of each other cell opens a row; the rest go out
        st.cell[threadIdx.x] = dcell;
        st.hcell[threadIdx.x] = h_cell;
        wave_sync_lds();
        const int gb = wbase + (lane & ~7);
        const int4 ca = *reinterpret_cast<const int4 *>(&st.cell[gb]);
        const int4 cb = *reinterpret_cast<const int4 *>(&st.cell[gb + 4]);
        const int4 ha = *reinterpret_cast<const int4 *>(&st.hcell[gb]);
        const int4 hb = *reinterpret_cast<const int4 *>(&st.hcell[gb + 4]);
        const int32_t C[8] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y, cb.z, cb.w};
        const int32_t H[8] = {ha.x, ha.y, ha.z, ha.w, hb.x, hb.y, hb.z, hb.w};
        const bool held = h_cell >= 0;
        bool keep = false, below = false;
        int hr = -1;   // the group place of the lane holding this lane's cell
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            keep = keep || (held && C[j] == h_cell);
            below = below || (j < go && C[j] == dcell);
            hr = dep && H[j] == dcell ? j : hr;
        }
        const bool owner = dep && !below;
        const uint64_t km = stage_rows(held && !keep, keep);
        if (owner) {
            // this lane's deposit, the deposits of the lanes above it into
            // its cell, and the open row of that cell
#pragma unroll
            for (int l = 0; l < NL; ++l) h_du[l] = st.du[l][threadIdx.x];
#pragma unroll
            for (int j = 1; j < 8; ++j) {
                if (j > go && C[j] == dcell) {
#pragma unroll
                    for (int l = 0; l < NL; ++l) h_du[l] += st.du[l][gb + j];
                }
            }
            if (hr >= 0) {
                const int hl = (lane & ~7) + hr;
                const int src = wbase + 63 - __popcll(km & ((1ull << hl) - 1ull));
#pragma unroll
                for (int l = 0; l < NL; ++l) h_du[l] += st.ed[l][src];
            }
        }
        h_cell = owner ? dcell : -1;
        if (!owner) {
#pragma unroll
            for (int l = 0; l < NL; ++l) h_du[l] = 0.f;
        }
        wave_sync_lds();
    }
    stage_rows(h_cell >= 0, false);
    wave_sync_lds();
    if (A.esc_dir) {
        // all rays of the item share direction r: one FP64 add per wavelength
        wave_sync_lds();
        if (lane < NL) {
            const double v = st.edir[w][lane];
            if (lane < nlc && v != 0.0)
                atomic_add_f64(A.esc_dir + (int64_t)(l0 + lane) * (12 << (2 * A.log2_nside_ray)) + r, v);
            st.edir[w][lane] = 0.0;
        }
        wave_sync_lds();
    }
}

// the wave's escaped-luminosity sums and counters into A's tallies
template <int NL>
__device__ void fixed_commit(const FixedArgs &A, FixedStage<NL> &st, FixedAcc<NL> &acc)
{
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int nl = A.lt->n_lambda;
    wave_sync_lds();
    if (lane < NL) {
        const double v = st.esc[w][lane];
        if (lane < A.nlc && v != 0.0) atomic_add_f64(&A.tally[(A.l0 + lane) * DARTRAY_N_TALLY + DARTRAY_T_ESCAPED], v);
        st.esc[w][lane] = 0.0;
    }
    wave_sync_lds();
    if (A.counters) {
        const uint64_t wc = wave_sum_u64(acc.ncross), wr = wave_sum_u64(acc.nrays), wm = wave_sum_u64(acc.nmax),
                       wu = wave_sum_u64(acc.nrows);
        if (lane == 0) {
            if (wu) atomicAdd((unsigned long long *)&A.counters[DARTRAY_C_U_ROWS], (unsigned long long)wu);
            if (wc) atomicAdd((unsigned long long *)&A.counters[DARTRAY_C_CROSSINGS], (unsigned long long)wc);
            if (wr) atomicAdd((unsigned long long *)&A.counters[DARTRAY_C_RAYS], (unsigned long long)wr);
            if (wr) atomicAdd((unsigned long long *)&A.counters[DARTRAY_C_ESCAPES], (unsigned long long)(wr - wm));
            if (wm) atomicAdd((unsigned long long *)&A.counters[DARTRAY_C_MAXSTEP], (unsigned long long)wm);
            // deposits count the counted crossings times the wavelengths carried
            if (wc) atomicAdd((unsigned long long *)&A.counters[DARTRAY_C_DEPOSITS], (unsigned long long)(wc * nl));
        }
    }
    acc.clear();
}

__device__ inline void fixed_item_index(const FixedArgs &A, int64_t it, int64_t ntiles, int64_t &tile, int &rl)
{
    if (A.order == 0) {
        tile = it / A.nb;
        rl = (int)(it - tile * A.nb);
    } else {
        rl = (int)(it / ntiles);
        tile = it - (int64_t)rl * ntiles;
    }
}

// The fixed march waits on dependent loads (each cell's record names the
// next), so occupancy pays for a small spill: up to 16 wavelengths it runs at
// 4 waves per SIMD (at 16 wavelengths 52 bytes per lane spill, and the 128^3
// clumpy march takes 0.83x the time it takes at 3 waves); at 32 wavelengths
// its LDS staging allows 2 anyway.
#define DR_FIXED_WAVES(NL) ((NL) <= 16 ? 4 : 1)

template <int NL, bool LIN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DR_FIXED_WAVES(NL), 8)))
void k_march_fixed(const FixedArgs A)
{
    __shared__ FixedStage<NL> st;
    const int64_t wid = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int nsrc = *A.n_src;
    const int64_t ntiles = (nsrc + 63) >> 6;
    const int64_t nitems = ntiles * A.nb;
    FixedAcc<NL> acc;
    acc.clear();
    if ((threadIdx.x & 63) < NL) {
        st.esc[threadIdx.x >> 6][threadIdx.x & 63] = 0.0;
        st.edir[threadIdx.x >> 6][threadIdx.x & 63] = 0.0;
    }
    for (int64_t it = wid; it < nitems; it += nw) {
        int64_t tile;
        int rl;
        fixed_item_index(A, it, ntiles, tile, rl);
        fixed_item<NL, LIN>(A, tile, rl, nsrc, st, acc);
    }
    fixed_commit<NL>(A, st, acc);
}

// Several models in one persistent launch.  The work items of model m are
// item_off[m] .. item_off[m + 1] - 1 (models in descending order of expected
// work); a wave strides over all of them and commits its tallies whenever it
// moves on to another model.
struct BatchMarch {
    const FixedArgs *models;     // [n_models], r0 / nb / l0 / nlc taken from here
    const int64_t *item_off;     // [n_models + 1]
    int32_t n_models;
    int32_t r0, nb, l0, nlc;
    int32_t count;               // 0: no counters in this launch
};

template <int NL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DR_FIXED_WAVES(NL), 8)))
void k_march_fixed_multi(const BatchMarch B)
{
    __shared__ FixedStage<NL> st;
    const int64_t wid = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t nitems = B.item_off[B.n_models];
    FixedAcc<NL> acc;
    acc.clear();
    if ((threadIdx.x & 63) < NL) {
        st.esc[threadIdx.x >> 6][threadIdx.x & 63] = 0.0;
        st.edir[threadIdx.x >> 6][threadIdx.x & 63] = 0.0;
    }
    int mcur = -1;
    FixedArgs A{};
    int nsrc = 0;
    int64_t ntiles = 0;
    for (int64_t it = wid; it < nitems; it += nw) {
        int m = mcur < 0 ? 0 : mcur;
        while (it >= B.item_off[m + 1]) ++m;
        m = __builtin_amdgcn_readfirstlane(m);
        if (m != mcur) {
            if (mcur >= 0) fixed_commit<NL>(A, st, acc);
            A = B.models[m];
            A.r0 = B.r0;
            A.nb = B.nb;
            A.l0 = B.l0;
            A.nlc = B.nlc;
            if (!B.count) A.counters = nullptr;
            nsrc = *A.n_src;
            ntiles = (nsrc + 63) >> 6;
            mcur = m;
        }
        int64_t tile;
        int rl;
        fixed_item_index(A, it - B.item_off[m], ntiles, tile, rl);
        fixed_item<NL, false>(A, tile, rl, nsrc, st, acc);
    }
    if (mcur >= 0) fixed_commit<NL>(A, st, acc);
}

// item_off[m + 1] = item_off[m] + ceil(n_src(model order[m]) / 64) nb
__global__ void k_batch_items(const FixedArgs *models, int n_models, int nb, int64_t *item_off)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t acc = 0;
    item_off[0] = 0;
    for (int m = 0; m < n_models; ++m) {
        acc += (int64_t)((*models[m].n_src + 63) >> 6) * nb;
        item_off[m + 1] = acc;
    }
}

// Flush of one direction batch:
//   U_k[c][l] += sum_r ubar[r][c][l]
//   S[l][c][p] += albedo kappa rho V c sum_r ubar[r][c][l] w_l(p|r)
// A block holds 256 / NLP cells x NLP wavelength slots (NLP = n_lambda rounded
// up to a power of two), so its bin reads are one contiguous range per
// direction; the block's pixel chunk is PCH pixels from by * PCH.  The phase
// weights of rb_stage directions are staged in LDS as
// [direction][wavelength][PCH + 1] (the odd row stride spreads the
// wavelengths over the banks).
struct FlushArgs {
    const float *ubar;
    const float *wtab;
    const LambdaTable *lt;
    const float *rho;
    const float *inv_vc;
    double *U_k;
    float *S_next;
    int64_t n;
    int32_t w_row;
    int32_t bx;                  // blocks along the cells (multi-model launch)
    int64_t block0;              // first block of this model (multi-model launch)
};

constexpr int kFlushStage = 16;   // most directions staged at once

template <int PCH>
__device__ void flush_block(const FlushArgs &F, float *ws, int64_t bx, int by, int r0, int nb, int log2_nlp,
                            int rb_stage)
{
    constexpr int PS = PCH + 1;
    const LambdaTable *lt = F.lt;
    const int nl = lt->n_lambda;
    __shared__ int s_npix[kMaxLambda], s_woff[kMaxLambda];
    if (threadIdx.x < nl) {
        s_npix[threadIdx.x] = lt->npix[threadIdx.x];
        s_woff[threadIdx.x] = lt->w_off[threadIdx.x];
    }
    __syncthreads();
    const int64_t n = F.n;
    const int l = threadIdx.x & ((1 << log2_nlp) - 1);
    const int64_t c = bx * (int64_t)(256 >> log2_nlp) + (threadIdx.x >> log2_nlp);
    const int p0 = by * PCH;
    const bool ok = c < n && l < nl;
    const int npix = ok ? lt->npix[l] : 0;
    const bool pix = ok && p0 < npix;
    float acc[PCH];
#pragma unroll
    for (int j = 0; j < PCH; ++j) acc[j] = 0.f;
    double accU = 0.0;           // sum over up to 768 direction bins
    const float *ub = F.ubar + (ok ? (size_t)c * nl + l : 0);
    const size_t rstride = (size_t)n * nl;
    const float *wsl = ws + (size_t)(ok ? l : 0) * PS;
    // the bins of the next stage are loaded while the current one is summed
    float un[kFlushStage];
#pragma unroll
    for (int i = 0; i < kFlushStage; ++i) un[i] = (ok && i < min(rb_stage, nb)) ? ub[(size_t)i * rstride] : 0.f;
    for (int rb = 0; rb < nb; rb += rb_stage) {
        const int cnt = min(rb_stage, nb - rb);
        float uc[kFlushStage];
#pragma unroll
        for (int i = 0; i < kFlushStage; ++i) {
            uc[i] = un[i];
            const int rn = rb + rb_stage + i;
            un[i] = (ok && i < rb_stage && rn < nb) ? ub[(size_t)rn * rstride] : 0.f;
        }
        __syncthreads();
        {
            // element e of the stage is weight j of row (direction i, wavelength
            // ll); eight independent loads in flight per thread
            const int total = cnt * nl * PCH;
            const float inv_nl = 1.f / (float)nl;
            for (int e0 = threadIdx.x; e0 < total; e0 += 8 * 256) {
                float v[8];
                int dst[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int e = e0 + k * 256;
                    const int row = e / PCH;
                    const int j = e - row * PCH;
                    const int i = (int)(((float)row + 0.5f) * inv_nl);
                    const int ll = row - i * nl;
                    const int p = p0 + j;
                    const bool in = e < total && p < s_npix[ll];
                    v[k] = in ? F.wtab[(int64_t)(r0 + rb + i) * F.w_row + s_woff[ll] + p] : 0.f;
                    dst[k] = e < total ? row * PS + j : -1;
                }
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (dst[k] >= 0) ws[dst[k]] = v[k];
            }
        }
        __syncthreads();
        if (ok) {
#pragma unroll
            for (int i = 0; i < kFlushStage; ++i) {
                if (i < cnt) {
                    const float u = uc[i];
                    accU += (double)u;
                    if (pix) {
                        const float *w = wsl + (size_t)i * nl * PS;
#pragma unroll
                        for (int j = 0; j < PCH; ++j) acc[j] = fmaf(u, w[j], acc[j]);
                    }
                }
            }
        }
    }
    if (!ok) return;
    if (pix) {
        const float f = lt->albedo[l] * lt->kappa[l] * F.rho[c] / F.inv_vc[c];
        float *srow = F.S_next + lt->s_off[l] + c * (int64_t)npix + p0;
#pragma unroll
        for (int j = 0; j < PCH; ++j)
            if (p0 + j < npix) srow[j] += f * acc[j];
    }
    if (by == 0) F.U_k[c * nl + l] += accU;
}

template <int PCH>
__global__ __launch_bounds__(256) void k_flush_fixed(const FlushArgs F, int r0, int nb, int log2_nlp, int rb_stage)
{
    extern __shared__ float ws[];
    flush_block<PCH>(F, ws, blockIdx.x, blockIdx.y, r0, nb, log2_nlp, rb_stage);
}

// all models of a batch: a flat grid, model m owning blocks block0 .. (its
// cell blocks x pixel chunks)
template <int PCH>
__global__ __launch_bounds__(256) void k_flush_fixed_multi(const FlushArgs *models, int n_models, int r0, int nb,
                                                            int log2_nlp, int rb_stage)
{
    extern __shared__ float ws[];
    int m = 0;
    while (m + 1 < n_models && (int64_t)blockIdx.x >= models[m + 1].block0) ++m;
    m = __builtin_amdgcn_readfirstlane(m);
    const FlushArgs F = models[m];
    const int64_t b = (int64_t)blockIdx.x - F.block0;
    const int64_t by = b / F.bx;
    flush_block<PCH>(F, ws, b - by * F.bx, (int)by, r0, nb, log2_nlp, rb_stage);
}

// ---------------------------------------------------------------------------
// Adaptive march (ray splitting and blocking, Sect. 3.1.1 / 3.2 / 3.5): the
// direct and scattering passes, and step 1 with ray merging (step 1 without
// merging runs k_step1_quad, below).
//
// A persistent kernel: each lane takes work items (top-level pixel r0,
// source) from a device counter, 64 at a time per wave, items ordered so that
// a wave starts on 64 Morton-consecutive sources with the same direction.  A
// lane walks the ray tree of its item depth first: a split replaces the ray
// by its four nested children (Nside doubled) that restart at the entry
// distance of the triggering crossing with a quarter of its luminosity.  The
// stack keeps one (distance, luminosity / 4) entry per level; the pixel of
// the next sibling is pix + 1 and the parent is pix >> 2.
//
// Every loop iteration advances each lane with a ray by one crossing; the
// energy density is deposited lane by lane, the scattered luminosity through
// the deposit log (expanded per cell after the launch) or, for what the log
// cannot take, cooperatively: for each depositing lane the whole wave adds
// that crossing's phase-weighted luminosity to the cell's HEALPix row, 64
// pixels per instruction.
// ---------------------------------------------------------------------------

struct AdaptArgs {
    Geo geo;
    const int32_t *src_list;
    const int32_t *n_src;
    const float4 *dirs;          // all-level direction table (FP32; j_sca pixels)
    const double4 *dirs64;       // all-level direction table (FP64; ray geometry)
    const float *invz;           // [entry][n_lambda]
    const float *emis_lum;
    const double *lum64;         // [n_lambda][n] 4 pi j V in FP64 (direct pass launch)
    const double4 *ps_pos;       // point sources (index n + k): position, fine units
    const int32_t *ps_cell;      // the leaf holding each point
    const float *ps_lum;         // [n_lambda][n_point] luminosity
    const double *ps_lum64;      // the same in FP64
    int32_t n_point;
    const float *S_pending;
    const float *ull_t;          // [n][n_lambda] copy of U_LL
    const int32_t *n_all;        // sources of the pass in the whole model (N_s of Eq. 11)
    const LambdaTable *lt;
    double *U_k;
    float *S_next;
    double *tally;
    uint64_t *counters;
    unsigned long long *queue;
    // deposit log (0 capacity: deposit with atomics)
    uint64_t *log_key;           // (cell << log_dir_bits) | direction entry
    int32_t log_dir_bits;
    float *log_du;
    unsigned long long *log_count;
    int64_t log_cap;
    int64_t log_limit;           // no new items once the log holds this many tuples
    int64_t n;
    int32_t mode;                // 0 step 1, 1 direct, 2 scatter
    int32_t nside0;
    int32_t log2_nside0;
    int32_t max_depth;           // levels above nside0 a ray may reach
    double n_rays;               // N_rays of Eq. 2
    double n_rays_max;           // N_rays^max of Eq. 3 (merging instances)
    double f_U;                  // < 0: 4 a_RT / N_s (Eq. 11)
    double a_RT;
    double c_light;
    double r_pre_fine64;         // step-1 extent in fine units
    double h_fine64;
    int64_t max_steps;
    int64_t hard_cap;
};

// a + b + c + d added in ascending order (the same sum for any order of the four)
template <typename T>
__device__ inline T sum4_sorted(T a, T b, T c, T d)
{
    T v[4] = {a, b, c, d};
#pragma unroll
    for (int i = 1; i < 4; ++i)
#pragma unroll
        for (int k = i; k > 0; --k)
            if (v[k] < v[k - 1]) {
                const T x = v[k];
                v[k] = v[k - 1];
                v[k - 1] = x;
            }
    return ((v[0] + v[1]) + v[2]) + v[3];
}

__device__ inline float readlane_f(float v, int j)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

__device__ inline int readlane_i(int v, int j) { return __builtin_amdgcn_readlane(v, j); }

// waves per SIMD the compiler must allow for the adaptive march (register
// budget): step 1, and the passes that scatter light
#ifndef DR_WAVES_STEP1
#define DR_WAVES_STEP1 4
#endif
#ifndef DR_WAVES_SCATTER
#define DR_WAVES_SCATTER 2
#endif
#ifndef DR_PENDING_MIN
#define DR_PENDING_MIN 4
#endif
#ifndef DR_FETCH_MIN_STEP1
#define DR_FETCH_MIN_STEP1 4
#endif
#ifndef DR_FETCH_MIN_SCATTER
#define DR_FETCH_MIN_SCATTER 32
#endif

// MERGE: ray merging (Eq. 3).  A ray's luminosity is then carried
// explicitly per wavelength (FP64 outside step 1), since a merged ray's is a
// sum over four paths; each split level keeps its group's paused children.
template <int NL, int MODE, bool MERGE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MODE == 0 ? DR_WAVES_STEP1 : DR_WAVES_SCATTER, 8)))
void k_march_adaptive(const AdaptArgs A)
{
    constexpr bool STEP1 = MODE == 0;
    constexpr int kBlock = 256;
    __shared__ float4 sca[STEP1 ? 1 : kScaDirs];
    __shared__ float s_kap[NL], s_alb[NL], s_hgA[NL], s_hgB[NL], s_hgC[NL];
    __shared__ double s_esc[NL], s_cut[NL], s_skp[NL];
    // per-thread deposit staging for the cooperative scattered-light deposit
    __shared__ float s_F[STEP1 ? 1 : NL][STEP1 ? 1 : kBlock];
    __shared__ float4 s_dep[STEP1 ? 1 : kBlock];     // direction xyz, cell id (bits) in w
    // energy-density deposits of the step, written out wave-cooperatively:
    // one atomic instruction stores the NL values of 64 / NL crossings
    __shared__ float s_du[NL][kBlock];
    __shared__ int32_t s_cell[kBlock];
    __shared__ uint8_t s_list[kBlock];
    const LambdaTable *lt = A.lt;
    const int nl = lt->n_lambda;
    if (!STEP1)
        for (int i = threadIdx.x; i < kScaDirs; i += blockDim.x) sca[i] = A.dirs[i];
    if (threadIdx.x < NL) {
        const int l = threadIdx.x;
        const float g = l < nl ? lt->g[l] : 0.f;
        s_kap[l] = l < nl ? lt->kappa[l] : 0.f;
        s_alb[l] = l < nl ? lt->albedo[l] : 0.f;
        s_hgA[l] = (1.f - g * g) / (4.f * 3.14159265358979f);   // Henyey-Greenstein prefactor
        s_hgB[l] = 1.f + g * g;
        s_hgC[l] = -2.f * g;
        s_esc[l] = 0.0;
        s_cut[l] = 0.0;
        s_skp[l] = 0.0;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wbase = threadIdx.x & ~63;
    const int nsrc = *A.n_src;
    const uint64_t nitems = (uint64_t)nsrc * (uint64_t)(12 * A.nside0 * A.nside0);
    double f_U = A.f_U;
    if (!(f_U >= 0.0)) {
        const int ns_all = *A.n_all;
        f_U = ns_all > 0 ? 4.0 * A.a_RT / (double)ns_all : 0.0;
    }

    float skp[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) skp[l] = 0.f;
    uint32_t n_cross = 0, n_rays = 0, n_split = 0, n_cut = 0, n_esc = 0, n_dep = 0, n_skip = 0, n_max = 0, n_merge = 0;

    // ray state.  Step 1 carries the ray's luminosity in FP32 (its decisions
    // are geometric).  The passes that take per-wavelength significance
    // decisions (Eq. 1 / Eq. 8) carry it in FP64 per wavelength, attenuated
    // crossing by crossing as in the oracle, so no decision rests on FP32
    // rounding or underflow.
    bool has_ray = false, has_item = false, pending = false, done = false;
    int32_t s = 0;
    int32_t own_c = -1;            // the source's own cell (no split or block test there)
    double o[3] = {0.0, 0.0, 0.0};
    int depth = 0;
    int pix = 0;
    double t = 0.0;                // distance from the source, fine units
    int32_t c = -1;
    int64_t e = 0;                 // direction table entry of the ray
    RayT<double> R;
    float L[STEP1 ? NL : 1];
    double L0[STEP1 ? 1 : NL];
    double st_t[kMaxDepthAdaptive + 1];
    int32_t st_c[kMaxDepthAdaptive + 1];   // cell in which the level's parent split
    float st_L[STEP1 ? kMaxDepthAdaptive + 1 : 1][STEP1 ? NL : 1];
    // the FP64 luminosity outside step 1 and what the children of each
    // level start with
    constexpr bool XL = !STEP1;
    double Lx[XL ? NL : 1];
    double st_Lx[XL ? kMaxDepthAdaptive + 1 : 1][XL ? NL : 1];
    // merging state (MERGE only): per level the paused children (bitmask,
    // distance, cell, luminosity), the plane they crossed (0 none yet, -1 not
    // all the same) and whether the level is resuming them; bit d of
    // can_low: the ray at depth d may pause
    constexpr int KD = MERGE ? kMaxDepthAdaptive + 1 : 1;
    uint8_t g_low[KD], g_res[KD];
    int32_t g_pl[KD];
    double g_t[KD][4];
    int32_t g_c[KD][4];
    float g_Ls[MERGE && STEP1 ? KD : 1][4][MERGE && STEP1 ? NL : 1];
    double g_Ld[MERGE && XL ? KD : 1][4][MERGE && XL ? NL : 1];
    uint32_t can_low = 0;
    int32_t entry_key = 0;         // plane through which the ray entered c: 1 + axis + 3 coordinate, 0 none
    int32_t start_c = -1;          // a resumed child starts in its own cell
#pragma unroll
    for (int l = 0; l < (XL ? NL : 1); ++l) Lx[l] = 0.0;
    int64_t steps = 0;
    double omega_hp = 0.0;
#pragma unroll
    for (int l = 0; l < (STEP1 ? NL : 1); ++l) L[l] = 0.f;
#pragma unroll
    for (int l = 0; l < (STEP1 ? 1 : NL); ++l) L0[l] = 0.0;
    // luminosity the ray carries at its current position, wavelength l
    auto lum = [&](int l) -> double {
        if constexpr (STEP1) return (double)L[l];
        else return Lx[l];
    };

    while (true) {
        // ---- lanes without a ray: next sibling from the stack
        if constexpr (MERGE) {
            if (!has_ray && !pending && has_item && depth > 0) {
                // next sibling, or the end of a group: merge, resume, pop
                for (;;) {
                    const int k = pix & 3;
                    if (!g_res[depth] && k < 3) {
                        ++pix;
                        t = st_t[depth];
                        if constexpr (STEP1) {
#pragma unroll
                            for (int l = 0; l < NL; ++l) L[l] = st_L[depth][l];
                        } else {
#pragma unroll
                            for (int l = 0; l < NL; ++l) Lx[l] = st_Lx[depth][l];
                        }
                        pending = true;
                        break;
                    }
                    if (!g_res[depth]) {
                        if (g_low[depth] == 15 && g_pl[depth] > 0) {
                            // four paused siblings across one plane: the
                            // parent carries on with their summed luminosity
                            // from their mean distance (sums in ascending order)
                            ++n_merge;
                            t = 0.25 * sum4_sorted(g_t[depth][0], g_t[depth][1], g_t[depth][2], g_t[depth][3]);
                            if constexpr (STEP1) {
#pragma unroll
                                for (int l = 0; l < NL; ++l)
                                    L[l] = sum4_sorted(g_Ls[depth][0][l], g_Ls[depth][1][l], g_Ls[depth][2][l],
                                                       g_Ls[depth][3][l]);
                            } else {
#pragma unroll
                                for (int l = 0; l < NL; ++l)
                                    Lx[l] = sum4_sorted(g_Ld[depth][0][l], g_Ld[depth][1][l], g_Ld[depth][2][l],
                                                        g_Ld[depth][3][l]);
                            }
                            --depth;
                            pix >>= 2;
                            pending = true;
                            break;
                        }
                        g_res[depth] = 1;
                    }
                    if (g_low[depth]) {
                        // a paused sibling of a group that does not merge
                        // continues from where it stopped, pausing no more
                        const int kk = __builtin_ctz((unsigned)g_low[depth]);
                        g_low[depth] &= (uint8_t)~(1u << kk);
                        pix = (pix & ~3) | kk;
                        t = g_t[depth][kk];
                        start_c = g_c[depth][kk];
                        if constexpr (STEP1) {
#pragma unroll
                            for (int l = 0; l < NL; ++l) L[l] = g_Ls[depth][kk][l];
                        } else {
#pragma unroll
                            for (int l = 0; l < NL; ++l) Lx[l] = g_Ld[depth][kk][l];
                        }
                        can_low &= ~(1u << depth);
                        pending = true;
                        break;
                    }
                    g_res[depth] = 0;
                    --depth;
                    pix >>= 2;
                    if (depth == 0) break;
                }
            }
        }
        if (!has_ray && !pending && has_item) {
            while (depth > 0 && (pix & 3) == 3) {
                --depth;
                pix >>= 2;
            }
            if (depth > 0) {
                ++pix;
                t = st_t[depth];
                if constexpr (STEP1) {
#pragma unroll
                    for (int l = 0; l < NL; ++l) L[l] = st_L[depth][l];
                } else {
#pragma unroll
                    for (int l = 0; l < NL; ++l) Lx[l] = st_Lx[depth][l];
                }
                pending = true;
            } else {
                has_item = false;
                // the item's skipped luminosity joins the block's FP64 sum:
                // per-lane FP32 sums over many items would lose low bits
#pragma unroll
                for (int l = 0; l < NL; ++l)
                    if (l < nl && skp[l] != 0.f) {
                        atomicAdd(&s_skp[l], (double)skp[l]);
                        skp[l] = 0.f;
                    }
            }
        }
        // ---- ... or a new item (top pixel r0, source), 64 at a time per wave
        const bool want = !has_ray && !pending && !has_item && !done;
        const uint64_t need = __ballot(want);
        // new items are taken several lanes at a time (their set-up is a
        // divergent stretch), or when no lane has anything else to do
        constexpr int kFetchMin = STEP1 ? DR_FETCH_MIN_STEP1 : DR_FETCH_MIN_SCATTER;
        if (need && (__popcll(need) >= kFetchMin || __ballot(has_ray || pending || has_item) == 0)) {
            const int leader = __ffsll((unsigned long long)need) - 1;
            unsigned long long base = 0;
            int stop = 0;
            if (lane == leader) {
                if (!STEP1 && A.log_cap > 0 &&
                    __hip_atomic_load(A.log_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
                        (unsigned long long)A.log_limit)
                    stop = 1;   // the log is nearly full: finish current items, take no new ones
                else
                    base = atomicAdd(A.queue, (unsigned long long)__popcll(need));
            }
            base = __shfl(base, leader, 64);
            stop = __shfl(stop, leader, 64);
            if (want) {
                const uint64_t it = base + __popcll(need & ((1ull << lane) - 1ull));
                if (stop || it >= nitems) {
                    done = true;
                } else {
                    const int r0 = (int)(it / (uint64_t)nsrc);
                    s = A.src_list[it - (uint64_t)r0 * nsrc];
                    if (s < A.n) {
                        // an emitting cell: rays start at its centre, it is its own cell
                        const int4 sb = A.geo.rec[s].box;
                        const double half = 0.5 * (double)sb.w;
                        o[0] = (double)sb.x + half;
                        o[1] = (double)sb.y + half;
                        o[2] = (double)sb.z + half;
                        own_c = s;
                    } else {
                        // a point source: rays start at the point, in the leaf holding it
                        const double4 pp = A.ps_pos[s - A.n];
                        o[0] = pp.x;
                        o[1] = pp.y;
                        o[2] = pp.z;
                        own_c = A.ps_cell[s - A.n];
                    }
                    const int32_t kp = s - (int32_t)A.n;   // point index when s >= n
                    double lsum = 0.0;
                    if constexpr (STEP1) {
                        const float inv_nray0 = 1.f / (float)(12 * A.nside0 * A.nside0);
#pragma unroll
                        for (int l = 0; l < NL; ++l) {
                            L[l] = l >= nl ? 0.f
                                   : s < A.n ? A.emis_lum[(int64_t)l * A.n + s] * inv_nray0
                                             : A.ps_lum[(int64_t)l * A.n_point + kp] * inv_nray0;
                            lsum += (double)L[l];
                        }
                    } else {
                        // launch luminosity in FP64: 4 pi j V / N_ray (direct light), or
                        // S N_pix / N_ray from the pixel holding the ray (scattered light;
                        // the sum over the pixels inside the ray when rays are coarser)
                        const double nray0 = 12.0 * (double)A.nside0 * (double)A.nside0;
#pragma unroll
                        for (int l = 0; l < NL; ++l) {
                            double v = 0.0;
                            if (l < nl) {
                                if (MODE != 2) {
                                    v = (s < A.n ? A.lum64[(int64_t)l * A.n + s]
                                                 : A.ps_lum64[(int64_t)l * A.n_point + kp]) / nray0;
                                } else {
                                    const int npix = lt->npix[l];
                                    const float *row = A.S_pending + lt->s_off[l] + (int64_t)s * npix;
                                    const int ls = 31 - __clz(lt->nside_sca[l]);
                                    if (A.log2_nside0 >= ls) {
                                        v = (double)row[r0 >> (2 * (A.log2_nside0 - ls))] * (double)npix / nray0;
                                    } else {
                                        const int sh = 2 * (ls - A.log2_nside0);
                                        for (int q = r0 << sh; q < ((r0 + 1) << sh); ++q) v += (double)row[q];
                                    }
                                }
                            }
                            L0[l] = v;
                            lsum += v;
                        }
                        if constexpr (XL) {
#pragma unroll
                            for (int l = 0; l < NL; ++l) Lx[l] = L0[l];
                        }
                    }
                    can_low = 0;
                    has_item = true;
                    depth = 0;
                    pix = r0;
                    t = 0.0;
                    st_c[0] = own_c;   // a ray merged back to the launch level starts its search here
                    if (lsum > 0.0) {
                        ++n_rays;
                        pending = true;
                    }
                }
            }
        }
        // ---- start pending rays: direction, first cell.  The start is a
        // divergent stretch of code, so it waits until DR_PENDING_MIN lanes
        // have a ray to start, or no lane has one to march
        const uint64_t pend_m = __ballot(pending);
        const bool start_now = __popcll(pend_m) >= DR_PENDING_MIN || __ballot(has_ray) == 0;
        if (pending && start_now) {
            pending = false;
            const int64_t N = (int64_t)A.nside0 << depth;
            e = entry_of(N, pix);
            const double4 nd = A.dirs64[e];
            R.n[0] = nd.x;
            R.n[1] = nd.y;
            R.n[2] = nd.z;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                R.o[a] = o[a];
                R.inv[a] = 1.0 / R.n[a];
            }
            omega_hp = kPi / (3.0 * (double)N * (double)N);   // 4 pi / (12 N^2)
            steps = 0;
            entry_key = 0;
            if (MERGE && start_c >= 0) {
                c = start_c;
                start_c = -1;
            } else if (t == 0.0) {
                c = own_c;
            } else {
                // a child starts at its parent's entry distance: mostly inside
                // the cell where the parent split, which then needs no descent
                const int fx = fine_coord<double>(fma(t, R.n[0], o[0]), R.n[0], A.geo.fine[0]);
                const int fy = fine_coord<double>(fma(t, R.n[1], o[1]), R.n[1], A.geo.fine[1]);
                const int fz = fine_coord<double>(fma(t, R.n[2], o[2]), R.n[2], A.geo.fine[2]);
                const int32_t cp = st_c[depth];
                const int4 pb = A.geo.rec[cp].box;
                const bool inside = fx >= pb.x && fx < pb.x + pb.w && fy >= pb.y && fy < pb.y + pb.w &&
                                    fz >= pb.z && fz < pb.z + pb.w;
                c = inside ? cp : locate_fine(A.geo, fx, fy, fz);
            }
            if (c >= 0) {
                has_ray = true;
            } else {
#pragma unroll
                for (int l = 0; l < NL; ++l)
                    if (l < nl) atomicAdd(&s_esc[l], lum(l));
                ++n_esc;
            }
        }
        if (__ballot(has_ray) == 0) {
            if (__ballot(has_item || pending) == 0) break;
            continue;
        }

        // ---- one crossing per lane with a ray
        bool deposit = false;
        bool udep = false;
        int dslot = 0;   // this lane's slot in the wave's compacted deposit staging
        if (has_ray) {
            const LeafRec &rc = A.geo.rec[c];
            const int4 b = rc.box;
            const float rho_c = rc.rho;
            int32_t nbc[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) nbc[q] = rc.nb[q];
            int axis;
            double te = exit_t<double>(R, b, axis);
            if (STEP1 && fabs(te - A.r_pre_fine64) <= 1e-9 * A.r_pre_fine64) {
                // HEALPix z components are rational and cell faces lie on an
                // integer lattice, so a face can sit exactly at the step-1
                // extent: take the correctly rounded quotient there, which is
                // exact whenever the exact distance is representable
                const double face = (R.n[axis] > 0.0) ? (double)((axis == 0 ? b.x : axis == 1 ? b.y : b.z) + b.w)
                                                       : (double)(axis == 0 ? b.x : axis == 1 ? b.y : b.z);
                te = (face - R.o[axis]) / R.n[axis];
            }
            const double len = te - t;
            int action = 0;   // 0 continue, 1 split, 2 cut
            if (!is_graze(len, te)) {
                const double t_in = t;
                // source-to-cell-centre offsets are exact half-integers in fine units
                const double dx = ((double)b.x + 0.5 * (double)b.w - o[0]);
                const double dy = ((double)b.y + 0.5 * (double)b.w - o[1]);
                const double dz = ((double)b.z + 0.5 * (double)b.w - o[2]);
                const double h = A.h_fine64;
                const double d2 = (dx * dx + dy * dy + dz * dz) * (h * h);
                const double side = (double)b.w * h;
                const float lp = (float)(len * h);
                // step 1: e^{-tau} - 1 per wavelength (FP32); other passes: the
                // mean luminosity over the crossing <L> = L (1 - e^{-tau}) / tau
                // in FP64, from which the deposit, the extinguished luminosity
                // and the transmission follow
                float em1[STEP1 ? NL : 1];
                double lavg64[STEP1 ? 1 : NL];
                uint32_t sigm = 0;
                const float *ull = A.ull_t + (int64_t)c * nl;
                if constexpr (STEP1) {
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        em1[l] = 0.f;
                        if (l < nl) {
                            const float tau = s_kap[l] * rho_c * lp;
                            bool thick;
                            float tr;
                            em1[l] = fast_em1(tau, thick, tr);
                            sigm |= 1u << l;
                        }
                    }
                } else {
                    // Eq. 8 estimate <L> / (Omega_HP d^2 c) against f_U U_LL (Eq. 1), in FP64
                    const double lenp = len * h;
                    const double inv_den = 1.0 / (omega_hp * d2 * A.c_light);
                    double tau[NL];
                    double tmax = 0.0;
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        tau[l] = (double)s_kap[l] * (double)rho_c * lenp;   // zero beyond n_lambda
                        tmax = fmax(tmax, tau[l]);
                    }
                    const bool thin = __ballot(tmax >= 0.5) == 0;
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        const double g = thin || tau[l] < 0.5 ? g_series64(tau[l]) : -expm1(-tau[l]) / tau[l];
                        const double lavg = lum(l) * g;
                        const bool sg = l < nl && lavg > 0.0 &&
                                        (c == own_c || lavg * inv_den >= f_U * (double)ull[l < nl ? l : 0]);
                        sigm |= (uint32_t)sg << l;
                        lavg64[l] = lavg;
                    }
                }
                if (STEP1 && t_in >= A.r_pre_fine64) {
                    action = 2;
                } else if (c != own_c && omega_hp * (double)A.n_rays * d2 > side * side) {   // Eq. 2
                    if (sigm && depth < A.max_depth) action = 1;
                    else if (!sigm) action = 2;
                } else if (MERGE && ((can_low >> depth) & 1u) && depth > 0 && c != own_c &&
                           omega_hp * A.n_rays_max * d2 < side * side) {                      // Eq. 3
                    action = 3;
                }
                if (action == 1) {
                    // split: child 0 starts next iteration, siblings wait on the stack
                    ++n_split;
                    ++depth;
                    st_t[depth] = t_in;
                    st_c[depth] = c;
                    if constexpr (STEP1) {
#pragma unroll
                        for (int l = 0; l < NL; ++l) {
                            L[l] *= 0.25f;
                            st_L[depth][l] = L[l];
                        }
                    } else {
#pragma unroll
                        for (int l = 0; l < NL; ++l) {
                            Lx[l] *= 0.25;
                            st_Lx[depth][l] = Lx[l];
                        }
                    }
                    if constexpr (MERGE) {
                        g_low[depth] = 0;
                        g_res[depth] = 0;
                        g_pl[depth] = 0;
                        can_low |= 1u << depth;
                    }
                    pix = 4 * pix;
                    t = t_in;
                    has_ray = false;
                    pending = true;
                } else if (MERGE && action == 3) {
                    // paused before this crossing, nothing deposited: the
                    // group decides at its end (merge, or carry on)
                    const int k = pix & 3;
                    g_t[depth][k] = t_in;
                    g_c[depth][k] = c;
                    if constexpr (STEP1) {
#pragma unroll
                        for (int l = 0; l < NL; ++l) g_Ls[depth][k][l] = L[l];
                    } else {
#pragma unroll
                        for (int l = 0; l < NL; ++l) g_Ld[depth][k][l] = Lx[l];
                    }
                    g_low[depth] |= (uint8_t)(1u << k);
                    const int32_t key = entry_key > 0 ? entry_key : -1;
                    g_pl[depth] = g_pl[depth] == 0 ? key : (g_pl[depth] == key ? key : -1);
                    has_ray = false;
                } else if (action == 2) {
                    ++n_cut;
#pragma unroll
                    for (int l = 0; l < NL; ++l)
                        if (l < nl) atomicAdd(&s_cut[l], lum(l));
                    has_ray = false;
                } else {
                    const float ivc = rc.ivc;
                    ++n_cross;
                    ++steps;   // the per-ray limit counts crossings of positive length
                    udep = true;
                    // the lanes depositing in this step fill the staging in lane order
                    dslot = wbase + __popcll(__ballot(true) & ((1ull << lane) - 1ull));
                    s_cell[dslot] = c;
                    const float *izr = A.invz + e * nl;
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        if (l < nl) {
                            if constexpr (STEP1) {
                                const float ext = -L[l] * em1[l];
                                const float alpha = s_kap[l] * rho_c;
                                s_du[l][dslot] = alpha > 0.f ? ext * ivc * __builtin_amdgcn_rcpf(alpha) : L[l] * lp * ivc;
                                ++n_dep;
                                // transmission, fused; e^{-tau} again in thick cells (1 + em1 cancels)
                                const float tau = alpha * lp;
                                L[l] = tau < 0.5f ? fmaf(L[l], em1[l], L[l])
                                                  : L[l] * __builtin_amdgcn_exp2f(-tau * 1.44269504088896341f);
                            } else {
                                // extinguished luminosity <L> tau, deposit <L> l / (V c)
                                const double lenp = len * h;
                                const double tau = (double)s_kap[l] * (double)rho_c * lenp;
                                const double ext = lavg64[l] * tau;
                                const float ext32 = (float)ext;
                                float Fl = 0.f;
                                float du = 0.f;
                                if ((sigm >> l) & 1u) {
                                    du = (float)(lavg64[l] * lenp * (double)ivc);
                                    ++n_dep;
                                    Fl = s_alb[l] * ext32 * izr[l] * s_hgA[l];
                                } else {
                                    skp[l] += ext32;
                                    ++n_skip;
                                }
                                // transmission: L - <L> tau = L e^{-tau} below tau 0.5, where
                                // it keeps extinguished + transmitted equal to the input
                                Lx[l] = tau < 0.5 ? Lx[l] - ext : Lx[l] * exp(-tau);
                                s_F[l][threadIdx.x] = Fl;
                                deposit |= Fl != 0.f;
                                s_du[l][dslot] = du;
                            }
                        }
                    }
                    if constexpr (!STEP1) {
                        if (deposit)
                            s_dep[threadIdx.x] =
                                make_float4((float)R.n[0], (float)R.n[1], (float)R.n[2], __int_as_float(c));
                    }
                    t = te;
                }
            }
            if (has_ray && action == 0) {
                const int32_t nx = next_leaf<double>(A.geo, R, b, nbc, axis, te);
                if (nx < 0) {
#pragma unroll
                    for (int l = 0; l < NL; ++l)
                        if (l < nl) atomicAdd(&s_esc[l], lum(l));
                    ++n_esc;
                    has_ray = false;
                } else if ((A.max_steps > 0 && steps >= A.max_steps) || steps >= A.hard_cap) {
                    ++n_max;
                    has_ray = false;
                } else {
                    if constexpr (MERGE) {
                        // the plane of the face the ray leaves c by
                        const bool pos = axis == 0 ? R.n[0] > 0.0 : axis == 1 ? R.n[1] > 0.0 : R.n[2] > 0.0;
                        const int lo_a = axis == 0 ? b.x : axis == 1 ? b.y : b.z;
                        entry_key = 1 + axis + 3 * (pos ? lo_a + b.w : lo_a);
                    }
                    c = nx;
                }
            }
        }

        // ---- energy-density deposits: lanes q of an instruction take value
        // q % NL of the (q / NL)-th depositing lane, so each crossing's NL
        // values go out as one contiguous request
        // ---- log the deposits (scattering passes); what does not fit in the
        // log is deposited with atomics below
        if (!STEP1 && A.log_cap > 0) {
            const uint64_t lm = __ballot(udep);
            if (lm) {
                const int leader = __ffsll((unsigned long long)lm) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(A.log_count, (unsigned long long)__popcll(lm));
                base = __shfl(base, leader, 64);
                if (udep) {
                    const unsigned long long slot = base + __popcll(lm & ((1ull << lane) - 1ull));
                    if (slot < (unsigned long long)A.log_cap) {
                        A.log_key[slot] = ((uint64_t)(uint32_t)s_cell[dslot] << A.log_dir_bits) | (uint64_t)e;
#pragma unroll
                        for (int l = 0; l < NL; ++l)
                            if (l < nl) A.log_du[(int64_t)l * A.log_cap + slot] = s_du[l][dslot];
                        udep = false;
                        deposit = false;
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        {
            // step 1: every depositing lane's row sits at its compacted slot;
            // other passes: the lanes the log did not take are listed by slot
            const uint64_t um = __ballot(udep);
            if (!STEP1 && udep) s_list[wbase + __popcll(um & ((1ull << lane) - 1ull))] = (uint8_t)(dslot - wbase);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int cnt = __popcll(um);
            constexpr int PER = 64 / NL;
            for (int k0 = 0; k0 < cnt; k0 += PER) {
                const int q = k0 + lane / NL;
                const int l = lane % NL;
                if (q < cnt && l < nl) {
                    const int j = STEP1 ? q : (int)s_list[wbase + q];
                    const float v = s_du[l][wbase + j];
                    // 32-bit row offsets: n * n_lambda < 2^32 is checked at grid creation
                    const uint32_t off = (uint32_t)s_cell[wbase + j] * (uint32_t)nl + (uint32_t)l;
                    if (STEP1 || v != 0.f) atomic_add_f64(A.U_k + off, (double)v);
                }
            }
        }

        // ---- cooperative scattered-light deposit: for each depositing lane,
        // the wave adds its phase-weighted luminosity to the cell's pixel row
        if (!STEP1) {
            uint64_t m = __ballot(deposit);
            while (m) {
                const int j = __ffsll((unsigned long long)m) - 1;
                m &= m - 1;
                const float4 dj = s_dep[wbase + j];
                const int cj = __float_as_int(dj.w);
                for (int l = 0; l < nl; ++l) {
                    const float Fj = s_F[l][wbase + j];
                    if (Fj == 0.f) continue;
                    const int npix = lt->npix[l];
                    const int base = (int)entry_of(lt->nside_sca[l], 0);
                    float *dst = A.S_next + lt->s_off[l] + (int64_t)cj * npix;
                    const float B = s_hgB[l], Cc = s_hgC[l];
                    for (int p = lane; p < npix; p += 64) {
                        const float4 v = sca[base + p];
                        const float mu = fmaf(v.x, dj.x, fmaf(v.y, dj.y, v.z * dj.z));
                        const float r = rsqrtf(fmaf(Cc, mu, B));
                        atomic_add_f32(dst + p, Fj * (r * r * r));
                    }
                }
            }
        }
    }
    (void)done;

    // ---- FP64 tallies per block (skipped: what the lanes still hold)
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        if (l < nl) {
            const double vs = wave_sum((double)skp[l]);
            if (vs != 0.0 && lane == 0) atomicAdd(&s_skp[l], vs);
        }
    }
    if (A.counters) {
        const uint64_t v[9] = {wave_sum_u64(n_cross), wave_sum_u64(n_rays), wave_sum_u64(n_split), wave_sum_u64(n_cut),
                               wave_sum_u64(n_esc), wave_sum_u64(n_dep), wave_sum_u64(n_skip), wave_sum_u64(n_max),
                               MERGE ? wave_sum_u64(n_merge) : 0};
        if (lane == 0)
            for (int i = 0; i < 9; ++i)
                if (v[i]) atomicAdd((unsigned long long *)&A.counters[i], (unsigned long long)v[i]);
    }
    __syncthreads();
    if (threadIdx.x < NL && threadIdx.x < nl) {
        const int l = threadIdx.x;
        if (s_esc[l] != 0.0) atomic_add_f64(&A.tally[l * DARTRAY_N_TALLY + DARTRAY_T_ESCAPED], s_esc[l]);
        if (s_cut[l] != 0.0) atomic_add_f64(&A.tally[l * DARTRAY_N_TALLY + DARTRAY_T_CUT], s_cut[l]);
        if (s_skp[l] != 0.0) atomic_add_f64(&A.tally[l * DARTRAY_N_TALLY + DARTRAY_T_SKIPPED], s_skp[l]);
    }
}

// ---------------------------------------------------------------------------
// Step 1 by teams of four lanes (step-1 rays of Sect. 3.2, split by Eq. 2).
//
// The four children of a split start at one point with nearly parallel
// directions and cross many cells together, so the four lanes of a quad
// march them side by side, one crossing each per iteration, and the
// crossings of an iteration that deposit into the same cell add their rows
// inside the quad (DPP moves) before one atomic row goes out.  A quad's work
// item is one source and four nested launch pixels 4m .. 4m+3, which also
// start together, at the source.  The quad walks the item's ray tree group
// by group, depth first: a ray that splits leaves its children's start
// (entry distance, split cell, quarter luminosity, parent pixel) in its
// lane's slot of the next level and stops; once all four lanes have stopped,
// the quad starts the children of the deepest level holding a slot (lowest
// lane first), or takes a new item.  A lane holds at most one slot per
// level: the slots of a level all come from the single group running one
// level above, and deeper levels are emptied before another group of that
// level starts.  Same rays, crossings and counters as the lane-per-item
// march; only the order of the FP64 atomic adds and the FP32 pre-sums of
// equal-cell rows differ.
// ---------------------------------------------------------------------------

template <int NL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DR_WAVES_STEP1, 8)))
void k_step1_quad(const AdaptArgs A)
{
    constexpr int kBlock = 256;
    constexpr int KD = kMaxDepthAdaptive + 1;
    __shared__ float s_kap[NL];
    __shared__ double s_esc[NL], s_cut[NL];
    __shared__ float s_du[NL][kBlock];
    __shared__ int32_t s_cell[kBlock];
    // a starting group's slot, one per quad
    __shared__ double g_t[kBlock / 4];
    __shared__ int32_t g_c[kBlock / 4], g_p[kBlock / 4];
    __shared__ float g_L[NL][kBlock / 4];
    const LambdaTable *lt = A.lt;
    const int nl = lt->n_lambda;
    if (threadIdx.x < NL) {
        const int l = threadIdx.x;
        s_kap[l] = l < nl ? lt->kappa[l] : 0.f;
        s_esc[l] = 0.0;
        s_cut[l] = 0.0;
    }
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wbase = threadIdx.x & ~63;
    const int qbase = lane & ~3;          // first lane of this lane's quad
    const int qk = lane & 3;              // place in the quad: the child index within a group
    const int qi = threadIdx.x >> 2;      // the quad's slot in the block
    const int nsrc = *A.n_src;
    const uint64_t nitems = (uint64_t)nsrc * (uint64_t)(3 * A.nside0 * A.nside0);
    // event counts of the wave (uniform: ballots of per-lane events)
    uint64_t n_cross = 0, n_rows = 0;
    uint32_t n_rays = 0, n_split = 0, n_cut = 0, n_esc = 0, n_max = 0;

    bool has_ray = false, pending = false, done = false;
    int32_t s = 0;
    int32_t own_c = -1;
    int depth = 0;
    int pix = 0;
    double t = 0.0;
    int32_t c = -1;
    int32_t hint_c = -1;              // the cell the parent split in (children start there mostly)
    RayT<double> R;              // origin set per item (all its rays start at the source)
#pragma unroll
    for (int a = 0; a < 3; ++a) R.o[a] = R.n[a] = R.inv[a] = 0.0;
    float L[NL];
    // luminosity of this lane's cut rays within the current item (FP32, a
    // few hundred rays), folded into the block's FP64 sums between items
    float cut_acc[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) L[l] = cut_acc[l] = 0.f;
    auto flush_cuts = [&]() {
#pragma unroll
        for (int l = 0; l < NL; ++l)
            if (l < nl && cut_acc[l] != 0.f) {
                atomicAdd(&s_cut[l], (double)cut_acc[l]);
                cut_acc[l] = 0.f;
            }
    };
    double omega_hp = 0.0;
    // solid angle of a launch pixel; a power of two smaller per level
    const double omega_hp0 = kPi / (3.0 * (double)A.nside0 * (double)A.nside0);
    int32_t steps = 0;
    // this lane's waiting children group per level
    double w_t[KD];
    int32_t w_c[KD], w_p[KD];
    float w_L[KD][NL];
    uint32_t w_mask = 0;
    // the row this lane holds for one more step: cell (-1 none), values
    int32_t h_cell = -1;
    float h_du[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) h_du[l] = 0.f;
    // the wave's rows go out as atomic requests of NL FP64 values: lanes q of
    // an instruction take value q % NL of the (q / NL)-th row
    auto emit_rows = [&](bool has, int32_t cell, const float *vals) {
        const uint64_t om = __ballot(has);
        if (has) {
            const int slot = wbase + __popcll(om & ((1ull << lane) - 1ull));
            s_cell[slot] = cell;
#pragma unroll
            for (int l = 0; l < NL; ++l) s_du[l][slot] = vals[l];
        }
        wave_sync_lds();
        const int cnt = __popcll(om);
        constexpr int PER = 64 / NL;
        for (int k0 = 0; k0 < cnt; k0 += PER) {
            const int q = k0 + lane / NL;
            const int l = lane % NL;
            if (q < cnt && l < nl) {
                const float v = s_du[l][wbase + q];
                // 32-bit row offsets: n * n_lambda < 2^32 is checked at grid creation
                const uint32_t off = (uint32_t)s_cell[wbase + q] * (uint32_t)nl + (uint32_t)l;
                atomic_add_f64(A.U_k + off, (double)v);
            }
        }
        wave_sync_lds();
    };

    while (true) {
        // ---- quads whose four lanes have stopped: the deepest waiting group
        const uint64_t busy = __ballot(has_ray || pending);
        const bool q_idle = ((busy >> qbase) & 0xFull) == 0 && !done;
        uint32_t qm = q_idle ? w_mask : 0u;
        qm |= (uint32_t)quad_rot<1>((int)qm);
        qm |= (uint32_t)quad_rot<2>((int)qm);
        if (__ballot(qm != 0u)) {
            const int D = qm ? 31 - __clz(qm) : 0;
            const bool has_D = qm != 0u && ((w_mask >> D) & 1u);
            const uint32_t nib = (uint32_t)(__ballot(has_D) >> qbase) & 0xFu;
            if (has_D && qk == __builtin_ctz(nib | 16u)) {
                g_t[qi] = w_t[D];
                g_c[qi] = w_c[D];
                g_p[qi] = w_p[D];
#pragma unroll
                for (int l = 0; l < NL; ++l) g_L[l][qi] = w_L[D][l];
                w_mask &= ~(1u << D);
            }
            wave_sync_lds();
            if (qm != 0u) {
                depth = D;
                pix = 4 * g_p[qi] + qk;
                t = g_t[qi];
                hint_c = g_c[qi];
#pragma unroll
                for (int l = 0; l < NL; ++l) L[l] = g_L[l][qi];
                pending = true;
            }
            wave_sync_lds();
        }
        // events of this step, counted per wave below
        bool ev_launch = false, ev_esc = false, ev_split = false, ev_cut = false, ev_max = false;
        // ---- ... or a new item (source, launch pixels 4m .. 4m+3)
        const bool q_new = q_idle && qm == 0u;
        const uint64_t need = __ballot(q_new && qk == 0);
        if (need) {
            const int leader = __ffsll((unsigned long long)need) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(A.queue, (unsigned long long)__popcll(need));
            base = __shfl(base, leader, 64);
            if (q_new) {
                flush_cuts();
                const uint64_t it = base + __popcll(need & ((1ull << qbase) - 1ull));
                if (it >= nitems) {
                    done = true;
                } else {
                    const int m = (int)(it / (uint64_t)nsrc);
                    s = A.src_list[it - (uint64_t)m * nsrc];
                    if (s < A.n) {
                        const int4 sb = A.geo.rec[s].box;
                        const double half = 0.5 * (double)sb.w;
                        R.o[0] = (double)sb.x + half;
                        R.o[1] = (double)sb.y + half;
                        R.o[2] = (double)sb.z + half;
                        own_c = s;
                    } else {
                        const double4 pp = A.ps_pos[s - A.n];
                        R.o[0] = pp.x;
                        R.o[1] = pp.y;
                        R.o[2] = pp.z;
                        own_c = A.ps_cell[s - A.n];
                    }
                    const int32_t kp = s - (int32_t)A.n;
                    const float inv_nray0 = 1.f / (float)(12 * A.nside0 * A.nside0);
                    double lsum = 0.0;
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        L[l] = l >= nl ? 0.f
                               : s < A.n ? A.emis_lum[(int64_t)l * A.n + s] * inv_nray0
                                         : A.ps_lum[(int64_t)l * A.n_point + kp] * inv_nray0;
                        lsum += (double)L[l];
                    }
                    depth = 0;
                    pix = 4 * m + qk;
                    t = 0.0;
                    hint_c = own_c;
                    pending = lsum > 0.0;
                    ev_launch = pending;
                }
            }
        }
        // ---- start the rays of new groups: direction, first cell
        if (pending) {
            pending = false;
            const int64_t N = (int64_t)A.nside0 << depth;
            const double4 nd = A.dirs64[entry_of(N, pix)];
            R.n[0] = nd.x;
            R.n[1] = nd.y;
            R.n[2] = nd.z;
#pragma unroll
            for (int a = 0; a < 3; ++a) R.inv[a] = 1.0 / R.n[a];
            omega_hp = ldexp(omega_hp0, -2 * depth);   // 4 pi / (12 N^2), exactly
            steps = 0;
            if (t == 0.0) {
                c = own_c;
            } else {
                const int fx = fine_coord<double>(fma(t, R.n[0], R.o[0]), R.n[0], A.geo.fine[0]);
                const int fy = fine_coord<double>(fma(t, R.n[1], R.o[1]), R.n[1], A.geo.fine[1]);
                const int fz = fine_coord<double>(fma(t, R.n[2], R.o[2]), R.n[2], A.geo.fine[2]);
                const int4 pb = A.geo.rec[hint_c].box;
                const bool inside = fx >= pb.x && fx < pb.x + pb.w && fy >= pb.y && fy < pb.y + pb.w &&
                                    fz >= pb.z && fz < pb.z + pb.w;
                c = inside ? hint_c : locate_fine(A.geo, fx, fy, fz);
            }
            if (c >= 0) {
                has_ray = true;
            } else {
#pragma unroll
                for (int l = 0; l < NL; ++l)
                    if (l < nl) atomicAdd(&s_esc[l], (double)L[l]);
                ev_esc = true;
            }
        }
        if (__ballot(!done) == 0) break;

        // ---- one crossing per lane with a ray
        bool udep = false;
        int32_t dcell = -1;
        float du[NL];
#pragma unroll
        for (int l = 0; l < NL; ++l) du[l] = 0.f;
        if (has_ray) {
            const LeafRec &rc = A.geo.rec[c];
            const int4 b = rc.box;
            const float rho_c = rc.rho;
            int32_t nbc[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) nbc[q] = rc.nb[q];
            int axis;
            double te = exit_t<double>(R, b, axis);
            if (fabs(te - A.r_pre_fine64) <= 1e-9 * A.r_pre_fine64) {
                // a face exactly at the step-1 extent (rational HEALPix z
                // components, faces on an integer lattice): the correctly
                // rounded quotient, exact when the distance is representable.
                // (Selects, not a runtime index into the ray, which would keep
                // the ray in scratch memory.)
                const double na = axis == 0 ? R.n[0] : axis == 1 ? R.n[1] : R.n[2];
                const double oa = axis == 0 ? R.o[0] : axis == 1 ? R.o[1] : R.o[2];
                const int la = axis == 0 ? b.x : axis == 1 ? b.y : b.z;
                const double face = (double)(na > 0.0 ? la + b.w : la);
                te = (face - oa) / na;
            }
            const double len = te - t;
            int action = 0;   // 0 continue, 1 split, 2 cut
            if (!is_graze(len, te)) {
                const double t_in = t;
                const double dx = ((double)b.x + 0.5 * (double)b.w - R.o[0]);
                const double dy = ((double)b.y + 0.5 * (double)b.w - R.o[1]);
                const double dz = ((double)b.z + 0.5 * (double)b.w - R.o[2]);
                const double h = A.h_fine64;
                const double d2 = (dx * dx + dy * dy + dz * dz) * (h * h);
                const double side = (double)b.w * h;
                const float lp = (float)(len * h);
                if (t_in >= A.r_pre_fine64) {
                    action = 2;
                } else if (c != own_c && omega_hp * (double)A.n_rays * d2 > side * side) {   // Eq. 2
                    if (nl > 0 && depth < A.max_depth) action = 1;
                    else if (nl == 0) action = 2;
                }
                if (action == 1) {
                    // split: the children's start waits in this lane's slot of the next level
                    ev_split = true;
                    const int d1 = depth + 1;
                    w_t[d1] = t_in;
                    w_c[d1] = c;
                    w_p[d1] = pix;
#pragma unroll
                    for (int l = 0; l < NL; ++l) w_L[d1][l] = 0.25f * L[l];
                    w_mask |= 1u << d1;
                    has_ray = false;
                } else if (action == 2) {
                    ev_cut = true;
#pragma unroll
                    for (int l = 0; l < NL; ++l) cut_acc[l] += L[l];
                    has_ray = false;
                } else {
                    const float lpv = lp * rc.ivc;
                    ++steps;   // the per-ray limit counts crossings of positive length
                    udep = true;
                    dcell = c;
                    // optical depths (zero beyond n_lambda, where L is zero too)
                    float tau[NL];
                    float tmax = 0.f;
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        tau[l] = s_kap[l] * rho_c * lp;
                        tmax = fmaxf(tmax, tau[l]);
                    }
                    // extinguished luminosity L tau g, energy density L g l / (V c)
                    // with g = (1 - e^{-tau}) / tau (1 when the cell is empty);
                    // when every crossing of the wave is optically thin the
                    // series serves all wavelengths without a branch
                    if (__ballot(tmax >= 0.5f) == 0) {
#pragma unroll
                        for (int l = 0; l < NL; ++l) {
                            const float Lg = L[l] * g_series(tau[l]);
                            du[l] = Lg * lpv;
                            L[l] = fmaf(-tau[l], Lg, L[l]);
                        }
                    } else {
#pragma unroll
                        for (int l = 0; l < NL; ++l) {
                            bool thick;
                            float tr;
                            const float Lg = L[l] * fast_g(tau[l], thick, tr);
                            du[l] = Lg * lpv;
                            L[l] = thick ? L[l] * tr : fmaf(-tau[l], Lg, L[l]);
                        }
                    }
                    t = te;
                }
            }
            if (has_ray && action == 0) {
                const int32_t nx = next_leaf<double>(A.geo, R, b, nbc, axis, te);
                if (nx < 0) {
#pragma unroll
                    for (int l = 0; l < NL; ++l)
                        if (l < nl) atomicAdd(&s_esc[l], (double)L[l]);
                    ev_esc = true;
                    has_ray = false;
                } else if ((A.max_steps > 0 && steps >= A.max_steps) || steps >= A.hard_cap) {
                    ev_max = true;
                    has_ray = false;
                } else {
                    c = nx;
                }
            }
        }

        n_cross += (uint64_t)__popcll(__ballot(udep));
        n_rays += (uint32_t)__popcll(__ballot(ev_launch));
        n_esc += (uint32_t)__popcll(__ballot(ev_esc));
        n_split += (uint32_t)__popcll(__ballot(ev_split));
        n_cut += (uint32_t)__popcll(__ballot(ev_cut));
        n_max += (uint32_t)__popcll(__ballot(ev_max));

        // ---- energy-density rows.  A row stays with its quad for one more
        // step: a sibling one crossing behind (it cut a corner its siblings
        // missed) still adds to it.  Then (1) the quad's deposits into cells
        // whose rows are held join them; (2) of the other deposits, the
        // lowest lane of each cell takes the row of that cell; (3) the held
        // rows go out; (4) the new rows are held.
        const int32_t c1 = quad_rot<1>(dcell), c2 = quad_rot<2>(dcell), c3 = quad_rot<3>(dcell);
        const int32_t h1 = quad_rot<1>(h_cell), h2 = quad_rot<2>(h_cell), h3 = quad_rot<3>(h_cell);
        const bool joined = udep && (dcell == h_cell || dcell == h1 || dcell == h2 || dcell == h3);
        const bool held = h_cell >= 0;
        // lane (k + r) & 3 deposits into this lane's held cell
        const bool p0 = held && dcell == h_cell, p1 = held && c1 == h_cell, p2 = held && c2 == h_cell,
                   p3 = held && c3 == h_cell;
        // cells equal to a fresh deposit's are fresh deposits too (held cells
        // are distinct within the quad)
        const bool fresh = udep && !joined;
        const bool e1 = fresh && c1 == dcell, e2 = fresh && c2 == dcell, e3 = fresh && c3 == dcell;
        // lane (k + r) & 3 lies below this one when k + r >= 4
        const bool owner = fresh && !(e1 && qk >= 3) && !(e2 && qk >= 2) && !(e3 && qk >= 1);
        const bool a1 = owner && e1 && qk < 3, a2 = owner && e2 && qk < 2, a3 = owner && e3 && qk < 1;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            const float v1 = quad_rot_f<1>(du[l]), v2 = quad_rot_f<2>(du[l]), v3 = quad_rot_f<3>(du[l]);
            float hv = h_du[l];
            if (p0) hv += du[l];
            if (p1) hv += v1;
            if (p2) hv += v2;
            if (p3) hv += v3;
            h_du[l] = hv;
            float v = du[l];
            if (a1) v += v1;
            if (a2) v += v2;
            if (a3) v += v3;
            du[l] = v;
        }
        emit_rows(held, h_cell, h_du);
        n_rows += (uint64_t)__popcll(__ballot(owner));
        h_cell = owner ? dcell : -1;
#pragma unroll
        for (int l = 0; l < NL; ++l) h_du[l] = du[l];
    }
    emit_rows(h_cell >= 0, h_cell, h_du);
    flush_cuts();

    if (A.counters) {
        // every deposit of step 1 covers all wavelengths
        const uint64_t v[10] = {n_cross, n_rays, n_split, n_cut, n_esc, n_cross * (uint64_t)nl, 0, n_max, 0, n_rows};
        if (lane == 0)
            for (int i = 0; i < 10; ++i)
                if (v[i]) atomicAdd((unsigned long long *)&A.counters[i], (unsigned long long)v[i]);
    }
    __syncthreads();
    if (threadIdx.x < NL && threadIdx.x < nl) {
        const int l = threadIdx.x;
        if (s_esc[l] != 0.0) atomic_add_f64(&A.tally[l * DARTRAY_N_TALLY + DARTRAY_T_ESCAPED], s_esc[l]);
        if (s_cut[l] != 0.0) atomic_add_f64(&A.tally[l * DARTRAY_N_TALLY + DARTRAY_T_CUT], s_cut[l]);
    }
}

// ---------------------------------------------------------------------------
// Expansion of the sorted deposit log.  Thread slots cover every
// (wavelength, j_sca pixel) pair, and the first n_lambda threads also sum the
// energy density; a block walks a contiguous range of tuples sorted by
// (cell, direction), accumulates each cell's contributions in compensated
// (Kahan) registers and adds them to S_next / U_k when the cell changes.
// Tuples of one cell and one direction (rays of different sources in the
// same pixel) are summed first and their phase function evaluated once.
// The scattered luminosity of a tuple is albedo c alpha V du w(p|n) (the
// deposit du = ext / (alpha V c)).
// ---------------------------------------------------------------------------

constexpr int kExpandSlots = 8;        // pixel slots per thread: up to 2048 per block
constexpr int kExpandBatch = 64;       // tuples staged in LDS at a time

__global__ void k_iota(uint32_t *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (uint32_t)i;
}

struct ExpandArgs {
    const uint64_t *key;       // sorted keys (cell << dir_bits) | direction entry
    const uint32_t *idx;       // tuple index of each sorted entry
    const float *du;           // [nl][cap]
    const float4 *dirs;
    const float *invz;
    const LambdaTable *lt;
    const LeafRec *rec;
    double *U_k;
    float *S_next;
    int64_t cnt;
    int64_t cap;
    int64_t chunk;
    int32_t w_row;
    int32_t dir_bits;
};

#ifndef DR_WAVES_EXPAND
#define DR_WAVES_EXPAND 4
#endif

template <int NL, int SLOTS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DR_WAVES_EXPAND, 8)))
void k_expand(const ExpandArgs X)
{
    __shared__ float4 sca[kScaDirs];
    __shared__ int32_t t_cell[kExpandBatch];
    __shared__ float4 t_n[kExpandBatch];
    __shared__ float t_a[NL + 1][kExpandBatch];   // du / Z per wavelength; row NL stays zero
    __shared__ float t_du[NL][kExpandBatch];
    __shared__ uint8_t t_same[kExpandBatch];     // same (cell, direction) as the tuple before
    __shared__ uint8_t t_head[kExpandBatch];     // the first tuple of each run, in order
    __shared__ int t_nhead;
    const LambdaTable *lt = X.lt;
    const int nl = lt->n_lambda;
    for (int i = threadIdx.x; i < kScaDirs; i += blockDim.x) sca[i] = X.dirs[i];
    if (threadIdx.x < kExpandBatch) t_a[NL][threadIdx.x] = 0.f;
    __syncthreads();

    // slot k of this thread is pixel slot threadIdx.x + 256 k of the
    // concatenated per-wavelength rows; the Henyey-Greenstein denominator is
    // hB + (hC n_p) . n, so each slot keeps hC n_p and hB.  Slots past the
    // rows read the zero row of t_a.
    int lam[SLOTS];
    float cx[SLOTS], cy[SLOTS], cz[SLOTS], hb[SLOTS], acc[SLOTS], cmp[SLOTS], part[SLOTS];
#pragma unroll
    for (int k = 0; k < SLOTS; ++k) {
        const int sl = threadIdx.x + 256 * k;
        lam[k] = NL;
        cx[k] = cy[k] = cz[k] = 0.f;
        hb[k] = 1.f;
        acc[k] = cmp[k] = part[k] = 0.f;
        if (sl < X.w_row) {
            int l = 0;
            while (l + 1 < nl && lt->w_off[l + 1] <= sl) ++l;
            lam[k] = l;
            const float4 v = sca[entry_of(lt->nside_sca[l], 0) + (sl - lt->w_off[l])];
            const float g = lt->g[l];
            const float hC = -2.f * g;
            cx[k] = hC * v.x;
            cy[k] = hC * v.y;
            cz[k] = hC * v.z;
            hb[k] = 1.f + g * g;
        }
    }
    // energy density: thread l < nl sums wavelength l
    float accU = 0.f, cmpU = 0.f, partU = 0.f;
    const int ul = threadIdx.x < nl ? (int)threadIdx.x : 0;

    // plain sums over at most one staged batch of tuples fold into the
    // compensated (Kahan) accumulators: acc holds the sum, cmp its rounding error
    auto fold = [&]() {
#pragma unroll
        for (int k = 0; k < SLOTS; ++k) {
            const float y = part[k] - cmp[k];
            const float t = acc[k] + y;
            cmp[k] = (t - acc[k]) - y;
            acc[k] = t;
            part[k] = 0.f;
        }
        const float y = partU - cmpU;
        const float t = accU + y;
        cmpU = (t - accU) - y;
        accU = t;
        partU = 0.f;
    };

    const int64_t i0 = blockIdx.x * X.chunk;
    const int64_t i1 = min(X.cnt, i0 + X.chunk);
    int32_t cur = -1;

    auto flush = [&]() {
        if (cur < 0) return;
        fold();
        const LeafRec &r = X.rec[cur];
#pragma unroll
        for (int k = 0; k < SLOTS; ++k) {
            const float v = acc[k] - cmp[k];
            if (lam[k] < NL && v != 0.f) {
                const int l = lam[k];
                const float g = lt->g[l];
                const float scale = lt->albedo[l] * lt->kappa[l] * r.rho / r.ivc * ((1.f - g * g) / (4.f * 3.14159265358979f));
                const int p = (int)threadIdx.x + 256 * k - lt->w_off[l];
                atomic_add_f32(X.S_next + lt->s_off[l] + (int64_t)cur * lt->npix[l] + p, scale * v);
            }
            acc[k] = cmp[k] = 0.f;
        }
        if (threadIdx.x < nl) {
            const float v = accU - cmpU;
            if (v != 0.f) atomic_add_f64(X.U_k + (int64_t)cur * nl + threadIdx.x, (double)v);
        }
        accU = cmpU = 0.f;
    };

    for (int64_t i = i0; i < i1; i += kExpandBatch) {
        const int nb = (int)min((int64_t)kExpandBatch, i1 - i);
        __syncthreads();
        if (threadIdx.x < nb) {
            const int64_t j = i + threadIdx.x;
            const uint32_t orig = X.idx[j];
            const uint64_t key = X.key[j];
            const uint32_t e = (uint32_t)(key & ((1ull << X.dir_bits) - 1ull));
            t_cell[threadIdx.x] = (int32_t)(key >> X.dir_bits);
            t_same[threadIdx.x] = threadIdx.x > 0 && X.key[j - 1] == key;
            t_n[threadIdx.x] = X.dirs[e];
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                if (l < nl) {
                    const float d = X.du[(int64_t)l * X.cap + orig];
                    t_du[l][threadIdx.x] = d;
                    t_a[l][threadIdx.x] = d * X.invz[(int64_t)e * nl + l];
                }
            }
        }
        __syncthreads();
        // each run of one (cell, direction) is summed into its first tuple
        // (thread l: wavelength l), and wave 0 lists the runs' first tuples
        if (threadIdx.x < NL && threadIdx.x < nl) {
            const int l = threadIdx.x;
            for (int jj = nb - 1; jj > 0; --jj)
                if (t_same[jj]) {
                    t_a[l][jj - 1] += t_a[l][jj];
                    t_du[l][jj - 1] += t_du[l][jj];
                }
        }
        if (threadIdx.x < 64) {
            const bool h = (int)threadIdx.x < nb && !t_same[threadIdx.x];
            const uint64_t hm = __ballot(h);
            if (h) t_head[__popcll(hm & ((1ull << threadIdx.x) - 1ull))] = (uint8_t)threadIdx.x;
            if (threadIdx.x == 0) t_nhead = __popcll(hm);
        }
        __syncthreads();
        const int nh = t_nhead;
        for (int q = 0; q < nh; ++q) {
            const int jj = t_head[q];
            const int32_t cell = t_cell[jj];
            if (cell != cur) {
                flush();
                cur = cell;
            }
            const float4 n = t_n[jj];
#pragma unroll
            for (int k = 0; k < SLOTS; ++k) {
                const float r = rsqrtf(fmaf(cx[k], n.x, fmaf(cy[k], n.y, fmaf(cz[k], n.z, hb[k]))));
                part[k] = fmaf(t_a[lam[k]][jj], r * r * r, part[k]);
            }
            partU += t_du[ul][jj];
        }
        fold();
    }
    flush();
}

// ---------------------------------------------------------------------------
// Adjoint of fixed-ray passes.  For a ray with luminosity L_0 l_m at the
// entry of crossing m (l_0 = 1), the loss-weighted deposit of the crossing is
// L_0 l_m a_m(tau_m) with
//   a_m(tau) = l E(tau) Ubar / (V c) + albedo (1 - e^{-tau}) sbar_m,
//   E(tau) = (1 - e^{-tau}) / tau,  sbar_m = sum_p w(p|n) Sbar_next(c_m, p).
// With G = sum_m l_m a_m and the prefix P_m = sum_{i<=m} l_i a_i,
//   dJ/dtau_m = L_0 (l_m a_m'(tau_m) - (G - P_m)),  dJ/drho += kappa l dJ/dtau,
// and dJ/dL_0 = G goes to the pending luminosity the ray was launched from.
// ---------------------------------------------------------------------------

// sig[(rl n + c) n_lambda + l] = sum_p w_l(p | r0 + rl) Sbar_l[c][p]: per
// wavelength, the direction weights (nb x npix) times the transposed gradient
// of the pending scattered light (npix x cells), a dense contraction on the
// matrix cores (FP32 MFMA 16x16x4).  Both operands pass through LDS in stages
// of kGK pixels (zero past npix); a block covers kGT directions x kGT cells,
// each of its four waves a 32 x 32 quarter as 2 x 2 MFMA tiles.  Grid (cells
// / kGT, directions / kGT).
constexpr int kGT = 64;
constexpr int kGK = 32;
typedef float float4v __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_sbar_gather(float *sig, const float *wtab, const LambdaTable *lt,
                                                      const float *Sbar, int64_t n, int r0, int nb, int w_row)
{
    __shared__ float sW[kGK][kGT + 4];
    __shared__ float sS[kGK][kGT + 4];
    const int nl = lt->n_lambda;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int dq = 32 * (wave >> 1), cq = 32 * (wave & 1);   // this wave's quarter of the tile
    const int li = lane & 15, lk = lane >> 4;                  // MFMA operand row / k of this lane
    const int64_t c0 = (int64_t)blockIdx.x * kGT;
    const int d0 = (int)blockIdx.y * kGT;
    for (int l = 0; l < nl; ++l) {
        const int npix = lt->npix[l];
        const float *S = Sbar + lt->s_off[l];
        const float *W = wtab + lt->w_off[l];
        float4v acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = float4v{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < npix; k0 += kGK) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kGT * kGK / 256; ++q) {
                const int e = tid + 256 * q;
                const int row = e / kGK, kk = e % kGK;
                const int k = k0 + kk;
                const int64_t c = c0 + row;
                const int d = d0 + row;
                sS[kk][row] = (c < n && k < npix) ? S[c * npix + k] : 0.f;
                sW[kk][row] = (d < nb && k < npix) ? W[(int64_t)(r0 + d) * w_row + k] : 0.f;
            }
            __syncthreads();
#pragma unroll
            for (int ks = 0; ks < kGK; ks += 4) {
                // A (16 directions x 4 pixels): lane holds A[li][lk];
                // B (4 pixels x 16 cells): lane holds B[lk][li]
                const float a0 = sW[ks + lk][dq + li], a1 = sW[ks + lk][dq + 16 + li];
                const float b0 = sS[ks + lk][cq + li], b1 = sS[ks + lk][cq + 16 + li];
                acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
            }
        }
        // result element v of this lane: row 4 lk + v, column li of the 16 x 16 tile
#pragma unroll
        for (int i = 0; i < 2; ++i) {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int64_t c = c0 + cq + 16 * j + li;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int d = d0 + dq + 16 * i + 4 * lk + v;
                    if (d < nb && c < n) sig[((int64_t)d * n + c) * nl + l] = acc[i][j][v];
                }
            }
        }
    }
}

struct AdjArgs {
    Geo geo;
    const int32_t *src_list;
    const int32_t *n_src;
    const double4 *dirs;         // FP64 directions of this Nside
    const float *emis_lum;       // direct pass
    const double4 *ps_pos;       // point sources of the direct pass (index n + k)
    const int32_t *ps_cell;
    const float *ps_lum;
    int32_t n_point;
    const float *S_pending;      // scattering pass: its emission
    const LambdaTable *lt;
    const float *ubar_t;         // dJ/dU, [n][n_lambda]
    const float *sig;            // sbar per (direction, cell, wavelength), or null
    double *rho_bar;
    float *sbar_k;               // dJ/dS of the pass's emission (scattering pass)
    const float *ebar;           // dJ/dF [n_lambda][nray] of the escaping luminosity, or null
    int64_t n;
    int32_t scatter;
    int32_t r0;
    int32_t nb;
    int32_t order;               // 0: tile-major items, 1: direction-major
    int32_t log2_nside_ray;
    float inv_nray;
    double h_fine;
    int64_t hard_cap;
};

// E(tau) = (1 - e^{-tau}) / tau and E'(tau) from em1 = e^{-tau} - 1
__device__ inline void eprime(float tau, float em1, float &E, float &dE)
{
    if (tau < 0.05f) {
        E = 1.f + tau * (-0.5f + tau * (1.f / 6.f + tau * (-1.f / 24.f + tau * (1.f / 120.f))));
        dE = -0.5f + tau * (1.f / 3.f + tau * (-0.125f + tau * (1.f / 30.f + tau * (-1.f / 144.f))));
    } else {
        E = -em1 / tau;
        dE = fmaf(em1, 1.f + tau, tau) / (tau * tau);
    }
}

// waves per SIMD the compiler must allow for the adjoint march: its loads
// depend on the previous crossing, so occupancy hides their latency
#ifndef DR_WAVES_ADJOINT
#define DR_WAVES_ADJOINT 4
#endif

template <int NL, bool UNIFORM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NL <= 4 ? DR_WAVES_ADJOINT : 2, 8)))
void k_march_adjoint(const AdjArgs A)
{
    const LambdaTable *lt = A.lt;
    const int nl = lt->n_lambda;
    const int lane = threadIdx.x & 63;
    (void)lane;
    const int64_t wid = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int nsrc = *A.n_src;
    const int64_t ntiles = (nsrc + 63) >> 6;
    const int64_t nitems = ntiles * A.nb;
    float kap[NL], alb[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
        kap[l] = l < nl ? lt->kappa[l] : 0.f;
        alb[l] = l < nl ? lt->albedo[l] : 0.f;
    }
    for (int64_t it = wid; it < nitems; it += nw) {
        // item order as in the forward march (tuning item_order)
        int64_t tile;
        int rl;
        if (A.order == 0) {
            tile = it / A.nb;
            rl = (int)(it - tile * A.nb);
        } else {
            rl = (int)(it / ntiles);
            tile = it - (int64_t)rl * ntiles;
        }
        const int r = A.r0 + rl;
        const int64_t si = tile * 64 + (threadIdx.x & 63);
        if (si >= nsrc) continue;
        const int32_t s = A.src_list[si];
        const double4 nd = A.dirs[r];
        RayT<double> R;              // FP64 geometry, as in the forward march
        R.n[0] = nd.x;
        R.n[1] = nd.y;
        R.n[2] = nd.z;
        int32_t c0 = s;              // the cell the ray starts in
        if (s < A.n) {
            const int4 sb = A.geo.rec[s].box;
            const double half = 0.5 * (double)sb.w;
            R.o[0] = (double)sb.x + half;
            R.o[1] = (double)sb.y + half;
            R.o[2] = (double)sb.z + half;
        } else {                     // a point source of the direct pass
            const double4 pp = A.ps_pos[s - A.n];
            R.o[0] = pp.x;
            R.o[1] = pp.y;
            R.o[2] = pp.z;
            c0 = A.ps_cell[s - A.n];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) R.inv[a] = 1.0 / R.n[a];
        float L0[NL];
        float lsum = 0.f;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            float v = 0.f;
            if (l < nl) {
                if (!A.scatter) {
                    v = (s < A.n ? A.emis_lum[(int64_t)l * A.n + s] : A.ps_lum[(int64_t)l * A.n_point + (s - A.n)]) *
                        A.inv_nray;
                } else {
                    const int npix = lt->npix[l];
                    const float *row = A.S_pending + lt->s_off[l] + (int64_t)s * npix;
                    const int ls = 31 - __clz(lt->nside_sca[l]);
                    if (A.log2_nside_ray >= ls) {
                        v = row[r >> (2 * (A.log2_nside_ray - ls))] * ((float)npix * A.inv_nray);
                    } else {
                        const int sh = 2 * (ls - A.log2_nside_ray);
                        for (int q = r << sh; q < ((r + 1) << sh); ++q) v += row[q];
                    }
                }
            }
            L0[l] = v;
            lsum += v;
        }
        // the direct pass's emission does not depend on rho: rays that carry
        // nothing contribute nothing; scattered light needs dJ/dL_0 regardless
        if (!A.scatter && !(lsum > 0.f)) continue;

        double G[NL], P[NL];
        float ell[NL];
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            G[l] = 0.0;
            P[l] = 0.0;
        }
        for (int walk = 0; walk < 2; ++walk) {
#pragma unroll
            for (int l = 0; l < NL; ++l) ell[l] = 1.f;
            int32_t c = c0;
            double t = 0.0;
            int64_t steps = 0;
            while (true) {
                const LeafRec &rc = A.geo.rec[c];
                const int4 b = rc.box;
                int32_t nbc[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) nbc[q] = rc.nb[q];
                int axis;
                const double te = exit_t(R, b, axis);
                const double len = te - t;
                if (!is_graze(len, te)) {
                    const float rho = rc.rho;
                    const float ivc = rc.ivc;
                    const float lp = (float)(len * A.h_fine);
                    double rb = 0.0;
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
                        if (l < nl) {
                            const float alpha = kap[l] * rho;
                            const float tau = alpha * lp;
                            bool thick;
                            float tr;
                            const float em1 = fast_em1(tau, thick, tr);
                            const float T = thick ? tr : 1.f + em1;   // e^{-tau}
                            float E, dE;
                            eprime(tau, em1, E, dE);
                            const float ub = A.ubar_t[(int64_t)c * nl + l];
                            const float sg = A.sig ? A.sig[((int64_t)rl * A.n + c) * nl + l] : 0.f;
                            const float a = lp * E * ivc * ub - alb[l] * em1 * sg;
                            if (walk == 0) {
                                G[l] += (double)ell[l] * (double)a;
                            } else {
                                const float ap = lp * dE * ivc * ub + alb[l] * T * sg;
                                P[l] += (double)ell[l] * (double)a;
                                const double dtau = (double)L0[l] * ((double)ell[l] * (double)ap - (G[l] - P[l]));
                                rb += (double)kap[l] * (double)lp * dtau;
                            }
                            ell[l] *= T;
                        }
                    }
                    if (walk == 1 && rb != 0.0) atomic_add_f64(A.rho_bar + c, rb);
                    t = te;
                }
                const int32_t nx = next_leaf<double>(A.geo, R, b, nbc, axis, te);
                if (nx < 0) break;
                if (++steps >= A.hard_cap) break;
                c = nx;
            }
            if (walk == 0 && A.ebar) {
                // loss on the escaping luminosity: the terminal value of the recursion
                const int64_t nray = (int64_t)12 << (2 * A.log2_nside_ray);
#pragma unroll
                for (int l = 0; l < NL; ++l)
                    if (l < nl) G[l] += (double)ell[l] * (double)A.ebar[(int64_t)l * nray + r];
            }
        }
        if (A.scatter) {
#pragma unroll
            for (int l = 0; l < NL; ++l) {
                if (l < nl && G[l] != 0.0) {
                    const int npix = lt->npix[l];
                    float *row = A.sbar_k + lt->s_off[l] + (int64_t)s * npix;
                    const int ls = 31 - __clz(lt->nside_sca[l]);
                    if (A.log2_nside_ray >= ls) {
                        atomic_add_f32(row + (r >> (2 * (A.log2_nside_ray - ls))),
                                       (float)(G[l] * ((double)npix * (double)A.inv_nray)));
                    } else {
                        const int sh = 2 * (ls - A.log2_nside_ray);
                        for (int q = r << sh; q < ((r + 1) << sh); ++q) atomic_add_f32(row + q, (float)G[l]);
                    }
                }
            }
        }
    }
}

__global__ void k_add_f32(float *a, const float *b, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] += b[i];
}

__global__ void k_to_f32(const double *a, float *out, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)a[i];
}

__global__ void k_rho_out(const double *rb, float *out, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)rb[i];
}

// U += U_k (and U_pass = U_k), absorbed / scattered tallies from U_k in FP64,
// U_LL <- U when requested.  grid.y = wavelength
// bit 0 of the device error word when any lane saw a non-finite value
__device__ inline void flag_nonfinite(bool bad, uint32_t *err)
{
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(err, 1u);
}

__global__ void k_finish_u(const double *U_k, float *U, float *U_pass, float *U_LL, int set_ull, int ull_only,
                           const LambdaTable *lt, const float *rho, const float *inv_vc, int64_t n, double *tally,
                           uint32_t *err)
{
    __shared__ double sh[16];
    const int l = blockIdx.y;
    double ext = 0.0;
    bool bad = false;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = (int64_t)l * n + c;
        const double ukd = U_k[c * lt->n_lambda + l];
        bad |= !isfinite(ukd);
        const float uk = (float)ukd;
        if (ull_only) {
            U_LL[i] = uk;
        } else {
            const float u = U[i] + uk;
            U[i] = u;
            if (U_pass) U_pass[i] = uk;
            if (set_ull) U_LL[i] = u;
        }
        ext += (double)lt->kappa[l] * (double)rho[c] / (double)inv_vc[c] * ukd;
    }
    flag_nonfinite(bad, err);
    const double b = block_sum(ext, sh);
    if (threadIdx.x == 0 && b != 0.0) {
        const double om = lt->albedo[l];
        atomic_add_f64(&tally[l * DARTRAY_N_TALLY + DARTRAY_T_ABSORBED], (1.0 - om) * b);
        atomic_add_f64(&tally[l * DARTRAY_N_TALLY + DARTRAY_T_SCATTERED], om * b);
    }
}

// S_total (=|+=) S_next, S_pending = S_next, per-wavelength FP64 sums of S_next
__global__ void k_finish_s(const float *S_next, float *S_total, float *S_pending, int accumulate,
                           const LambdaTable *lt, int64_t s_size, double *ssum, uint32_t *err)
{
    __shared__ double sh[16];
    const int l = blockIdx.y;
    const int64_t lo = lt->s_off[l], hi = lt->s_off[l + 1];
    double acc = 0.0;
    bool bad = false;
    for (int64_t i = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < hi; i += (int64_t)gridDim.x * blockDim.x) {
        const float v = S_next[i];
        bad |= !isfinite(v);
        S_total[i] = accumulate ? S_total[i] + v : v;
        S_pending[i] = v;
        acc += v;
    }
    flag_nonfinite(bad, err);
    const double b = block_sum(acc, sh);
    if (threadIdx.x == 0 && b != 0.0) atomic_add_f64(&ssum[l], b);
}

// [nl][n] -> [n][nl]
__global__ void k_transpose_ull(const float *U_LL, float *ull_t, int64_t n, int nl)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * nl; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i / nl;
        const int l = (int)(i - c * nl);
        ull_t[i] = U_LL[(int64_t)l * n + c];
    }
}

__global__ void k_set_rho(LeafRec *rec, float *rho_arr, const float *rho, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        rec[i].rho = rho[i];
        rho_arr[i] = rho[i];
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

static double hg_fwhm_closed(double g)
{
    if (g <= 0.0) return 0.0;
    const double f0 = std::pow(1.0 + g * g - 2.0 * g, -1.5);
    const double fpi = std::pow(1.0 + g * g + 2.0 * g, -1.5);
    const double half = fpi + 0.5 * (f0 - fpi);
    const double c = (1.0 + g * g - std::pow(half, -2.0 / 3.0)) / (2.0 * g);
    return 2.0 * std::acos(std::max(-1.0, std::min(1.0, c)));
}

// Eq. 5-6: k = 0.5 log2(4 pi / (12 theta_min^2)), theta_min = FWHM / n_fwhm,
// integer part, clamped to [0, k_max]
static int nside_from_rule(double g, double n_fwhm, int k_max)
{
    const double fwhm = hg_fwhm_closed(g);
    if (fwhm <= 0.0) return 1;
    const double tmin = fwhm / n_fwhm;
    double k = std::floor(0.5 * std::log2(4.0 * kPi / (12.0 * tmin * tmin)));
    k = std::max(0.0, std::min((double)k_max, k));   // k_max <= 3 is checked at grid creation
    return 1 << (int)k;
}

static uint64_t spread3(uint64_t x)
{
    x &= 0x1FFFFF;
    x = (x | (x << 32)) & 0x1F00000000FFFFull;
    x = (x | (x << 16)) & 0x1F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

template <typename T>
static int dalloc(Grid &g, T **p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * count);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(DARTRAY_E_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    g.bytes += sizeof(T) * count;
    return DARTRAY_OK;
}

static void free_grid(Grid &g)
{
    for (hipEvent_t e : g.ev_pool) (void)hipEventDestroy(e);
    g.ev_pool.clear();
    void *ptrs[] = {g.mir, g.first, g.reps, g.pmir, g.esc_tmp, g.dust_word, g.ps_pos, g.ps_xyz, g.ps_cell, g.ps_lum, g.ps_lum64, g.rec, g.ull_t, g.rho_bar, g.own.esc64, g.sbar[0], g.sbar[1], g.leaf_box, g.rho, g.inv_vc, g.emis_lum, g.lum64, g.own.n_all, g.own.err_word, g.root_tab, g.nodes, g.morton, g.by_level, g.d_lt, g.own.U_k,
                    g.own.flags, g.cell_flag, g.own.src_list, g.own.scan_blocks, g.own.n_src, g.own.dsum, g.s1_sum, g.own.ubar, g.dir_all, g.dir64, g.invz, g.sca64, g.wtab, g.queue, g.log_key, g.log_key2,
                    g.log_idx, g.log_idx2, g.log_du, g.log_count, g.sort_tmp};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
}

static int validate_desc(const dartray_grid_desc *d)
{
    if (!d) return fail(DARTRAY_E_INVALID, "null grid description");
    if (d->n_leaves <= 0 || d->n_leaves > (int64_t)INT32_MAX) return fail(DARTRAY_E_INVALID, "n_leaves out of range");
    if (d->n_lambda <= 0 || d->n_lambda > kMaxLambda) return fail(DARTRAY_E_INVALID, "n_lambda must be 1..64");
    if (d->n_leaves * (int64_t)d->n_lambda >= ((int64_t)1 << 32))
        return fail(DARTRAY_E_UNSUPPORTED, "n_leaves x n_lambda must be below 2^32");
    if (!(d->root_size > 0.0) || !std::isfinite(d->root_size)) return fail(DARTRAY_E_INVALID, "root_size must be > 0");
    if (!(d->c_light > 0.0)) return fail(DARTRAY_E_INVALID, "c_light must be > 0");
    for (int a = 0; a < 3; ++a)
        if (d->nroot[a] <= 0 || !std::isfinite(d->lo[a])) return fail(DARTRAY_E_INVALID, "bad root block");
    if (!d->leaf_level || !d->leaf_ijk || !d->rho || !d->emis || !d->kappa || !d->albedo || !d->g || !d->nside_sca)
        return fail(DARTRAY_E_INVALID, "null array in grid description");
    for (int l = 0; l < d->n_lambda; ++l) {
        if (!(d->kappa[l] >= 0.f) || !std::isfinite(d->kappa[l])) return fail(DARTRAY_E_INVALID, "kappa must be finite and >= 0");
        if (!(d->albedo[l] >= 0.f && d->albedo[l] <= 1.f)) return fail(DARTRAY_E_INVALID, "albedo must lie in [0, 1]");
        if (!(d->g[l] > -1.f && d->g[l] < 1.f)) return fail(DARTRAY_E_INVALID, "g must lie in (-1, 1)");
        const int ns = d->nside_sca[l];
        if (ns < 0 || (ns > 0 && (ns & (ns - 1))) || ns > kMaxNsideSca) return fail(DARTRAY_E_INVALID, "nside_sca must be 0 or a power of two <= 8");
    }
    if (d->nside_max < 0 || d->nside_max > kMaxNsideCap || (d->nside_max & (d->nside_max - 1)))
        return fail(DARTRAY_E_INVALID, "nside_max must be 0 or a power of two <= 1024");
    if (d->k_max < 0) return fail(DARTRAY_E_INVALID, "k_max must be >= 0");
    if (d->n_point < 0 || (d->n_point > 0 && (!d->point_pos || !d->point_lum)))
        return fail(DARTRAY_E_INVALID, "point sources: n_point >= 0 with both arrays given");
    if (d->n_leaves + (int64_t)d->n_point > (int64_t)INT32_MAX) return fail(DARTRAY_E_INVALID, "too many sources");
    for (int32_t k = 0; k < d->n_point; ++k) {
        for (int a = 0; a < 3; ++a) {
            const double x = d->point_pos[3 * k + a];
            const double hi = d->lo[a] + d->nroot[a] * d->root_size;
            if (!std::isfinite(x) || !(x >= d->lo[a] && x < hi))
                return fail(DARTRAY_E_INVALID, "point sources must lie inside the root block");
        }
        for (int l = 0; l < d->n_lambda; ++l) {
            const float v = d->point_lum[(int64_t)l * d->n_point + k];
            if (!(v >= 0.f) || !std::isfinite(v)) return fail(DARTRAY_E_INVALID, "point luminosities must be finite and >= 0");
        }
    }
    for (int l = 0; l < d->n_lambda; ++l)
        if (d->nside_sca[l] == 0 && d->k_max > 3)
            return fail(DARTRAY_E_UNSUPPORTED, "the Eq. 5 rule is applied with k_max <= 3 (Nside_sca <= 8)");
    if (!(d->n_fwhm > 0.0)) {
        for (int l = 0; l < d->n_lambda; ++l)
            if (d->nside_sca[l] == 0) return fail(DARTRAY_E_INVALID, "n_fwhm must be > 0 with nside_sca = 0");
    }
    return DARTRAY_OK;
}

}  // namespace dr

using namespace dr;

extern "C" {

const char *dartray_last_error(void) { return g_last_error.c_str(); }

const char *dartray_version(void) { return DR_VERSION; }

int dartray_grid_destroy(dartray_grid *grid)
{
    if (!grid) return DARTRAY_OK;
    if (grid->g.stream) (void)hipStreamSynchronize(grid->g.stream);
    else (void)hipDeviceSynchronize();
    free_grid(grid->g);
    delete grid;
    return DARTRAY_OK;
}

int dartray_grid_create(const dartray_grid_desc *d, void *stream, dartray_grid **out)
{
    if (!out) return fail(DARTRAY_E_INVALID, "null output handle");
    *out = nullptr;
    int rc = validate_desc(d);
    if (rc) return rc;
    const int64_t n = d->n_leaves;
    const int nl = d->n_lambda;

    // --- host-side checks and the locator -------------------------------
    int lmax = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int lv = d->leaf_level[i];
        if (lv < 0 || lv > 20) return fail(DARTRAY_E_INVALID, "leaf level out of range 0..20");
        lmax = std::max(lmax, lv);
    }
    int64_t fine[3];
    for (int a = 0; a < 3; ++a) {
        fine[a] = (int64_t)d->nroot[a] << lmax;
        if (fine[a] > (1 << 21)) return fail(DARTRAY_E_INVALID, "more than 2^21 finest-level cells along an axis");
    }
    const int64_t nroot = (int64_t)d->nroot[0] * d->nroot[1] * d->nroot[2];
    // codes: >= 0 internal node, < 0 leaf; root table starts "unset"
    const int32_t kUnset = INT32_MIN;
    std::vector<int32_t> root_tab((size_t)nroot, kUnset);
    std::vector<int32_t> nodes;
    std::vector<int4> boxes((size_t)n);
    std::vector<float> inv_vc((size_t)n);
    std::vector<uint64_t> keys((size_t)n);
    int64_t covered = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int lv = d->leaf_level[i];
        const int64_t span = (int64_t)1 << (lmax - lv);
        int64_t c[3];
        for (int a = 0; a < 3; ++a) {
            c[a] = d->leaf_ijk[3 * i + a];
            if (c[a] < 0 || (c[a] + 1) * span > fine[a])
                return fail(DARTRAY_E_INVALID, "leaf outside the root block");
        }
        if (!(d->rho[i] >= 0.f) || !std::isfinite(d->rho[i])) return fail(DARTRAY_E_INVALID, "rho must be finite and >= 0");
        for (int l = 0; l < nl; ++l) {
            const float e = d->emis[(int64_t)l * n + i];
            if (!(e >= 0.f) || !std::isfinite(e)) return fail(DARTRAY_E_INVALID, "emis must be finite and >= 0");
        }
        boxes[i] = make_int4((int)(c[0] * span), (int)(c[1] * span), (int)(c[2] * span), (int)span);
        const double side = d->root_size / (double)((int64_t)1 << lv);
        inv_vc[i] = (float)(1.0 / (side * side * side * d->c_light));
        keys[i] = spread3((uint64_t)(c[0] * span)) | (spread3((uint64_t)(c[1] * span)) << 1) |
                  (spread3((uint64_t)(c[2] * span)) << 2);
        covered += span * span * span;
        // insert into the locator; a slot is an index into root_tab (in_nodes
        // false) or into nodes (true), so it survives reallocation of nodes
        const int64_t root = ((c[2] >> lv) * d->nroot[1] + (c[1] >> lv)) * d->nroot[0] + (c[0] >> lv);
        bool in_nodes = false;
        size_t slot = (size_t)root;
        auto at = [&](void) -> int32_t & { return in_nodes ? nodes[slot] : root_tab[slot]; };
        for (int lev = 0; lev < lv; ++lev) {
            int32_t code = at();
            if (code == kUnset) {
                code = (int32_t)(nodes.size() / 8);
                at() = code;
                nodes.resize(nodes.size() + 8, kUnset);
            } else if (code < 0) {
                return fail(DARTRAY_E_INVALID, "leaves overlap");
            }
            const int bit = lv - lev - 1;
            const int oct = (int)(((c[0] >> bit) & 1) | (((c[1] >> bit) & 1) << 1) | (((c[2] >> bit) & 1) << 2));
            in_nodes = true;
            slot = (size_t)code * 8 + oct;
        }
        if (at() != kUnset) return fail(DARTRAY_E_INVALID, "leaves overlap");
        at() = -(int32_t)i - 1;
    }
    if (covered != fine[0] * fine[1] * fine[2]) return fail(DARTRAY_E_INVALID, "leaves do not tile the root block");
    for (int32_t v : root_tab)
        if (v == kUnset) return fail(DARTRAY_E_INVALID, "leaves do not tile the root block");
    for (int32_t v : nodes)
        if (v == kUnset) return fail(DARTRAY_E_INVALID, "leaves do not tile the root block");

    // leaf records with face-neighbour codes
    auto region_code = [&](int lv, const int64_t q[3]) -> int32_t {
        for (int a = 0; a < 3; ++a)
            if (q[a] < 0 || q[a] >= ((int64_t)d->nroot[a] << lv)) return -1;
        const int64_t root = ((q[2] >> lv) * d->nroot[1] + (q[1] >> lv)) * d->nroot[0] + (q[0] >> lv);
        int32_t code = root_tab[(size_t)root];
        for (int lev = 0; lev < lv; ++lev) {
            if (code < 0) return -code - 1;          // a coarser leaf covers the region
            const int bit = lv - lev - 1;
            const int oct = (int)(((q[0] >> bit) & 1) | (((q[1] >> bit) & 1) << 1) | (((q[2] >> bit) & 1) << 2));
            code = nodes[(size_t)code * 8 + oct];
        }
        return code < 0 ? (-code - 1) : -(code + 2);
    };
    std::vector<LeafRec> recs((size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        LeafRec &r = recs[(size_t)i];
        std::memset(&r, 0, sizeof(r));
        r.box = boxes[(size_t)i];
        r.rho = d->rho[i];
        r.ivc = inv_vc[(size_t)i];
        r.level = d->leaf_level[i];
        const int lv = d->leaf_level[i];
        for (int a = 0; a < 3; ++a)
            for (int dir = 0; dir < 2; ++dir) {
                int64_t q[3] = {d->leaf_ijk[3 * i], d->leaf_ijk[3 * i + 1], d->leaf_ijk[3 * i + 2]};
                q[a] += dir ? 1 : -1;
                r.nb[2 * a + dir] = region_code(lv, q);
            }
    }

    std::vector<int32_t> morton((size_t)n);
    for (int64_t i = 0; i < n; ++i) morton[i] = (int32_t)i;
    std::stable_sort(morton.begin(), morton.end(), [&](int32_t a, int32_t b) { return keys[a] < keys[b]; });
    // source order of the adaptive passes: a source's ray tree grows with the
    // fineness of the cells around it, so the finest levels go first and the
    // work queue ends on the lightest items (Morton order within a level)
    std::vector<int32_t> by_level(morton);
    std::stable_sort(by_level.begin(), by_level.end(),
                     [&](int32_t a, int32_t b) { return d->leaf_level[a] > d->leaf_level[b]; });
    // point sources follow the cells in both source orders (index n + k)
    const int32_t np = d->n_point;
    for (int32_t k = 0; k < np; ++k) {
        morton.push_back((int32_t)(n + k));
        by_level.push_back((int32_t)(n + k));
    }
    // the leaf holding each point source: fine-cell index (a point on a face
    // belongs to the upper side), then down the locator
    std::vector<double4> ps_pos((size_t)std::max(np, 1)), ps_xyz((size_t)std::max(np, 1));
    std::vector<int32_t> ps_cell((size_t)std::max(np, 1));
    std::vector<float> ps_lum((size_t)std::max<int64_t>(1, (int64_t)np * nl));
    std::vector<double> ps_lum64((size_t)std::max<int64_t>(1, (int64_t)np * nl));
    {
        const double hf = d->root_size / (double)((int64_t)1 << lmax);
        for (int32_t k = 0; k < np; ++k) {
            double f[3];
            int64_t q[3];
            for (int a = 0; a < 3; ++a) {
                f[a] = (d->point_pos[3 * k + a] - d->lo[a]) / hf;
                q[a] = std::min<int64_t>(fine[a] - 1, std::max<int64_t>(0, (int64_t)std::floor(f[a])));
            }
            ps_pos[(size_t)k] = make_double4(f[0], f[1], f[2], 0.0);
            ps_xyz[(size_t)k] = make_double4(d->point_pos[3 * k], d->point_pos[3 * k + 1], d->point_pos[3 * k + 2], 0.0);
            int32_t v = root_tab[(size_t)(((q[2] >> lmax) * d->nroot[1] + (q[1] >> lmax)) * d->nroot[0] + (q[0] >> lmax))];
            int bit = lmax - 1;
            while (v >= 0) {
                const int oct = (int)(((q[0] >> bit) & 1) | (((q[1] >> bit) & 1) << 1) | (((q[2] >> bit) & 1) << 2));
                v = nodes[(size_t)v * 8 + oct];
                --bit;
            }
            ps_cell[(size_t)k] = -v - 1;
            for (int l = 0; l < nl; ++l) {
                ps_lum[(size_t)l * np + k] = d->point_lum[(int64_t)l * np + k];
                ps_lum64[(size_t)l * np + k] = (double)d->point_lum[(int64_t)l * np + k];
            }
        }
    }
    const int64_t n_src_max = n + np;

    LambdaTable lt{};
    lt.n_lambda = nl;
    lt.s_off[0] = 0;
    lt.w_off[0] = 0;
    for (int l = 0; l < nl; ++l) {
        lt.kappa[l] = d->kappa[l];
        lt.albedo[l] = d->albedo[l];
        lt.g[l] = d->g[l];
        int ns = d->nside_sca[l];
        if (ns == 0) ns = nside_from_rule(d->g[l], d->n_fwhm, d->k_max);
        lt.nside_sca[l] = ns;
        lt.npix[l] = 12 * ns * ns;
        lt.s_off[l + 1] = lt.s_off[l] + n * (int64_t)lt.npix[l];
        lt.w_off[l + 1] = lt.w_off[l] + lt.npix[l];
    }

    // luminosity 4 pi j V of each cell: FP64 (launch luminosity of the passes
    // that take FP64 significance decisions) and rounded to FP32
    std::vector<float> emis_lum((size_t)(nl * n));
    std::vector<double> lum64((size_t)(nl * n));
    for (int l = 0; l < nl; ++l)
        for (int64_t i = 0; i < n; ++i) {
            const double side = d->root_size / (double)((int64_t)1 << d->leaf_level[i]);
            const double v = 4.0 * kPi * (double)d->emis[(int64_t)l * n + i] * side * side * side;
            lum64[(size_t)(l * n + i)] = v;
            emis_lum[(size_t)(l * n + i)] = (float)v;
        }

    // --- device side ------------------------------------------------------
    dartray_grid *h = new dartray_grid();
    Grid &g = h->g;
    g.n = n;
    g.n_lambda = nl;
    g.n_point = np;
    for (int a = 0; a < 3; ++a) {
        g.nroot[a] = d->nroot[a];
        g.fine[a] = (int32_t)fine[a];
        g.lo[a] = d->lo[a];
    }
    g.max_level = lmax;
    g.root_size = d->root_size;
    g.h_fine = d->root_size / (double)((int64_t)1 << lmax);
    g.c_light = d->c_light;
    g.uniform = (lmax == 0);
    // leaf i at root position i, x fastest: the fixed march then finds a
    // cell's neighbours by index arithmetic
    g.linear = g.uniform && n == nroot;
    for (int64_t i = 0; g.linear && i < nroot; ++i) g.linear = root_tab[(size_t)i] == (int32_t)(-i - 1);
    g.n_internal = (int64_t)(nodes.size() / 8);
    g.lt = lt;
    g.s_size = lt.s_off[nl];
    g.w_row = lt.w_off[nl];
    g.stream = (hipStream_t)stream;
    if (hipGetDevice(&g.device) != hipSuccess) g.device = 0;

    const size_t nray_w = 12 * (size_t)kMaxNsideWTable * kMaxNsideWTable;
    const int32_t cap = std::max(64, (int)d->nside_max);
    const int64_t ndir = 4 * (4 * (int64_t)cap * cap - 1);   // all levels 1 .. cap
    // direction-binned work array: all 768 Nside-8 directions when they fit
    // in half the free device memory (at most 128 GiB), else as many as fit
    const size_t per_dir = (size_t)nl * (size_t)n;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || free_b == 0) free_b = (size_t)16 << 30;
    const size_t bin_budget = std::min<size_t>(free_b / 2, (size_t)128 << 30);
    size_t nb_cap = std::min<size_t>(768, std::max<size_t>(1, bin_budget / (4 * per_dir)));
    int rcs[] = {
        dalloc(g, &g.leaf_box, (size_t)n), dalloc(g, &g.rho, (size_t)n), dalloc(g, &g.inv_vc, (size_t)n),
        dalloc(g, &g.rec, (size_t)n), dalloc(g, &g.ull_t, (size_t)(nl * n)), dalloc(g, &g.rho_bar, (size_t)n), dalloc(g, &g.own.esc64, (size_t)nl * 12 * kMaxNsideWTable * kMaxNsideWTable),
        dalloc(g, &g.sbar[0], (size_t)lt.s_off[nl]), dalloc(g, &g.sbar[1], (size_t)lt.s_off[nl]),
        dalloc(g, &g.emis_lum, (size_t)(nl * n)), dalloc(g, &g.lum64, (size_t)(nl * n)), dalloc(g, &g.root_tab, (size_t)nroot),
        dalloc(g, &g.own.n_all, 1), dalloc(g, &g.own.err_word, 1), dalloc(g, &g.dust_word, 2),
        dalloc(g, &g.mir, (size_t)n * 8), dalloc(g, &g.first, (size_t)n), dalloc(g, &g.reps, (size_t)(n / 8 + 1)),
        dalloc(g, &g.pmir, (size_t)entry_of(32, 0) * 8), dalloc(g, &g.esc_tmp, (size_t)nl * 12 * 16 * 16),
        dalloc(g, &g.ps_pos, (size_t)std::max(np, 1)), dalloc(g, &g.ps_xyz, (size_t)std::max(np, 1)), dalloc(g, &g.ps_cell, (size_t)std::max(np, 1)),
        dalloc(g, &g.ps_lum, (size_t)std::max<int64_t>(1, (int64_t)np * nl)),
        dalloc(g, &g.ps_lum64, (size_t)std::max<int64_t>(1, (int64_t)np * nl)),
        dalloc(g, &g.nodes, nodes.size()), dalloc(g, &g.morton, (size_t)n_src_max), dalloc(g, &g.by_level, (size_t)n_src_max), dalloc(g, &g.d_lt, 1),
        dalloc(g, &g.own.U_k, (size_t)(nl * n)), dalloc(g, &g.own.flags, (size_t)n_src_max), dalloc(g, &g.cell_flag, (size_t)n), dalloc(g, &g.own.src_list, (size_t)n_src_max),
        dalloc(g, &g.own.scan_blocks, (size_t)((n_src_max + kScanBlock - 1) / kScanBlock)), dalloc(g, &g.own.n_src, 1),
        dalloc(g, &g.own.dsum, 4 * kMaxLambda), dalloc(g, &g.s1_sum, kMaxLambda),
        dalloc(g, &g.own.ubar, nb_cap * per_dir), dalloc(g, &g.dir_all, (size_t)ndir), dalloc(g, &g.dir64, (size_t)ndir),
        dalloc(g, &g.invz, (size_t)ndir * nl), dalloc(g, &g.sca64, 3 * (size_t)kScaDirs),
        dalloc(g, &g.wtab, nray_w * (size_t)g.w_row), dalloc(g, &g.queue, 1),
    };
    for (int r : rcs)
        if (r) {
            std::string msg = g_last_error;
            free_grid(g);
            delete h;
            return fail(DARTRAY_E_OOM, msg);
        }
    g.own.ubar_floats = nb_cap * per_dir;
    g.w = g.own;
    g.nside_cap = cap;
    g.ndir_all = ndir;
    // deposit log for the scattering passes of adaptive rays (wavelength rows
    // of at most 2048 slots per expansion block)
    if (nl <= 16 && g.w_row <= 256 * kExpandSlots) {
        // up to 1024 tuples per cell within an eighth of the free memory (at
        // most 16 GiB): fewer log-full restarts of the march per pass
        size_t fr = 0, tt = 0;
        if (hipMemGetInfo(&fr, &tt) != hipSuccess || fr == 0) fr = (size_t)16 << 30;
        const int64_t per_tuple = 24 + 4 * (int64_t)nl;
        const int64_t by_mem = (int64_t)(std::min<size_t>(fr / 8, (size_t)16 << 30) / (size_t)per_tuple);
        const int64_t lcap = std::max<int64_t>((int64_t)1 << 16,
                                               std::min<int64_t>(std::min<int64_t>((int64_t)1 << 28, 1024 * n), by_mem));
        int rl[] = {dalloc(g, &g.log_key, (size_t)lcap), dalloc(g, &g.log_key2, (size_t)lcap),
                    dalloc(g, &g.log_idx, (size_t)lcap), dalloc(g, &g.log_idx2, (size_t)lcap),
                    dalloc(g, &g.log_du, (size_t)lcap * nl), dalloc(g, &g.log_count, 1)};
        int bad = 0;
        for (int r : rl) bad |= r;
        int cell_bits = 1;
        while ((1ll << cell_bits) < n) ++cell_bits;
        while ((1ll << g.dir_bits) < g.ndir_all) ++g.dir_bits;
        g.key_bits = cell_bits + g.dir_bits;
        if (!bad) {
            hipcub::DoubleBuffer<uint64_t> kb(g.log_key, g.log_key2);
            hipcub::DoubleBuffer<uint32_t> vb(g.log_idx, g.log_idx2);
            size_t tb = 0;
            hipError_t qe = hipcub::DeviceRadixSort::SortPairs(nullptr, tb, kb, vb, (int)lcap, 0, g.key_bits, g.stream);
            if (qe != hipSuccess) bad = 1;
            else bad = dalloc(g, (char **)&g.sort_tmp, tb);
            g.sort_tmp_bytes = tb;
        }
        if (bad) {
            std::string msg = g_last_error;
            free_grid(g);
            delete h;
            return fail(DARTRAY_E_OOM, "deposit log: " + msg);
        }
        g.log_cap = lcap;
    }
    hipStream_t s = g.stream;
    hipError_t e = hipSuccess;
    std::vector<float> rho_f(d->rho, d->rho + n);
    auto cp = [&](void *dst, const void *src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    };
    cp(g.leaf_box, boxes.data(), sizeof(int4) * n);
    cp(g.rec, recs.data(), sizeof(LeafRec) * n);
    cp(g.rho, rho_f.data(), sizeof(float) * n);
    cp(g.inv_vc, inv_vc.data(), sizeof(float) * n);
    cp(g.emis_lum, emis_lum.data(), sizeof(float) * nl * n);
    cp(g.lum64, lum64.data(), sizeof(double) * nl * n);
    cp(g.root_tab, root_tab.data(), sizeof(int32_t) * nroot);
    cp(g.nodes, nodes.data(), sizeof(int32_t) * nodes.size());
    cp(g.morton, morton.data(), sizeof(int32_t) * n_src_max);
    cp(g.by_level, by_level.data(), sizeof(int32_t) * n_src_max);
    if (np > 0) {
        cp(g.ps_pos, ps_pos.data(), sizeof(double4) * np);
        cp(g.ps_xyz, ps_xyz.data(), sizeof(double4) * np);
        cp(g.ps_cell, ps_cell.data(), sizeof(int32_t) * np);
        cp(g.ps_lum, ps_lum.data(), sizeof(float) * np * nl);
        cp(g.ps_lum64, ps_lum64.data(), sizeof(double) * np * nl);
    }
    cp(g.d_lt, &lt, sizeof(LambdaTable));
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // host vectors go out of scope
    if (e != hipSuccess) {
        int r = hip_fail(e, "grid upload");
        free_grid(g);
        delete h;
        return r;
    }
    *out = h;
    return DARTRAY_OK;
}

int dartray_grid_info(const dartray_grid *grid, int64_t *n_leaves, int32_t *n_lambda, int64_t *s_size)
{
    if (!grid) return fail(DARTRAY_E_INVALID, "null grid");
    if (n_leaves) *n_leaves = grid->g.n;
    if (n_lambda) *n_lambda = grid->g.n_lambda;
    if (s_size) *s_size = grid->g.s_size;
    return DARTRAY_OK;
}

int dartray_nside_sca(const dartray_grid *grid, int32_t l, int32_t *nside)
{
    if (!grid || !nside) return fail(DARTRAY_E_INVALID, "null argument");
    if (l < 0 || l >= grid->g.n_lambda) return fail(DARTRAY_E_INVALID, "wavelength index out of range");
    *nside = grid->g.lt.nside_sca[l];
    return DARTRAY_OK;
}

int64_t dartray_s_offset(const dartray_grid *grid, int32_t l)
{
    if (!grid || l < 0 || l > grid->g.n_lambda) return -1;
    return grid->g.lt.s_off[l];
}

int dartray_profile_enable(dartray_grid *grid, int32_t kinds)
{
    if (!grid) return fail(DARTRAY_E_INVALID, "null grid");
    grid->g.prof = kinds & DARTRAY_PROF_ALL;
    grid->g.ev_used = 0;
    return DARTRAY_OK;
}

int dartray_profile_read(dartray_grid *grid, double *march_ms, int64_t *launches)
{
    if (!grid || !march_ms || !launches) return fail(DARTRAY_E_INVALID, "null argument");
    Grid &g = grid->g;
    DR_HIP(hipStreamSynchronize(g.stream));
    double total = 0.0;
    for (size_t i = 0; i + 1 < g.ev_used; i += 2) {
        float ms = 0.f;
        DR_HIP(hipEventElapsedTime(&ms, g.ev_pool[i], g.ev_pool[i + 1]));
        total += ms;
    }
    *march_ms = total;
    *launches = (int64_t)(g.ev_used / 2);
    return DARTRAY_OK;
}

int dartray_workspace_bytes(const dartray_grid *grid, const dartray_trace_opts *opts, size_t *bytes)
{
    if (!grid || !bytes) return fail(DARTRAY_E_INVALID, "null argument");
    const Grid &g = grid->g;
    if (!opts) {
        *bytes = g.bytes;
        return DARTRAY_OK;
    }
    const size_t n = (size_t)g.n, nl = (size_t)g.n_lambda;
    // every pass: FP64 energy-density accumulators, source selection, tables
    size_t b = n * nl * sizeof(double) + n * (2 * sizeof(int32_t) + 1) + (size_t)g.ndir_all * (sizeof(float4) + sizeof(double4)) +
               3 * (size_t)kScaDirs * sizeof(double);
    const bool step1 = opts->adaptive && opts->mode == DARTRAY_MODE_STEP1;
    if (!opts->adaptive) {
        const int64_t nray = 12 * (int64_t)opts->nside * opts->nside;
        const size_t nb = (size_t)std::min<int64_t>(nray, (int64_t)(g.w.ubar_floats / std::max<size_t>(1, n * nl)));
        b += nb * n * nl * sizeof(float) + (size_t)nray * (size_t)g.w_row * sizeof(float);
    } else if (!step1) {
        b += n * nl * sizeof(float) + (size_t)g.ndir_all * nl * sizeof(float);   // U_LL copy, phase normalisation
        if (g.log_cap > 0)
            b += (size_t)g.log_cap * (2 * sizeof(uint64_t) + 2 * sizeof(uint32_t) + nl * sizeof(float)) + g.sort_tmp_bytes;
    }
    *bytes = b;
    return DARTRAY_OK;
}

int dartray_set_tuning(dartray_grid *grid, const dartray_tuning *t)
{
    if (!grid || !t) return fail(DARTRAY_E_INVALID, "null argument");
    const int lt = t->lambda_tile;
    if (!(lt == 0 || lt == 1 || lt == 4 || lt == 8 || lt == 16 || lt == 32 || lt == 64))
        return fail(DARTRAY_E_INVALID, "lambda_tile must be 0, 1, 4, 8, 16, 32 or 64");
    if (!(t->block_waves == 0 || t->block_waves == 1 || t->block_waves == 2 || t->block_waves == 4))
        return fail(DARTRAY_E_INVALID, "block_waves must be 0, 1, 2 or 4");
    if (t->grid_blocks < 0 || t->grid_blocks > 65536) return fail(DARTRAY_E_INVALID, "grid_blocks out of range");
    if (t->dir_batch < 0) return fail(DARTRAY_E_INVALID, "dir_batch must be >= 0");
    if (t->item_order != 0 && t->item_order != 1) return fail(DARTRAY_E_INVALID, "item_order must be 0 or 1");
    grid->g.tune = *t;
    return DARTRAY_OK;
}

int dartray_get_tuning(const dartray_grid *grid, dartray_tuning *t)
{
    if (!grid || !t) return fail(DARTRAY_E_INVALID, "null argument");
    *t = grid->g.tune;
    return DARTRAY_OK;
}

int dartray_grid_set_rho(dartray_grid *grid, const float *rho_device)
{
    if (!grid || !rho_device) return fail(DARTRAY_E_INVALID, "null argument");
    Grid &g = grid->g;
    hipLaunchKernelGGL(k_set_rho, dim3((unsigned)std::min<int64_t>((g.n + 255) / 256, 4096)), dim3(256), 0, g.stream,
                       g.rec, g.rho, rho_device, g.n);
    DR_LAUNCH_CHECK("k_set_rho");
    g.mirror_ok = false;
    return DARTRAY_OK;
}

int dartray_debug_ray_cells(dartray_grid *grid, int32_t n_rays, const double *origin, const double *dir,
                            int32_t max_cross, int64_t *cells, double *lengths, int32_t *counts)
{
    if (!grid || !origin || !dir || !cells || !lengths || !counts || n_rays <= 0 || max_cross <= 0)
        return fail(DARTRAY_E_INVALID, "bad argument");
    Grid &g = grid->g;
    // origins and directions in fine-cell units
    std::vector<double> o((size_t)3 * n_rays), dd((size_t)3 * n_rays);
    for (int i = 0; i < n_rays; ++i) {
        double nrm = 0.0;
        for (int a = 0; a < 3; ++a) nrm += dir[3 * i + a] * dir[3 * i + a];
        if (!(nrm > 0.0)) return fail(DARTRAY_E_INVALID, "zero direction");
        for (int a = 0; a < 3; ++a) {
            o[3 * i + a] = (origin[3 * i + a] - g.lo[a]) / g.h_fine;
            dd[3 * i + a] = dir[3 * i + a] / std::sqrt(nrm);
        }
    }
    double *d_o = nullptr, *d_d = nullptr;
    int64_t *d_c = nullptr;
    double *d_l = nullptr;
    int32_t *d_n = nullptr;
    const size_t tot = (size_t)n_rays * max_cross;
    hipError_t e = hipMalloc((void **)&d_o, sizeof(double) * 3 * n_rays);
    if (e == hipSuccess) e = hipMalloc((void **)&d_d, sizeof(double) * 3 * n_rays);
    if (e == hipSuccess) e = hipMalloc((void **)&d_c, sizeof(int64_t) * tot);
    if (e == hipSuccess) e = hipMalloc((void **)&d_l, sizeof(double) * tot);
    if (e == hipSuccess) e = hipMalloc((void **)&d_n, sizeof(int32_t) * n_rays);
    if (e == hipSuccess) e = hipMemcpyAsync(d_o, o.data(), sizeof(double) * 3 * n_rays, hipMemcpyHostToDevice, g.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_d, dd.data(), sizeof(double) * 3 * n_rays, hipMemcpyHostToDevice, g.stream);
    if (e == hipSuccess) {
        Geo geo{g.rec, g.root_tab, g.nodes, {g.fine[0], g.fine[1], g.fine[2]},
                {g.nroot[0], g.nroot[1], g.nroot[2]}, g.max_level};
        hipLaunchKernelGGL(k_debug_cells, dim3((n_rays + 63) / 64), dim3(64), 0, g.stream, geo, n_rays, d_o, d_d,
                           max_cross, d_c, d_l, d_n);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(cells, d_c, sizeof(int64_t) * tot, hipMemcpyDeviceToHost, g.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(lengths, d_l, sizeof(double) * tot, hipMemcpyDeviceToHost, g.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(counts, d_n, sizeof(int32_t) * n_rays, hipMemcpyDeviceToHost, g.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g.stream);
    (void)hipFree(d_o);
    (void)hipFree(d_d);
    (void)hipFree(d_c);
    (void)hipFree(d_l);
    (void)hipFree(d_n);
    if (e != hipSuccess) return hip_fail(e, "debug_ray_cells");
    for (int i = 0; i < n_rays; ++i)
        for (int m = 0; m < counts[i]; ++m) lengths[(size_t)i * max_cross + m] *= g.h_fine;
    return DARTRAY_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Pass driver
// ---------------------------------------------------------------------------

namespace dr {

static int check_opts(const Grid &g, const dartray_trace_opts *o, const dartray_fields *f, bool scatter)
{
    if (!o || !f) return fail(DARTRAY_E_INVALID, "null opts or fields");
    if (o->nside <= 0 || (o->nside & (o->nside - 1))) return fail(DARTRAY_E_INVALID, "nside must be a power of two");
    if (!scatter && o->mode != DARTRAY_MODE_STEP1 && o->mode != DARTRAY_MODE_DIRECT)
        return fail(DARTRAY_E_INVALID, "unknown mode");
    if (o->max_steps < 0) return fail(DARTRAY_E_INVALID, "max_steps must be >= 0");
    if (!f->tally) return fail(DARTRAY_E_INVALID, "tally buffer required");
    const bool step1 = !scatter && o->mode == DARTRAY_MODE_STEP1;
    if (step1) {
        if (!o->adaptive) return fail(DARTRAY_E_INVALID, "step 1 needs adaptive rays");
        if (!f->U_LL) return fail(DARTRAY_E_INVALID, "step 1 writes U_LL");
    } else {
        if (!f->U || !f->S_total || !f->S_pending || !f->S_next) return fail(DARTRAY_E_INVALID, "U and S buffers required");
        if (o->adaptive && !f->U_LL) return fail(DARTRAY_E_INVALID, "adaptive passes need U_LL");
    }
    if (o->nside > g.nside_cap) return fail(DARTRAY_E_INVALID, "nside above the grid's nside_max");
    if (o->flags & DARTRAY_FLAG_2D) {
        bool ident = true, zero = true;
        for (int i = 0; i < 9; ++i) {
            ident &= o->frame[i] == ((i % 4 == 0) ? 1.0 : 0.0);
            zero &= o->frame[i] == 0.0;
        }
        if (!(ident || zero)) return fail(DARTRAY_E_UNSUPPORTED, "2D mode needs the unrotated frame");
        if (o->source_mask) return fail(DARTRAY_E_UNSUPPORTED, "2D mode selects its own sources (no source_mask)");
        if (g.n_point > 0) return fail(DARTRAY_E_UNSUPPORTED, "2D mode: no point sources");
        if (f->escape && !o->adaptive && o->nside > 16) return fail(DARTRAY_E_UNSUPPORTED, "2D mode: escape by direction up to Nside 16");
    }
    if (o->adaptive) {
        if (o->nside_max < o->nside || (o->nside_max & (o->nside_max - 1)) || o->nside_max > g.nside_cap)
            return fail(DARTRAY_E_INVALID, "adaptive nside_max must be a power of two in [nside, grid nside_max]");
        int depth = 0;
        while ((o->nside << depth) < o->nside_max) ++depth;
        if (depth > kMaxDepthAdaptive) return fail(DARTRAY_E_INVALID, "more than 12 split levels");
        if (!(o->n_rays_min > 0.0) || !std::isfinite(o->n_rays_min)) return fail(DARTRAY_E_INVALID, "n_rays_min must be > 0");
        if (!std::isfinite(o->f_U) || (!(o->f_U >= 0.0) && !(o->a_RT > 0.0 && std::isfinite(o->a_RT))))
            return fail(DARTRAY_E_INVALID, "f_U must be >= 0, or < 0 with a_RT > 0 (Eq. 11)");
        if (!std::isfinite(o->r_pre)) return fail(DARTRAY_E_INVALID, "r_pre must be finite");
        if (!(o->n_rays_max == 0.0 || (o->n_rays_max >= 4.0 * o->n_rays_min && std::isfinite(o->n_rays_max))))
            return fail(DARTRAY_E_INVALID, "n_rays_max must be 0 or >= 4 n_rays_min (Eq. 3)");
        // merging has been run on trees of at most 3 split levels; a run with
        // 8 levels faulted the device and the cause is not yet found
        if (o->n_rays_max > 0.0 && depth > kMaxDepthMerge)
            return fail(DARTRAY_E_UNSUPPORTED, "ray merging is limited to 3 split levels (nside_max <= 8 nside)");
        if (g.n_lambda > 16) return fail(DARTRAY_E_UNSUPPORTED, "adaptive rays carry at most 16 wavelengths");
    }
    if (f->escape && o->adaptive) return fail(DARTRAY_E_UNSUPPORTED, "escape by direction covers fixed rays only");
    if ((f->counters == nullptr) && (o->flags & DARTRAY_FLAG_COUNTERS))
        return fail(DARTRAY_E_INVALID, "counters buffer required by DARTRAY_FLAG_COUNTERS");
    if (scatter && !g.have_s1) return fail(DARTRAY_E_STATE, "scatter_iter needs a prior direct pass");
    return DARTRAY_OK;
}

static void frame_of(const dartray_trace_opts *o, Frame &f)
{
    bool zero = true;
    for (int i = 0; i < 9; ++i) {
        f.R[i] = o->frame[i];
        zero &= o->frame[i] == 0.0;
    }
    if (zero)
        for (int i = 0; i < 9; ++i) f.R[i] = (i % 4 == 0) ? 1.0 : 0.0;
}

static int ensure_dirs(Grid &g, const Frame &f)
{
    if (g.dirs_valid && std::memcmp(g.dirs_frame, f.R, sizeof(f.R)) == 0) return DARTRAY_OK;
    hipLaunchKernelGGL(k_dir_all, dim3((unsigned)((g.ndir_all + 255) / 256)), dim3(256), 0, g.stream, g.dir_all,
                       g.dir64, g.ndir_all, f);
    DR_LAUNCH_CHECK("k_dir_all");
    hipLaunchKernelGGL(k_sca64, dim3((kScaDirs + 255) / 256), dim3(256), 0, g.stream, g.sca64, f);
    DR_LAUNCH_CHECK("k_sca64");
    g.dirs_valid = true;
    g.invz_valid = false;
    g.wtab_valid = false;
    std::memcpy(g.dirs_frame, f.R, sizeof(f.R));
    return DARTRAY_OK;
}

static int ensure_wtab(Grid &g, int nside, const Frame &f)
{
    if (g.wtab_valid && g.wtab_nside == nside) return DARTRAY_OK;
    if (nside > kMaxNsideWTable) return fail(DARTRAY_E_UNSUPPORTED, "fixed-mode nside above 16");
    const int64_t nray = 12 * (int64_t)nside * nside;
    const int64_t tot = nray * g.n_lambda;
    hipLaunchKernelGGL(k_wtab, dim3((unsigned)((tot + 63) / 64)), dim3(64), 0, g.stream, g.wtab, g.d_lt, g.sca64, nside,
                       nray, g.w_row, f);
    DR_LAUNCH_CHECK("k_wtab");
    g.wtab_valid = true;
    g.wtab_nside = nside;
    return DARTRAY_OK;
}

static int ensure_invz(Grid &g, const Frame &f)
{
    if (g.invz_valid) return DARTRAY_OK;
    hipLaunchKernelGGL(k_invz, dim3((unsigned)((g.ndir_all + 127) / 128)), dim3(128), 0, g.stream, g.invz, g.d_lt,
                       g.sca64, (int64_t)0, g.ndir_all, f);
    DR_LAUNCH_CHECK("k_invz");
    g.invz_valid = true;
    return DARTRAY_OK;
}

// blocks per wavelength for sweeps over the scattered-luminosity arrays:
// about 16 elements per thread, at most 1024
static unsigned s_blocks(const Grid &g)
{
    int64_t longest = 0;
    for (int l = 0; l < g.n_lambda; ++l) longest = std::max<int64_t>(longest, g.lt.s_off[l + 1] - g.lt.s_off[l]);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(1024, (longest + 4095) / 4096));
}

static int select_sources(Grid &g, const dartray_trace_opts *o, const dartray_fields *f, bool scatter)
{
    // point sources emit in step 1 and the direct pass only
    const int64_t n = g.n + (scatter ? 0 : g.n_point);
    const unsigned nblk = (unsigned)((n + kScanBlock - 1) / kScanBlock);
    // the order in which sources become work items
    const int32_t *order = o->adaptive ? g.by_level : g.morton;
    int rc = fill<int32_t>(g, g.w.n_all, 1, 0);
    if (rc) return rc;
    if ((rc = fill<uint32_t>(g, g.w.err_word, 1, 0u))) return rc;   // the pass's own error word
    if (!scatter) {
        hipLaunchKernelGGL(k_source_flags, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, g.stream, g.w.flags, order,
                           g.n, g.n_point, g.d_lt, g.emis_lum, g.ps_lum, o->source_mask, f->tally, g.w.n_all);
        DR_LAUNCH_CHECK("k_source_flags");
    } else {
        if ((rc = fill<uint8_t>(g, g.cell_flag, (size_t)n, (uint8_t)0))) return rc;
        hipLaunchKernelGGL(k_sflag_sweep, dim3(s_blocks(g), g.n_lambda), dim3(256), 0, g.stream, f->S_pending, g.d_lt,
                           o->source_mask, g.cell_flag, f->tally);
        DR_LAUNCH_CHECK("k_sflag_sweep");
        hipLaunchKernelGGL(k_sflag_gather, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)), dim3(256), 0,
                           g.stream, g.w.flags, order, g.cell_flag, o->source_mask, n, g.w.n_all);
        DR_LAUNCH_CHECK("k_sflag_gather");
    }
    hipLaunchKernelGGL(k_scan_count, dim3(nblk), dim3(kScanBlock), 0, g.stream, g.w.flags, n, g.w.scan_blocks);
    DR_LAUNCH_CHECK("k_scan_count");
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(64), 0, g.stream, g.w.scan_blocks, (int64_t)nblk, g.w.n_src);
    DR_LAUNCH_CHECK("k_scan_blocks");
    hipLaunchKernelGGL(k_scan_scatter, dim3(nblk), dim3(kScanBlock), 0, g.stream, g.w.flags, order, n,
                       g.w.scan_blocks, g.w.src_list);
    DR_LAUNCH_CHECK("k_scan_scatter");
    return DARTRAY_OK;
}

// record a timing event on the grid's stream (profiling only)
static int prof_mark(Grid &g)
{
    if (!(g.prof & g.prof_kind)) return DARTRAY_OK;
    if (g.ev_used == g.ev_pool.size()) {
        hipEvent_t e;
        DR_HIP(hipEventCreate(&e));
        g.ev_pool.push_back(e);
    }
    DR_HIP(hipEventRecord(g.ev_pool[g.ev_used++], g.stream));
    return DARTRAY_OK;
}

static int nl_template(int k) { return k <= 1 ? 1 : k <= 4 ? 4 : k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : 64; }

static void launch_fixed(const FixedArgs &A, int nlt, hipStream_t s, unsigned blocks, unsigned threads)
{
#define DR_LAUNCH_FIXED(N)                                                                           \
    do {                                                                                             \
        if (A.linear) hipLaunchKernelGGL((k_march_fixed<N, true>), dim3(blocks), dim3(threads), 0, s, A);  \
        else hipLaunchKernelGGL((k_march_fixed<N, false>), dim3(blocks), dim3(threads), 0, s, A);          \
    } while (0)
    switch (nlt) {
    case 1: DR_LAUNCH_FIXED(1); break;
    case 4: DR_LAUNCH_FIXED(4); break;
    case 8: DR_LAUNCH_FIXED(8); break;
    case 16: DR_LAUNCH_FIXED(16); break;
    case 32: DR_LAUNCH_FIXED(32); break;
    default: DR_LAUNCH_FIXED(64); break;
    }
#undef DR_LAUNCH_FIXED
}

// wavelengths per march launch under the grid's tuning
static int lambda_chunk(const Grid &g)
{
    const int t = g.tune.lambda_tile > 0 ? g.tune.lambda_tile : g.n_lambda;
    return std::min(t, g.n_lambda);
}

// directions binned between two flushes
static int dir_batch(const Grid &g, int64_t nray)
{
    const size_t per_dir = (size_t)g.n_lambda * (size_t)g.n;
    int64_t nb = std::min<int64_t>(nray, (int64_t)(g.w.ubar_floats / per_dir));
    if (g.tune.dir_batch > 0) nb = std::min<int64_t>(nb, g.tune.dir_batch);
    return (int)std::max<int64_t>(nb, 1);
}

static FixedArgs fixed_args(Grid &g, const dartray_trace_opts *o, dartray_fields *f, bool scatter)
{
    const int64_t nray = 12 * (int64_t)o->nside * o->nside;
    int log2n = 0;
    while ((1 << log2n) < o->nside) ++log2n;
    FixedArgs A{};
    A.geo = Geo{g.rec, g.root_tab, g.nodes, {g.fine[0], g.fine[1], g.fine[2]}, {g.nroot[0], g.nroot[1], g.nroot[2]},
                g.max_level};
    A.linear = g.linear ? 1 : 0;
    A.src_list = g.w.src_list;
    A.n_src = g.w.n_src;
    A.dirs = g.dir64 + entry_of(o->nside, 0);
    A.emis_lum = g.emis_lum;
    A.ps_pos = g.ps_pos;
    A.ps_cell = g.ps_cell;
    A.ps_lum = g.ps_lum;
    A.n_point = g.n_point;
    A.S_pending = f->S_pending;
    A.lt = g.d_lt;
    A.ubar = g.w.ubar;
    A.tally = f->tally;
    A.counters = (o->flags & DARTRAY_FLAG_COUNTERS) ? f->counters : nullptr;
    A.esc_dir = f->escape ? g.w.esc64 : nullptr;
    A.n = g.n;
    A.scatter = scatter ? 1 : 0;
    A.order = g.tune.item_order;
    A.nside_ray = o->nside;
    A.log2_nside_ray = log2n;
    A.inv_nray = (float)(1.0 / (double)nray);
    A.h_fine = g.h_fine;
    A.max_steps = o->max_steps;
    A.hard_cap = 4 * ((int64_t)g.fine[0] + g.fine[1] + g.fine[2]) + 64;
    return A;
}

// one march launch per wavelength chunk over directions r0 .. r0 + nb - 1
static int march_fixed_batch(Grid &g, FixedArgs A, int r0, int nb)
{
    const int chunk = lambda_chunk(g);
    const unsigned threads = 64u * (unsigned)(g.tune.block_waves > 0 ? g.tune.block_waves : 4);
    const unsigned blocks = (unsigned)(g.tune.grid_blocks > 0 ? g.tune.grid_blocks : 2048);
    uint64_t *counters = A.counters;
    A.r0 = r0;
    A.nb = nb;
    int rc;
    for (int l0 = 0; l0 < g.n_lambda; l0 += chunk) {
        A.l0 = l0;
        A.nlc = std::min(chunk, g.n_lambda - l0);
        A.counters = l0 == 0 ? counters : nullptr;
        if ((rc = prof_mark(g))) return rc;
        launch_fixed(A, nl_template(A.nlc), g.stream, blocks, threads);
        DR_LAUNCH_CHECK("k_march_fixed");
        if ((rc = prof_mark(g))) return rc;
    }
    return DARTRAY_OK;
}

// flush launch shape shared by single- and multi-model passes
struct FlushShape {
    int log2_nlp, pch, rb_stage, max_npix;
    int64_t per_block;
    size_t lds;
};

static FlushShape flush_shape(const Grid &g)
{
    FlushShape f{};
    const int nl = g.n_lambda;
    while ((1 << f.log2_nlp) < nl) ++f.log2_nlp;
    int min_npix = 1 << 30;
    for (int l = 0; l < nl; ++l) {
        min_npix = std::min(min_npix, g.lt.npix[l]);
        f.max_npix = std::max(f.max_npix, g.lt.npix[l]);
    }
    f.pch = (min_npix % 48 == 0) ? 48 : 12;
    f.rb_stage = 16;
    while (f.rb_stage > 1 && (size_t)f.rb_stage * nl * (f.pch + 1) * sizeof(float) > (size_t)48 * 1024) f.rb_stage >>= 1;
    f.lds = (size_t)f.rb_stage * nl * (f.pch + 1) * sizeof(float);
    f.per_block = 256 >> f.log2_nlp;
    return f;
}

static FlushArgs flush_args(Grid &g, float *S_next)
{
    FlushArgs F{};
    F.ubar = g.w.ubar;
    F.wtab = g.wtab;
    F.lt = g.d_lt;
    F.rho = g.rho;
    F.inv_vc = g.inv_vc;
    F.U_k = g.w.U_k;
    F.S_next = S_next;
    F.n = g.n;
    F.w_row = g.w_row;
    return F;
}

static int flush_fixed_batch(Grid &g, float *S_next, int r0, int nb)
{
    const FlushShape fs = flush_shape(g);
    const FlushArgs F = flush_args(g, S_next);
    const dim3 grid((unsigned)((g.n + fs.per_block - 1) / fs.per_block), (unsigned)(fs.max_npix / fs.pch));
    if (fs.pch == 48)
        hipLaunchKernelGGL(k_flush_fixed<48>, grid, dim3(256), fs.lds, g.stream, F, r0, nb, fs.log2_nlp, fs.rb_stage);
    else
        hipLaunchKernelGGL(k_flush_fixed<12>, grid, dim3(256), fs.lds, g.stream, F, r0, nb, fs.log2_nlp, fs.rb_stage);
    DR_LAUNCH_CHECK("k_flush_fixed");
    return DARTRAY_OK;
}

static int run_fixed_pass(Grid &g, const dartray_trace_opts *o, dartray_fields *f, bool scatter)
{
    const int nl = g.n_lambda;
    const int64_t n = g.n;
    Frame fr;
    frame_of(o, fr);
    int rc = ensure_dirs(g, fr);
    if (rc) return rc;
    if ((rc = ensure_wtab(g, o->nside, fr))) return rc;
    const int64_t nray = 12 * (int64_t)o->nside * o->nside;

    if ((rc = fill<double>(g, g.w.U_k, (size_t)nl * n, 0.0))) return rc;
    if ((rc = fill<float>(g, f->S_next, (size_t)g.s_size, 0.f))) return rc;
    if ((rc = fill<double>(g, f->tally, (size_t)nl * DARTRAY_N_TALLY, 0.0))) return rc;
    if (f->counters && (rc = fill<uint64_t>(g, f->counters, DARTRAY_N_COUNT, 0))) return rc;
    if (f->escape && (rc = fill<double>(g, g.w.esc64, (size_t)nl * nray, 0.0))) return rc;
    if ((rc = select_sources(g, o, f, scatter))) return rc;

    const size_t per_dir = (size_t)nl * n;
    const int nb_max = dir_batch(g, nray);
    g.prof_kind = DARTRAY_PROF_FIXED;
    const FixedArgs A = fixed_args(g, o, f, scatter);
    for (int64_t r0 = 0; r0 < nray; r0 += nb_max) {
        const int nb = (int)std::min<int64_t>(nb_max, nray - r0);
        if ((rc = fill<float>(g, g.w.ubar, (size_t)nb * per_dir, 0.f))) return rc;
        if ((rc = march_fixed_batch(g, A, (int)r0, nb))) return rc;
        if ((rc = flush_fixed_batch(g, f->S_next, (int)r0, nb))) return rc;
    }
    return DARTRAY_OK;
}

template <int NL>
static void launch_expand_nl(const ExpandArgs &X, int slots, hipStream_t s, unsigned blocks)
{
    switch (slots) {
    case 1: hipLaunchKernelGGL((k_expand<NL, 1>), dim3(blocks), dim3(256), 0, s, X); break;
    case 2: hipLaunchKernelGGL((k_expand<NL, 2>), dim3(blocks), dim3(256), 0, s, X); break;
    case 3: hipLaunchKernelGGL((k_expand<NL, 3>), dim3(blocks), dim3(256), 0, s, X); break;
    case 4: hipLaunchKernelGGL((k_expand<NL, 4>), dim3(blocks), dim3(256), 0, s, X); break;
    case 5: hipLaunchKernelGGL((k_expand<NL, 5>), dim3(blocks), dim3(256), 0, s, X); break;
    case 6: hipLaunchKernelGGL((k_expand<NL, 6>), dim3(blocks), dim3(256), 0, s, X); break;
    case 7: hipLaunchKernelGGL((k_expand<NL, 7>), dim3(blocks), dim3(256), 0, s, X); break;
    default: hipLaunchKernelGGL((k_expand<NL, 8>), dim3(blocks), dim3(256), 0, s, X); break;
    }
}

// expansion with ceil(w_row / 256) pixel slots per thread (at most 8)
static void launch_expand(const ExpandArgs &X, int nl, int slots, hipStream_t s, unsigned blocks)
{
    if (nl <= 1) launch_expand_nl<1>(X, slots, s, blocks);
    else if (nl <= 4) launch_expand_nl<4>(X, slots, s, blocks);
    else if (nl <= 8) launch_expand_nl<8>(X, slots, s, blocks);
    else launch_expand_nl<16>(X, slots, s, blocks);
}

template <int NL>
static void launch_adaptive(const AdaptArgs &A, int mode, hipStream_t s, unsigned blocks)
{
    const bool merge = A.n_rays_max > 0.0;
    if (mode == 0) {
        if (merge) hipLaunchKernelGGL((k_march_adaptive<NL, 0, true>), dim3(blocks), dim3(256), 0, s, A);
        else hipLaunchKernelGGL((k_step1_quad<NL>), dim3(blocks), dim3(256), 0, s, A);
    } else if (mode == 1) {
        if (merge) hipLaunchKernelGGL((k_march_adaptive<NL, 1, true>), dim3(blocks), dim3(256), 0, s, A);
        else hipLaunchKernelGGL((k_march_adaptive<NL, 1, false>), dim3(blocks), dim3(256), 0, s, A);
    } else {
        if (merge) hipLaunchKernelGGL((k_march_adaptive<NL, 2, true>), dim3(blocks), dim3(256), 0, s, A);
        else hipLaunchKernelGGL((k_march_adaptive<NL, 2, false>), dim3(blocks), dim3(256), 0, s, A);
    }
}

static int run_adaptive_pass(Grid &g, const dartray_trace_opts *o, dartray_fields *f, bool scatter)
{
    const int nl = g.n_lambda;
    const int64_t n = g.n;
    const bool step1 = !scatter && o->mode == DARTRAY_MODE_STEP1;
    Frame fr;
    frame_of(o, fr);
    int rc = ensure_dirs(g, fr);
    if (rc) return rc;
    if (!step1 && (rc = ensure_invz(g, fr))) return rc;
    if ((rc = fill<double>(g, g.w.U_k, (size_t)nl * n, 0.0))) return rc;
    if (!step1 && (rc = fill<float>(g, f->S_next, (size_t)g.s_size, 0.f))) return rc;
    if ((rc = fill<double>(g, f->tally, (size_t)nl * DARTRAY_N_TALLY, 0.0))) return rc;
    if (f->counters && (rc = fill<uint64_t>(g, f->counters, DARTRAY_N_COUNT, 0))) return rc;
    if ((rc = fill<unsigned long long>(g, g.queue, 1, 0ull))) return rc;
    if ((rc = select_sources(g, o, f, scatter))) return rc;
    if (!step1) {
        hipLaunchKernelGGL(k_transpose_ull, dim3((unsigned)std::min<int64_t>((n * nl + 255) / 256, 8192)), dim3(256), 0,
                           g.stream, f->U_LL, g.ull_t, n, nl);
        DR_LAUNCH_CHECK("k_transpose_ull");
    }

    AdaptArgs A{};
    A.geo = Geo{g.rec, g.root_tab, g.nodes, {g.fine[0], g.fine[1], g.fine[2]}, {g.nroot[0], g.nroot[1], g.nroot[2]},
                g.max_level};
    A.src_list = g.w.src_list;
    A.n_src = g.w.n_src;
    A.dirs = g.dir_all;
    A.invz = g.invz;
    A.emis_lum = g.emis_lum;
    A.lum64 = g.lum64;
    A.ps_pos = g.ps_pos;
    A.ps_cell = g.ps_cell;
    A.ps_lum = g.ps_lum;
    A.ps_lum64 = g.ps_lum64;
    A.n_point = g.n_point;
    A.S_pending = f->S_pending;
    A.ull_t = g.ull_t;
    A.n_all = g.w.n_all;
    A.lt = g.d_lt;
    A.U_k = g.w.U_k;
    A.S_next = f->S_next;
    A.tally = f->tally;
    A.counters = (o->flags & DARTRAY_FLAG_COUNTERS) ? f->counters : nullptr;
    A.queue = g.queue;
    A.n = n;
    A.mode = step1 ? 0 : (scatter ? 2 : 1);
    A.nside0 = o->nside;
    int l2 = 0;
    while ((1 << l2) < o->nside) ++l2;
    A.log2_nside0 = l2;
    int depth = 0;
    while ((o->nside << depth) < o->nside_max) ++depth;
    A.max_depth = depth;
    A.n_rays = o->n_rays_min;
    A.n_rays_max = o->n_rays_max;
    A.f_U = o->f_U;
    A.a_RT = o->a_RT;
    A.r_pre_fine64 = o->r_pre / g.h_fine;
    A.h_fine64 = g.h_fine;
    A.dirs64 = g.dir64;
    A.c_light = g.c_light;
    A.max_steps = o->max_steps;
    A.hard_cap = 4 * ((int64_t)g.fine[0] + g.fine[1] + g.fine[2]) + 64;
    const unsigned blocks = 2048;
    const bool use_log = !step1 && g.log_cap > 0;
    g.prof_kind = step1 ? DARTRAY_PROF_STEP1 : DARTRAY_PROF_SCATTERING;
    A.log_key = g.log_key;
    A.log_dir_bits = g.dir_bits;
    A.log_du = g.log_du;
    A.log_count = g.log_count;
    A.log_cap = use_log ? g.log_cap : 0;
    A.log_limit = use_log ? g.log_cap - g.log_cap / 4 : 0;
    int32_t nsrc_h = 0;
    if (use_log) {
        DR_HIP(hipMemcpyAsync(&nsrc_h, g.w.n_src, sizeof(int32_t), hipMemcpyDeviceToHost, g.stream));
        DR_HIP(hipStreamSynchronize(g.stream));
    }
    const unsigned long long nitems = (unsigned long long)nsrc_h * (unsigned long long)(12 * o->nside * o->nside);
    g.log_chunks = 0;
    while (true) {
        if (use_log && (rc = fill<unsigned long long>(g, g.log_count, 1, 0ull))) return rc;
        if ((rc = prof_mark(g))) return rc;
        if (nl <= 1) launch_adaptive<1>(A, A.mode, g.stream, blocks);
        else if (nl <= 4) launch_adaptive<4>(A, A.mode, g.stream, blocks);
        else if (nl <= 8) launch_adaptive<8>(A, A.mode, g.stream, blocks);
        else launch_adaptive<16>(A, A.mode, g.stream, blocks);
        DR_LAUNCH_CHECK("k_march_adaptive");
        if ((rc = prof_mark(g))) return rc;
        ++g.log_chunks;
        if (!use_log) break;
        unsigned long long hc[2] = {0, 0};
        DR_HIP(hipMemcpyAsync(&hc[0], g.log_count, sizeof(unsigned long long), hipMemcpyDeviceToHost, g.stream));
        DR_HIP(hipMemcpyAsync(&hc[1], g.queue, sizeof(unsigned long long), hipMemcpyDeviceToHost, g.stream));
        DR_HIP(hipStreamSynchronize(g.stream));
        const int64_t cnt = (int64_t)std::min<unsigned long long>(hc[0], (unsigned long long)g.log_cap);
        if (cnt > 0) {
            hipLaunchKernelGGL(k_iota, dim3((unsigned)std::min<int64_t>((cnt + 255) / 256, 8192)), dim3(256), 0,
                               g.stream, g.log_idx, cnt);
            DR_LAUNCH_CHECK("k_iota");
            hipcub::DoubleBuffer<uint64_t> kb(g.log_key, g.log_key2);
            hipcub::DoubleBuffer<uint32_t> vb(g.log_idx, g.log_idx2);
            size_t tb = g.sort_tmp_bytes;
            DR_HIP(hipcub::DeviceRadixSort::SortPairs(g.sort_tmp, tb, kb, vb, (int)cnt, 0, g.key_bits, g.stream));
            ExpandArgs X{};
            X.key = kb.Current();
            X.idx = vb.Current();
            X.dir_bits = g.dir_bits;
            X.du = g.log_du;
            X.dirs = g.dir_all;
            X.invz = g.invz;
            X.lt = g.d_lt;
            X.rec = g.rec;
            X.U_k = g.w.U_k;
            X.S_next = f->S_next;
            X.cnt = cnt;
            X.cap = g.log_cap;
            X.chunk = 2048;
            X.w_row = g.w_row;
            const unsigned eb = (unsigned)((cnt + X.chunk - 1) / X.chunk);
            launch_expand(X, nl, (g.w_row + 255) / 256, g.stream, eb);
            DR_LAUNCH_CHECK("k_expand");
        }
        if (hc[1] >= nitems) break;
    }
    return DARTRAY_OK;
}

static int finish_pass(Grid &g, const dartray_trace_opts *o, dartray_fields *f, bool scatter)
{
    const int nl = g.n_lambda;
    const int64_t n = g.n;
    const bool step1 = !scatter && o->mode == DARTRAY_MODE_STEP1;
    hipLaunchKernelGGL(k_finish_u, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1024), nl), dim3(256), 0,
                       g.stream, g.w.U_k, f->U, f->U_pass, f->U_LL, o->adaptive ? 1 : 0, step1 ? 1 : 0, g.d_lt, g.rho,
                       g.inv_vc, n, f->tally, g.w.err_word);
    DR_LAUNCH_CHECK("k_finish_u");
    if (f->escape && !o->adaptive) {
        const int64_t ne = (int64_t)nl * 12 * o->nside * o->nside;
        hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, g.stream, g.w.esc64, f->escape, ne);
        DR_LAUNCH_CHECK("k_to_f32");
    }
    if (step1) return DARTRAY_OK;
    int rc;
    double *ssum = g.w.dsum;
    if ((rc = fill<double>(g, ssum, (size_t)nl, 0.0))) return rc;
    hipLaunchKernelGGL(k_finish_s, dim3(s_blocks(g), nl), dim3(256), 0, g.stream, f->S_next, f->S_total, f->S_pending,
                       (scatter || (o->flags & DARTRAY_FLAG_CONTINUE)) ? 1 : 0, g.d_lt, g.s_size, ssum, g.w.err_word);
    DR_LAUNCH_CHECK("k_finish_s");
    if (!scatter) {
        DR_HIP(hipMemcpyAsync(g.s1_sum, ssum, sizeof(double) * nl, hipMemcpyDeviceToDevice, g.stream));
        g.have_s1 = true;
    }
    return DARTRAY_OK;
}

// ---------------------------------------------------------------------------
// 2D mode (Sect. 3.6): a model symmetric across the three planes through
// the block centre.  The first octant's sources are traced as usual; then
// every orbit {M c} of cells (and {(M c, M p)} of cells and scattered-light
// pixels, {M d} of escape directions) takes the sum of what the traced rays
// left over the orbit, which is what the 7 mirror images of each traced
// source would have left there.  Orbits are disjoint, so each thread owns
// one and the folds run in place, summing in FP64 in a fixed order.
// ---------------------------------------------------------------------------

__global__ void k_mirror_check(const int32_t *mir, const float *rho, const float *emis_lum, int64_t n, int nl,
                               uint32_t *bad)
{
    bool b = false;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        for (int M = 1; M < 8; ++M) {
            const int32_t m = mir[8 * c + M];
            b |= rho[m] != rho[c];
            for (int l = 0; l < nl; ++l) b |= emis_lum[(int64_t)l * n + m] != emis_lum[(int64_t)l * n + c];
        }
    }
    if (__ballot(b) && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
}

// U_k [n][nl]
__global__ void k_mirror_u(double *U_k, const int32_t *mir, const int32_t *reps, int64_t n_reps, int nl)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_reps * nl;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = reps[i / nl];
        const int l = (int)(i % nl);
        int32_t cm[8];
        double v = 0.0;
        for (int M = 0; M < 8; ++M) {
            cm[M] = mir[8 * r + M];
            v += U_k[(int64_t)cm[M] * nl + l];
        }
        for (int M = 0; M < 8; ++M) U_k[(int64_t)cm[M] * nl + l] = v;
    }
}

// the block of wavelength blockIdx.y of an S array
__global__ void k_mirror_s(float *S, const LambdaTable *lt, const int32_t *mir, const int32_t *reps, int64_t n_reps,
                           const int32_t *pmir)
{
    const int l = blockIdx.y;
    const int np = lt->npix[l];
    const int64_t e0 = entry_of(lt->nside_sca[l], 0);
    float *blk = S + lt->s_off[l];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_reps * np;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = reps[i / np];
        const int64_t p = i % np;
        int64_t at[8];
        double v = 0.0;
        for (int M = 0; M < 8; ++M) {
            at[M] = (int64_t)mir[8 * r + M] * np + pmir[8 * (e0 + p) + M];
            v += (double)blk[at[M]];
        }
        const float f = (float)v;
        for (int M = 0; M < 8; ++M) blk[at[M]] = f;
    }
}

// escape by direction [nl][12 nside^2], from a copy
__global__ void k_mirror_esc(double *esc, const double *tmp, int nl, int nside, const int32_t *pmir)
{
    const int64_t np = 12 * (int64_t)nside * nside;
    const int64_t e0 = entry_of(nside, 0);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np * nl; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t l = i / np, p = i % np;
        double v = 0.0;
        for (int M = 0; M < 8; ++M) v += tmp[l * np + pmir[8 * (e0 + p) + M]];
        esc[i] = v;
    }
}

// the luminosity tallies the march counted for the traced sources, for all 8 images
__global__ void k_tally_x8(double *tally, int nl)
{
    const int l = threadIdx.x;
    if (l >= nl) return;
    const int cols[4] = {DARTRAY_T_EMITTED, DARTRAY_T_ESCAPED, DARTRAY_T_CUT, DARTRAY_T_SKIPPED};
    for (int k = 0; k < 4; ++k) tally[l * DARTRAY_N_TALLY + cols[k]] *= 8.0;
}

// Mirror tables (on first use) and the symmetry of density and emission
// (after every change of either).  Synchronises.
static int ensure_mirror(Grid &g)
{
    if (!g.mirror_geo) {
        const int64_t n = g.n;
        for (int a = 0; a < 3; ++a)
            if (g.fine[a] >= (1 << 21)) return fail(DARTRAY_E_UNSUPPORTED, "2D mode: grid above 2^21 finest cells per axis");
        std::vector<int4> box((size_t)n);
        DR_HIP(hipMemcpyAsync(box.data(), g.leaf_box, sizeof(int4) * n, hipMemcpyDeviceToHost, g.stream));
        DR_HIP(hipStreamSynchronize(g.stream));
        // leaves tile the block, so a lower corner names one leaf
        auto key = [](int64_t x, int64_t y, int64_t z) { return (uint64_t)x | ((uint64_t)y << 21) | ((uint64_t)z << 42); };
        std::unordered_map<uint64_t, int32_t> at;
        at.reserve((size_t)n * 2);
        for (int64_t c = 0; c < n; ++c) at.emplace(key(box[c].x, box[c].y, box[c].z), (int32_t)c);
        std::vector<int32_t> mir((size_t)n * 8), reps;
        std::vector<uint8_t> first((size_t)n);
        for (int64_t c = 0; c < n; ++c) {
            const int4 b = box[c];
            const int64_t lo[3] = {b.x, b.y, b.z};
            bool up = true;
            for (int a = 0; a < 3; ++a) {
                const int64_t F = g.fine[a];
                if (2 * lo[a] < F && F < 2 * (lo[a] + b.w))
                    return fail(DARTRAY_E_INVALID, "2D mode: a leaf lies across a plane through the block centre");
                up &= 2 * lo[a] + b.w > F;
            }
            first[c] = up ? 1 : 0;
            if (up) reps.push_back((int32_t)c);
            for (int M = 0; M < 8; ++M) {
                int64_t q[3];
                for (int a = 0; a < 3; ++a) q[a] = ((M >> a) & 1) ? g.fine[a] - lo[a] - b.w : lo[a];
                auto it = at.find(key(q[0], q[1], q[2]));
                if (it == at.end() || box[it->second].w != b.w)
                    return fail(DARTRAY_E_INVALID, "2D mode: the leaves are not mirror symmetric");
                mir[(size_t)c * 8 + M] = it->second;
            }
        }
        if ((int64_t)reps.size() * 8 != n) return fail(DARTRAY_E_INVALID, "2D mode: the leaves are not mirror symmetric");
        // mirror images of the pixels, Nside 1 .. 16: the pixel holding the
        // reflected centre, which is that pixel's own centre bit for bit
        const int64_t ne = entry_of(32, 0);
        std::vector<int32_t> pm((size_t)ne * 8);
        const double I[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        for (int64_t N = 1; N <= 16; N *= 2)
            for (int64_t p = 0; p < 12 * N * N; ++p) {
                double v[3], w[3], back[3];
                dr_pix_vec(N, p, I, v);
                for (int M = 0; M < 8; ++M) {
                    for (int a = 0; a < 3; ++a) w[a] = ((M >> a) & 1) ? -v[a] : v[a];
                    const int64_t q = dr_vec_pix(N, w);
                    dr_pix_vec(N, q, I, back);
                    if (back[0] != w[0] || back[1] != w[1] || back[2] != w[2])
                        return fail(DARTRAY_E_DEVICE, "2D mode: pixel set not mirror symmetric");
                    pm[(size_t)(entry_of(N, p) * 8 + M)] = (int32_t)q;
                }
            }
        DR_HIP(hipMemcpyAsync(g.mir, mir.data(), sizeof(int32_t) * mir.size(), hipMemcpyHostToDevice, g.stream));
        DR_HIP(hipMemcpyAsync(g.first, first.data(), (size_t)n, hipMemcpyHostToDevice, g.stream));
        DR_HIP(hipMemcpyAsync(g.reps, reps.data(), sizeof(int32_t) * reps.size(), hipMemcpyHostToDevice, g.stream));
        DR_HIP(hipMemcpyAsync(g.pmir, pm.data(), sizeof(int32_t) * pm.size(), hipMemcpyHostToDevice, g.stream));
        DR_HIP(hipStreamSynchronize(g.stream));
        g.n_reps = (int64_t)reps.size();
        g.mirror_geo = true;
    }
    if (!g.mirror_ok) {
        int rc = fill<uint32_t>(g, g.w.err_word, 1, 0u);
        if (rc) return rc;
        hipLaunchKernelGGL(k_mirror_check, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>((g.n + 255) / 256, 4096))),
                           dim3(256), 0, g.stream, g.mir, g.rho, g.emis_lum, g.n, g.n_lambda, g.w.err_word);
        DR_LAUNCH_CHECK("k_mirror_check");
        uint32_t bad = 0;
        DR_HIP(hipMemcpyAsync(&bad, g.w.err_word, sizeof(bad), hipMemcpyDeviceToHost, g.stream));
        DR_HIP(hipStreamSynchronize(g.stream));
        if (bad) return fail(DARTRAY_E_INVALID, "2D mode: density or emission not mirror symmetric");
        g.mirror_ok = true;
    }
    return DARTRAY_OK;
}

// the opts a 2D-mode pass runs with: the first octant as the source mask
static int prepare_2d(Grid &g, const dartray_trace_opts *o, dartray_trace_opts &o2)
{
    int rc = ensure_mirror(g);
    if (rc) return rc;
    o2 = *o;
    o2.source_mask = g.first;
    return DARTRAY_OK;
}

// after the march of a 2D-mode pass, before finish_pass
static int fold_2d(Grid &g, const dartray_trace_opts *o, dartray_fields *f, bool scatter)
{
    const int nl = g.n_lambda;
    const unsigned ub = (unsigned)std::max<int64_t>(1, std::min<int64_t>((g.n_reps * nl + 255) / 256, 4096));
    hipLaunchKernelGGL(k_mirror_u, dim3(ub), dim3(256), 0, g.stream, g.w.U_k, g.mir, g.reps, g.n_reps, nl);
    DR_LAUNCH_CHECK("k_mirror_u");
    const bool step1 = !scatter && o->mode == DARTRAY_MODE_STEP1;
    if (!step1) {
        int64_t widest = 0;
        for (int l = 0; l < nl; ++l) widest = std::max<int64_t>(widest, g.lt.npix[l]);
        const unsigned sb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((g.n_reps * widest + 255) / 256, 2048));
        hipLaunchKernelGGL(k_mirror_s, dim3(sb, nl), dim3(256), 0, g.stream, f->S_next, g.d_lt, g.mir, g.reps,
                           g.n_reps, g.pmir);
        DR_LAUNCH_CHECK("k_mirror_s");
    }
    if (f->escape && !o->adaptive) {
        const int64_t ne = (int64_t)nl * 12 * o->nside * o->nside;
        DR_HIP(hipMemcpyAsync(g.esc_tmp, g.w.esc64, sizeof(double) * ne, hipMemcpyDeviceToDevice, g.stream));
        hipLaunchKernelGGL(k_mirror_esc, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, g.stream, g.w.esc64,
                           (const double *)g.esc_tmp, nl, o->nside, g.pmir);
        DR_LAUNCH_CHECK("k_mirror_esc");
    }
    hipLaunchKernelGGL(k_tally_x8, dim3(1), dim3(64), 0, g.stream, f->tally, nl);
    DR_LAUNCH_CHECK("k_tally_x8");
    return DARTRAY_OK;
}

// Read the pass's device error word (synchronises the stream).
static int check_err(Grid &g)
{
    uint32_t w = 0;
    DR_HIP(hipMemcpyAsync(&w, g.w.err_word, sizeof(w), hipMemcpyDeviceToHost, g.stream));
    DR_HIP(hipStreamSynchronize(g.stream));
    if (w & 1u) return fail(DARTRAY_E_NUMERIC, "the pass produced a non-finite energy density or scattered luminosity");
    return DARTRAY_OK;
}

}  // namespace dr

extern "C" {

int dartray_trace_direct(dartray_grid *grid, const dartray_trace_opts *opts, dartray_fields *fields)
{
    if (!grid) return fail(DARTRAY_E_INVALID, "null grid");
    Grid &g = grid->g;
    int rc = check_opts(g, opts, fields, false);
    if (rc) return rc;
    dartray_trace_opts o2;
    const bool two_d = (opts->flags & DARTRAY_FLAG_2D) != 0;
    if (two_d && (rc = prepare_2d(g, opts, o2))) return rc;
    const dartray_trace_opts *o = two_d ? &o2 : opts;
    rc = o->adaptive ? run_adaptive_pass(g, o, fields, false) : run_fixed_pass(g, o, fields, false);
    if (rc) return rc;
    if (two_d && (rc = fold_2d(g, o, fields, false))) return rc;
    if ((rc = finish_pass(g, o, fields, false))) return rc;
    if ((o->flags & DARTRAY_FLAG_CHECK) || o->adaptive) return check_err(g);
    return DARTRAY_OK;
}

int dartray_scatter_iter(dartray_grid *grid, const dartray_trace_opts *opts, dartray_fields *fields, double *r_k)
{
    if (!grid) return fail(DARTRAY_E_INVALID, "null grid");
    Grid &g = grid->g;
    int rc = check_opts(g, opts, fields, true);
    if (rc) return rc;
    dartray_trace_opts o2;
    const bool two_d = (opts->flags & DARTRAY_FLAG_2D) != 0;
    if (two_d && (rc = prepare_2d(g, opts, o2))) return rc;
    const dartray_trace_opts *o = two_d ? &o2 : opts;
    rc = o->adaptive ? run_adaptive_pass(g, o, fields, true) : run_fixed_pass(g, o, fields, true);
    if (rc) return rc;
    if (two_d && (rc = fold_2d(g, o, fields, true))) return rc;
    if ((rc = finish_pass(g, o, fields, true))) return rc;
    if (r_k) {
        const int nl = g.n_lambda;
        double a[kMaxLambda], b[kMaxLambda];
        DR_HIP(hipMemcpyAsync(a, g.w.dsum, sizeof(double) * nl, hipMemcpyDeviceToHost, g.stream));
        DR_HIP(hipMemcpyAsync(b, g.s1_sum, sizeof(double) * nl, hipMemcpyDeviceToHost, g.stream));
        DR_HIP(hipStreamSynchronize(g.stream));
        double sa = 0.0, sb = 0.0;
        for (int l = 0; l < nl; ++l) {
            sa += a[l];
            sb += b[l];
        }
        *r_k = sb > 0.0 ? sa / sb : 0.0;
    }
    if ((opts->flags & DARTRAY_FLAG_CHECK) || opts->adaptive || r_k) return check_err(g);
    return DARTRAY_OK;
}

int dartray_trace_adjoint(dartray_grid *grid, const dartray_trace_opts *opts, int32_t n_scatter,
                          const float *const *S_hist, const float *dJ_dU, const float *dJ_dS, const float *dJ_desc,
                          float *dJ_drho)
{
    if (!grid) return fail(DARTRAY_E_INVALID, "null grid");
    Grid &g = grid->g;
    if (!opts || !dJ_drho || n_scatter < 0 || (n_scatter > 0 && !S_hist))
        return fail(DARTRAY_E_INVALID, "bad argument");
    for (int k = 0; k < n_scatter; ++k)
        if (!S_hist[k]) return fail(DARTRAY_E_INVALID, "null S_hist entry");
    if (opts->adaptive) return fail(DARTRAY_E_UNSUPPORTED, "the adjoint covers fixed rays only");
    if (opts->flags & DARTRAY_FLAG_2D) return fail(DARTRAY_E_UNSUPPORTED, "the adjoint has no 2D mode");
    if (opts->nside <= 0 || (opts->nside & (opts->nside - 1)) || opts->nside > kMaxNsideWTable)
        return fail(DARTRAY_E_INVALID, "adjoint nside must be a power of two <= 16");
    if (g.n_lambda > 8) return fail(DARTRAY_E_UNSUPPORTED, "the adjoint carries at most 8 wavelengths");
    const int nl = g.n_lambda;
    const int64_t n = g.n;
    Frame fr;
    frame_of(opts, fr);
    int rc = ensure_dirs(g, fr);
    if (rc) return rc;
    if ((rc = ensure_wtab(g, opts->nside, fr))) return rc;
    const int64_t nray = 12 * (int64_t)opts->nside * opts->nside;
    int log2n = 0;
    while ((1 << log2n) < opts->nside) ++log2n;
    if ((rc = fill<double>(g, g.rho_bar, (size_t)n, 0.0))) return rc;
    if (dJ_dU) {
        hipLaunchKernelGGL(k_transpose_ull, dim3((unsigned)std::min<int64_t>((n * nl + 255) / 256, 8192)), dim3(256), 0,
                           g.stream, dJ_dU, g.ull_t, n, nl);
        DR_LAUNCH_CHECK("k_transpose_ull");
    } else if ((rc = fill<float>(g, g.ull_t, (size_t)n * nl, 0.f))) {
        return rc;
    }
    const size_t per_dir = (size_t)nl * n;
    const int nb_max = (int)std::min<int64_t>(nray, (int64_t)(g.w.ubar_floats / per_dir));
    AdjArgs A{};
    A.geo = Geo{g.rec, g.root_tab, g.nodes, {g.fine[0], g.fine[1], g.fine[2]}, {g.nroot[0], g.nroot[1], g.nroot[2]},
                g.max_level};
    A.src_list = g.w.src_list;
    A.n_src = g.w.n_src;
    A.dirs = g.dir64 + entry_of(opts->nside, 0);
    A.emis_lum = g.emis_lum;
    A.ps_pos = g.ps_pos;
    A.ps_cell = g.ps_cell;
    A.ps_lum = g.ps_lum;
    A.n_point = g.n_point;
    A.lt = g.d_lt;
    A.ubar_t = g.ull_t;
    A.rho_bar = g.rho_bar;
    A.ebar = dJ_desc;
    A.n = n;
    A.order = g.tune.item_order;
    A.log2_nside_ray = log2n;
    A.inv_nray = (float)(1.0 / (double)nray);
    A.h_fine = g.h_fine;
    A.hard_cap = 4 * ((int64_t)g.fine[0] + g.fine[1] + g.fine[2]) + 64;
    // S_total holds every order S_1 .. S_{K+1}: dJ/dS_total reaches each of
    // them directly, the last (never re-emitted) one only directly
    const float *sbar_next = dJ_dS;
    g.prof_kind = DARTRAY_PROF_ADJOINT;
    for (int k = n_scatter; k >= 0; --k) {
        const bool scatter = k > 0;
        float *sbar_k = scatter ? g.sbar[k & 1] : nullptr;
        if (scatter) {
            if ((rc = fill<float>(g, sbar_k, (size_t)g.s_size, 0.f))) return rc;
            // every cell may feed scattered light back: all cells are sources
            DR_HIP(hipMemcpyAsync(g.w.src_list, g.morton, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, g.stream));
            if ((rc = fill<int32_t>(g, g.w.n_src, 1, (int32_t)n))) return rc;
        } else {
            dartray_fields tmp{};
            tmp.tally = g.w.dsum;   // emitted luminosity sums are not needed here
            if ((rc = fill<double>(g, g.w.dsum, (size_t)nl * DARTRAY_N_TALLY, 0.0))) return rc;
            if ((rc = select_sources(g, opts, &tmp, false))) return rc;
        }
        A.scatter = scatter ? 1 : 0;
        A.S_pending = scatter ? S_hist[k - 1] : nullptr;
        A.sbar_k = sbar_k;
        for (int64_t r0 = 0; r0 < nray; r0 += nb_max) {
            const int nb = (int)std::min<int64_t>(nb_max, nray - r0);
            A.r0 = (int)r0;
            A.nb = nb;
            A.sig = nullptr;
            if (sbar_next) {
                hipLaunchKernelGGL(k_sbar_gather, dim3((unsigned)((n + kGT - 1) / kGT), (unsigned)((nb + kGT - 1) / kGT)),
                                   dim3(256), 0, g.stream, g.w.ubar, g.wtab, g.d_lt, sbar_next, n, (int)r0, nb, g.w_row);
                DR_LAUNCH_CHECK("k_sbar_gather");
                A.sig = g.w.ubar;
            }
            const unsigned blocks = 2048;
            if ((rc = prof_mark(g))) return rc;
            if (nl <= 1) {
                if (g.uniform) hipLaunchKernelGGL((k_march_adjoint<1, true>), dim3(blocks), dim3(256), 0, g.stream, A);
                else hipLaunchKernelGGL((k_march_adjoint<1, false>), dim3(blocks), dim3(256), 0, g.stream, A);
            } else if (nl <= 4) {
                if (g.uniform) hipLaunchKernelGGL((k_march_adjoint<4, true>), dim3(blocks), dim3(256), 0, g.stream, A);
                else hipLaunchKernelGGL((k_march_adjoint<4, false>), dim3(blocks), dim3(256), 0, g.stream, A);
            } else {
                if (g.uniform) hipLaunchKernelGGL((k_march_adjoint<8, true>), dim3(blocks), dim3(256), 0, g.stream, A);
                else hipLaunchKernelGGL((k_march_adjoint<8, false>), dim3(blocks), dim3(256), 0, g.stream, A);
            }
            DR_LAUNCH_CHECK("k_march_adjoint");
            if ((rc = prof_mark(g))) return rc;
        }
        if (scatter && dJ_dS) {
            hipLaunchKernelGGL(k_add_f32, dim3((unsigned)std::min<int64_t>((g.s_size + 255) / 256, 8192)), dim3(256), 0,
                               g.stream, sbar_k, dJ_dS, g.s_size);
            DR_LAUNCH_CHECK("k_add_f32");
        }
        sbar_next = sbar_k;
    }
    hipLaunchKernelGGL(k_rho_out, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0, g.stream,
                       g.rho_bar, dJ_drho, n);
    DR_LAUNCH_CHECK("k_rho_out");
    return DARTRAY_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of models: every pass of every model in one persistent march launch
// and one flush launch per direction batch, optionally recorded once as a HIP
// graph and replayed.
// ---------------------------------------------------------------------------

struct dartray_batch {
    std::vector<dartray_grid *> grids;   // processing order: descending expected work
    std::vector<int> caller;             // caller's index of each processed model
    hipStream_t stream = nullptr;
    int32_t n_lambda = 0;
    dr::FixedArgs *d_args = nullptr;     // [2][n_models]: direct-pass and scattering-pass arguments
    dr::FlushArgs *d_flush = nullptr;    // [n_models]
    int64_t *d_item_off = nullptr;       // [n_models + 1]
    std::vector<dr::FixedArgs> h_args;
    std::vector<dr::FlushArgs> h_flush;
    int64_t flush_blocks = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace dr {

static void batch_free(dartray_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_args) (void)hipFree(b->d_args);
    if (b->d_flush) (void)hipFree(b->d_flush);
    if (b->d_item_off) (void)hipFree(b->d_item_off);
    delete b;
}

static void launch_fixed_multi(const BatchMarch &B, int nlt, hipStream_t s, unsigned blocks, unsigned threads)
{
    switch (nlt) {
    case 1: hipLaunchKernelGGL((k_march_fixed_multi<1>), dim3(blocks), dim3(threads), 0, s, B); break;
    case 4: hipLaunchKernelGGL((k_march_fixed_multi<4>), dim3(blocks), dim3(threads), 0, s, B); break;
    case 8: hipLaunchKernelGGL((k_march_fixed_multi<8>), dim3(blocks), dim3(threads), 0, s, B); break;
    case 16: hipLaunchKernelGGL((k_march_fixed_multi<16>), dim3(blocks), dim3(threads), 0, s, B); break;
    case 32: hipLaunchKernelGGL((k_march_fixed_multi<32>), dim3(blocks), dim3(threads), 0, s, B); break;
    default: hipLaunchKernelGGL((k_march_fixed_multi<64>), dim3(blocks), dim3(threads), 0, s, B); break;
    }
}

// argument checks and the device copies of every model's pass arguments;
// fields[k] belongs to the caller's model k
static int batch_prepare(dartray_batch *b, const dartray_trace_opts *o, dartray_fields *const *fields,
                         const std::vector<int> &caller_index)
{
    if (!o || !fields) return fail(DARTRAY_E_INVALID, "null opts or fields");
    if (o->adaptive) return fail(DARTRAY_E_UNSUPPORTED, "batches run fixed rays only");
    if (o->mode != DARTRAY_MODE_DIRECT) return fail(DARTRAY_E_INVALID, "batches start with the direct pass");
    if (o->source_mask) return fail(DARTRAY_E_UNSUPPORTED, "batches take no source mask");
    const size_t nm = b->grids.size();
    for (size_t k = 0; k < nm; ++k) {
        Grid &g = b->grids[k]->g;
        dartray_fields *f = fields[caller_index[k]];
        int rc = check_opts(g, o, f, false);
        if (rc) return rc;
        if (o->nside > kMaxNsideWTable) return fail(DARTRAY_E_UNSUPPORTED, "fixed-mode nside above 16");
        Frame fr;
        frame_of(o, fr);
        if ((rc = ensure_dirs(g, fr))) return rc;
        if ((rc = ensure_wtab(g, o->nside, fr))) return rc;
        b->h_args[k] = fixed_args(g, o, f, false);
        b->h_args[nm + k] = fixed_args(g, o, f, true);
        b->h_flush[k] = flush_args(g, f->S_next);
    }
    // flat flush grid: model k owns (cell blocks) x (pixel chunks) blocks
    const FlushShape fs0 = flush_shape(b->grids[0]->g);
    int pch = fs0.pch;
    for (size_t k = 0; k < nm; ++k) pch = std::min(pch, flush_shape(b->grids[k]->g).pch);
    int64_t blk = 0;
    for (size_t k = 0; k < nm; ++k) {
        const Grid &g = b->grids[k]->g;
        const FlushShape fs = flush_shape(g);
        const int64_t bx = (g.n + fs.per_block - 1) / fs.per_block;
        b->h_flush[k].bx = (int32_t)bx;
        b->h_flush[k].block0 = blk;
        blk += bx * (fs.max_npix / pch);
    }
    if (blk > (int64_t)INT32_MAX) return fail(DARTRAY_E_UNSUPPORTED, "batch too large for one flush launch");
    b->flush_blocks = blk;
    DR_HIP(hipMemcpyAsync(b->d_args, b->h_args.data(), sizeof(FixedArgs) * 2 * nm, hipMemcpyHostToDevice, b->stream));
    DR_HIP(hipMemcpyAsync(b->d_flush, b->h_flush.data(), sizeof(FlushArgs) * nm, hipMemcpyHostToDevice, b->stream));
    DR_HIP(hipStreamSynchronize(b->stream));
    return DARTRAY_OK;
}

// the pass sequence: direct pass, then n_scatter scattering iterations
static int batch_sequence(dartray_batch *b, const dartray_trace_opts *o, dartray_fields *const *fields,
                          const std::vector<int> &caller_index, int n_scatter)
{
    const int nm = (int)b->grids.size();
    const int nl = b->n_lambda;
    const int64_t nray = 12 * (int64_t)o->nside * o->nside;
    Grid &g0 = b->grids[0]->g;
    int nb = (int)nray;
    for (int k = 0; k < nm; ++k) nb = std::min(nb, dir_batch(b->grids[k]->g, nray));
    const FlushShape fs0 = flush_shape(g0);
    int pch = fs0.pch;
    size_t lds = 0;
    for (int k = 0; k < nm; ++k) {
        const FlushShape fs = flush_shape(b->grids[k]->g);
        pch = std::min(pch, fs.pch);
    }
    int rb_stage = 16;
    while (rb_stage > 1 && (size_t)rb_stage * nl * (pch + 1) * sizeof(float) > (size_t)48 * 1024) rb_stage >>= 1;
    lds = (size_t)rb_stage * nl * (pch + 1) * sizeof(float);
    const int chunk = lambda_chunk(g0);
    const unsigned threads = 64u * (unsigned)(g0.tune.block_waves > 0 ? g0.tune.block_waves : 4);
    const unsigned blocks = (unsigned)(g0.tune.grid_blocks > 0 ? g0.tune.grid_blocks : 2048);
    const bool counting = (o->flags & DARTRAY_FLAG_COUNTERS) != 0;
    int rc;
    for (int pass = 0; pass <= n_scatter; ++pass) {
        const bool scatter = pass > 0;
        for (int k = 0; k < nm; ++k) {
            Grid &g = b->grids[k]->g;
            dartray_fields *f = fields[caller_index[k]];
            if ((rc = fill<double>(g, g.w.U_k, (size_t)nl * g.n, 0.0))) return rc;
            if ((rc = fill<float>(g, f->S_next, (size_t)g.s_size, 0.f))) return rc;
            if ((rc = fill<double>(g, f->tally, (size_t)nl * DARTRAY_N_TALLY, 0.0))) return rc;
            if (counting && (rc = fill<uint64_t>(g, f->counters, DARTRAY_N_COUNT, 0))) return rc;
            if (f->escape && (rc = fill<double>(g, g.w.esc64, (size_t)nl * nray, 0.0))) return rc;
            if ((rc = select_sources(g, o, f, scatter))) return rc;
        }
        const FixedArgs *args = b->d_args + (scatter ? nm : 0);
        for (int64_t r0 = 0; r0 < nray; r0 += nb) {
            const int nbb = (int)std::min<int64_t>(nb, nray - r0);
            for (int k = 0; k < nm; ++k) {
                Grid &g = b->grids[k]->g;
                if ((rc = fill<float>(g, g.w.ubar, (size_t)nbb * nl * g.n, 0.f))) return rc;
            }
            hipLaunchKernelGGL(k_batch_items, dim3(1), dim3(64), 0, b->stream, args, nm, nbb, b->d_item_off);
            DR_LAUNCH_CHECK("k_batch_items");
            for (int l0 = 0; l0 < nl; l0 += chunk) {
                BatchMarch B{};
                B.models = args;
                B.item_off = b->d_item_off;
                B.n_models = nm;
                B.r0 = (int)r0;
                B.nb = nbb;
                B.l0 = l0;
                B.nlc = std::min(chunk, nl - l0);
                B.count = l0 == 0 ? 1 : 0;
                launch_fixed_multi(B, nl_template(B.nlc), b->stream, blocks, threads);
                DR_LAUNCH_CHECK("k_march_fixed_multi");
            }
            if (pch == 48)
                hipLaunchKernelGGL(k_flush_fixed_multi<48>, dim3((unsigned)b->flush_blocks), dim3(256), lds, b->stream,
                                   b->d_flush, nm, (int)r0, nbb, fs0.log2_nlp, rb_stage);
            else
                hipLaunchKernelGGL(k_flush_fixed_multi<12>, dim3((unsigned)b->flush_blocks), dim3(256), lds, b->stream,
                                   b->d_flush, nm, (int)r0, nbb, fs0.log2_nlp, rb_stage);
            DR_LAUNCH_CHECK("k_flush_fixed_multi");
        }
        for (int k = 0; k < nm; ++k) {
            Grid &g = b->grids[k]->g;
            if ((rc = finish_pass(g, o, fields[caller_index[k]], scatter))) return rc;
        }
    }
    return DARTRAY_OK;
}

}  // namespace dr

extern "C" {

int dartray_batch_create(dartray_grid *const *grids, int32_t n_models, dartray_batch **out)
{
    if (!out) return fail(DARTRAY_E_INVALID, "null out");
    *out = nullptr;
    if (!grids || n_models <= 0) return fail(DARTRAY_E_INVALID, "need at least one grid");
    for (int m = 0; m < n_models; ++m) {
        if (!grids[m]) return fail(DARTRAY_E_INVALID, "null grid in batch");
        if (grids[m]->g.stream != grids[0]->g.stream) return fail(DARTRAY_E_INVALID, "grids of a batch share one stream");
        if (grids[m]->g.n_lambda != grids[0]->g.n_lambda)
            return fail(DARTRAY_E_INVALID, "grids of a batch carry the same number of wavelengths");
        for (int k = 0; k < m; ++k)
            if (grids[k] == grids[m]) return fail(DARTRAY_E_INVALID, "a grid appears twice in the batch");
    }
    auto *b = new dartray_batch;
    b->stream = grids[0]->g.stream;
    b->n_lambda = grids[0]->g.n_lambda;
    // descending expected work: sources x rays x path length ~ n^(4/3)
    std::vector<int> idx(n_models);
    for (int m = 0; m < n_models; ++m) idx[m] = m;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) { return grids[a]->g.n > grids[c]->g.n; });
    for (int m : idx) {
        b->grids.push_back(grids[m]);
        b->caller.push_back(m);
    }
    b->h_args.resize(2 * (size_t)n_models);
    b->h_flush.resize(n_models);
    if (hipMalloc(&b->d_args, sizeof(dr::FixedArgs) * 2 * n_models) != hipSuccess ||
        hipMalloc(&b->d_flush, sizeof(dr::FlushArgs) * n_models) != hipSuccess ||
        hipMalloc(&b->d_item_off, sizeof(int64_t) * (n_models + 1)) != hipSuccess) {
        (void)hipGetLastError();
        dr::batch_free(b);
        return fail(DARTRAY_E_OOM, "batch argument arrays");
    }
    *out = b;
    return DARTRAY_OK;
}

int dartray_batch_destroy(dartray_batch *b)
{
    if (b) dr::batch_free(b);
    return DARTRAY_OK;
}

int dartray_batch_run(dartray_batch *b, const dartray_trace_opts *opts, dartray_fields *const *fields,
                      int32_t n_scatter)
{
    if (!b) return fail(DARTRAY_E_INVALID, "null batch");
    if (opts && (opts->flags & DARTRAY_FLAG_2D)) return fail(DARTRAY_E_UNSUPPORTED, "batches have no 2D mode");
    if (n_scatter < 0) return fail(DARTRAY_E_INVALID, "n_scatter must be >= 0");
    int rc = dr::batch_prepare(b, opts, fields, b->caller);
    if (rc) return rc;
    return dr::batch_sequence(b, opts, fields, b->caller, n_scatter);
}

int dartray_batch_capture(dartray_batch *b, const dartray_trace_opts *opts, dartray_fields *const *fields,
                          int32_t n_scatter)
{
    if (!b) return fail(DARTRAY_E_INVALID, "null batch");
    if (opts && (opts->flags & DARTRAY_FLAG_2D)) return fail(DARTRAY_E_UNSUPPORTED, "batches have no 2D mode");
    if (n_scatter < 0) return fail(DARTRAY_E_INVALID, "n_scatter must be >= 0");
    int rc = dr::batch_prepare(b, opts, fields, b->caller);
    if (rc) return rc;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    // no event records inside the graph
    std::vector<int32_t> prof(b->grids.size());
    for (size_t k = 0; k < b->grids.size(); ++k) {
        prof[k] = b->grids[k]->g.prof;
        b->grids[k]->g.prof = 0;
    }
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) rc = hip_fail(e, "hipStreamBeginCapture");
    int rs = rc ? rc : dr::batch_sequence(b, opts, fields, b->caller, n_scatter);
    if (!rc) {
        hipGraph_t gr = nullptr;
        e = hipStreamEndCapture(b->stream, &gr);
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamEndCapture");
        else if (rs) {
            (void)hipGraphDestroy(gr);
            rc = rs;
        } else {
            b->graph = gr;
            e = hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                b->exec = nullptr;
                rc = hip_fail(e, "hipGraphInstantiate");
            }
        }
    }
    for (size_t k = 0; k < b->grids.size(); ++k) b->grids[k]->g.prof = prof[k];
    return rc;
}

int dartray_batch_replay(dartray_batch *b)
{
    if (!b) return fail(DARTRAY_E_INVALID, "null batch");
    if (!b->exec) return fail(DARTRAY_E_STATE, "no captured graph");
    hipError_t e = hipGraphLaunch(b->exec, b->stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return DARTRAY_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Direct pass that allocates nothing.  Its work arrays (energy-density
// accumulators, direction bins, source list, scan sums, tallies' scratch,
// error word) are carved from `scratch`, a static device array of
// kScratchBytes per GPU, instead of the handle's own arrays; the kernels are
// those of dartray_trace_direct.
// ---------------------------------------------------------------------------

namespace dr {

constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
static void *g_scratch_ptr[kMaxScratchDevices];
static std::mutex g_scratch_mu;

// Device address of the current device's copy of `scratch`, looked up once
// per device (with that device current) and kept: in host code the array's
// name is only a stand-in, never a device address.
static int scratch_base(char **out)
{
    int dev = 0;
    DR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(DARTRAY_E_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(DARTRAY_E_DEVICE, "hipGetSymbolAddress(scratch) returned a null address");
        g_scratch_ptr[dev] = p;
    }
    *out = (char *)g_scratch_ptr[dev];
    return DARTRAY_OK;
}

// Work arrays of a fixed-ray direct pass laid out in the scratch array: the
// fixed-size parts first, the direction bins take what remains (at least one
// direction).  Sizes beyond kScratchBytes are refused.
static int scratch_work(const Grid &g, const dartray_trace_opts *o, const dartray_fields *f, char *base, PassWork &w)
{
    const size_t n = (size_t)g.n, nl = (size_t)g.n_lambda;
    const size_t ns = n + (size_t)g.n_point;       // cells and point sources
    const size_t nray = 12 * (size_t)o->nside * (size_t)o->nside;
    const size_t nblk = (ns + kScanBlock - 1) / kScanBlock;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        const size_t at = off;
        off += bytes;
        return at;
    };
    const size_t o_uk = take(n * nl * sizeof(double)), o_flags = take(ns * sizeof(int32_t)),
                 o_src = take(ns * sizeof(int32_t)), o_scan = take(nblk * sizeof(int32_t)), o_nsrc = take(sizeof(int32_t)),
                 o_nall = take(sizeof(int32_t)), o_err = take(sizeof(uint32_t)),
                 o_dsum = take(4 * (size_t)kMaxLambda * sizeof(double)),
                 o_esc = f->escape ? take(nl * nray * sizeof(double)) : 0;
    off = (off + 255) & ~(size_t)255;
    const size_t per_dir = n * nl * sizeof(float);
    if (off + per_dir > kScratchBytes) {
        return fail(DARTRAY_E_UNSUPPORTED, "the allocation-free direct pass needs " + std::to_string(off + per_dir) +
                                               " bytes of scratch for this grid; its limit is " +
                                               std::to_string(kScratchBytes) + " bytes");
    }
    w.U_k = (double *)(base + o_uk);
    w.flags = (int32_t *)(base + o_flags);
    w.src_list = (int32_t *)(base + o_src);
    w.scan_blocks = (int32_t *)(base + o_scan);
    w.n_src = (int32_t *)(base + o_nsrc);
    w.n_all = (int32_t *)(base + o_nall);
    w.err_word = (uint32_t *)(base + o_err);
    w.dsum = (double *)(base + o_dsum);
    w.esc64 = f->escape ? (double *)(base + o_esc) : nullptr;
    w.ubar = (float *)(base + off);
    w.ubar_floats = (kScratchBytes - off) / sizeof(float);
    return DARTRAY_OK;
}

}  // namespace dr

extern "C" {

int dartray_trace_direct_noalloc(dartray_grid *grid, const dartray_trace_opts *opts, dartray_fields *fields)
{
    if (!grid) return fail(DARTRAY_E_INVALID, "null grid");
    Grid &g = grid->g;
    int rc = check_opts(g, opts, fields, false);
    if (rc) return rc;
    if (opts->adaptive || opts->mode != DARTRAY_MODE_DIRECT)
        return fail(DARTRAY_E_UNSUPPORTED, "the allocation-free direct pass covers fixed rays only");
    if (opts->flags & DARTRAY_FLAG_2D) return fail(DARTRAY_E_UNSUPPORTED, "the allocation-free direct pass has no 2D mode");
    if (opts->nside > kMaxNsideWTable) return fail(DARTRAY_E_UNSUPPORTED, "fixed-mode nside above 16");
    int prev = 0;
    DR_HIP(hipGetDevice(&prev));
    if (prev != g.device) DR_HIP(hipSetDevice(g.device));
    char *base = nullptr;
    PassWork w{};
    rc = scratch_base(&base);
    if (!rc) rc = scratch_work(g, opts, fields, base, w);
    if (!rc) {
        // the pass runs on the scratch work set; no timing events are created
        const int32_t prof = g.prof;
        g.prof = 0;
        g.w = w;
        rc = run_fixed_pass(g, opts, fields, false);
        if (!rc) rc = finish_pass(g, opts, fields, false);
        if (!rc && (opts->flags & DARTRAY_FLAG_CHECK)) rc = check_err(g);
        g.w = g.own;
        g.prof = prof;
    }
    if (prev != g.device) (void)hipSetDevice(prev);
    return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Observer maps (Sect. 2: I_obs = I_0 e^{-tau} from every cell; Sect. 3.6:
// internal-observer HEALPix maps).  A gather march: one lane per cell walks
// from the cell centre towards the observer (or out of the block for a
// distant one) summing rho l in FP64, then adds the cell's luminosity per
// steradian towards the observer -- j V, plus S[p] N_pix / (4 pi) for the
// j_sca pixel p holding that direction -- times e^{-kappa sum rho l} to its
// map pixel (FP64 atomics).  Cells are taken in Morton order, so the lanes
// of a wave start from neighbouring cells.
// ---------------------------------------------------------------------------

namespace dr {

struct ObsArgs {
    Geo geo;
    const int32_t *morton;
    const LambdaTable *lt;
    const double *lum64;          // [n_lambda][n] 4 pi j V
    const double4 *ps_pos;        // point sources (item n + k), fine units
    const double4 *ps_xyz;        // the same, model units as given
    const int32_t *ps_cell;
    const double *ps_lum64;       // [n_lambda][n_point]
    int32_t n_point;
    const float *S;               // S_total, or null
    double *map;                  // [n_lambda][npix]
    int64_t n;
    int64_t npix;
    int32_t kind;                 // DARTRAY_OBS_*
    int32_t nx, ny;
    int32_t nside_map;
    int32_t obs_cell;             // internal: the leaf holding the observer (left out)
    double dir[3];                // distant: unit vector towards the observer
    double e1[3], e2[3];          // distant: image axes
    double centre[3];             // distant: image centre, model units
    double pos[3];                // internal: observer, model units
    double pixel;                 // distant: pixel edge, model units
    double pix_weight;            // distant: 1 / pixel area; internal: 1 / map-pixel solid angle
    double lo[3];                 // model-space corner of the grid
    double h_fine;
    double R[9];                  // frame of the j_sca pixel directions
    int64_t hard_cap;
};

// Where a source lands on the map, from its model-space position, in plain
// FP64 steps without fused multiply-adds: a source whose projection falls on a
// pixel edge (a cell row seen face-on, say) goes to the pixel that ordinary
// rounding of these steps selects, whatever the compiler would contract.
__device__ __noinline__ int64_t obs_locate(const ObsArgs &A, const double xc[3], double nv[3], double &dist)
{
#pragma clang fp contract(off)
    if (A.kind == DARTRAY_OBS_DISTANT) {
        double u = 0.0, w = 0.0;
        for (int a = 0; a < 3; ++a) {
            nv[a] = A.dir[a];
            u += (xc[a] - A.centre[a]) * A.e1[a];
            w += (xc[a] - A.centre[a]) * A.e2[a];
        }
        const double fx = floor(u / A.pixel + 0.5 * A.nx), fy = floor(w / A.pixel + 0.5 * A.ny);
        if (!(fx >= 0.0 && fy >= 0.0 && fx < (double)A.nx && fy < (double)A.ny)) return -1;
        dist = __builtin_huge_val();
        return (int64_t)fy * A.nx + (int64_t)fx;
    }
    for (int a = 0; a < 3; ++a) nv[a] = A.pos[a] - xc[a];
    dist = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    if (!(dist > 0.0)) return -1;
    for (int a = 0; a < 3; ++a) nv[a] /= dist;
    const double away[3] = {-nv[0], -nv[1], -nv[2]};   // from the observer towards the source
    return dr_vec_pix(A.nside_map, away);
}

// model-space centre of a leaf: corner + (fine offset of the centre) x h
__device__ __noinline__ void obs_centre(const ObsArgs &A, const int4 b, double xc[3])
{
#pragma clang fp contract(off)
    const double half = 0.5 * (double)b.w;
    xc[0] = A.lo[0] + ((double)b.x + half) * A.h_fine;
    xc[1] = A.lo[1] + ((double)b.y + half) * A.h_fine;
    xc[2] = A.lo[2] + ((double)b.z + half) * A.h_fine;
}

__global__ __launch_bounds__(256) void k_observe(const ObsArgs A)
{
    const LambdaTable *lt = A.lt;
    const int nl = lt->n_lambda;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < A.n + A.n_point;
         i += (int64_t)gridDim.x * blockDim.x) {
        // a cell (Morton order), or point source i - n
        const bool point = i >= A.n;
        const int32_t c = point ? A.ps_cell[i - A.n] : A.morton[i];
        if (!point && c == A.obs_cell) continue;
        RayT<double> R;
        double xc[3];
        if (point) {
            const double4 pp = A.ps_pos[i - A.n];
            R.o[0] = pp.x;
            R.o[1] = pp.y;
            R.o[2] = pp.z;
            const double4 px = A.ps_xyz[i - A.n];
            xc[0] = px.x;
            xc[1] = px.y;
            xc[2] = px.z;
        } else {
            const int4 b = A.geo.rec[c].box;
            const double half = 0.5 * (double)b.w;
            R.o[0] = (double)b.x + half;
            R.o[1] = (double)b.y + half;
            R.o[2] = (double)b.z + half;
            obs_centre(A, b, xc);
        }
        double dist;
        const int64_t pix = obs_locate(A, xc, R.n, dist);
        if (pix < 0) continue;
        // the march runs in fine units; it ends at the observer (internal) or
        // leaves the block (distant)
        const double stop = dist / A.h_fine;
        const double weight = A.kind == DARTRAY_OBS_DISTANT ? A.pix_weight : A.pix_weight / (dist * dist);
        for (int a = 0; a < 3; ++a) R.inv[a] = 1.0 / R.n[a];
        // optical depth towards the observer: sum of rho l over the crossings
        double colr = 0.0, t = 0.0;
        int32_t cc = c;
        for (int64_t steps = 0; cc >= 0 && t < stop && steps < A.hard_cap; ++steps) {
            const LeafRec &rc = A.geo.rec[cc];
            const int4 bb = rc.box;
            int32_t nbc[6];
            for (int q = 0; q < 6; ++q) nbc[q] = rc.nb[q];
            int axis;
            const double te = exit_t<double>(R, bb, axis);
            const double len = te - t;
            if (!is_graze(len, te)) {
                const double seg = (te < stop ? te : stop) - t;
                colr += (double)rc.rho * (seg * A.h_fine);
                t = te;
            }
            cc = next_leaf<double>(A.geo, R, bb, nbc, axis, te);
        }
        // the j_sca pixel holding the direction towards the observer, in the rotated frame
        const double loc[3] = {A.R[0] * R.n[0] + A.R[3] * R.n[1] + A.R[6] * R.n[2],
                               A.R[1] * R.n[0] + A.R[4] * R.n[1] + A.R[7] * R.n[2],
                               A.R[2] * R.n[0] + A.R[5] * R.n[1] + A.R[8] * R.n[2]};
        for (int l = 0; l < nl; ++l) {
            if (point) {
                const double dl = A.ps_lum64[(int64_t)l * A.n_point + (i - A.n)] / (4.0 * kPi);
                if (dl != 0.0)
                    atomic_add_f64(A.map + (int64_t)l * A.npix + pix, dl * exp(-(double)lt->kappa[l] * colr) * weight);
                continue;
            }
            double dl = A.lum64[(int64_t)l * A.n + c] / (4.0 * kPi);
            if (A.S) {
                const int np = lt->npix[l];
                dl += (double)A.S[lt->s_off[l] + (int64_t)c * np + dr_vec_pix(lt->nside_sca[l], loc)] * (double)np /
                      (4.0 * kPi);
            }
            if (dl == 0.0) continue;
            atomic_add_f64(A.map + (int64_t)l * A.npix + pix, dl * exp(-(double)lt->kappa[l] * colr) * weight);
        }
    }
}

}  // namespace dr

extern "C" {

int dartray_observe(dartray_grid *grid, const dartray_observer *obs, const float *S_total, double *map)
{
    if (!grid || !obs || !map) return fail(DARTRAY_E_INVALID, "null argument");
    Grid &g = grid->g;
    ObsArgs A{};
    A.geo = Geo{g.rec, g.root_tab, g.nodes, {g.fine[0], g.fine[1], g.fine[2]}, {g.nroot[0], g.nroot[1], g.nroot[2]},
                g.max_level};
    A.morton = g.morton;
    A.lt = g.d_lt;
    A.lum64 = g.lum64;
    A.ps_pos = g.ps_pos;
    A.ps_xyz = g.ps_xyz;
    A.ps_cell = g.ps_cell;
    A.ps_lum64 = g.ps_lum64;
    A.n_point = g.n_point;
    A.S = S_total;
    A.map = map;
    A.n = g.n;
    A.kind = obs->kind;
    A.h_fine = g.h_fine;
    for (int a = 0; a < 3; ++a) A.lo[a] = g.lo[a];
    A.obs_cell = -1;
    A.hard_cap = 4 * ((int64_t)g.fine[0] + g.fine[1] + g.fine[2]) + 64;
    bool zero = true;
    for (int i = 0; i < 9; ++i) zero &= obs->frame[i] == 0.0;
    for (int i = 0; i < 9; ++i) A.R[i] = zero ? ((i % 4 == 0) ? 1.0 : 0.0) : obs->frame[i];
    if (obs->kind == DARTRAY_OBS_DISTANT) {
        if (obs->nx <= 0 || obs->ny <= 0 || !(obs->pixel_size > 0.0) || !std::isfinite(obs->pixel_size))
            return fail(DARTRAY_E_INVALID, "distant observer: image size and pixel size must be positive");
        double d[3], up[3];
        for (int a = 0; a < 3; ++a) {
            d[a] = obs->dir[a];
            up[a] = obs->up[a];
        }
        const double dn = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (!(dn > 0.0) || !std::isfinite(dn)) return fail(DARTRAY_E_INVALID, "distant observer: zero direction");
        for (int a = 0; a < 3; ++a) d[a] /= dn;
        const double ud = up[0] * d[0] + up[1] * d[1] + up[2] * d[2];
        double e2[3], n2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            e2[a] = up[a] - ud * d[a];
            n2 += e2[a] * e2[a];
        }
        if (!(n2 > 1e-24)) return fail(DARTRAY_E_INVALID, "distant observer: up parallel to the direction");
        for (int a = 0; a < 3; ++a) e2[a] /= std::sqrt(n2);
        const double e1[3] = {e2[1] * d[2] - e2[2] * d[1], e2[2] * d[0] - e2[0] * d[2], e2[0] * d[1] - e2[1] * d[0]};
        for (int a = 0; a < 3; ++a) {
            A.dir[a] = d[a];
            A.e1[a] = e1[a];
            A.e2[a] = e2[a];
            A.centre[a] = obs->centre[a];
        }
        A.nx = obs->nx;
        A.ny = obs->ny;
        A.npix = (int64_t)obs->nx * obs->ny;
        A.pixel = obs->pixel_size;
        A.pix_weight = 1.0 / (obs->pixel_size * obs->pixel_size);
    } else if (obs->kind == DARTRAY_OBS_INTERNAL) {
        const int ns = obs->nside_map;
        if (ns <= 0 || (ns & (ns - 1)) || ns > 8192) return fail(DARTRAY_E_INVALID, "internal observer: nside_map must be a power of two <= 8192");
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(obs->pos[a])) return fail(DARTRAY_E_INVALID, "internal observer: position not finite");
            A.pos[a] = obs->pos[a];
        }
        A.nside_map = ns;
        A.npix = 12 * (int64_t)ns * ns;
        A.pix_weight = (double)A.npix / (4.0 * kPi);
        // the leaf holding the observer (points on a face belong to the upper side)
        int f[3];
        bool inside = true;
        for (int a = 0; a < 3; ++a) {
            const double u = std::floor((obs->pos[a] - g.lo[a]) / g.h_fine);
            inside &= u >= 0.0 && u < (double)g.fine[a];
            f[a] = inside ? (int)u : 0;
        }
        if (inside) {
            std::vector<int4> boxes((size_t)g.n);
            // the observer's leaf: one host search over the leaf boxes (set-up, not the march)
            DR_HIP(hipMemcpyAsync(boxes.data(), g.leaf_box, sizeof(int4) * g.n, hipMemcpyDeviceToHost, g.stream));
            DR_HIP(hipStreamSynchronize(g.stream));
            for (int64_t c = 0; c < g.n; ++c) {
                const int4 bx = boxes[(size_t)c];
                if (f[0] >= bx.x && f[0] < bx.x + bx.w && f[1] >= bx.y && f[1] < bx.y + bx.w && f[2] >= bx.z &&
                    f[2] < bx.z + bx.w) {
                    A.obs_cell = (int32_t)c;
                    break;
                }
            }
        }
    } else {
        return fail(DARTRAY_E_INVALID, "unknown observer kind");
    }
    int rc = fill<double>(g, map, (size_t)(g.n_lambda * A.npix), 0.0);
    if (rc) return rc;
    hipLaunchKernelGGL(k_observe, dim3((unsigned)std::min<int64_t>((g.n + g.n_point + 255) / 256, 8192)), dim3(256), 0,
                       g.stream, A);
    DR_LAUNCH_CHECK("k_observe");
    return DARTRAY_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Dust emission and the self-heating loop (Sect. 3.3)
// ---------------------------------------------------------------------------
// Every wavelength of a grid is a band.  A cell absorbs (1 - albedo) kappa
// rho V c U per band; the equilibrium grain re-emits the sum over the
// emitting grid's bands as 4 pi rho V kappa_i (1 - albedo_i) B(lambda_i, T)
// dlambda_i.  One thread per cell: the temperature is a bisection of
// [0, t_max] down to adjacent doubles, some 60-70 steps of n_lambda expm1
// each, negligible next to a ray pass.

namespace dr {

struct DustBand {
    double kabs;                  // kappa (1 - albedo)
    double lam, dlam;             // band centre and width
};

struct DustArgs {
    const float *rho;
    const int4 *leaf_box;
    double h_fine;
    int64_t n;
    int32_t nl;
    double b0, x0, t_max;
    DustBand band[kMaxLambda];
    const double *A;              // absorbed luminosity [n]
    double *T;                    // [n]
    double *j;                    // [nl][n]
    const double *j_prev;         // [nl][n] or null
    double *dj;                   // [nl][n] max(j - j_prev, 0), with j_prev
    unsigned long long *word;     // [0] max dj / j_prev (FP64 bits), [1] bracket overflow
};

__device__ inline double dust_planck(const DustArgs &D, double lam, double T)
{
    if (!(T > 0.0)) return 0.0;
    return D.b0 / (lam * lam * lam * lam * lam) / expm1(D.x0 / (lam * T));
}

// power a unit dust mass emits at temperature T over every band
__device__ inline double dust_power(const DustArgs &D, double T)
{
    double p = 0.0;
    for (int l = 0; l < D.nl; ++l) p += 4.0 * kPi * D.band[l].kabs * dust_planck(D, D.band[l].lam, T) * D.band[l].dlam;
    return p;
}

__global__ __launch_bounds__(256) void k_dust_emis(const DustArgs D)
{
    double qmax = 0.0;
    const double p_top = dust_power(D, D.t_max);
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < D.n; c += (int64_t)gridDim.x * blockDim.x) {
        const double side = (double)D.leaf_box[c].w * D.h_fine;
        const double vol = side * side * side;
        const double rho = (double)D.rho[c];
        const double a = D.A[c];
        double t = 0.0;
        if (rho > 0.0 && a > 0.0) {
            const double target = a / (rho * vol);
            if (!(p_top >= target)) {
                atomicMax(&D.word[1], 1ull);
            } else {
                double lo = 0.0, hi = D.t_max;
                for (;;) {
                    const double mid = 0.5 * (lo + hi);
                    if (!(mid > lo && mid < hi)) break;
                    if (dust_power(D, mid) < target)
                        lo = mid;
                    else
                        hi = mid;
                }
                t = hi;
            }
        }
        D.T[c] = t;
        for (int l = 0; l < D.nl; ++l) {
            const int64_t i = (int64_t)l * D.n + c;
            const double jl = rho * D.band[l].kabs * dust_planck(D, D.band[l].lam, t) * D.band[l].dlam;
            D.j[i] = jl;
            if (D.j_prev) {
                const double jp = D.j_prev[i];
                const double d = jl > jp ? jl - jp : 0.0;
                D.dj[i] = d;
                const double q = jp > 0.0 ? d / jp : (d > 0.0 ? __builtin_huge_val() : 0.0);
                qmax = q > qmax ? q : qmax;
            }
        }
    }
    if (D.j_prev) {
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(qmax, off);
            qmax = o > qmax ? o : qmax;
        }
        // non-negative doubles order as their bit patterns
        if ((threadIdx.x & 63) == 0 && qmax > 0.0) atomicMax(&D.word[0], (unsigned long long)__double_as_longlong(qmax));
    }
}

// A[c] = (base ? base[c] : A[c]) + sum_l (1 - albedo_l) kappa_l rho_c V_c c U[l][c]
__global__ __launch_bounds__(256) void k_absorbed(const LambdaTable *lt, const float *rho, const int4 *leaf_box,
                                                  double h_fine, double c_light, const float *U, const double *base,
                                                  double *A, int64_t n)
{
    const int nl = lt->n_lambda;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
        const double side = (double)leaf_box[c].w * h_fine;
        const double vol = side * side * side;
        const double r = (double)rho[c];
        double s = 0.0;
        for (int l = 0; l < nl; ++l)
            s += (1.0 - (double)lt->albedo[l]) * (double)lt->kappa[l] * r * vol * c_light * (double)U[(int64_t)l * n + c];
        A[c] = (base ? base[c] : A[c]) + s;
    }
}

// 4 pi j V of every cell, FP64 and FP32: the launch luminosity of later passes
__global__ __launch_bounds__(256) void k_set_emis(const double *j, const int4 *leaf_box, double h_fine, int64_t n,
                                                  int32_t nl, float *emis_lum, double *lum64)
{
    const int64_t tot = (int64_t)nl * n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i % n;
        const double side = (double)leaf_box[c].w * h_fine;
        const double v = 4.0 * kPi * j[i] * side * side * side;
        lum64[i] = v;
        emis_lum[i] = (float)v;
    }
}

// bit 0: some j not finite or negative
__global__ __launch_bounds__(256) void k_check_emis(const double *j, int64_t tot, uint32_t *bad)
{
    bool b = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < tot; i += (int64_t)gridDim.x * blockDim.x)
        b |= !(j[i] >= 0.0) || !isfinite(j[i]);
    if (__ballot(b) && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
}

__global__ void k_add_f64(double *a, const double *b, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] += b[i];
}

static unsigned sweep_blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

static int dust_args(const Grid &g, const dartray_dust_model *dm, DustArgs &D)
{
    if (!dm || !dm->lambda || !dm->dlambda) return fail(DARTRAY_E_INVALID, "dust model: null argument");
    if (!(dm->b0 > 0.0) || !std::isfinite(dm->b0) || !(dm->x0 > 0.0) || !std::isfinite(dm->x0) ||
        !(dm->t_max > 0.0) || !std::isfinite(dm->t_max))
        return fail(DARTRAY_E_INVALID, "dust model: b0, x0 and t_max must be finite and > 0");
    D = DustArgs{};
    D.rho = g.rho;
    D.leaf_box = g.leaf_box;
    D.h_fine = g.h_fine;
    D.n = g.n;
    D.nl = g.n_lambda;
    D.b0 = dm->b0;
    D.x0 = dm->x0;
    D.t_max = dm->t_max;
    for (int l = 0; l < g.n_lambda; ++l) {
        if (!(dm->lambda[l] > 0.0) || !std::isfinite(dm->lambda[l]) || !(dm->dlambda[l] > 0.0) ||
            !std::isfinite(dm->dlambda[l]))
            return fail(DARTRAY_E_INVALID, "dust model: band centres and widths must be finite and > 0");
        D.band[l].kabs = (double)g.lt.kappa[l] * (1.0 - (double)g.lt.albedo[l]);
        D.band[l].lam = dm->lambda[l];
        D.band[l].dlam = dm->dlambda[l];
    }
    return DARTRAY_OK;
}

// one emission update; with j_prev also dj and max dj / j_prev (*ratio, host)
static int dust_update(Grid &g, DustArgs D, double *ratio)
{
    int rc = fill<unsigned long long>(g, g.dust_word, 2, 0ull);
    if (rc) return rc;
    D.word = g.dust_word;
    hipLaunchKernelGGL(k_dust_emis, dim3(sweep_blocks(g.n)), dim3(256), 0, g.stream, D);
    DR_LAUNCH_CHECK("k_dust_emis");
    unsigned long long w[2] = {0, 0};
    DR_HIP(hipMemcpyAsync(w, g.dust_word, sizeof(w), hipMemcpyDeviceToHost, g.stream));
    DR_HIP(hipStreamSynchronize(g.stream));
    if (w[1]) return fail(DARTRAY_E_NUMERIC, "dust temperature above t_max");
    if (ratio) {
        double q;
        std::memcpy(&q, &w[0], sizeof(q));
        *ratio = q;
    }
    return DARTRAY_OK;
}

static void set_emis(Grid &g, const double *j)
{
    g.mirror_ok = false;
    hipLaunchKernelGGL(k_set_emis, dim3(sweep_blocks((int64_t)g.n_lambda * g.n)), dim3(256), 0, g.stream, j, g.leaf_box,
                       g.h_fine, g.n, g.n_lambda, g.emis_lum, g.lum64);
}

}  // namespace dr

extern "C" {

int dartray_absorbed(const dartray_grid *grid, const float *U, double *A)
{
    if (!grid || !U || !A) return fail(DARTRAY_E_INVALID, "null argument");
    const Grid &g = grid->g;
    hipLaunchKernelGGL(k_absorbed, dim3(sweep_blocks(g.n)), dim3(256), 0, g.stream, g.d_lt, g.rho, g.leaf_box, g.h_fine,
                       g.c_light, U, (const double *)nullptr, A, g.n);
    DR_LAUNCH_CHECK("k_absorbed");
    return DARTRAY_OK;
}

int dartray_dust_emission(dartray_grid *grid, const dartray_dust_model *dm, const double *A, double *T, double *j)
{
    if (!grid || !A || !T || !j) return fail(DARTRAY_E_INVALID, "null argument");
    Grid &g = grid->g;
    DustArgs D;
    int rc = dust_args(g, dm, D);
    if (rc) return rc;
    D.A = A;
    D.T = T;
    D.j = j;
    return dust_update(g, D, nullptr);
}

int dartray_grid_set_emis(dartray_grid *grid, const double *j)
{
    if (!grid || !j) return fail(DARTRAY_E_INVALID, "null argument");
    Grid &g = grid->g;
    const int64_t tot = (int64_t)g.n_lambda * g.n;
    int rc = fill<uint32_t>(g, g.w.err_word, 1, 0u);
    if (rc) return rc;
    hipLaunchKernelGGL(k_check_emis, dim3(sweep_blocks(tot)), dim3(256), 0, g.stream, j, tot, g.w.err_word);
    DR_LAUNCH_CHECK("k_check_emis");
    uint32_t bad = 0;
    DR_HIP(hipMemcpyAsync(&bad, g.w.err_word, sizeof(bad), hipMemcpyDeviceToHost, g.stream));
    DR_HIP(hipStreamSynchronize(g.stream));
    if (bad) return fail(DARTRAY_E_INVALID, "emission must be finite and >= 0");
    set_emis(g, j);
    DR_LAUNCH_CHECK("k_set_emis");
    return DARTRAY_OK;
}

int dartray_dust_selfheat(dartray_grid *grid, const dartray_trace_opts *opts, const dartray_selfheat_opts *so,
                          const dartray_dust_model *dm, const double *A_star, dartray_fields *fields, double *T,
                          double *j, double *j_traced, double *work, double *ratios, int32_t *n_rt)
{
    if (!grid || !opts || !so || !A_star || !fields || !T || !j || !j_traced || !work || !ratios || !n_rt)
        return fail(DARTRAY_E_INVALID, "null argument");
    Grid &g = grid->g;
    if (so->max_iter < 1 || so->max_iter > 1000) return fail(DARTRAY_E_INVALID, "max_iter must be 1..1000");
    if (so->n_scatter < 0) return fail(DARTRAY_E_INVALID, "n_scatter must be >= 0");
    if (!(so->conv > 0.0) || !std::isfinite(so->conv)) return fail(DARTRAY_E_INVALID, "conv must be finite and > 0");
    if (!(so->f_L >= 0.0) || !std::isfinite(so->f_L)) return fail(DARTRAY_E_INVALID, "f_L must be finite and >= 0");
    if (!fields->U || !fields->U_LL || !fields->S_total) return fail(DARTRAY_E_INVALID, "fields: U, U_LL and S_total required");
    DustArgs D;
    int rc = dust_args(g, dm, D);
    if (rc) return rc;
    dartray_trace_opts o = *opts;
    o.mode = DARTRAY_MODE_DIRECT;
    o.flags &= ~DARTRAY_FLAG_CONTINUE;
    if ((rc = check_opts(g, &o, fields, false))) return rc;
    *n_rt = 0;
    const int64_t n = g.n, nln = (int64_t)g.n_lambda * g.n;
    double *A = work, *dj = work + n;
    // the loop's energy density starts empty, and so does what it has traced
    if ((rc = fill<float>(g, fields->U, (size_t)nln, 0.f))) return rc;
    if ((rc = fill<double>(g, j_traced, (size_t)nln, 0.0))) return rc;
    // 1. emission from the stellar heating alone: dj = j (j_traced is zero)
    DR_HIP(hipMemcpyAsync(A, A_star, sizeof(double) * n, hipMemcpyDeviceToDevice, g.stream));
    D.A = A;
    D.T = T;
    D.j = j;
    D.j_prev = j_traced;
    D.dj = dj;
    double q = 0.0;
    if ((rc = dust_update(g, D, &q))) return rc;
    set_emis(g, dj);
    DR_LAUNCH_CHECK("k_set_emis");
    for (int it = 0; it < so->max_iter; ++it) {
        // 2 / 5. a dust RT calculation of dj
        o.flags = opts->flags & ~DARTRAY_FLAG_CONTINUE;
        if (it == 0 && o.adaptive) {
            if (so->step1) {
                o.mode = DARTRAY_MODE_STEP1;
                if ((rc = dartray_trace_direct(grid, &o, fields))) return rc;
            } else if ((rc = fill<float>(g, fields->U_LL, (size_t)nln, 0.f))) {
                return rc;
            }
        }
        // later calculations continue S_total; U_LL = U was left by the previous pass
        if (it > 0) o.flags |= DARTRAY_FLAG_CONTINUE;
        o.mode = DARTRAY_MODE_DIRECT;
        if ((rc = dartray_trace_direct(grid, &o, fields))) return rc;
        o.flags &= ~DARTRAY_FLAG_CONTINUE;
        for (int k = 0; k < so->n_scatter; ++k) {
            double rk = 0.0;
            if ((rc = dartray_scatter_iter(grid, &o, fields, so->f_L > 0.0 ? &rk : nullptr))) return rc;
            if (so->f_L > 0.0 && rk < so->f_L) break;
        }
        hipLaunchKernelGGL(k_add_f64, dim3(sweep_blocks(nln)), dim3(256), 0, g.stream, j_traced, (const double *)dj, nln);
        DR_LAUNCH_CHECK("k_add_f64");
        // 3. emission from the stellar plus the dust light absorbed; 4. dj
        hipLaunchKernelGGL(k_absorbed, dim3(sweep_blocks(n)), dim3(256), 0, g.stream, g.d_lt, g.rho, g.leaf_box,
                           g.h_fine, g.c_light, (const float *)fields->U, A_star, A, n);
        DR_LAUNCH_CHECK("k_absorbed");
        if ((rc = dust_update(g, D, &q))) return rc;
        ratios[it] = q;
        *n_rt = it + 1;
        // 6. converged at every cell and band
        if (q < so->conv) break;
        set_emis(g, dj);
        DR_LAUNCH_CHECK("k_set_emis");
    }
    return DARTRAY_OK;
}

}  // extern "C"
