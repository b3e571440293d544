// Internal declarations of the gfx950 ray-march library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstddef>
#include <string>
#include <vector>

#include "dartray.h"

namespace dr {

constexpr int kWave = 64;                 // CDNA wavefront width
constexpr int kMaxLambda = 64;            // wavelengths per grid
constexpr int kMaxDepthMerge = 3;         // split levels of adaptive trees with ray merging
constexpr int kMaxNsideWTable = 16;       // fixed-mode ray Nside with a tabulated phase table
constexpr int kMaxNsideCap = 1024;        // largest ray Nside of any table
constexpr int kMaxNsideSca = 8;           // largest Nside of the scattered source function
constexpr int kScaDirs = 1020;            // pixels of Nside 1, 2, 4 and 8 together
constexpr int kMaxDepthAdaptive = 12;     // split levels an adaptive ray tree may use
constexpr double kPi = 3.14159265358979323846;

// Per-wavelength constants used by every kernel (constant memory image).
struct LambdaTable {
    int32_t n_lambda;
    int32_t pad;
    float kappa[kMaxLambda];
    float albedo[kMaxLambda];
    float g[kMaxLambda];
    int32_t nside_sca[kMaxLambda];
    int32_t npix[kMaxLambda];
    int64_t s_off[kMaxLambda + 1];        // start of wavelength block l in S
    int32_t w_off[kMaxLambda + 1];        // start of wavelength l in a per-direction weight row
};

// One leaf, one 64-byte record: box in finest-level units, density,
// 1/(V c), and the six face-neighbour codes (index 2*axis + (direction > 0)):
// a leaf id (>= 0) when one leaf covers the same-size region across the face,
// -1 outside the root block, -(node + 2) when that region is subdivided.
struct alignas(64) LeafRec {
    int4 box;          // x, y, z lower corner, span
    float rho;
    float ivc;         // 1 / (V c)
    int32_t nb[6];
    int32_t level;
    int32_t pad[3];
};
static_assert(sizeof(LeafRec) == 64, "leaf record must be one 64-byte line");

// Per-pass work arrays (device): everything a fixed-ray direct pass writes
// besides the caller's fields and the handle's persistent state.
struct PassWork {
    double *U_k = nullptr;                // [n][nl] (wavelength fastest), FP64 accumulator of FP32 deposits
    int32_t *flags = nullptr;             // [n] source flags, then scan
    int32_t *src_list = nullptr;          // [n] compacted sources
    int32_t *scan_blocks = nullptr;       // block sums
    int32_t *n_src = nullptr;             // [1] sources the pass traces (after the source mask)
    int32_t *n_all = nullptr;             // [1] sources of the pass in the whole model (N_s of Eq. 11)
    uint32_t *err_word = nullptr;         // [1] device error word: bit 0 non-finite U or S
    double *dsum = nullptr;               // [4 * kMaxLambda] FP64 scratch sums
    double *esc64 = nullptr;              // [nl][12 * 16^2] FP64 escape by direction (fixed rays)
    float *ubar = nullptr;                // direction-binned energy density (fixed mode)
    size_t ubar_floats = 0;
};

struct Grid {
    // geometry
    int64_t n = 0;
    int32_t n_lambda = 0;
    int32_t nroot[3] = {0, 0, 0};
    int32_t max_level = 0;
    int32_t fine[3] = {0, 0, 0};          // finest-level cells per axis
    double lo[3] = {0, 0, 0};
    double root_size = 0;
    double h_fine = 0;                    // physical edge of a finest-level cell
    double c_light = 1;
    bool uniform = true;                  // no refinement anywhere
    bool linear = false;                  // uniform, leaf i at root position i (x fastest)
    int64_t n_internal = 0;
    LambdaTable lt{};
    int64_t s_size = 0;
    int32_t w_row = 0;                    // sum over wavelengths of npix

    hipStream_t stream = nullptr;
    int device = 0;                       // device current at creation (the stream's device)

    // device arrays owned by the handle
    int4 *leaf_box = nullptr;             // lower corner in fine units + span
    LeafRec *rec = nullptr;               // [n] leaf records
    float *rho = nullptr;
    float *inv_vc = nullptr;              // 1 / (V c)
    int32_t n_point = 0;                  // point sources: source index n + k
    double4 *ps_pos = nullptr;            // [n_point] positions, fine units
    double4 *ps_xyz = nullptr;            // [n_point] positions as given, model units
    int32_t *ps_cell = nullptr;           // [n_point] leaf holding each point
    float *ps_lum = nullptr;              // [nl][n_point] luminosity
    double *ps_lum64 = nullptr;           // [nl][n_point] luminosity, FP64
    float *emis_lum = nullptr;            // [nl][n] 4 pi j V
    double *lum64 = nullptr;              // [nl][n] 4 pi j V in FP64 (launch luminosity of the FP64-decision passes)
    int32_t *root_tab = nullptr;          // root cell -> node code
    int32_t *nodes = nullptr;             // [8 * n_internal] child codes
    int32_t *morton = nullptr;            // leaves in Morton order, then the point sources n .. n + n_point - 1
    int32_t *by_level = nullptr;          // leaves finest level first, Morton order within a level, then the point sources
    LambdaTable *d_lt = nullptr;

    // work arrays of a pass: `own` is what dartray_grid_create allocated,
    // `w` the set the pass functions use (own, except inside the entry point
    // that allocates nothing, which points w into its static scratch array)
    PassWork own{};
    PassWork w{};
    float *ull_t = nullptr;               // [n][nl] copy of U_LL for the march
    uint8_t *cell_flag = nullptr;         // [n] scattering-pass source flags by cell
    double *s1_sum = nullptr;             // [kMaxLambda] sum of S after the direct pass
    bool have_s1 = false;
    // direction tables: entry 4 (N^2 - 1) + pix holds nested pixel pix at
    // Nside N, for N = 1, 2, 4, ... nside_cap, rotated by the current frame
    int32_t nside_cap = 64;
    int64_t ndir_all = 0;
    float4 *dir_all = nullptr;
    double4 *dir64 = nullptr;             // the same directions in FP64
    float *invz = nullptr;                // [entry][n_lambda] 1 / sum_p Phi(n_p . n)
    double *sca64 = nullptr;              // FP64 scattered-light pixel directions, first kScaDirs entries
    double dirs_frame[9] = {0};
    bool dirs_valid = false;
    bool invz_valid = false;
    float *wtab = nullptr;                // fixed-mode phase weights [r][w_row]
    int32_t wtab_nside = 0;
    bool wtab_valid = false;
    unsigned long long *queue = nullptr;  // work counter of the adaptive march
    unsigned long long *dust_word = nullptr;  // [2] dust emission: max dj / j_prev (FP64 bits), bracket overflow
    // 2D mode (mirror symmetry through the block centre), built on first use
    bool mirror_geo = false;              // leaf and pixel mirror tables built
    bool mirror_ok = false;               // density and emission checked symmetric since the last change
    int32_t *mir = nullptr;               // [n][8] mirror image M (bits x, y, z) of each leaf
    uint8_t *first = nullptr;             // [n] 1 for the leaves of the first octant
    int32_t *reps = nullptr;              // [n / 8] the first-octant leaves
    int64_t n_reps = 0;
    int32_t *pmir = nullptr;              // [direction entry][8] mirror images of the HEALPix pixels, Nside <= 16
    double *esc_tmp = nullptr;            // [nl][12 * 16^2] escape by direction before folding

    // deposit log of the adaptive passes that scatter light: one tuple
    // (cell and direction entry as one key, per-wavelength energy-density
    // deposit) per depositing crossing, radix-sorted by (cell, direction) and
    // expanded per cell, once per run of one direction
    int64_t log_cap = 0;
    uint64_t *log_key = nullptr, *log_key2 = nullptr;   // (cell << dir_bits) | direction entry
    uint32_t *log_idx = nullptr, *log_idx2 = nullptr;
    float *log_du = nullptr;              // [nl][log_cap]
    unsigned long long *log_count = nullptr;
    void *sort_tmp = nullptr;
    size_t sort_tmp_bytes = 0;
    int32_t key_bits = 1;                 // bits of the sort key
    int32_t dir_bits = 1;                 // bits of a direction entry
    int64_t log_chunks = 0;               // launches of the last adaptive pass


    // adjoint work arrays
    double *rho_bar = nullptr;            // [n] FP64 accumulator of dJ/drho
    float *sbar[2] = {nullptr, nullptr};  // [s_size] dJ/dS of consecutive orders

    size_t bytes = 0;
    dartray_tuning tune{};                // fixed-ray launch parameters (zero = default)

    // march-kernel timing
    int32_t prof = 0;                     // DARTRAY_PROF_* mask
    int32_t prof_kind = 0;                // kind of the launch being marked
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
};

// error handling
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

}  // namespace dr

struct dartray_grid {
    dr::Grid g;
};

// ---------------------------------------------------------------------------
// HEALPix nested pixel centres (Gorski et al. 2005), device and host.
// ---------------------------------------------------------------------------

__host__ __device__ inline uint32_t dr_compact_bits(uint64_t v)
{
    // gather the even bits of v into the low half
    v &= 0x5555555555555555ull;
    v = (v | (v >> 1)) & 0x3333333333333333ull;
    v = (v | (v >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v >> 4)) & 0x00FF00FF00FF00FFull;
    v = (v | (v >> 8)) & 0x0000FFFF0000FFFFull;
    v = (v | (v >> 16)) & 0x00000000FFFFFFFFull;
    return (uint32_t)v;
}

// Centre of nested pixel `pix` at resolution `nside`: z, and the longitude
// as the fraction num / den of a quarter turn.
__host__ __device__ inline void dr_pix_zq(int64_t nside, int64_t pix, double *z_out, int64_t *num, int64_t *den)
{
    // base pixels are numbered 0..11: four around the north pole, four on
    // the equator, four around the south pole
    const int64_t npf = nside * nside;
    const int face = (int)(pix / npf);
    const uint64_t in_face = (uint64_t)(pix - (int64_t)face * npf);
    const int64_t x = dr_compact_bits(in_face);
    const int64_t y = dr_compact_bits(in_face >> 1);
    const int row = face >> 2;                       // 0 north, 1 equator, 2 south
    const int col = face & 3;
    // ring index counted from the north pole: the face's south vertex lies on
    // ring (row + 2) * nside
    const int64_t ring = (int64_t)(row + 2) * nside - x - y - 1;
    int64_t q;                                       // pixels per quarter ring
    double z;
    int64_t half_shift;                              // 1 when the ring starts half a pixel later
    if (ring < nside) {
        q = ring;
        z = 1.0 - (double)(q * q) / (3.0 * (double)npf);
        half_shift = 0;
    } else if (ring > 3 * nside) {
        q = 4 * nside - ring;
        z = (double)(q * q) / (3.0 * (double)npf) - 1.0;
        half_shift = 0;
    } else {
        q = nside;
        z = 2.0 * (double)(2 * nside - ring) / (3.0 * (double)nside);
        half_shift = (ring - nside) & 1;
    }
    // longitude of the face centre in units of half a quarter-ring pixel
    const int64_t face_phi = (row == 1) ? 2 * col : 2 * col + 1;
    int64_t j = (face_phi * q + x - y + 1 + half_shift) / 2;   // 1-based position in the ring
    if (j > 4 * q) j -= 4 * q;
    if (j < 1) j += 4 * q;
    *z_out = z;
    *num = 2 * j - 1 - half_shift;                   // phi = (pi / 2) num / den
    *den = 2 * q;
}

// Unit vector of nested pixel `pix`, rotated by R.  cos and sin of the
// longitude come from the angle to the nearest axis of its quarter turn, so
// that reflecting the direction across the x, y or z plane gives exactly the
// vector of the reflected pixel (the unrotated direction set is then
// mirror symmetric bit for bit).
__host__ __device__ inline void dr_pix_vec(int64_t nside, int64_t pix, const double *R, double v[3])
{
    double z;
    int64_t num, den;
    dr_pix_zq(nside, pix, &z, &num, &den);
    const int64_t quarter = num / den, m = num - quarter * den;
    double c, s;
    if (2 * m < den) {
        const double t = (0.5 * dr::kPi) * (double)m / (double)den;
        c = cos(t);
        s = sin(t);
    } else if (2 * m > den) {
        const double t = (0.5 * dr::kPi) * (double)(den - m) / (double)den;
        c = sin(t);
        s = cos(t);
    } else {
        c = s = sqrt(0.5);
    }
    const double st = sqrt((1.0 - z) * (1.0 + z));
    const double cx = quarter == 0 ? c : quarter == 1 ? -s : quarter == 2 ? -c : s;
    const double cy = quarter == 0 ? s : quarter == 1 ? c : quarter == 2 ? -s : -c;
    const double a[3] = {st * cx, st * cy, z};
    for (int i = 0; i < 3; ++i) v[i] = R[3 * i] * a[0] + R[3 * i + 1] * a[1] + R[3 * i + 2] * a[2];
}

__host__ __device__ inline uint64_t dr_spread_bits(uint32_t v)
{
    // put bit k of v at bit 2k
    uint64_t x = v;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

// Nested pixel at resolution `nside` that contains direction v (any length).
// Between |z| = 2/3 the pixel boundaries are the lines of constant
// phi / (pi/2) + 3z/4 and phi / (pi/2) - 3z/4 (in units of 1/nside), whose
// integer parts give the base pixel and the in-face indices; in the polar
// caps they are the lines of constant (phi / (pi/2) - q) sqrt(3 (1 - |z|))
// and (1 - phi / (pi/2) + q) sqrt(3 (1 - |z|)) within quarter q.
__host__ __device__ inline int64_t dr_vec_pix(int64_t nside, const double v[3])
{
    const double len = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const double z = v[2] / len;
    double phi = atan2(v[1], v[0]);
    if (phi < 0.0) phi += 2.0 * dr::kPi;
    double u = phi * (2.0 / dr::kPi);                 // longitude in quarter turns, [0, 4)
    if (u >= 4.0) u -= 4.0;
    const double N = (double)nside;
    int64_t face, x, y;
    if (z <= 2.0 / 3.0 && z >= -2.0 / 3.0) {
        const int64_t up = (int64_t)floor(N * (0.5 + u) - 0.75 * N * z);    // ascending boundary index
        const int64_t down = (int64_t)floor(N * (0.5 + u) + 0.75 * N * z);  // descending boundary index
        const int64_t fu = up / nside, fd = down / nside;
        face = fu == fd ? 4 + (fu & 3) : (fu < fd ? (fu & 3) : 8 + (fd & 3));
        x = down - fd * nside;
        y = nside - 1 - (up - fu * nside);
    } else {
        int64_t q = (int64_t)floor(u);
        if (q > 3) q = 3;
        const double frac = u - (double)q;
        const double s = N * sqrt(3.0 * (1.0 - fabs(z)));
        int64_t a = (int64_t)floor(frac * s), b = (int64_t)floor((1.0 - frac) * s);
        if (a > nside - 1) a = nside - 1;
        if (b > nside - 1) b = nside - 1;
        if (z > 0.0) {
            face = q;
            x = nside - 1 - b;
            y = nside - 1 - a;
        } else {
            face = 8 + q;
            x = a;
            y = b;
        }
    }
    return face * nside * nside + (int64_t)(dr_spread_bits((uint32_t)x) | (dr_spread_bits((uint32_t)y) << 1));
}
