/*
 * FP64 reference ("oracle") for the ray-march of DART-Ray V2
 * (Natale et al. 2017, "Ray-tracing 3D dust radiative transfer with DART-Ray:
 * code upgrade and public release", arXiv:1709.03802).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the package smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or constant with the GPU library, and is deliberately plain:
 * one ray at a time, one crossing at a time, every deposit written out, in
 * double precision.
 *
 * What it computes (paper Sect. 2): for every radiation source (an emitting
 * cell, or a dusty cell holding scattered luminosity) rays are cast along the
 * HEALPix directions (Sect. 3.1.1, Gorski et al. 2005) from the cell centre.
 * Each ray-cell crossing attenuates the ray, adds to the radiation-field
 * energy density U of the crossed cell and adds the scattered part of the
 * extinguished luminosity to that cell's angular scattered-luminosity array
 * through the Henyey-Greenstein phase function (Eq. 4).  Rays may be split
 * when the beam is too large (Eq. 2) and blocked when their contribution is
 * negligible (Eq. 1, with the source-contribution estimate of Eq. 8); during
 * step 1 the block test is replaced by the fixed extent R_pre (caption of the
 * ray-density flowchart figure).  Multi-wavelength rays are blocked only when
 * negligible at every wavelength and skip deposits at negligible wavelengths
 * (Sect. 3.2).  With N_rays^max set, rays whose beam is too small for the
 * crossed cell pause in a low list and four siblings merge (Eq. 3).  Observer
 * maps, point sources (Sect. 2, Sect. 3.6) and the dust emission of the
 * self-heating loop (Sect. 3.3) close the file.
 *
 * Readings where the paper is silent (each one also listed in the design
 * notes of the repository):
 *  - rays start at the source-cell centre and the source cell is crossed from
 *    the centre to its exit like any other cell;
 *  - the per-ray luminosity is L_s / N_ray (direct) and, for scattered light,
 *    the luminosity held in the j_sca pixel that contains the ray direction,
 *    shared evenly among the rays inside that pixel;
 *  - the energy-density deposit of one crossing is ext / (alpha V c), where
 *    ext = L_in (1 - exp(-tau)), which equals the per-ray expression
 *    <I> A_EM Omega_HP dL / (V c) of Sect. 3.5 with <I> the path-averaged
 *    intensity;
 *  - the scattered luminosity of a crossing is albedo * ext, spread over the
 *    j_sca pixels with weights Phi(n_p . n) / sum_q Phi(n_q . n);
 *  - the estimate of Eq. 8 becomes <L> / (Omega_HP d^2 c), with d the
 *    distance from the source to the crossed cell centre and
 *    Omega_INT = L_c^2 / d^2 (infinite in the source's own cell);
 *  - a wavelength is significant when its path-averaged luminosity is > 0 and
 *    that estimate is >= f_U * U_LL;
 *  - a ray is split (4 children, each with a quarter of its luminosity,
 *    starting at the entry distance of the triggering crossing) when the beam
 *    is too large and the ray is significant at some wavelength, blocked when
 *    the beam is too large and no wavelength is significant, and otherwise
 *    deposits the significant wavelengths and carries on;
 *  - traversal: the exit face is the axis with the smallest exit distance
 *    (exact ties resolved x before y before z) and the next leaf is the face
 *    neighbour across it that contains the exit point (points on a face
 *    belong to the side the direction points to; a ray lying in the face
 *    plane, with a zero component, takes the side away from the block's
 *    central plane, which keeps mirror-image rays on mirror-image cells, and
 *    the upper side on the central plane itself); a ray through an edge or
 *    corner therefore crosses zero-length segments;
 *  - a segment whose length is zero up to the rounding of its two end
 *    distances -- no longer than 2^-46 of its exit distance, some 32 to 64
 *    units in the last place of an FP64 distance -- is an edge or corner
 *    graze: a ray through an edge or corner of a cell crosses it with zero
 *    length in exact arithmetic, and the paper is silent on such crossings.
 *    A graze deposits nothing, counts as no crossing and takes no split or
 *    block decision; the ray's distance is not advanced, so the rounding
 *    residue folds into the next segment.  The forward passes and the
 *    adjoint walk rays with this same rule (orc_is_graze);
 *  - ray merging (Eq. 3 and the text after it): a ray below the launch
 *    resolution, outside its source's cell, whose beam is smaller than
 *    Omega_INT / N_rays^max pauses before the crossing (nothing deposited);
 *    the four children of one split that all pause having crossed the same
 *    grid plane merge into one ray in the parent pixel carrying the sum of
 *    their luminosities (the average intensity of a four times wider beam)
 *    from the mean of their distances, and the parent's walk continues with
 *    it; paused children of a group that does not merge continue from where
 *    they stopped and no longer pause.  Merging never goes below the launch
 *    Nside, and N_rays^max >= 4 N_rays so that a merged beam is not at once
 *    too large;
 *  - outputs beyond the paper: the luminosity a ray carries out of the root
 *    block, by the launch pixel it descends from, and the adjoint of
 *    fixed-ray passes (orc_adjoint_pass).
 *
 * Pins (CPU tests), by function:
 *  - orc_healpix_vec: ring closed forms of Gorski et al. (z and phi per ring),
 *    an independently written ang2pix (children inside their parent), the
 *    symmetry of the pixel set;
 *  - orc_hg, orc_hg_fwhm, orc_k_hp: normalisation over the sphere by
 *    quadrature, the g = 0 limit, the FWHM against its closed form, and the
 *    Eq. 5 resolution putting between 3 and 30 pixel centres inside the FWHM
 *    around any direction (Sect. 3.1.2: several points sample the peak);
 *  - orc_step, orc_trace_cells, orc_crossings, orc_is_graze: brute-force slab
 *    intersection on uniform grids and random octrees; a segment 1e-9 of a
 *    cell long is a crossing; graze lengths fold so that crossings add up to
 *    the chord;
 *  - orc_run_pass, fixed rays: exp(-tau) through a cube and a layered slab,
 *    the thin-medium sum U V c = sum L d, the 1/(4 pi r^2 c) field, exact
 *    luminosity balance, albedo and g limits, symmetry, additivity,
 *    linearity, escape by direction, the launch rule when rays are coarser
 *    than the j_sca pixels;
 *  - orc_run_pass, adaptive rays (orc_follow): hand-built rows of cells where
 *    Eq. 2 must split at a known crossing or must not, the Nside scaling of
 *    the beam, the Eq. 8 estimate a part in 1e9 above and below the threshold,
 *    blocking only when insignificant at every wavelength, brute force of all
 *    rays and their children, luminosity balance with cut and skipped terms,
 *    the fixed-ray limit, every ray ending once, the step-1 extent, and Eq. 11
 *    (N_s counted independently; the a_RT 0.05 / 0.005 property of Sect. 5);
 *  - orc_split (merging): brute force of every ray of a source on an octree
 *    where rays split and merge (U, S, counts), no pauses reproducing the
 *    unmerged run, balance and every ray ending once with merges, 2D mode
 *    equal to 3D with merging;
 *  - 2D mode (orc_mirror_tables): mirror-exact pixel vectors, 3D passes of
 *    symmetric models symmetric, 2D passes equal to 3D passes;
 *  - orc_adjoint_pass: central differences on every cell (also in a frame
 *    with near-ties), a dot-product test, zero gradient at the target;
 *  - orc_healpix_pix, orc_observe: an independent ang2pix and the round trip
 *    through pixel centres; transparent images integrating to the luminosity,
 *    a face-on slab as a geometric series, the inverse-square all-sky map,
 *    scattered light seen only inside its pixel;
 *  - point sources: a point at a cell centre is that emitting cell, escape
 *    and path sums in a transparent medium, balance, Eq. 11 counts, a point
 *    seen by an observer, the adjoint against central differences;
 *  - orc_absorbed, orc_dust_power, orc_dust_emission: the absorbed tally of
 *    the march, the one-band closed-form temperature, emission equal to
 *    absorption in every cell; the self-heating loop (Python side) by energy
 *    conservation over its updates, linearity of the incremental processing,
 *    the transparent limit and warming only.
 */

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_E_INVALID (-1)
#define ORC_E_OOM (-2)

enum { ORC_STEP1 = 0, ORC_DIRECT = 1, ORC_SCATTER = 2 };
enum { T_EMITTED = 0, T_ABSORBED, T_SCATTERED, T_ESCAPED, T_CUT, T_SKIPPED, N_TALLY = 8 };
enum { C_CROSS = 0, C_RAYS, C_SPLITS, C_CUTS, C_ESCAPES, C_DEPOSITS, C_SKIPS, C_MAXSTEP, C_MERGES, N_COUNT = 16 };

typedef struct {
    int32_t nroot[3];
    double lo[3];
    double root_size;
    int64_t n_leaves;
    const int32_t *level;   /* [n] */
    const int64_t *ijk;     /* [n][3] cell coordinates at the leaf's level */
    const double *rho;      /* [n] */
    const double *emis;     /* [n_lambda][n] */
    int32_t n_lambda;
    const double *kappa;    /* [n_lambda] */
    const double *albedo;   /* [n_lambda] */
    const double *g;        /* [n_lambda] */
    const int32_t *nside_sca; /* [n_lambda], 0 selects Eq. 5 */
    double n_fwhm;
    int32_t k_max;
    double c_light;
    int64_t n_point;        /* point sources (Sect. 3.6) */
    const double *point_pos; /* [n_point][3] positions inside the root block */
    const double *point_lum; /* [n_lambda][n_point] luminosity */
} orc_grid_desc;

typedef struct {
    orc_grid_desc d;
    int max_level;
    int64_t fine[3];        /* finest-level cells along each axis */
    double h_fine;
    int32_t *fine_map;      /* finest-level cell -> leaf */
    double *centre;         /* [n][3] */
    double *side;           /* [n] */
    int32_t *nside_sca;     /* [n_lambda] effective */
    int64_t *s_offset;      /* [n_lambda + 1] start of each wavelength block of S */
    int64_t *point_cell;    /* [n_point] leaf holding each point source */
} orc_model;

typedef struct {
    int32_t mode;           /* ORC_STEP1, ORC_DIRECT, ORC_SCATTER */
    int32_t adaptive;       /* 0: fixed Nside, 1: split/block rays */
    int32_t nside;          /* fixed Nside, or the initial Nside */
    int32_t nside_max;
    double n_rays_min;      /* N_rays of Eq. 2 */
    double f_U;             /* Eq. 1 */
    double r_pre;           /* step-1 extent */
    double frame[9];        /* rotation applied to every HEALPix direction */
    const uint8_t *source_mask; /* [n] or NULL */
    int64_t max_steps;      /* per ray, crossings of positive length; <= 0 means unlimited */
    int32_t n_threads;
    double a_RT;            /* accuracy parameter of Eq. 11, used when f_U < 0 */
    int32_t mode_2d;        /* 2D mode (Sect. 3.6): first-octant sources, deposits mirrored */
    double n_rays_max;      /* N_rays^max of Eq. 3 (ray merging); 0: no merging */
} orc_pass_opts;

/* ------------------------------------------------------------------------ */
/* HEALPix, nested scheme (Gorski et al. 2005, Sect. 4-5 of that paper).      */
/* ------------------------------------------------------------------------ */

/* Base-pixel layout: ring index of the base pixel's southern-most corner
 * row (in units of Nside) and its longitude offset, for faces 0..11. */
static const int orc_face_ring[12] = {2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4};
static const int orc_face_phi[12] = {1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7};

static void orc_deinterleave(int64_t v, int64_t *x, int64_t *y)
{
    int64_t a = 0, b = 0;
    for (int bit = 0; bit < 31; ++bit) {
        a |= ((v >> (2 * bit)) & 1) << bit;
        b |= ((v >> (2 * bit + 1)) & 1) << bit;
    }
    *x = a;
    *y = b;
}

/* Unit vector of the centre of nested pixel `pix` at resolution `nside`. */
void orc_healpix_vec(int64_t nside, int64_t pix, double v[3])
{
    int64_t npface = nside * nside;
    int face = (int)(pix / npface);
    int64_t ix, iy;
    orc_deinterleave(pix % npface, &ix, &iy);
    /* ring number counted from the north pole, 1 .. 4 nside - 1 */
    int64_t ring = (int64_t)orc_face_ring[face] * nside - ix - iy - 1;
    int64_t nr;           /* pixels in a quarter of this ring */
    double z;
    int shifted;          /* ring whose first pixel centre is offset by half a pixel less */
    if (ring < nside) {                       /* north polar cap */
        nr = ring;
        z = 1.0 - (double)(nr * nr) / (3.0 * (double)npface);
        shifted = 0;
    } else if (ring > 3 * nside) {            /* south polar cap */
        nr = 4 * nside - ring;
        z = -(1.0 - (double)(nr * nr) / (3.0 * (double)npface));
        shifted = 0;
    } else {                                  /* equatorial belt */
        nr = nside;
        z = (double)(2 * nside - ring) * 2.0 / (3.0 * (double)nside);
        shifted = (int)((ring - nside) & 1);
    }
    int64_t jp = ((int64_t)orc_face_phi[face] * nr + ix - iy + 1 + shifted) / 2;
    if (jp > 4 * nr) jp -= 4 * nr;
    if (jp < 1) jp += 4 * nr;
    /* phi = (pi / 2) num / den: quarter turn q, and the angle m / den of a
     * quarter turn within it.  cos and sin come from the angle measured from
     * the nearer axis, so that the mirror images of a pixel (x, y or z
     * reflected) give exactly the mirrored vector: a mirror-symmetric model
     * then casts mirror-symmetric rays. */
    int64_t num = 2 * jp - 1 - shifted, den = 2 * nr;
    int64_t q = num / den, m = num - q * den;
    double a, b;
    if (2 * m < den) {
        double t = (M_PI / 2.0) * (double)m / (double)den;
        a = cos(t);
        b = sin(t);
    } else if (2 * m > den) {
        double u = (M_PI / 2.0) * (double)(den - m) / (double)den;
        a = sin(u);
        b = cos(u);
    } else {
        a = b = sqrt(0.5);
    }
    double st = sqrt((1.0 - z) * (1.0 + z));
    double x = q == 0 ? a : q == 1 ? -b : q == 2 ? -a : b;
    double y = q == 0 ? b : q == 1 ? a : q == 2 ? -b : -a;
    v[0] = st * x;
    v[1] = st * y;
    v[2] = z;
}

/* Nested pixel at `nside` containing the direction v (need not be unit
 * length), following the construction of Gorski et al. 2005: the
 * equatorial belt (|z| <= 2/3) is cut by the two families of lines
 * phi / (pi / 2) -+ (3/4) z = const, which give the face and the in-face
 * coordinates; the polar caps by the lines of constant (1 - |z|) phi within
 * each quarter. */
int64_t orc_healpix_pix(int64_t nside, const double v[3])
{
    double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double z = v[2] / r;
    double phi = atan2(v[1], v[0]);
    if (phi < 0.0) phi += 2.0 * M_PI;
    double tt = phi / (0.5 * M_PI);             /* in [0, 4] */
    if (tt >= 4.0) tt -= 4.0;
    int64_t face, ix, iy;
    if (fabs(z) <= 2.0 / 3.0) {
        double a = (double)nside * (0.5 + tt), b = 0.75 * (double)nside * z;
        int64_t jp = (int64_t)floor(a - b);     /* index of the ascending edge line */
        int64_t jm = (int64_t)floor(a + b);     /* index of the descending edge line */
        int64_t fp = jp / nside, fm = jm / nside;
        if (fp == fm) face = (fp % 4) + 4;      /* an equatorial face */
        else if (fp < fm) face = fp % 4;        /* a northern face */
        else face = (fm % 4) + 8;               /* a southern face */
        ix = jm % nside;
        iy = nside - 1 - (jp % nside);
    } else {
        int64_t q = (int64_t)floor(tt);
        if (q > 3) q = 3;
        double tp = tt - (double)q;
        double w = (double)nside * sqrt(3.0 * (1.0 - fabs(z)));
        int64_t jp = (int64_t)floor(tp * w), jm = (int64_t)floor((1.0 - tp) * w);
        if (jp > nside - 1) jp = nside - 1;
        if (jm > nside - 1) jm = nside - 1;
        if (z > 0.0) {
            face = q;
            ix = nside - 1 - jm;
            iy = nside - 1 - jp;
        } else {
            face = q + 8;
            ix = jp;
            iy = jm;
        }
    }
    int64_t sub = 0;
    for (int bit = 0; bit < 31; ++bit) {
        sub |= ((ix >> bit) & 1) << (2 * bit);
        sub |= ((iy >> bit) & 1) << (2 * bit + 1);
    }
    return face * nside * nside + sub;
}

static void orc_rotate(const double R[9], const double a[3], double b[3])
{
    b[0] = R[0] * a[0] + R[1] * a[1] + R[2] * a[2];
    b[1] = R[3] * a[0] + R[4] * a[1] + R[5] * a[2];
    b[2] = R[6] * a[0] + R[7] * a[1] + R[8] * a[2];
}

/* ------------------------------------------------------------------------ */
/* Henyey-Greenstein phase function (Eq. 4) and the j_sca resolution rule     */
/* (Eq. 5 with theta_min = FWHM[Phi - Phi(pi)] / n_FWHM).                    */
/* ------------------------------------------------------------------------ */

double orc_hg(double g, double cos_theta)
{
    double den = 1.0 + g * g - 2.0 * g * cos_theta;
    return (1.0 - g * g) / (4.0 * M_PI * den * sqrt(den));
}

/* Full width at half maximum of Phi(theta) - Phi(pi), in radians.
 * Zero when the profile has no forward peak (g <= 0). */
double orc_hg_fwhm(double g)
{
    if (g <= 0.0) return 0.0;
    double top = orc_hg(g, 1.0) - orc_hg(g, -1.0);
    double a = 0.0, b = M_PI;   /* Phi is decreasing in theta for g > 0 */
    for (int it = 0; it < 200; ++it) {
        double m = 0.5 * (a + b);
        double f = orc_hg(g, cos(m)) - orc_hg(g, -1.0) - 0.5 * top;
        if (f > 0.0) a = m; else b = m;
    }
    return 2.0 * 0.5 * (a + b);
}

/* Real-valued k of Eq. 5 (before taking the integer part). */
double orc_k_hp_real(double g, double n_fwhm)
{
    double fwhm = orc_hg_fwhm(g);
    if (fwhm <= 0.0) return 0.0;
    double tmin = fwhm / n_fwhm;
    return 0.5 * log2(4.0 * M_PI / (12.0 * tmin * tmin));
}

/* Integer k of Eq. 5: integer part, clamped to [0, k_max]. */
int orc_k_hp(double g, double n_fwhm, int k_max)
{
    double k = floor(orc_k_hp_real(g, n_fwhm));
    if (k < 0.0) k = 0.0;
    if (k > (double)k_max) k = (double)k_max;
    return (int)k;
}

/* Weights w(p | n) = Phi(n_p . n) / sum_q Phi(n_q . n) over `npix` j_sca
 * pixels whose (rotated) centre vectors are pv[3p..3p+2]. */
static void orc_hg_weights_tab(int64_t npix, const double *pv, double g, const double n[3], double *w)
{
    double sum = 0.0;
    for (int64_t p = 0; p < npix; ++p) {
        w[p] = orc_hg(g, pv[3 * p] * n[0] + pv[3 * p + 1] * n[1] + pv[3 * p + 2] * n[2]);
        sum += w[p];
    }
    for (int64_t p = 0; p < npix; ++p) w[p] /= sum;
}

/* Rotated centre vectors of the nested pixels at `nside`: out[3p..3p+2]. */
static void orc_pixel_table(int64_t nside, const double frame[9], double *out)
{
    for (int64_t p = 0; p < 12 * nside * nside; ++p) {
        double v0[3];
        orc_healpix_vec(nside, p, v0);
        orc_rotate(frame, v0, out + 3 * p);
    }
}

/* Weights w(p | n) over the j_sca pixels at `nside_sca`, pixel centres
 * rotated by `frame`. */
void orc_hg_weights(int nside_sca, double g, const double n[3], const double frame[9], double *w)
{
    int64_t npix = 12 * (int64_t)nside_sca * nside_sca;
    double *pv = (double *)malloc(sizeof(double) * 3 * (size_t)npix);
    if (!pv) return;
    orc_pixel_table(nside_sca, frame, pv);
    orc_hg_weights_tab(npix, pv, g, n, w);
    free(pv);
}

/* ------------------------------------------------------------------------ */
/* Grid model                                                                */
/* ------------------------------------------------------------------------ */

void orc_model_destroy(orc_model *m)
{
    if (!m) return;
    free(m->fine_map);
    free(m->centre);
    free(m->side);
    free(m->nside_sca);
    free(m->s_offset);
    free(m->point_cell);
    free(m);
}

static int is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int64_t orc_locate(const orc_model *m, const double p[3], const double d[3]);

int orc_model_create(const orc_grid_desc *d, orc_model **out)
{
    *out = NULL;
    if (d->n_leaves <= 0 || d->n_lambda <= 0 || d->root_size <= 0.0 || d->c_light <= 0.0) return ORC_E_INVALID;
    for (int a = 0; a < 3; ++a) if (d->nroot[a] <= 0) return ORC_E_INVALID;
    orc_model *m = (orc_model *)calloc(1, sizeof(orc_model));
    if (!m) return ORC_E_OOM;
    m->d = *d;
    int lmax = 0;
    for (int64_t i = 0; i < d->n_leaves; ++i) {
        if (d->level[i] < 0 || d->level[i] > 20) { orc_model_destroy(m); return ORC_E_INVALID; }
        if (d->level[i] > lmax) lmax = d->level[i];
    }
    m->max_level = lmax;
    for (int a = 0; a < 3; ++a) m->fine[a] = (int64_t)d->nroot[a] << lmax;
    m->h_fine = d->root_size / (double)((int64_t)1 << lmax);
    int64_t nfine = m->fine[0] * m->fine[1] * m->fine[2];
    m->fine_map = (int32_t *)malloc(sizeof(int32_t) * (size_t)nfine);
    m->centre = (double *)malloc(sizeof(double) * 3 * (size_t)d->n_leaves);
    m->side = (double *)malloc(sizeof(double) * (size_t)d->n_leaves);
    m->nside_sca = (int32_t *)malloc(sizeof(int32_t) * (size_t)d->n_lambda);
    m->s_offset = (int64_t *)malloc(sizeof(int64_t) * (size_t)(d->n_lambda + 1));
    if (!m->fine_map || !m->centre || !m->side || !m->nside_sca || !m->s_offset) { orc_model_destroy(m); return ORC_E_OOM; }
    for (int64_t f = 0; f < nfine; ++f) m->fine_map[f] = -1;
    /* every finest-level cell must belong to exactly one leaf */
    for (int64_t i = 0; i < d->n_leaves; ++i) {
        int lv = d->level[i];
        int64_t span = (int64_t)1 << (lmax - lv);
        double side = d->root_size / (double)((int64_t)1 << lv);
        m->side[i] = side;
        for (int a = 0; a < 3; ++a) {
            int64_t c = d->ijk[3 * i + a];
            if (c < 0 || (c + 1) * span > m->fine[a]) { orc_model_destroy(m); return ORC_E_INVALID; }
            m->centre[3 * i + a] = d->lo[a] + ((double)c + 0.5) * side;
        }
        if (!(d->rho[i] >= 0.0) || !isfinite(d->rho[i])) { orc_model_destroy(m); return ORC_E_INVALID; }
        for (int l = 0; l < d->n_lambda; ++l) {
            double e = d->emis[(int64_t)l * d->n_leaves + i];
            if (!(e >= 0.0) || !isfinite(e)) { orc_model_destroy(m); return ORC_E_INVALID; }
        }
        int64_t x0 = d->ijk[3 * i] * span, y0 = d->ijk[3 * i + 1] * span, z0 = d->ijk[3 * i + 2] * span;
        for (int64_t z = z0; z < z0 + span; ++z)
            for (int64_t y = y0; y < y0 + span; ++y)
                for (int64_t x = x0; x < x0 + span; ++x) {
                    int64_t f = (z * m->fine[1] + y) * m->fine[0] + x;
                    if (m->fine_map[f] != -1) { orc_model_destroy(m); return ORC_E_INVALID; }
                    m->fine_map[f] = (int32_t)i;
                }
    }
    for (int64_t f = 0; f < nfine; ++f)
        if (m->fine_map[f] < 0) { orc_model_destroy(m); return ORC_E_INVALID; }
    m->s_offset[0] = 0;
    for (int l = 0; l < d->n_lambda; ++l) {
        int ns = d->nside_sca[l];
        if (ns == 0) ns = 1 << orc_k_hp(d->g[l], d->n_fwhm, d->k_max);
        if (!is_pow2(ns) || !(d->kappa[l] >= 0.0) || !(d->albedo[l] >= 0.0 && d->albedo[l] <= 1.0) ||
            !(d->g[l] > -1.0 && d->g[l] < 1.0)) { orc_model_destroy(m); return ORC_E_INVALID; }
        m->nside_sca[l] = ns;
        m->s_offset[l + 1] = m->s_offset[l] + d->n_leaves * 12 * (int64_t)ns * ns;
    }
    /* point sources: inside the root block, finite non-negative luminosity;
     * each belongs to the leaf holding it (a point on a face to the upper side) */
    if (d->n_point < 0 || (d->n_point > 0 && (!d->point_pos || !d->point_lum))) { orc_model_destroy(m); return ORC_E_INVALID; }
    m->point_cell = (int64_t *)malloc(sizeof(int64_t) * (size_t)(d->n_point > 0 ? d->n_point : 1));
    if (!m->point_cell) { orc_model_destroy(m); return ORC_E_OOM; }
    for (int64_t k = 0; k < d->n_point; ++k) {
        const double up[3] = {1.0, 1.0, 1.0};   /* a point on a face belongs to the upper side */
        for (int l = 0; l < d->n_lambda; ++l) {
            double v = d->point_lum[(int64_t)l * d->n_point + k];
            if (!(v >= 0.0) || !isfinite(v)) { orc_model_destroy(m); return ORC_E_INVALID; }
        }
        m->point_cell[k] = orc_locate(m, &d->point_pos[3 * k], up);
        if (m->point_cell[k] < 0) { orc_model_destroy(m); return ORC_E_INVALID; }
    }
    *out = m;
    return ORC_OK;
}

int64_t orc_model_s_size(const orc_model *m) { return m->s_offset[m->d.n_lambda]; }
int32_t orc_model_nside_sca(const orc_model *m, int l) { return m->nside_sca[l]; }
int64_t orc_model_s_offset(const orc_model *m, int l) { return m->s_offset[l]; }

/* Finest-level cell index of point p along each axis; a point on a cell face
 * belongs to the cell that the direction d points into (upper cell when the
 * component is zero).  Returns 0 outside the root block. */
static int orc_fine_index(const orc_model *m, const double p[3], const double d[3], int64_t f[3])
{
    int inside = 1;
    for (int a = 0; a < 3; ++a) {
        double u = (p[a] - m->d.lo[a]) / m->h_fine;
        double fl = floor(u);
        int64_t i = (fl < -1.0) ? -1 : (fl > (double)m->fine[a]) ? m->fine[a] : (int64_t)fl;
        /* on a plane of the fine grid: the side the direction points to; a
         * ray lying in the plane (zero component) takes the side away from
         * the block's central plane, so that mirror-image rays take
         * mirror-image cells (on the central plane itself: the upper side) */
        if (u == fl && (d[a] < 0.0 || (d[a] == 0.0 && 2.0 * fl < (double)m->fine[a]))) i -= 1;
        if (i < 0 || i >= m->fine[a]) inside = 0;
        f[a] = i;
    }
    return inside;
}

static int64_t orc_leaf_at(const orc_model *m, const int64_t f[3])
{
    for (int a = 0; a < 3; ++a)
        if (f[a] < 0 || f[a] >= m->fine[a]) return -1;
    return m->fine_map[(f[2] * m->fine[1] + f[1]) * m->fine[0] + f[0]];
}

/* Leaf containing point p (tie rule above); -1 outside the root block. */
int64_t orc_locate(const orc_model *m, const double p[3], const double d[3])
{
    int64_t f[3];
    if (!orc_fine_index(m, p, d, f)) return -1;
    return orc_leaf_at(m, f);
}

/* Exit of leaf c along o + t d: exit distance and next leaf (-1 when the ray
 * leaves the root block).  The next leaf is the face neighbour across the
 * exit face that contains the exit point: on the exit axis its index follows
 * from the leaf's integer coordinates, on the other axes the exit point is
 * located and kept within the leaf's own extent. */
static int64_t orc_step_axis(const orc_model *m, int64_t c, const double o[3], const double d[3], double *t_exit,
                             int *exit_axis);

static int64_t orc_step(const orc_model *m, int64_t c, const double o[3], const double d[3], double *t_exit)
{
    int axis;
    return orc_step_axis(m, c, o, d, t_exit, &axis);
}

static int64_t orc_step_axis(const orc_model *m, int64_t c, const double o[3], const double d[3], double *t_exit,
                             int *exit_axis)
{
    double lo[3], hi[3];
    int64_t span = (int64_t)1 << (m->max_level - m->d.level[c]);
    for (int a = 0; a < 3; ++a) {
        lo[a] = m->centre[3 * c + a] - 0.5 * m->side[c];
        hi[a] = m->centre[3 * c + a] + 0.5 * m->side[c];
    }
    double best = INFINITY;
    int axis = -1;
    for (int a = 0; a < 3; ++a) {
        double t;
        if (d[a] > 0.0) t = (hi[a] - o[a]) / d[a];
        else if (d[a] < 0.0) t = (lo[a] - o[a]) / d[a];
        else continue;
        if (t < best) { best = t; axis = a; }
    }
    *t_exit = best;
    *exit_axis = axis;
    double p[3];
    int64_t f[3];
    for (int a = 0; a < 3; ++a) p[a] = o[a] + best * d[a];
    orc_fine_index(m, p, d, f);
    for (int a = 0; a < 3; ++a) {
        int64_t first = m->d.ijk[3 * c + a] * span, last = first + span - 1;
        if (a == axis) f[a] = d[a] > 0.0 ? last + 1 : first - 1;
        else if (f[a] < first) f[a] = first;
        else if (f[a] > last) f[a] = last;
    }
    return orc_leaf_at(m, f);
}

/* Cells crossed by the ray o + t d from t = t0: leaf ids, path lengths and
 * entry distances (zero-length segments included).  Returns the count, at
 * most max_cross. */
int64_t orc_trace_cells(const orc_model *m, const double o[3], const double d[3], double t0,
                        int64_t max_cross, int64_t *cells, double *lengths, double *t_in)
{
    double p[3];
    for (int a = 0; a < 3; ++a) p[a] = o[a] + t0 * d[a];
    int64_t c = orc_locate(m, p, d);
    double t = t0;
    int64_t n = 0;
    while (c >= 0 && n < max_cross) {
        double te;
        int64_t nx = orc_step(m, c, o, d, &te);
        cells[n] = c;
        lengths[n] = te > t ? te - t : 0.0;
        t_in[n] = t;
        ++n;
        if (te > t) t = te;
        c = nx;
    }
    return n;
}

/* A segment [t, te] whose length is zero up to the rounding of t and te: a
 * ray through an edge or corner of a cell (Sect. 2 is silent on these).  The
 * bound is 2^-46 of the exit distance, a few tens of units in the last place
 * of an FP64 distance: the exit distances of one exact tie, each computed
 * from an exact face position and a direction rounded to FP64, differ by a
 * few units in the last place. */
int orc_is_graze(double len, double te)
{
    return !(len > 0x1p-46 * te);
}

/* Crossings of positive length of the ray o + t d from t = t0, walked as a
 * radiative-transfer pass walks it: grazes are skipped without advancing the
 * distance, so their length folds into the next crossing.  Writes leaf ids,
 * lengths and entry distances; returns the count, at most max_cross. */
int64_t orc_crossings(const orc_model *m, const double o[3], const double d[3], double t0,
                      int64_t max_cross, int64_t *cells, double *lengths, double *t_in)
{
    double p[3];
    for (int a = 0; a < 3; ++a) p[a] = o[a] + t0 * d[a];
    int64_t c = orc_locate(m, p, d);
    double t = t0;
    int64_t n = 0;
    while (c >= 0 && n < max_cross) {
        double te;
        int64_t nx = orc_step(m, c, o, d, &te);
        double len = te > t ? te - t : 0.0;
        if (!orc_is_graze(len, te)) {
            cells[n] = c;
            lengths[n] = len;
            t_in[n] = t;
            ++n;
            t = te;
        }
        c = nx;
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* One radiative-transfer pass                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    double *U;          /* private or shared accumulators */
    double *S;
    int atomic;
    double tally[64 * N_TALLY];
    int64_t count[N_COUNT];
    double *w;          /* [sum npix] weights of the current ray */
    const double *pv;   /* [sum npix][3] j_sca pixel vectors of each wavelength's block */
    double *esc;        /* [n_lambda][nray0] escaping luminosity per launch pixel, or NULL */
    int64_t nray0;
    int nmir;           /* 8 in 2D mode, else 1 */
    const int64_t *mir; /* 2D mode: [n][8] the mirror images of each leaf */
    const int64_t *pmir;/* 2D mode: [sum npix][8] mirror images of the j_sca pixels */
    const int64_t *emir;/* 2D mode: [nray0][8] mirror images of the launch pixels */
} orc_thread;

static inline void orc_add(double *p, double v, int atomic)
{
    if (atomic) {
#pragma omp atomic
        *p += v;
    } else {
        *p += v;
    }
}

/* Luminosity launched along ray pixel `pix` at `nside_ray` from source s at
 * wavelength l, for the direct pass or from the pending scattered light. */
static double orc_launch(const orc_model *m, const orc_pass_opts *o, const double *S_pending,
                         int64_t s, int l, int64_t nside_ray, int64_t pix)
{
    const orc_grid_desc *d = &m->d;
    double nray = 12.0 * (double)nside_ray * (double)nside_ray;
    if (s >= d->n_leaves)   /* a point source: its luminosity spread evenly over the rays */
        return o->mode != ORC_SCATTER ? d->point_lum[(int64_t)l * d->n_point + (s - d->n_leaves)] / nray : 0.0;
    if (o->mode != ORC_SCATTER)
        return 4.0 * M_PI * d->emis[(int64_t)l * d->n_leaves + s] * m->side[s] * m->side[s] * m->side[s] / nray;
    int64_t ns = m->nside_sca[l];
    int64_t npix = 12 * ns * ns;
    const double *row = S_pending + m->s_offset[l] + s * npix;
    if (nside_ray >= ns) {
        int64_t shift = 0;
        while ((ns << shift) < nside_ray) ++shift;
        return row[pix >> (2 * shift)] * (double)npix / nray;
    }
    int64_t shift = 0;
    while ((nside_ray << shift) < ns) ++shift;
    int64_t nchild = (int64_t)1 << (2 * shift);
    double sum = 0.0;
    for (int64_t q = pix * nchild; q < (pix + 1) * nchild; ++q) sum += row[q];
    return sum;
}

static void orc_ray_dir(const orc_pass_opts *o, int64_t nside, int64_t pix, double n[3])
{
    double v[3];
    orc_healpix_vec(nside, pix, v);
    orc_rotate(o->frame, v, n);
}

/* Where the rays of source s start: the centre of emitting cell s, or the
 * position of point source s - n. */
static const double *orc_source_origin(const orc_model *m, int64_t s)
{
    return s < m->d.n_leaves ? &m->centre[3 * s] : &m->d.point_pos[3 * (s - m->d.n_leaves)];
}

/* The source's own cell: the emitting cell itself, or the leaf holding the
 * point source.  There the crossed cell fills the whole sky of the source
 * (Omega_INT infinite): no split or block test, and every wavelength counts
 * as significant. */
static int64_t orc_source_cell(const orc_model *m, int64_t s)
{
    return s < m->d.n_leaves ? s : m->point_cell[s - m->d.n_leaves];
}

/* A ray paused in the low list (Eq. 3): the cell it was about to cross,
 * the entry distance there, the grid plane it crossed to enter that cell
 * (axis -1: none, it started inside) and its luminosity. */
typedef struct {
    int64_t c;
    double t;
    int axis;
    double plane;
    double L[64];
} orc_low;

static int orc_follow(const orc_model *m, const orc_pass_opts *o, const double *U_LL, int64_t s, int level,
                      int64_t pix, double t_start, int64_t start_cell, const double *L_in, int can_low,
                      orc_thread *th, orc_low *low);

/* the j_sca weights w(p | n) of a ray along n, per wavelength block */
static void orc_ray_weights(const orc_model *m, const orc_pass_opts *o, const double n[3], orc_thread *th)
{
    if (o->mode == ORC_STEP1) return;
    for (int l = 0; l < m->d.n_lambda; ++l) {
        int64_t woff = m->s_offset[l] / m->d.n_leaves;
        orc_hg_weights_tab(12 * (int64_t)m->nside_sca[l] * m->nside_sca[l], th->pv + 3 * woff, m->d.g[l], n,
                           th->w + woff);
    }
}

/* v[0] + v[1] + v[2] + v[3] added in ascending order */
static double orc_sum4(double v[4])
{
    for (int i = 1; i < 4; ++i)
        for (int k = i; k > 0 && v[k] < v[k - 1]; --k) {
            double x = v[k];
            v[k] = v[k - 1];
            v[k - 1] = x;
        }
    return ((v[0] + v[1]) + v[2]) + v[3];
}

/*
 * The four children of a ray split at entry distance t_in (Eq. 2), each
 * with a quarter of its luminosity, followed one after the other.  When all
 * four end up in the low list having crossed the same grid plane, they merge
 * (Eq. 3 and the text after it): one ray in the parent's pixel carrying the
 * sum of their luminosities (the average intensity over a beam four times
 * wider), from the mean of their distances; orc_split then returns 1 with
 * that state in *merged and the parent's walk carries on with it.
 * Otherwise the paused children carry on from where they stopped, no longer
 * entering the low list, and orc_split returns 0 (the parent has ended).
 */
static int orc_split(const orc_model *m, const orc_pass_opts *o, const double *U_LL, int64_t s, int level,
                     int64_t pix, double t_in, const double *L, orc_thread *th, orc_low *merged)
{
    const int nl = m->d.n_lambda;
    th->count[C_SPLITS]++;
    orc_low kid[4];
    int paused[4], all = 1;
    double Lc[64];
    for (int l = 0; l < nl; ++l) Lc[l] = 0.25 * L[l];
    for (int k = 0; k < 4; ++k) {
        paused[k] = orc_follow(m, o, U_LL, s, level + 1, 4 * pix + k, t_in, -1, Lc, 1, th, &kid[k]);
        all &= paused[k];
    }
    if (all) {
        for (int k = 0; k < 4; ++k)
            if (kid[k].axis < 0 || kid[k].axis != kid[0].axis || kid[k].plane != kid[0].plane) all = 0;
    }
    if (all) {
        th->count[C_MERGES]++;
        /* sums over the four in ascending order, so that mirror-image groups
         * (the same siblings in another order) give the same ray */
        double v[4];
        for (int l = 0; l < nl; ++l) {
            for (int k = 0; k < 4; ++k) v[k] = kid[k].L[l];
            merged->L[l] = orc_sum4(v);
        }
        for (int k = 0; k < 4; ++k) v[k] = kid[k].t;
        merged->t = 0.25 * orc_sum4(v);
        return 1;
    }
    for (int k = 0; k < 4; ++k)
        if (paused[k]) orc_follow(m, o, U_LL, s, level + 1, 4 * pix + k, kid[k].t, kid[k].c, kid[k].L, 0, th, NULL);
    return 0;
}

/*
 * Follow one ray of source s (pixel pix at Nside nside0 2^level) from
 * distance t_start -- in start_cell, or the leaf found at that point when
 * -1 -- until it escapes, is blocked, is split (its children are followed
 * through orc_split) or, when can_low, pauses in the low list (returns 1).
 */
static int orc_follow(const orc_model *m, const orc_pass_opts *o, const double *U_LL, int64_t s, int level,
                      int64_t pix, double t_start, int64_t start_cell, const double *L_in, int can_low,
                      orc_thread *th, orc_low *low)
{
    const orc_grid_desc *d = &m->d;
    const int nl = d->n_lambda;
    const double cl = d->c_light;
    int64_t nside = (int64_t)o->nside << level;
    double omega_hp = 4.0 * M_PI / (12.0 * (double)nside * (double)nside);
    double n[3];
    orc_ray_dir(o, nside, pix, n);
    const double *xs = orc_source_origin(m, s);
    const int64_t own = orc_source_cell(m, s);
    orc_ray_weights(m, o, n, th);
    int64_t c = start_cell;
    if (c < 0) {
        double p[3];
        for (int a = 0; a < 3; ++a) p[a] = xs[a] + t_start * n[a];
        c = orc_locate(m, p, n);
    }
    double t = t_start;
    double L[64];
    for (int l = 0; l < nl; ++l) L[l] = L_in[l];
    double tau[64], ext[64];
    int sig[64];
    int64_t steps = 0;
    int entry_axis = -1;      /* the grid plane crossed to enter cell c */
    double entry_plane = 0.0;
    while (c >= 0) {
        /* the per-ray limit counts crossings of positive length: a ray that has
         * made max_steps of them stops before its next cell */
        if (o->max_steps > 0 && steps >= o->max_steps) { th->count[C_MAXSTEP]++; return 0; }
        double te;
        int axis;
        int64_t next = orc_step_axis(m, c, xs, n, &te, &axis);
        double len = te > t ? te - t : 0.0;
        /* a graze of an edge or corner: nothing is deposited, no decision is
         * taken and t is not advanced */
        if (!orc_is_graze(len, te)) {
            double t_in = t;
            double dc2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                double q = m->centre[3 * c + a] - xs[a];
                dc2 += q * q;
            }
            double vol = m->side[c] * m->side[c] * m->side[c];
            int any_sig = 0;
            for (int l = 0; l < nl; ++l) {
                double alpha = d->kappa[l] * d->rho[c];
                tau[l] = alpha * len;
                ext[l] = L[l] * (-expm1(-tau[l]));
                if (!o->adaptive || o->mode == ORC_STEP1) {
                    sig[l] = 1;
                } else {
                    double lavg = tau[l] > 0.0 ? ext[l] / tau[l] : L[l];
                    if (!(lavg > 0.0)) sig[l] = 0;
                    else if (c == own) sig[l] = 1;
                    else sig[l] = lavg / (omega_hp * dc2 * cl) >= o->f_U * U_LL[(int64_t)l * d->n_leaves + c];
                }
                any_sig |= sig[l];
            }
            if (o->adaptive) {
                if (o->mode == ORC_STEP1 && t_in >= o->r_pre) {
                    for (int l = 0; l < nl; ++l) th->tally[l * N_TALLY + T_CUT] += L[l];
                    th->count[C_CUTS]++;
                    return 0;
                }
                double omega_int = c == own ? INFINITY : m->side[c] * m->side[c] / dc2;
                if (omega_hp > omega_int / o->n_rays_min) {           /* Eq. 2: the beam is too large */
                    if (any_sig && nside < o->nside_max) {
                        orc_low mg;
                        if (!orc_split(m, o, U_LL, s, level, pix, t_in, L, th, &mg)) return 0;
                        /* the merged ray continues this walk from the mean distance
                         * (the children left their own phase weights behind) */
                        orc_ray_weights(m, o, n, th);
                        t = mg.t;
                        for (int l = 0; l < nl; ++l) L[l] = mg.L[l];
                        double p[3];
                        for (int a = 0; a < 3; ++a) p[a] = xs[a] + t * n[a];
                        c = orc_locate(m, p, n);
                        entry_axis = -1;
                        continue;
                    }
                    if (!any_sig) {
                        for (int l = 0; l < nl; ++l) th->tally[l * N_TALLY + T_CUT] += L[l];
                        th->count[C_CUTS]++;
                        return 0;
                    }
                }
                /* Eq. 3: the beam is too small for this cell; merging never
                 * goes below the launch resolution */
                if (can_low && o->n_rays_max > 0.0 && level > 0 && c != own && omega_hp < omega_int / o->n_rays_max) {
                    low->c = c;
                    low->t = t_in;
                    low->axis = entry_axis;
                    low->plane = entry_plane;
                    for (int l = 0; l < nl; ++l) low->L[l] = L[l];
                    return 1;
                }
            }
            th->count[C_CROSS]++;
            ++steps;
            for (int l = 0; l < nl; ++l) {
                double alpha = d->kappa[l] * d->rho[c];
                if (sig[l]) {
                    double du = alpha > 0.0 ? ext[l] / (alpha * vol * cl) : L[l] * len / (vol * cl);
                    /* 2D mode: the same deposit by each mirror image of the source */
                    for (int M = 0; M < th->nmir; ++M) {
                        int64_t cm = th->mir ? th->mir[8 * c + M] : c;
                        orc_add(&th->U[(int64_t)l * d->n_leaves + cm], du, th->atomic);
                    }
                    double om = d->albedo[l];
                    th->tally[l * N_TALLY + T_ABSORBED] += (1.0 - om) * ext[l];
                    th->tally[l * N_TALLY + T_SCATTERED] += om * ext[l];
                    th->count[C_DEPOSITS]++;
                    if (o->mode != ORC_STEP1 && om * ext[l] != 0.0) {
                        int64_t npix = 12 * (int64_t)m->nside_sca[l] * m->nside_sca[l];
                        int64_t woff = m->s_offset[l] / d->n_leaves;
                        const double *w = th->w + woff;
                        double ds = om * ext[l];
                        for (int M = 0; M < th->nmir; ++M) {
                            int64_t cm = th->mir ? th->mir[8 * c + M] : c;
                            double *row = th->S + m->s_offset[l] + cm * npix;
                            for (int64_t q = 0; q < npix; ++q) {
                                int64_t qm = th->pmir ? th->pmir[8 * (woff + q) + M] : q;
                                orc_add(&row[qm], ds * w[q], th->atomic);
                            }
                        }
                    }
                } else {
                    th->tally[l * N_TALLY + T_SKIPPED] += ext[l];
                    th->count[C_SKIPS]++;
                }
                L[l] *= exp(-tau[l]);
            }
            t = te;
        }
        /* the plane through which the ray leaves c is the one it enters the next cell by */
        entry_axis = axis;
        entry_plane = n[axis] > 0.0 ? m->centre[3 * c + axis] + 0.5 * m->side[c]
                                    : m->centre[3 * c + axis] - 0.5 * m->side[c];
        c = next;
    }
    for (int l = 0; l < nl; ++l) th->tally[l * N_TALLY + T_ESCAPED] += L[l];
    th->count[C_ESCAPES]++;
    if (th->esc) {
        /* attributed to the launch pixel the ray descends from */
        int64_t top = pix >> (2 * level);
        for (int M = 0; M < th->nmir; ++M) {
            int64_t tm = th->emir ? th->emir[8 * top + M] : top;
            for (int l = 0; l < nl; ++l) th->esc[(int64_t)l * th->nray0 + tm] += L[l];
        }
    }
    return 0;
}

/* Luminosity source s emits at wavelength l in this pass: 4 pi j V for the
 * direct light and step 1, the pending scattered luminosity of the cell summed
 * over its j_sca pixels in a scattering pass. */
static double orc_emitted(const orc_model *m, int mode, const double *S_pending, int64_t s, int l)
{
    const orc_grid_desc *d = &m->d;
    if (s >= d->n_leaves)
        return mode != ORC_SCATTER ? d->point_lum[(int64_t)l * d->n_point + (s - d->n_leaves)] : 0.0;
    if (mode != ORC_SCATTER)
        return 4.0 * M_PI * d->emis[(int64_t)l * d->n_leaves + s] * m->side[s] * m->side[s] * m->side[s];
    int64_t npix = 12 * (int64_t)m->nside_sca[l] * m->nside_sca[l];
    double e = 0.0;
    for (int64_t q = 0; q < npix; ++q) e += S_pending[m->s_offset[l] + s * npix + q];
    return e;
}

/* N_s of Eq. 11: the radiation sources of the pass in the whole model (cells
 * emitting at some wavelength), whatever subset of them a pass traces. */
int64_t orc_count_sources(const orc_model *m, int mode, const double *S_pending)
{
    int64_t ns = 0;
    for (int64_t s = 0; s < m->d.n_leaves + m->d.n_point; ++s) {
        int any = 0;
        for (int l = 0; l < m->d.n_lambda && !any; ++l) any = orc_emitted(m, mode, S_pending, s, l) > 0.0;
        ns += any;
    }
    return ns;
}

/* Run one pass.  Outputs (overwritten): U_k [n_lambda][n], S_next [S size]
 * (untouched in step 1), tally [n_lambda][8], counters [8], and escape
 * [n_lambda][12 nside^2] when not NULL: the luminosity leaving the root block,
 * by the launch pixel of the ray (the initial Nside).  Inputs: S_pending
 * (scatter pass), U_LL (adaptive direct/scatter passes). */
/*
 * 2D mode (Sect. 3.6): an axisymmetric model on a Cartesian grid is mirror
 * symmetric about the three planes through the block centre.  Only the
 * sources of the first octant (centre above the block centre on every axis)
 * are traced; every deposit is repeated by the 7 mirror images of the source
 * into the mirror images of the crossed cell (and of the j_sca pixel, and of
 * the launch pixel for the escape by direction), and the luminosity tallies
 * count all 8 sources.  The grid must be mirror symmetric (leaves, density
 * and emission), with no leaf across a mirror plane, no point sources, no
 * source mask and the unrotated frame.  Mirror image M (bits 0, 1, 2: x, y, z
 * reflected) of leaf c is mir[8 c + M].
 */
int64_t orc_healpix_pix(int64_t nside, const double v[3]);

static int orc_mirror_tables(const orc_model *m, const orc_pass_opts *o, int64_t nray0, int64_t **mir_out,
                             int64_t **pmir_out, int64_t **emir_out, uint8_t **first_out)
{
    const orc_grid_desc *d = &m->d;
    const int64_t n = d->n_leaves;
    const int nl = d->n_lambda;
    double cb[3];
    for (int a = 0; a < 3; ++a) cb[a] = d->lo[a] + 0.5 * d->nroot[a] * d->root_size;
    for (int i = 0; i < 9; ++i)
        if (o->frame[i] != ((i % 4 == 0) ? 1.0 : 0.0)) return ORC_E_INVALID;
    if (d->n_point > 0 || o->source_mask) return ORC_E_INVALID;
    int64_t wsize = m->s_offset[nl] / n;
    int64_t *mir = (int64_t *)malloc(sizeof(int64_t) * 8 * (size_t)n);
    int64_t *pmir = (int64_t *)malloc(sizeof(int64_t) * 8 * (size_t)(wsize > 0 ? wsize : 1));
    int64_t *emir = (int64_t *)malloc(sizeof(int64_t) * 8 * (size_t)nray0);
    uint8_t *first = (uint8_t *)malloc((size_t)n);
    int bad = !mir || !pmir || !emir || !first;
    for (int64_t c = 0; c < n && !bad; ++c) {
        const double *x = &m->centre[3 * c];
        first[c] = 1;
        for (int a = 0; a < 3; ++a) {
            if (fabs(x[a] - cb[a]) < 0.5 * m->side[c]) bad = 1;   /* across a mirror plane */
            if (!(x[a] > cb[a])) first[c] = 0;
        }
        for (int M = 0; M < 8 && !bad; ++M) {
            double p[3], dir[3] = {1.0, 1.0, 1.0};
            for (int a = 0; a < 3; ++a) p[a] = ((M >> a) & 1) ? 2.0 * cb[a] - x[a] : x[a];
            int64_t cm = orc_locate(m, p, dir);
            if (cm < 0 || d->level[cm] != d->level[c] || d->rho[cm] != d->rho[c]) {
                bad = 1;
                break;
            }
            for (int l = 0; l < nl; ++l)
                if (d->emis[(int64_t)l * n + cm] != d->emis[(int64_t)l * n + c]) bad = 1;
            mir[8 * c + M] = cm;
        }
    }
    /* mirror images of HEALPix pixels: the pixel holding the reflected centre */
    for (int pass = 0; pass < 2 && !bad; ++pass) {
        for (int l = 0; l < (pass == 0 ? nl : 1) && !bad; ++l) {
            int64_t ns = pass == 0 ? m->nside_sca[l] : o->nside;
            int64_t np = 12 * ns * ns;
            int64_t *tab = pass == 0 ? pmir + 8 * (m->s_offset[l] / n) : emir;
            for (int64_t q = 0; q < np; ++q) {
                double v[3], w[3], back[3];
                orc_healpix_vec(ns, q, v);
                for (int M = 0; M < 8; ++M) {
                    for (int a = 0; a < 3; ++a) w[a] = ((M >> a) & 1) ? -v[a] : v[a];
                    int64_t qm = orc_healpix_pix(ns, w);
                    orc_healpix_vec(ns, qm, back);
                    for (int a = 0; a < 3; ++a)
                        if (fabs(back[a] - w[a]) > 1e-12) bad = 1;   /* the pixel set is symmetric */
                    tab[8 * q + M] = qm;
                }
            }
        }
    }
    if (bad) {
        free(mir);
        free(pmir);
        free(emir);
        free(first);
        return mir && pmir && emir && first ? ORC_E_INVALID : ORC_E_OOM;
    }
    *mir_out = mir;
    *pmir_out = pmir;
    *emir_out = emir;
    *first_out = first;
    return ORC_OK;
}

int orc_run_pass(const orc_model *m, const orc_pass_opts *o, const double *S_pending, const double *U_LL,
                 double *U_k, double *S_next, double *tally, int64_t *counters, double *escape)
{
    const orc_grid_desc *d = &m->d;
    const int nl = d->n_lambda;
    const int64_t n = d->n_leaves;
    if (nl > 64 || o->nside <= 0 || !is_pow2(o->nside)) return ORC_E_INVALID;
    if (o->adaptive && (o->nside_max < o->nside || !is_pow2(o->nside_max) || !(o->n_rays_min > 0.0))) return ORC_E_INVALID;
    /* a merged beam (four times a child's) must not be too large at once (Eq. 2 against Eq. 3) */
    if (o->n_rays_max != 0.0 && !(o->n_rays_max >= 4.0 * o->n_rays_min)) return ORC_E_INVALID;
    if (o->mode == ORC_SCATTER && !S_pending) return ORC_E_INVALID;
    if (o->adaptive && o->mode != ORC_STEP1 && !U_LL) return ORC_E_INVALID;
    orc_pass_opts eff = *o;
    if (o->adaptive && o->mode != ORC_STEP1 && o->f_U < 0.0) {
        /* Eq. 11: f_U = 4 a_RT / N_s */
        if (!(o->a_RT > 0.0)) return ORC_E_INVALID;
        int64_t ns = orc_count_sources(m, o->mode, S_pending);
        eff.f_U = ns > 0 ? 4.0 * o->a_RT / (double)ns : 0.0;
    }
    o = &eff;
    int64_t ssize = m->s_offset[nl];
    int64_t wsize = ssize / n;
    /* point sources emit in step 1 and the direct pass; a source mask covers
     * the cells, then the point sources */
    const int64_t n_src_points = o->mode == ORC_SCATTER ? 0 : d->n_point;
    int64_t nray0_ = 12 * (int64_t)o->nside * o->nside;
    int64_t *mir = NULL, *pmir = NULL, *emir = NULL;
    uint8_t *first = NULL;
    if (o->mode_2d) {
        int rc = orc_mirror_tables(m, o, nray0_, &mir, &pmir, &emir, &first);
        if (rc != ORC_OK) return rc;
    }
    int nthreads = o->n_threads > 0 ? o->n_threads : omp_get_max_threads();
    /* private accumulators when they fit comfortably, shared atomics otherwise */
    double per_thread = 8.0 * ((double)nl * n + (o->mode == ORC_STEP1 ? 0.0 : (double)ssize));
    int atomic = per_thread * nthreads > 6.0e9;
    memset(U_k, 0, sizeof(double) * (size_t)(nl * n));
    if (o->mode != ORC_STEP1) memset(S_next, 0, sizeof(double) * (size_t)ssize);
    memset(tally, 0, sizeof(double) * (size_t)(nl * N_TALLY));
    memset(counters, 0, sizeof(int64_t) * N_COUNT);
    int64_t nray0 = 12 * (int64_t)o->nside * o->nside;
    if (escape) memset(escape, 0, sizeof(double) * (size_t)(nl * nray0));
    int failed = 0;
    /* j_sca pixel centre vectors, one block per wavelength (rotated frame) */
    double *pv = (double *)malloc(sizeof(double) * 3 * (size_t)(wsize > 0 ? wsize : 1));
    if (!pv) {
        free(mir);
        free(pmir);
        free(emir);
        free(first);
        return ORC_E_OOM;
    }
    for (int l = 0; l < nl; ++l) orc_pixel_table(m->nside_sca[l], o->frame, pv + 3 * (m->s_offset[l] / n));

#pragma omp parallel num_threads(nthreads)
    {
        orc_thread th;
        memset(&th, 0, sizeof(th));
        th.atomic = atomic;
        th.pv = pv;
        th.nmir = mir ? 8 : 1;
        th.mir = mir;
        th.pmir = pmir;
        th.emir = emir;
        if (atomic) {
            th.U = U_k;
            th.S = S_next;
        } else {
            th.U = (double *)calloc((size_t)(nl * n), sizeof(double));
            th.S = o->mode == ORC_STEP1 ? NULL : (double *)calloc((size_t)ssize, sizeof(double));
        }
        th.w = (double *)malloc(sizeof(double) * (size_t)(wsize > 0 ? wsize : 1));
        th.nray0 = nray0;
        th.esc = escape ? (double *)calloc((size_t)(nl * nray0), sizeof(double)) : NULL;
        int ok = th.w && th.U && (o->mode == ORC_STEP1 || th.S) && (!escape || th.esc);
        if (!ok) {
#pragma omp atomic write
            failed = 1;
        }
        if (ok) {
#pragma omp for schedule(dynamic, 1)
            for (int64_t s = 0; s < n + n_src_points; ++s) {
                if (o->source_mask && !o->source_mask[s]) continue;
                if (first && !first[s]) continue;   /* 2D mode: first-octant sources only */
                /* emitted luminosity of this source */
                double emitted_any = 0.0;
                for (int l = 0; l < nl; ++l) {
                    double e = orc_emitted(m, o->mode, S_pending, s, l);
                    th.tally[l * N_TALLY + T_EMITTED] += e;
                    emitted_any += e;
                }
                if (!(emitted_any > 0.0)) continue;
                for (int64_t r = 0; r < nray0; ++r) {
                    double L0[64];
                    double lsum = 0.0;
                    for (int l = 0; l < nl; ++l) {
                        L0[l] = orc_launch(m, o, S_pending, s, l, o->nside, r);
                        lsum += L0[l];
                    }
                    if (!(lsum > 0.0)) continue;
                    th.count[C_RAYS]++;
                    orc_low unused;
                    orc_follow(m, o, U_LL, s, 0, r, 0.0, orc_source_cell(m, s), L0, 0, &th, &unused);
                }
            }
#pragma omp critical
            {
                if (!atomic) {
                    for (int64_t i = 0; i < nl * n; ++i) U_k[i] += th.U[i];
                    if (o->mode != ORC_STEP1)
                        for (int64_t i = 0; i < ssize; ++i) S_next[i] += th.S[i];
                }
                for (int i = 0; i < nl * N_TALLY; ++i) tally[i] += th.tally[i];
                for (int i = 0; i < N_COUNT; ++i) counters[i] += th.count[i];
                if (escape)
                    for (int64_t i = 0; i < nl * nray0; ++i) escape[i] += th.esc[i];
            }
        }
        if (!atomic) {
            free(th.U);
            free(th.S);
        }
        free(th.w);
        free(th.esc);
    }
    free(pv);
    if (mir) {
        /* the tallies of all 8 mirror images of the traced sources */
        for (int i = 0; i < nl * N_TALLY; ++i) tally[i] *= 8.0;
        free(mir);
        free(pmir);
        free(emir);
        free(first);
    }
    return failed ? ORC_E_OOM : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of one fixed-Nside pass (reverse mode, FP64).                      */
/*                                                                            */
/* For a ray with crossings m = 0..M-1 of length l_m in cells c_m, luminosity  */
/* L_m at entry (L_{m+1} = L_m e^{-tau_m}) and tau_m = kappa rho_{c_m} l_m, the */
/* pass contributes J_ray = sum_m L_m a_m(tau_m) with                          */
/*   a_m(tau) = l_m E(tau) Ubar(c_m) / (V c) + albedo (1 - e^{-tau}) sbar_m,    */
/*   E(tau) = (1 - e^{-tau}) / tau,  sbar_m = sum_p w(p|n) Sbar_next(c_m, p),   */
/* where Ubar = dJ/dU and Sbar_next = dJ/dS of the luminosity this pass        */
/* scatters.  A loss on the escaping luminosity adds L_M Ebar(r) for the ray's */
/* pixel r, L_M being what leaves the block.  With                             */
/* G_m = a_m + e^{-tau_m} G_{m+1} and G_M = Ebar(r) (zero without that loss):  */
/*   dJ/dtau_m = L_m (a_m'(tau_m) - e^{-tau_m} G_{m+1}),                       */
/*   dJ/drho_c += kappa l_m dJ/dtau_m over the crossings in c,                 */
/*   dJ/dL_0 = G_0, which for a scattering pass flows to the pending           */
/*   luminosity the ray was launched from (the inverse of the launch rule).    */
/* ------------------------------------------------------------------------ */

static void orc_E(double tau, double *E, double *dE)
{
    if (tau < 1e-4) {
        *E = 1.0 - tau / 2.0 + tau * tau / 6.0;
        *dE = -0.5 + tau / 3.0 - tau * tau / 8.0;
    } else {
        double em = exp(-tau);
        *E = -expm1(-tau) / tau;
        *dE = (em * (1.0 + tau) - 1.0) / (tau * tau);
    }
}

/* Ubar [n_lambda][n]; Sbar_next [S size] or NULL (zero); Ebar
 * [n_lambda][12 nside^2] or NULL (zero); S_pending: the pass's emission
 * (scattering pass) or NULL (direct pass); rho_bar [n] is accumulated; Sbar_k
 * [S size] is overwritten for scattering passes. */
int orc_adjoint_pass(const orc_model *m, const orc_pass_opts *o, const double *S_pending, const double *Ubar,
                     const double *Sbar_next, const double *Ebar, double *rho_bar, double *Sbar_k)
{
    const orc_grid_desc *d = &m->d;
    const int nl = d->n_lambda;
    const int64_t n = d->n_leaves;
    if (o->adaptive || nl > 64 || o->nside <= 0 || !is_pow2(o->nside)) return ORC_E_INVALID;
    const int scatter = o->mode == ORC_SCATTER;
    if (scatter && (!S_pending || !Sbar_k)) return ORC_E_INVALID;
    int64_t ssize = m->s_offset[nl];
    int64_t wsize = ssize / n;
    int64_t nside = o->nside;
    int64_t nray = 12 * nside * nside;
    if (scatter) memset(Sbar_k, 0, sizeof(double) * (size_t)ssize);
    double *pv = (double *)malloc(sizeof(double) * 3 * (size_t)(wsize > 0 ? wsize : 1));
    if (!pv) return ORC_E_OOM;
    for (int l = 0; l < nl; ++l) orc_pixel_table(m->nside_sca[l], o->frame, pv + 3 * (m->s_offset[l] / n));
    int nthreads = o->n_threads > 0 ? o->n_threads : omp_get_max_threads();
    int64_t maxc = 4 * (m->fine[0] + m->fine[1] + m->fine[2]) + 64;
    int failed = 0;
#pragma omp parallel num_threads(nthreads)
    {
        double *w = (double *)malloc(sizeof(double) * (size_t)(wsize > 0 ? wsize : 1));
        int64_t *cells = (int64_t *)malloc(sizeof(int64_t) * (size_t)maxc);
        double *lens = (double *)malloc(sizeof(double) * (size_t)maxc);
        double *tins = (double *)malloc(sizeof(double) * (size_t)maxc);
        double *Lm = (double *)malloc(sizeof(double) * (size_t)maxc);
        if (!w || !cells || !lens || !tins || !Lm) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t s = 0; s < n + (scatter ? 0 : d->n_point); ++s) {
                if (!scatter && o->source_mask && !o->source_mask[s]) continue;
                const double *xs = orc_source_origin(m, s);
                for (int64_t r = 0; r < nray; ++r) {
                    double nvec[3];
                    orc_ray_dir(o, nside, r, nvec);
                    /* the crossings of the forward pass: grazes skipped and folded */
                    int64_t nc = orc_crossings(m, xs, nvec, 0.0, maxc, cells, lens, tins);
                    for (int l = 0; l < nl; ++l)
                        orc_hg_weights_tab(12 * (int64_t)m->nside_sca[l] * m->nside_sca[l], pv + 3 * (m->s_offset[l] / n),
                                           d->g[l], nvec, w + m->s_offset[l] / n);
                    for (int l = 0; l < nl; ++l) {
                        /* rays with zero launch luminosity still carry sensitivity
                         * (dJ/dL_0 = G_0) back to the pending luminosity */
                        double L0 = orc_launch(m, o, S_pending, s, l, nside, r);
                        if (!scatter && !(L0 > 0.0)) continue;
                        const double kap = d->kappa[l], om = d->albedo[l], cl = d->c_light;
                        int64_t npix = 12 * (int64_t)m->nside_sca[l] * m->nside_sca[l];
                        const double *wl = w + m->s_offset[l] / n;
                        /* forward: luminosity at entry of each crossing */
                        double L = L0;
                        for (int64_t k = 0; k < nc; ++k) {
                            Lm[k] = L;
                            L *= exp(-kap * d->rho[cells[k]] * lens[k]);
                        }
                        /* backward suffix recursion from the escaping end */
                        double G = Ebar ? Ebar[(int64_t)l * nray + r] : 0.0;
                        for (int64_t k = nc - 1; k >= 0; --k) {
                            int64_t c = cells[k];
                            double len = lens[k];
                            double vol = m->side[c] * m->side[c] * m->side[c];
                            double tau = kap * d->rho[c] * len;
                            double em = exp(-tau), E, dE;
                            orc_E(tau, &E, &dE);
                            double sb = 0.0;
                            if (Sbar_next) {
                                const double *row = Sbar_next + m->s_offset[l] + c * npix;
                                for (int64_t q = 0; q < npix; ++q) sb += wl[q] * row[q];
                            }
                            double ub = Ubar[(int64_t)l * n + c];
                            double a = len * E * ub / (vol * cl) + om * (1.0 - em) * sb;
                            double da = len * dE * ub / (vol * cl) + om * em * sb;
                            double dtau = Lm[k] * (da - em * G);
                            G = a + em * G;
                            double v = kap * len * dtau;
#pragma omp atomic
                            rho_bar[c] += v;
                        }
                        if (scatter) {
                            int64_t ns = m->nside_sca[l];
                            double *srow = Sbar_k + m->s_offset[l] + s * npix;
                            if (nside >= ns) {
                                int64_t shift = 0;
                                while ((ns << shift) < nside) ++shift;
                                double v = G * (double)npix / (double)nray;
#pragma omp atomic
                                srow[r >> (2 * shift)] += v;
                            } else {
                                int64_t shift = 0;
                                while ((nside << shift) < ns) ++shift;
                                int64_t nch = (int64_t)1 << (2 * shift);
                                for (int64_t q = r * nch; q < (r + 1) * nch; ++q) {
#pragma omp atomic
                                    srow[q] += G;
                                }
                            }
                        }
                    }
                }
            }
        }
        free(w);
        free(cells);
        free(lens);
        free(tins);
        free(Lm);
    }
    free(pv);
    return failed ? ORC_E_OOM : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Observer maps (Sect. 2: I_obs = I_0 e^{-tau}; Sect. 3.6: internal-observer */
/* all-sky HEALPix maps).                                                     */
/*                                                                            */
/* Every cell is a source of luminosity per unit solid angle towards the      */
/* observer, j V (stellar emission, isotropic) plus S[p] N_pix / (4 pi) for   */
/* the j_sca pixel p containing that direction (scattered light), emitted at  */
/* its centre and attenuated by the optical depth from the centre to the      */
/* observer (the cell's own half included).  A distant observer along `dir`   */
/* sees it on an image pixel of the plane normal to dir (surface brightness:  */
/* the sum over the cells of a pixel over the pixel's area); an internal      */
/* observer at `pos` sees it in the map pixel containing the direction to the */
/* cell, as a flux over the distance squared, per the pixel's solid angle.    */
/* The observer's own cell is left out of an internal map.                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t kind;           /* 0 distant, 1 internal */
    double dir[3];          /* distant: unit vector from the model towards the observer */
    double up[3];           /* distant: image up direction */
    double centre[3];       /* distant: model point at the image centre */
    double pixel_size;      /* distant: image pixel edge */
    int32_t nx, ny;         /* distant: image pixels */
    double pos[3];          /* internal: observer position */
    int32_t nside_map;      /* internal: map Nside */
    double frame[9];        /* rotation of the j_sca pixel directions */
} orc_observer;

static void orc_normalise(double v[3])
{
    double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int a = 0; a < 3; ++a) v[a] /= r;
}

/* map [n_lambda][npix] is overwritten; S_total (S layout) may be NULL. */
int orc_observe(const orc_model *m, const orc_observer *ob, const double *S_total, double *map)
{
    const orc_grid_desc *d = &m->d;
    const int nl = d->n_lambda;
    const int64_t n = d->n_leaves;
    int64_t npix;
    double e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0}, dir[3] = {0, 0, 0};
    int64_t obs_cell = -1;
    if (ob->kind == 0) {
        if (ob->nx <= 0 || ob->ny <= 0 || !(ob->pixel_size > 0.0)) return ORC_E_INVALID;
        npix = (int64_t)ob->nx * ob->ny;
        for (int a = 0; a < 3; ++a) dir[a] = ob->dir[a];
        orc_normalise(dir);
        double ud = ob->up[0] * dir[0] + ob->up[1] * dir[1] + ob->up[2] * dir[2];
        for (int a = 0; a < 3; ++a) e2[a] = ob->up[a] - ud * dir[a];
        orc_normalise(e2);
        e1[0] = e2[1] * dir[2] - e2[2] * dir[1];   /* e1 = e2 x dir */
        e1[1] = e2[2] * dir[0] - e2[0] * dir[2];
        e1[2] = e2[0] * dir[1] - e2[1] * dir[0];
    } else if (ob->kind == 1) {
        if (ob->nside_map <= 0 || !is_pow2(ob->nside_map)) return ORC_E_INVALID;
        npix = 12 * (int64_t)ob->nside_map * ob->nside_map;
        double up0[3] = {1.0, 1.0, 1.0};   /* a point on a face belongs to the upper side */
        obs_cell = orc_locate(m, ob->pos, up0);
    } else {
        return ORC_E_INVALID;
    }
    memset(map, 0, sizeof(double) * (size_t)(nl * npix));
    int64_t maxc = 4 * (m->fine[0] + m->fine[1] + m->fine[2]) + 64;
    int failed = 0;
#pragma omp parallel
    {
        int64_t *cells = (int64_t *)malloc(sizeof(int64_t) * (size_t)maxc);
        double *lens = (double *)malloc(sizeof(double) * (size_t)maxc);
        double *tins = (double *)malloc(sizeof(double) * (size_t)maxc);
        double *acc = (double *)calloc((size_t)(nl * npix), sizeof(double));
        if (!cells || !lens || !tins || !acc) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (int64_t c = 0; c < n + d->n_point; ++c) {
                if (c == obs_cell) continue;
                /* a cell, or a point source (index n + k) */
                const double *xc = orc_source_origin(m, c);
                double nv[3], dist = INFINITY;
                if (ob->kind == 0) {
                    for (int a = 0; a < 3; ++a) nv[a] = dir[a];
                } else {
                    for (int a = 0; a < 3; ++a) nv[a] = ob->pos[a] - xc[a];
                    dist = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
                    if (!(dist > 0.0)) continue;
                    for (int a = 0; a < 3; ++a) nv[a] /= dist;
                }
                int64_t pix;
                double weight;   /* map value per unit luminosity per steradian reaching the observer */
                if (ob->kind == 0) {
                    double u = 0.0, w = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        u += (xc[a] - ob->centre[a]) * e1[a];
                        w += (xc[a] - ob->centre[a]) * e2[a];
                    }
                    double fx = floor(u / ob->pixel_size + 0.5 * ob->nx), fy = floor(w / ob->pixel_size + 0.5 * ob->ny);
                    if (fx < 0.0 || fy < 0.0 || fx >= ob->nx || fy >= ob->ny) continue;
                    pix = (int64_t)fy * ob->nx + (int64_t)fx;
                    weight = 1.0 / (ob->pixel_size * ob->pixel_size);
                } else {
                    double away[3] = {-nv[0], -nv[1], -nv[2]};   /* from the observer towards the cell */
                    pix = orc_healpix_pix(ob->nside_map, away);
                    weight = 1.0 / (dist * dist * (4.0 * M_PI / (double)npix));
                }
                /* optical depth from the cell centre to the observer (or out of the block) */
                int64_t nc = orc_crossings(m, xc, nv, 0.0, maxc, cells, lens, tins);
                double colr = 0.0;   /* sum of rho l */
                for (int64_t k = 0; k < nc; ++k) {
                    double len = lens[k];
                    if (tins[k] >= dist) break;
                    if (tins[k] + len > dist) len = dist - tins[k];
                    colr += d->rho[cells[k]] * len;
                }
                if (c >= n) {
                    /* a point source: its luminosity per steradian, isotropic */
                    for (int l = 0; l < nl; ++l) {
                        double dl = d->point_lum[(int64_t)l * d->n_point + (c - n)] / (4.0 * M_PI);
                        if (dl != 0.0) acc[(int64_t)l * npix + pix] += dl * exp(-d->kappa[l] * colr) * weight;
                    }
                    continue;
                }
                double vol = m->side[c] * m->side[c] * m->side[c];
                /* the j_sca pixel holding the direction towards the observer, in the rotated frame */
                double loc[3];
                for (int a = 0; a < 3; ++a)
                    loc[a] = ob->frame[a] * nv[0] + ob->frame[3 + a] * nv[1] + ob->frame[6 + a] * nv[2];
                for (int l = 0; l < nl; ++l) {
                    double dl = d->emis[(int64_t)l * n + c] * vol;
                    if (S_total) {
                        int64_t ns = m->nside_sca[l];
                        int64_t np = 12 * ns * ns;
                        dl += S_total[m->s_offset[l] + c * np + orc_healpix_pix(ns, loc)] * (double)np / (4.0 * M_PI);
                    }
                    if (dl == 0.0) continue;
                    acc[(int64_t)l * npix + pix] += dl * exp(-d->kappa[l] * colr) * weight;
                }
            }
#pragma omp critical
            for (int64_t i = 0; i < nl * npix; ++i) map[i] += acc[i];
        }
        free(cells);
        free(lens);
        free(tins);
        free(acc);
    }
    return failed ? ORC_E_OOM : ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Dust emission (Sect. 3.3): absorbed luminosity, equilibrium temperature,   */
/* emission of a toy modified-blackbody grain                                  */
/* ------------------------------------------------------------------------- */
/*
 * Every wavelength of a grid stands for a band: U, j and the tallies are
 * band-integrated.  The dust of a cell absorbs (1 - albedo) of what it
 * extinguishes, so with the deposit rule (U = ext / (alpha V c)) the band
 * absorbs (1 - albedo) kappa rho V c U.  In equilibrium the grain re-emits
 * that power in the emission bands as kappa_abs B_lambda(T) (Kirchhoff), band
 * i carrying 4 pi rho V kappa_i (1 - albedo_i) B(lambda_i, T) dlambda_i, with
 * the Planck-shaped B(lambda, T) = b0 lambda^-5 / (exp(x0 / (lambda T)) - 1).
 * The paper leaves the grain model to the user (equilibrium or stochastic
 * heating, its Sect. 3.3); this one stands in for it.
 */
typedef struct {
    double b0;              /* scale of B */
    double x0;              /* h c / k in the units of lambda times temperature */
    double t_max;           /* upper end of the temperature bracket */
    const double *lambda;   /* [n_lambda of the emitting grid] band centres */
    const double *dlambda;  /* [n_lambda of the emitting grid] band widths */
} orc_dust_model;

/* A[c] += sum_l (1 - albedo_l) kappa_l rho_c V_c c U[l][c] */
void orc_absorbed(const orc_model *m, const double *U, double *A)
{
    const orc_grid_desc *d = &m->d;
    for (int64_t c = 0; c < d->n_leaves; ++c) {
        double vol = m->side[c] * m->side[c] * m->side[c];
        for (int l = 0; l < d->n_lambda; ++l)
            A[c] += (1.0 - d->albedo[l]) * d->kappa[l] * d->rho[c] * vol * d->c_light * U[(int64_t)l * d->n_leaves + c];
    }
}

static double orc_planck(const orc_dust_model *dm, double lambda, double T)
{
    if (!(T > 0.0)) return 0.0;
    return dm->b0 / (lambda * lambda * lambda * lambda * lambda) / expm1(dm->x0 / (lambda * T));
}

/* power emitted per unit mass (rho V = 1) at temperature T, over every band */
double orc_dust_power(const orc_model *m, const orc_dust_model *dm, double T)
{
    const orc_grid_desc *d = &m->d;
    double p = 0.0;
    for (int l = 0; l < d->n_lambda; ++l)
        p += 4.0 * M_PI * d->kappa[l] * (1.0 - d->albedo[l]) * orc_planck(dm, dm->lambda[l], T) * dm->dlambda[l];
    return p;
}

/*
 * Equilibrium temperature of every cell of the emitting grid m from its
 * absorbed luminosity A (the power per unit mass A / (rho V) equals
 * orc_dust_power(T)), by bisection of [0, t_max] down to adjacent doubles,
 * and the emission j[l][c] = rho kappa_l (1 - albedo_l) B(lambda_l, T) dlambda_l
 * (per unit volume and steradian, band-integrated).  Cells without dust or
 * without absorbed light get T = 0 and no emission.  A cell that would need
 * more than t_max gives ORC_E_INVALID.
 */
int orc_dust_emission(const orc_model *m, const orc_dust_model *dm, const double *A, double *T, double *j)
{
    const orc_grid_desc *d = &m->d;
    const int64_t n = d->n_leaves;
    int bad = 0;
    if (orc_dust_power(m, dm, dm->t_max) <= 0.0) return ORC_E_INVALID;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t c = 0; c < n; ++c) {
        double vol = m->side[c] * m->side[c] * m->side[c];
        double t = 0.0;
        if (d->rho[c] > 0.0 && A[c] > 0.0) {
            double target = A[c] / (d->rho[c] * vol);
            double lo = 0.0, hi = dm->t_max;
            if (orc_dust_power(m, dm, hi) < target) {
                bad = 1;
            } else {
                for (;;) {
                    double mid = 0.5 * (lo + hi);
                    if (!(mid > lo && mid < hi)) break;
                    if (orc_dust_power(m, dm, mid) < target)
                        lo = mid;
                    else
                        hi = mid;
                }
                t = hi;
            }
        }
        T[c] = t;
        for (int l = 0; l < d->n_lambda; ++l)
            j[(int64_t)l * n + c] =
                d->rho[c] * d->kappa[l] * (1.0 - d->albedo[l]) * orc_planck(dm, dm->lambda[l], t) * dm->dlambda[l];
    }
    return bad ? ORC_E_INVALID : ORC_OK;
}
