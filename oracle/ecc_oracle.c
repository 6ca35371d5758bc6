/*
 * ecc_oracle.c -- reference ("oracle") computation of the Euler characteristic
 * curve of a grayscale image of 1 to 8 dimensions (the definitions are the same
 * in every dimension, Sec. 2.1).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously correct CPU
 * implementation used to check the GPU library bit for bit.  It shares no code,
 * header, table or constant with the GPU library, and the library never calls it.
 * Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * load it.
 *
 * What is computed (Wang, Wagner, Chen, "GPU Computation of the Euler
 * Characteristic Curve for Imaging Data", SoCG 2022):
 *
 *   1. every voxel value is mapped to an integer bin in [0, nbins)   (the paper
 *      indexes its histogram by gray level, Sec. 4 and Algorithm 2; the mapping
 *      for 16-bit and float data is this library's own reading, stated below);
 *   2. every cell of the cubical complex gets a filtration value (Sec. 2.1):
 *        - ORACLE_VERTEX: voxels are the vertices of the complex, a cell is a
 *          block of 2^k voxels and takes the MAXIMUM bin over its vertices;
 *        - ORACLE_TOP:    voxels are the top-dimensional cells (closed unit
 *          cubes), lower cells are the faces of the vertex lattice and take the
 *          MINIMUM bin over the voxels that contain them (Sec. 2.1, last
 *          paragraph);
 *   3. VCEC[j] = sum over cells with value j of (-1)^dim            (Sec. 2.3,
 *      "Tracking the VCEC"; Eq. (1) for the alternating sum);
 *   4. ECC[i]  = sum_{j <= i} VCEC[j]                               (Sec. 2.3).
 *
 * Step 2/3 enumerate every cell explicitly (no per-voxel "introduced faces"
 * bookkeeping as in Algorithm 1), so the oracle is independent of the
 * tie-breaking argument the fast path relies on.
 *
 * Binning (the paper is silent for data that is not 0..255 integers):
 *   integer data (u8, u16), integer range [lo, hi]:
 *       a = clamp(v, lo, hi) - lo ;  bin = (a * nbins) / (hi - lo + 1)   (exact)
 *   float data (f32), range [lo, hi] given as doubles:
 *       NaN               -> nbins - 1
 *       hi == lo          -> (x > hi) ? nbins - 1 : 0
 *       otherwise t = ((double)x - lo) * scale, scale = (double)nbins / (hi - lo),
 *       each operation rounded once in IEEE double (no fused multiply-add),
 *       bin = clamp(floor(t), 0, nbins - 1).
 *   Range modes: DEFAULT = [0,255] for u8 and AUTO otherwise; AUTO = [min, max]
 *   over the image (over the finite values for f32; [0,0] if there are none).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORACLE_U8 = 0, ORACLE_U16 = 1, ORACLE_F32 = 2 };
enum { ORACLE_VERTEX = 0, ORACLE_TOP = 1 };
enum { ORACLE_RANGE_DEFAULT = 0, ORACLE_RANGE_EXPLICIT = 1, ORACLE_RANGE_AUTO = 2 };

#define ORACLE_MAX_NDIM 8

/* ---------------------------------------------------------------- binning */

/* Resolves the range mode into an explicit [lo, hi]. Returns 0 on success. */
int oracle_resolve_range(const void* data, int dtype, int64_t nvox, int range_mode,
                         double lo_in, double hi_in, double* lo_out, double* hi_out)
{
    if (range_mode == ORACLE_RANGE_DEFAULT) {
        if (dtype == ORACLE_U8) { *lo_out = 0.0; *hi_out = 255.0; return 0; }
        range_mode = ORACLE_RANGE_AUTO;
    }
    if (range_mode == ORACLE_RANGE_EXPLICIT) {
        *lo_out = lo_in;
        *hi_out = hi_in;
        return 0;
    }
    if (range_mode != ORACLE_RANGE_AUTO) return -1;
    double lo = 0.0, hi = 0.0;
    int found = 0;
    for (int64_t i = 0; i < nvox; ++i) {
        double v;
        if (dtype == ORACLE_U8) v = ((const uint8_t*)data)[i];
        else if (dtype == ORACLE_U16) v = ((const uint16_t*)data)[i];
        else {
            float f = ((const float*)data)[i];
            if (!isfinite(f)) continue;
            v = f;
        }
        if (!found) { lo = hi = v; found = 1; }
        else { if (v < lo) lo = v; if (v > hi) hi = v; }
    }
    *lo_out = lo;
    *hi_out = hi;
    return 0;
}

static int32_t bin_integer(int64_t v, int64_t lo, int64_t hi, int64_t nbins)
{
    if (v < lo) v = lo;
    if (v > hi) v = hi;
    int64_t a = v - lo;
    return (int32_t)((a * nbins) / (hi - lo + 1));
}

static int32_t bin_float(float x, double lo, double hi, double scale, int32_t nbins)
{
    if (isnan(x)) return nbins - 1;
    if (hi == lo) return ((double)x > hi) ? nbins - 1 : 0;
    volatile double d = (double)x - lo;   /* volatile: one rounding per operation */
    volatile double t = d * scale;
    if (!(t >= 0.0)) return 0;            /* negative (incl. -inf) */
    if (t >= (double)nbins) return nbins - 1;
    return (int32_t)floor(t);
}

/* Maps every voxel to its bin. Returns 0 on success, -1 on a bad argument. */
int oracle_bins(const void* data, int dtype, int64_t nvox, int32_t nbins, int range_mode,
                double lo_in, double hi_in, int32_t* bins_out, double* lo_used, double* hi_used)
{
    if (nbins < 1 || nbins > 65535) return -1;
    double lo, hi;
    if (oracle_resolve_range(data, dtype, nvox, range_mode, lo_in, hi_in, &lo, &hi)) return -1;
    if (!(lo <= hi)) return -1;
    if (lo_used) *lo_used = lo;
    if (hi_used) *hi_used = hi;
    if (dtype == ORACLE_U8 || dtype == ORACLE_U16) {
        /* integer data: the range must be integers inside the type's range */
        double maxval = (dtype == ORACLE_U8) ? 255.0 : 65535.0;
        if (!(lo >= 0.0) || !(hi <= maxval)) return -1;
        int64_t ilo = (int64_t)lo, ihi = (int64_t)hi;
        if ((double)ilo != lo || (double)ihi != hi) return -1;
        for (int64_t i = 0; i < nvox; ++i) {
            int64_t v = (dtype == ORACLE_U8) ? ((const uint8_t*)data)[i] : ((const uint16_t*)data)[i];
            bins_out[i] = bin_integer(v, ilo, ihi, nbins);
        }
        return 0;
    }
    if (dtype != ORACLE_F32) return -1;
    if (!isfinite(lo) || !isfinite(hi)) return -1;
    double scale = (hi > lo) ? (double)nbins / (hi - lo) : 0.0;
    for (int64_t i = 0; i < nvox; ++i)
        bins_out[i] = bin_float(((const float*)data)[i], lo, hi, scale, nbins);
    return 0;
}

/* ----------------------------------------------------- cell enumeration */

typedef struct {
    const int32_t* bins;
    int ndim;
    int64_t n[ORACLE_MAX_NDIM];      /* voxel counts per axis, axis 0 slowest */
    int64_t stride[ORACLE_MAX_NDIM]; /* row-major voxel strides */
    int32_t nbins;
    int construction;
    int64_t a0_begin, a0_end;        /* slab of axis-0 anchors for this worker */
    int64_t* hist;                   /* int64[nbins], owned by the worker */
} oracle_job;

/* Advances the anchor a[1..d-1] through [0, lim[i]) (last axis fastest) and then
 * a[0] through [a0_begin, a0_end).  Returns 0 when every anchor was visited. */
static int next_anchor(int64_t* a, const int64_t* lim, int d, int64_t a0_end)
{
    for (int i = d - 1; i >= 1; --i) {
        if (++a[i] < lim[i]) return 1;
        a[i] = 0;
    }
    return ++a[0] < a0_end;
}

/* VERTEX construction.  A cell is the block of voxels  a + {0..s_0} x ... ,
 * s in {0,1}^d, lying inside the image; its dimension is |s| and its value is
 * the maximum bin over its 2^|s| voxels (its vertices). Each cell has exactly one
 * anchor a (its lowest corner), so iterating (a, s) visits every cell once. */
static void cells_vertex(oracle_job* J)
{
    const int d = J->ndim;
    int64_t a[ORACLE_MAX_NDIM] = {0};
    int64_t lim[ORACLE_MAX_NDIM];
    for (int i = 0; i < d; ++i) lim[i] = J->n[i];
    if (J->a0_begin >= J->a0_end) return;
    a[0] = J->a0_begin;
    do {
        for (int s = 0; s < (1 << d); ++s) {
            int ok = 1, dim = 0;
            for (int i = 0; i < d; ++i)
                if (s >> i & 1) { ++dim; if (a[i] + 1 >= J->n[i]) ok = 0; }
            if (!ok) continue;
            int32_t value = -1;
            for (int t = 0; t < (1 << d); ++t) {        /* vertices: t subset of s */
                if ((t & s) != t) continue;
                int64_t idx = 0;
                for (int i = 0; i < d; ++i) idx += (a[i] + (t >> i & 1)) * J->stride[i];
                int32_t b = J->bins[idx];
                if (b > value) value = b;
            }
            J->hist[value] += (dim & 1) ? -1 : 1;
        }
    } while (next_anchor(a, lim, d, J->a0_end));
}

/* TOP construction (the paper's).  Voxel v is the closed cube prod [v_i, v_i+1].
 * A cell is a face of the vertex lattice: per axis either the interval
 * [a_i, a_i+1] (non-degenerate, needs a_i < n_i; contained only in voxels with
 * coordinate a_i) or the point a_i in [0, n_i] (degenerate; contained in the
 * voxels with coordinate a_i - 1 or a_i that exist).  Dimension = number of
 * non-degenerate axes; value = minimum bin over the voxels containing it. */
static void cells_top(oracle_job* J)
{
    const int d = J->ndim;
    int64_t a[ORACLE_MAX_NDIM] = {0};
    int64_t lim[ORACLE_MAX_NDIM];
    for (int i = 0; i < d; ++i) lim[i] = J->n[i] + 1;   /* lattice points 0..n_i */
    if (J->a0_begin >= J->a0_end) return;
    a[0] = J->a0_begin;
    do {
        for (int s = 0; s < (1 << d); ++s) {
            int ok = 1, dim = 0;
            int64_t vlo[ORACLE_MAX_NDIM], vhi[ORACLE_MAX_NDIM];  /* voxel range per axis */
            for (int i = 0; i < d; ++i) {
                if (s >> i & 1) {
                    ++dim;
                    if (a[i] >= J->n[i]) ok = 0;
                    vlo[i] = vhi[i] = a[i];
                } else {
                    vlo[i] = a[i] - 1 < 0 ? 0 : a[i] - 1;
                    vhi[i] = a[i] > J->n[i] - 1 ? J->n[i] - 1 : a[i];
                }
            }
            if (!ok) continue;
            /* minimum over the box of voxels vlo..vhi (at most 2 per axis) */
            int32_t value = J->nbins;   /* larger than any bin */
            for (int t = 0; t < (1 << d); ++t) {
                int64_t idx = 0;
                int inside = 1;
                for (int i = 0; i < d; ++i) {
                    const int64_t v = vlo[i] + (t >> i & 1);
                    if (v > vhi[i]) { inside = 0; break; }
                    idx += v * J->stride[i];
                }
                if (inside && J->bins[idx] < value) value = J->bins[idx];
            }
            J->hist[value] += (dim & 1) ? -1 : 1;
        }
    } while (next_anchor(a, lim, d, J->a0_end));
}

static void* oracle_worker(void* arg)
{
    oracle_job* J = (oracle_job*)arg;
    if (J->construction == ORACLE_VERTEX) cells_vertex(J);
    else cells_top(J);
    return NULL;
}

/* VCEC from precomputed bins; every cell enumerated once.  `threads` workers
 * split the anchors of axis 0 into slabs and keep private histograms that are
 * summed at the end (integer sums, so the result does not depend on `threads`).
 * Returns 0 on success. */
int oracle_vcec_from_bins(const int32_t* bins, int ndim, const int64_t* dims, int32_t nbins,
                          int construction, int threads, int64_t* vcec_out)
{
    if (ndim < 1 || ndim > ORACLE_MAX_NDIM || nbins < 1) return -1;
    if (construction != ORACLE_VERTEX && construction != ORACLE_TOP) return -1;
    oracle_job base;
    memset(&base, 0, sizeof base);
    base.bins = bins;
    base.ndim = ndim;
    base.nbins = nbins;
    base.construction = construction;
    for (int i = 0; i < ndim; ++i) {
        if (dims[i] < 1) return -1;
        base.n[i] = dims[i];
    }
    {
        int64_t s = 1;
        for (int i = ndim - 1; i >= 0; --i) { base.stride[i] = s; s *= base.n[i]; }
    }
    int64_t a0_count = (construction == ORACLE_VERTEX) ? base.n[0] : base.n[0] + 1;
    if (threads < 1) threads = 1;
    if (threads > a0_count) threads = (int)a0_count;
    oracle_job* jobs = (oracle_job*)calloc((size_t)threads, sizeof(oracle_job));
    pthread_t* tids = (pthread_t*)calloc((size_t)threads, sizeof(pthread_t));
    int64_t* hists = (int64_t*)calloc((size_t)threads * (size_t)nbins, sizeof(int64_t));
    if (!jobs || !tids || !hists) { free(jobs); free(tids); free(hists); return -2; }
    for (int t = 0; t < threads; ++t) {
        jobs[t] = base;
        jobs[t].a0_begin = a0_count * t / threads;
        jobs[t].a0_end = a0_count * (t + 1) / threads;
        jobs[t].hist = hists + (size_t)t * (size_t)nbins;
    }
    int spawned = 0;
    for (int t = 1; t < threads; ++t)
        if (pthread_create(&tids[t], NULL, oracle_worker, &jobs[t]) == 0) spawned = t;
        else { oracle_worker(&jobs[t]); tids[t] = 0; }
    oracle_worker(&jobs[0]);
    for (int t = 1; t <= spawned; ++t)
        if (tids[t]) pthread_join(tids[t], NULL);
    for (int j = 0; j < nbins; ++j) {
        int64_t s = 0;
        for (int t = 0; t < threads; ++t) s += hists[(size_t)t * (size_t)nbins + j];
        vcec_out[j] = s;
    }
    free(jobs);
    free(tids);
    free(hists);
    return 0;
}

/* ECC_i = sum_{j <= i} VCEC_j  (Sec. 2.3). */
void oracle_prefix(const int64_t* vcec, int32_t nbins, int64_t* ecc_out)
{
    int64_t acc = 0;
    for (int32_t i = 0; i < nbins; ++i) { acc += vcec[i]; ecc_out[i] = acc; }
}

/* Whole path: bins -> VCEC -> ECC. Returns 0 on success. */
int oracle_ecc(const void* data, int dtype, int ndim, const int64_t* dims, int32_t nbins,
               int construction, int range_mode, double lo, double hi, int threads,
               int64_t* ecc_out)
{
    if (ndim < 1 || ndim > ORACLE_MAX_NDIM) return -1;
    int64_t nvox = 1;
    for (int i = 0; i < ndim; ++i) { if (dims[i] < 1) return -1; nvox *= dims[i]; }
    int32_t* bins = (int32_t*)malloc((size_t)nvox * sizeof(int32_t));
    int64_t* vcec = (int64_t*)calloc((size_t)(nbins > 0 ? nbins : 1), sizeof(int64_t));
    if (!bins || !vcec) { free(bins); free(vcec); return -2; }
    int rc = oracle_bins(data, dtype, nvox, nbins, range_mode, lo, hi, bins, NULL, NULL);
    if (rc == 0) rc = oracle_vcec_from_bins(bins, ndim, dims, nbins, construction, threads, vcec);
    if (rc == 0) oracle_prefix(vcec, nbins, ecc_out);
    free(bins);
    free(vcec);
    return rc;
}

/* Separable 13-tap smoothing of a 2D float32 image, the smoothing step of the
 * pipeline workload (Sec. 5, "Pipeline" and "Gaussian smoothing
 * implementation": a discrete Gaussian convolution of width 13, applied along
 * one axis and then the other).  The paper fixes neither the boundary nor the
 * evaluation order; this library's reading:
 *   rows:    tmp[y][x] = sum_{k=0..12} w[k] * in[y][clamp(x + k - 6)]
 *   columns: out[y][x] = sum_{k=0..12} w[k] * tmp[clamp(y + k - 6)][x]
 * clamp() repeats the border pixel; every sum starts from 0.0f and adds the
 * terms in the order k = 0..12, each product and each sum rounded once in IEEE
 * float32 (no fused multiply-add).  `out` may be `in`.  Returns 0, or -1 for an
 * empty image, -2 if memory runs out. */
static int64_t clamp_index(int64_t i, int64_t n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

int oracle_smooth13(const float* in, float* out, int64_t n1, int64_t n2, const float* w)
{
    if (n1 < 1 || n2 < 1) return -1;
    float* tmp = (float*)malloc((size_t)n1 * (size_t)n2 * sizeof(float));
    if (!tmp) return -2;
    for (int64_t y = 0; y < n1; ++y)
        for (int64_t x = 0; x < n2; ++x) {
            float acc = 0.0f;
            for (int k = 0; k < 13; ++k) {
                const float p = w[k] * in[y * n2 + clamp_index(x + k - 6, n2)];
                acc = acc + p;
            }
            tmp[y * n2 + x] = acc;
        }
    for (int64_t y = 0; y < n1; ++y)
        for (int64_t x = 0; x < n2; ++x) {
            float acc = 0.0f;
            for (int k = 0; k < 13; ++k) {
                const float p = w[k] * tmp[clamp_index(y + k - 6, n1) * n2 + x];
                acc = acc + p;
            }
            out[y * n2 + x] = acc;
        }
    free(tmp);
    return 0;
}
