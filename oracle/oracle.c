/*
 * Plain FP64 CPU oracle for convolutional gridding and degridding.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition the GPU library is checked against.  Only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the product
 * path never calls it.  It shares no code, header or table with the GPU
 * library.
 *
 * Definition followed (Chapter 2 of the thesis):
 *   - grid origin at the centre pixel, N*dl = 1 normalisation
 *     (Section 2.1.2, "Grids and normalisation");
 *   - the oversampled kernel is read by nearest-neighbour lookup into a table
 *     sampled every 1/beta cells (Section 2.3.6, "GCF oversampling"); by the
 *     equivalence theorem of Section 2.4.2 (Algorithm "Equivalent Algorithm
 *     for Convolutional Gridding with GCF Oversampling") this is the same as
 *     moving the record to its nearest pixel q/beta of the beta-oversampled
 *     grid and sampling the kernel at integer cell offsets from there;
 *   - nearest pixel: rect is 1 on the half-open interval (-1/(2 beta),
 *     1/(2 beta)] (helper functions, Section 2.1.4), hence
 *     q = floor(beta*x + 1/2), ties rounding up;
 *   - the footprint is the S cells whose offset from q/beta lies in
 *     (-S/2, S/2] (support, Section 2.3.4 "The form of the GCF");
 *   - records whose footprint leaves the grid are skipped (the Bounded
 *     Records Assumption, Section 2.3.1);
 *   - Gridding Step: W = [F * C] sampled on the grid (Algorithm "General
 *     Convolutional Gridding", Section 2.3), every polarisation gridded the
 *     same way (Section 1.1);
 *   - W-projection: the kernel of plane p is the table of plane
 *     p = round(|w| / dw), conjugated for w < 0 (the W-term relation of
 *     Section 1.3: gbar_{-w} = conj(gbar_w) with a real symmetric taper);
 *   - degridding is the exact adjoint: V_out = sum conj(weight) * G.
 *
 * All arithmetic in double, compiled with -ffp-contract=off so that the
 * index rule rounds exactly as written.  Records are visited in input order.
 *
 * orc_grid_window_par is the same gridder run on several host threads, for
 * the CPU rate only: the window's rows are cut into bands, every band is
 * owned by one thread and visits, in input order, the records whose
 * footprint reaches it, so each cell receives its contributions in the same
 * order as in orc_grid_window and the two agree bit for bit.
 *
 * Hybrid Gridding and column pruning (NEXT to the convolutional gridder, at
 * the end of this file) follow the same rules; their pins tie them to it.
 *
 * Parity pins (in tests/): delta kernel at integer cells, brute-force
 * footprint enumeration, the equivalence theorem (NN onto the beta grid,
 * then a discrete convolution), equal-offset exactness against a direct DFT
 * (component analysis, Section 2.3.2), Hermitian mirror symmetry, linearity
 * and the adjoint identity.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)

/* Floor division for a possibly negative numerator and positive divisor. */
static int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0)))
        q -= 1;
    return q;
}

typedef struct {
    int64_t k_lo;   /* first cell of the footprint        */
    int64_t t0;     /* table index of the first tap, 1..beta */
    int ok;
} axis_index;

/* One axis: position in cells -> footprint start and first tap.
 * x = coord * scale + n/2; q = floor(x*beta + 1/2);
 * k_lo = floor((q - beta*S/2) / beta) + 1; t0 = k_lo*beta - q + beta*S/2. */
static axis_index index_axis(double coord, double scale, int32_t n, int32_t beta, int32_t S)
{
    axis_index r = {0, 0, 0};
    double x = coord * scale;
    x = x + (double)(n / 2);
    double xb = x * (double)beta;
    xb = xb + 0.5;
    double fq = floor(xb);
    if (!(fabs(fq) < 4.0e15))
        return r;
    int64_t q = (int64_t)fq;
    int64_t half = (int64_t)beta * S / 2;
    r.k_lo = floor_div(q - half, beta) + 1;
    r.t0 = r.k_lo * beta - q + half;
    r.ok = (r.k_lo >= 0) && (r.k_lo + S - 1 <= (int64_t)n - 1);
    return r;
}

typedef struct {
    int32_t nu, nv, beta;
    double scale_u, scale_v;
    int32_t nplanes;              /* 0: separable kernel */
    const int32_t *plane_support; /* [nplanes] */
    double inv_dw;
    int32_t support;              /* separable support */
} orc_geom;

typedef struct {
    int64_t k_lo_u, k_lo_v, t0_u, t0_v;
    int32_t plane, S, conj, valid;
} rec_index;

static rec_index index_record(const orc_geom *g, const double *uvw)
{
    rec_index r;
    memset(&r, 0, sizeof r);
    r.plane = -1;
    double u = uvw[0], v = uvw[1], w = uvw[2];
    if (!isfinite(u) || !isfinite(v) || !isfinite(w))
        return r;
    int32_t S = g->support;
    if (g->nplanes > 0) {
        double a = fabs(w) * g->inv_dw;
        a = a + 0.5;
        double fp = floor(a);
        int32_t p = (fp >= (double)(g->nplanes - 1)) ? g->nplanes - 1 : (int32_t)fp;
        r.plane = p;
        r.conj = (w < 0.0);
        S = g->plane_support[p];
    }
    r.S = S;
    axis_index au = index_axis(u, g->scale_u, g->nu, g->beta, S);
    axis_index av = index_axis(v, g->scale_v, g->nv, g->beta, S);
    r.k_lo_u = au.k_lo;
    r.k_lo_v = av.k_lo;
    r.t0_u = au.t0;
    r.t0_v = av.t0;
    r.valid = au.ok && av.ok;
    return r;
}

static int check_geom(const orc_geom *g)
{
    if (g->nu <= 0 || g->nv <= 0 || g->beta <= 0)
        return ORC_EINVAL;
    if (g->nplanes == 0) {
        if (g->support <= 0 || ((int64_t)g->beta * g->support) % 2)
            return ORC_EINVAL;
    } else {
        for (int p = 0; p < g->nplanes; ++p)
            if (g->plane_support[p] <= 0 || ((int64_t)g->beta * g->plane_support[p]) % 2)
                return ORC_EINVAL;
    }
    return ORC_OK;
}

#define GEOM_ARGS int32_t nu, int32_t nv, int32_t beta, double scale_u, double scale_v, \
    int32_t nplanes, const int32_t *plane_support, double inv_dw, int32_t support
#define GEOM_INIT {nu, nv, beta, scale_u, scale_v, nplanes, plane_support, inv_dw, support}

/* Per-record indices (for parity of the integer part of the map).
 * o = t0 - 1 in [0, beta-1].  plane = -1 for a separable kernel.
 * Returns the number of skipped records, or ORC_EINVAL. */
int64_t orc_index(GEOM_ARGS, int64_t nrec, const double *uvw,
                  int32_t *k_lo_u, int32_t *k_lo_v, int32_t *o_u, int32_t *o_v,
                  int32_t *plane, uint8_t *valid)
{
    orc_geom g = GEOM_INIT;
    if (check_geom(&g))
        return ORC_EINVAL;
    int64_t skipped = 0;
    for (int64_t r = 0; r < nrec; ++r) {
        rec_index ix = index_record(&g, uvw + 3 * r);
        k_lo_u[r] = (int32_t)ix.k_lo_u;
        k_lo_v[r] = (int32_t)ix.k_lo_v;
        o_u[r] = (int32_t)(ix.t0_u - 1);
        o_v[r] = (int32_t)(ix.t0_v - 1);
        plane[r] = ix.plane;
        valid[r] = (uint8_t)ix.valid;
        skipped += !ix.valid;
    }
    return skipped;
}

/* Weight of tap (i, j) of a record: real for a separable table (taps[t]),
 * complex for a W-projection plane (taps interleaved re, im). */
static void tap_weight(const orc_geom *g, const double *taps, const int64_t *plane_offset,
                       const rec_index *ix, int32_t i, int32_t j, double *wr, double *wi)
{
    int64_t tu = ix->t0_u + (int64_t)i * g->beta;
    int64_t tv = ix->t0_v + (int64_t)j * g->beta;
    if (g->nplanes == 0) {
        *wr = taps[tu] * taps[tv];
        *wi = 0.0;
    } else {
        int64_t width = (int64_t)g->beta * ix->S + 1;
        const double *k = taps + 2 * (plane_offset[ix->plane] + tv * width + tu);
        *wr = k[0];
        *wi = ix->conj ? -k[1] : k[1];
    }
}

/* Grid only the cells inside the window [u0, u0+wu) x [v0, v0+wv) of the
 * full nv x nu grid.  out: complex128 [npol][wv][wu], ACCUMULATED.
 * vis: complex128 [nrec][npol].  The full-grid gridder is the window that
 * covers the whole grid.  Returns the number of skipped records. */
int64_t orc_grid_window(GEOM_ARGS, const double *taps, const int64_t *plane_offset,
                        int64_t nrec, const double *uvw, int32_t npol, const double *vis,
                        int32_t u0, int32_t v0, int32_t wu, int32_t wv, double *out)
{
    orc_geom g = GEOM_INIT;
    if (check_geom(&g) || npol < 1)
        return ORC_EINVAL;
    int64_t skipped = 0;
    for (int64_t r = 0; r < nrec; ++r) {
        rec_index ix = index_record(&g, uvw + 3 * r);
        if (!ix.valid) {
            ++skipped;
            continue;
        }
        for (int32_t j = 0; j < ix.S; ++j) {
            int64_t cv = ix.k_lo_v + j - v0;
            if (cv < 0 || cv >= wv)
                continue;
            for (int32_t i = 0; i < ix.S; ++i) {
                int64_t cu = ix.k_lo_u + i - u0;
                if (cu < 0 || cu >= wu)
                    continue;
                double wr, wi;
                tap_weight(&g, taps, plane_offset, &ix, i, j, &wr, &wi);
                for (int32_t pol = 0; pol < npol; ++pol) {
                    const double *V = vis + 2 * (r * npol + pol);
                    double *G = out + 2 * (((int64_t)pol * wv + cv) * wu + cu);
                    G[0] += wr * V[0] - wi * V[1];
                    G[1] += wr * V[1] + wi * V[0];
                }
            }
        }
    }
    return skipped;
}

/* Degridding, the adjoint of gridding:
 * vis_out[r][pol] = sum_{j,i} conj(weight_ij) * grid[pol][k_lo_v+j][k_lo_u+i]
 * (rows j outer, columns i inner); skipped records get 0.
 * grid: complex128 [npol][nv][nu]; vis_out: complex128 [nrec][npol],
 * OVERWRITTEN.  Returns the number of skipped records. */
int64_t orc_degrid(GEOM_ARGS, const double *taps, const int64_t *plane_offset,
                   int64_t nrec, const double *uvw, int32_t npol, const double *grid,
                   double *vis_out)
{
    orc_geom g = GEOM_INIT;
    if (check_geom(&g) || npol < 1)
        return ORC_EINVAL;
    int64_t skipped = 0;
    for (int64_t r = 0; r < nrec; ++r) {
        rec_index ix = index_record(&g, uvw + 3 * r);
        double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (!ix.valid) {
            ++skipped;
        } else {
            for (int32_t j = 0; j < ix.S; ++j) {
                for (int32_t i = 0; i < ix.S; ++i) {
                    double wr, wi;
                    tap_weight(&g, taps, plane_offset, &ix, i, j, &wr, &wi);
                    for (int32_t pol = 0; pol < npol; ++pol) {
                        const double *G = grid + 2 * (((int64_t)pol * nv + ix.k_lo_v + j) * nu
                                                      + ix.k_lo_u + i);
                        /* conj(w) * G = (wr - j wi)(gr + j gi) */
                        acc[2 * pol] += wr * G[0] + wi * G[1];
                        acc[2 * pol + 1] += wr * G[1] - wi * G[0];
                    }
                }
            }
        }
        for (int32_t pol = 0; pol < npol; ++pol) {
            vis_out[2 * (r * npol + pol)] = acc[2 * pol];
            vis_out[2 * (r * npol + pol) + 1] = acc[2 * pol + 1];
        }
    }
    return skipped;
}

/* Direct Fourier sum (the DFT of the problem statement, Section 2.2) at
 * positions given in cells from the grid centre:
 * image[iy][ix] = sum_r F_r exp(+j 2 pi (pu_r * l + pv_r * m)),
 * l = (ix - nx/2)/nx, m = (iy - ny/2)/ny.  Sign: the image-from-visibility
 * direction of the direct imaging sum I_D (Section 1.7).
 * pos: [nrec][2] in cells; F: complex128 [nrec]; image: complex128 [ny][nx]. */
void orc_dft(int64_t nrec, const double *pos, const double *F, int32_t nx, int32_t ny,
             double *image)
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int32_t iy = 0; iy < ny; ++iy) {
        double m = (double)(iy - ny / 2) / (double)ny;
        for (int32_t ix = 0; ix < nx; ++ix) {
            double l = (double)(ix - nx / 2) / (double)nx;
            double sr = 0.0, si = 0.0;
            for (int64_t r = 0; r < nrec; ++r) {
                double ph = two_pi * (pos[2 * r] * l + pos[2 * r + 1] * m);
                double c = cos(ph), s = sin(ph);
                sr += F[2 * r] * c - F[2 * r + 1] * s;
                si += F[2 * r] * s + F[2 * r + 1] * c;
            }
            image[2 * ((int64_t)iy * nx + ix)] = sr;
            image[2 * ((int64_t)iy * nx + ix) + 1] = si;
        }
    }
}

/* Band-parallel gridding for the CPU rate (same result as orc_grid_window,
 * bit for bit).  The window's wv rows are split into nbands bands of equal
 * height; pass 1 indexes every record once and counts it in each band its
 * footprint rows reach; pass 2 lets the threads take bands (dynamically) and
 * apply, in input order, the taps of the band's records that fall on the
 * band's rows.  nthreads <= 0 uses the OpenMP default.  Returns the skipped
 * count, ORC_EINVAL, or -2 if the record lists cannot be allocated. */
int64_t orc_grid_window_par(GEOM_ARGS, const double *taps, const int64_t *plane_offset,
                            int64_t nrec, const double *uvw, int32_t npol, const double *vis,
                            int32_t u0, int32_t v0, int32_t wu, int32_t wv, double *out,
                            int32_t nthreads, int32_t nbands)
{
    orc_geom g = GEOM_INIT;
    if (check_geom(&g) || npol < 1 || nbands < 1 || wv < 1)
        return ORC_EINVAL;
    if (nbands > wv)
        nbands = wv;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const int64_t bh = ((int64_t)wv + nbands - 1) / nbands;   /* rows per band */
    int64_t *cnt = calloc((size_t)nbands + 1, sizeof(int64_t));
    int32_t *first = malloc(sizeof(int32_t) * (size_t)(nrec > 0 ? nrec : 1));
    int32_t *last = malloc(sizeof(int32_t) * (size_t)(nrec > 0 ? nrec : 1));
    if (!cnt || !first || !last) {
        free(cnt); free(first); free(last);
        return -2;
    }
    int64_t skipped = 0;
    /* pass 1: band range of every valid record (first > last: none) */
#pragma omp parallel for schedule(static) reduction(+ : skipped)
    for (int64_t r = 0; r < nrec; ++r) {
        rec_index ix = index_record(&g, uvw + 3 * r);
        first[r] = 1;
        last[r] = 0;
        if (!ix.valid) {
            ++skipped;
            continue;
        }
        int64_t lo = ix.k_lo_v - v0, hi = ix.k_lo_v + ix.S - 1 - v0;
        int64_t cu_lo = ix.k_lo_u - u0, cu_hi = ix.k_lo_u + ix.S - 1 - u0;
        if (hi < 0 || lo >= wv || cu_hi < 0 || cu_lo >= wu)
            continue;
        if (lo < 0)
            lo = 0;
        if (hi >= wv)
            hi = wv - 1;
        first[r] = (int32_t)(lo / bh);
        last[r] = (int32_t)(hi / bh);
    }
    for (int64_t r = 0; r < nrec; ++r)
        for (int32_t b = first[r]; b <= last[r]; ++b)
            cnt[b + 1]++;
    for (int32_t b = 0; b < nbands; ++b)
        cnt[b + 1] += cnt[b];
    int64_t *list = malloc(sizeof(int64_t) * (size_t)(cnt[nbands] > 0 ? cnt[nbands] : 1));
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)nbands);
    if (!list || !fill) {
        free(cnt); free(first); free(last); free(list); free(fill);
        return -2;
    }
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)nbands);
    for (int64_t r = 0; r < nrec; ++r)          /* input order inside every band */
        for (int32_t b = first[r]; b <= last[r]; ++b)
            list[fill[b]++] = r;
    /* pass 2: every band's records, rows of the band only */
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t b = 0; b < nbands; ++b) {
        const int64_t row_lo = (int64_t)b * bh;
        const int64_t row_hi = row_lo + bh < wv ? row_lo + bh : wv;   /* exclusive */
        for (int64_t e = cnt[b]; e < cnt[b + 1]; ++e) {
            const int64_t r = list[e];
            rec_index ix = index_record(&g, uvw + 3 * r);
            for (int32_t j = 0; j < ix.S; ++j) {
                int64_t cv = ix.k_lo_v + j - v0;
                if (cv < row_lo || cv >= row_hi)
                    continue;
                for (int32_t i = 0; i < ix.S; ++i) {
                    int64_t cu = ix.k_lo_u + i - u0;
                    if (cu < 0 || cu >= wu)
                        continue;
                    double wr, wi;
                    tap_weight(&g, taps, plane_offset, &ix, i, j, &wr, &wi);
                    for (int32_t pol = 0; pol < npol; ++pol) {
                        const double *V = vis + 2 * (r * npol + pol);
                        double *G = out + 2 * (((int64_t)pol * wv + cv) * wu + cu);
                        G[0] += wr * V[0] - wi * V[1];
                        G[1] += wr * V[1] + wi * V[0];
                    }
                }
            }
        }
    }
    free(cnt); free(first); free(last); free(list); free(fill);
    return skipped;
}

/* Threads the OpenMP runtime would use (1 without OpenMP). */
int32_t orc_max_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------
 * Hybrid Gridding (Algorithm "The studied Hybrid Gridding Algorithm",
 * Section 2.4.4): the Gridding Step convolves with C_hy = C_co(u) rect(v),
 * i.e. along u the oversampled separable kernel of support S sampled at the
 * integer cells (exactly as in the convolutional gridder above), along v
 * nearest-neighbour interpolation onto the v axis oversampled by beta.  The
 * output grid has nv * beta rows (row q = the nearest pixel of the
 * beta-oversampled v axis, q = floor(beta x_v + 1/2), x_v = v scale_v +
 * nv/2, the same rule as for the convolutional gridder) and nu columns; the
 * origin u = v = 0 is at column nu/2, row beta nv / 2.  A record is gridded
 * if uvw is finite, its u footprint lies inside [0, nu) and 0 <= q < beta
 * nv.  out: complex128 [npol][wv][wu], the window [u0, u0 + wu) x
 * [v0, v0 + wv) of the [npol][beta nv][nu] grid, ACCUMULATED.  Returns the
 * number of skipped records, or ORC_EINVAL. */
int64_t orc_hybrid_grid_window(int32_t nu, int32_t nv, int32_t beta, double scale_u,
                               double scale_v, int32_t support, const double *taps,
                               int64_t nrec, const double *uvw, int32_t npol, const double *vis,
                               int32_t u0, int32_t v0, int32_t wu, int32_t wv, double *out)
{
    if (nu <= 0 || nv <= 0 || beta <= 0 || support <= 0 || npol < 1 ||
        ((int64_t)beta * support) % 2)
        return ORC_EINVAL;
    const int64_t rows = (int64_t)beta * nv;
    int64_t skipped = 0;
    for (int64_t r = 0; r < nrec; ++r) {
        const double u = uvw[3 * r], v = uvw[3 * r + 1], w = uvw[3 * r + 2];
        if (!isfinite(u) || !isfinite(v) || !isfinite(w)) {
            ++skipped;
            continue;
        }
        axis_index au = index_axis(u, scale_u, nu, beta, support);
        double x = v * scale_v;
        x = x + (double)(nv / 2);
        double xb = x * (double)beta;
        xb = xb + 0.5;
        const double fq = floor(xb);
        if (!au.ok || !(fq >= 0.0) || !(fq < (double)rows)) {
            ++skipped;
            continue;
        }
        const int64_t q = (int64_t)fq;
        const int64_t cv = q - v0;
        if (cv < 0 || cv >= wv)
            continue;
        for (int32_t i = 0; i < support; ++i) {
            const int64_t cu = au.k_lo + i - u0;
            if (cu < 0 || cu >= wu)
                continue;
            const double wr = taps[au.t0 + (int64_t)i * beta];
            for (int32_t pol = 0; pol < npol; ++pol) {
                const double *V = vis + 2 * (r * npol + pol);
                double *G = out + 2 * (((int64_t)pol * wv + cv) * wu + cu);
                G[0] += wr * V[0];
                G[1] += wr * V[1];
            }
        }
    }
    return skipped;
}

/* Column pruning (Convolution-Based FFT Pruning of Algorithm "A General
 * Algorithm for Convolution-based FFT Pruning in one dimension", Section
 * 2.5.2, applied down every column, as the Column Pruner of Section 7.1):
 * each column of M = nrows values is circularly convolved with the pruning
 * kernel and downsampled by alpha,
 *   out[j] = sum_{s=0}^{Sz-1} sum_{a=0}^{alpha-1} c(alpha (s - Sz/2) + a)
 *            in[(alpha (j - Sz/2 + s) + a) mod M],   j = 0 .. M/alpha - 1,
 * with c(d) = ztaps[d + alpha Sz / 2], a table of alpha Sz + 1 real values
 * (entry e at offset (e - alpha Sz/2) / alpha output samples; the last entry
 * is not used).  in: complex128 [npol][M][ncols]; out: complex128
 * [npol][M / alpha][ncols], OVERWRITTEN.  Requires M divisible by alpha and
 * Sz even.  Returns 0 or ORC_EINVAL. */
int64_t orc_prune_columns(int32_t npol, int64_t nrows, int32_t ncols, int32_t alpha,
                          int32_t support_z, const double *ztaps, const double *in,
                          double *out)
{
    if (npol < 1 || nrows < 1 || ncols < 1 || alpha < 1 || support_z < 1 ||
        nrows % alpha || support_z % 2)
        return ORC_EINVAL;
    const int64_t nout = nrows / alpha;
    const int64_t half = (int64_t)alpha * support_z / 2;
    for (int32_t pol = 0; pol < npol; ++pol) {
        for (int64_t j = 0; j < nout; ++j) {
            for (int32_t col = 0; col < ncols; ++col) {
                double sr = 0.0, si = 0.0;
                for (int32_t s = 0; s < support_z; ++s) {
                    for (int32_t a = 0; a < alpha; ++a) {
                        const int64_t d = (int64_t)alpha * (s - support_z / 2) + a;
                        const double c = ztaps[d + half];
                        int64_t row = ((int64_t)alpha * (j - support_z / 2 + s) + a) % nrows;
                        if (row < 0)
                            row += nrows;
                        const double *x = in + 2 * (((int64_t)pol * nrows + row) * ncols + col);
                        sr += c * x[0];
                        si += c * x[1];
                    }
                }
                double *o = out + 2 * (((int64_t)pol * nout + j) * ncols + col);
                o[0] = sr;
                o[1] = si;
            }
        }
    }
    return 0;
}
