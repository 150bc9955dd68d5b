/*
 * CPU FP64 direct correlation for the FDAS oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load this library.  It shares no code with the GPU path.
 *
 * What it computes is Eq. (1) of Dimoudi & Armour (Sec. 2), written out as a
 * plain sum with no FFT and no segmentation: for every template iz and output
 * bin k,
 *
 *     Y[iz][k] = sum_{q=-h}^{h} X[k - q] * T[iz][q],   X = 0 outside [0, nb)
 *     P[iz][k] = |Y[iz][k]|^2
 *
 * where X is the (normalised) complex spectrum and T[iz][q] the template taps
 * (already conjugated: Sec. 2 correlates with the complex conjugate of the
 * constant-acceleration response).  Output bin k plays the role of
 * the paper's reference frequency r0 and k - q that of its summation index.
 *
 * Layouts: complex arrays are interleaved (re, im) doubles; taps are
 * nz x (2h+1) complex, tap q stored at column q + h; the plane is nz x nb
 * doubles, row-major (template-major).
 */
#include <stdint.h>

static void corr_one(const double *spec, int64_t nb, const double *taps_row,
                     int32_t h, int64_t k, double *out_re, double *out_im)
{
    double yr = 0.0, yi = 0.0;
    for (int32_t q = -h; q <= h; ++q) {
        int64_t src = k - q;
        if (src < 0 || src >= nb)
            continue;
        double xr = spec[2 * src], xi = spec[2 * src + 1];
        double tr = taps_row[2 * (q + h)], ti = taps_row[2 * (q + h) + 1];
        yr += xr * tr - xi * ti;
        yi += xr * ti + xi * tr;
    }
    *out_re = yr;
    *out_im = yi;
}

/* Whole plane. */
void oracle_correlate_plane(const double *spec, int64_t nb, const double *taps,
                            int32_t nz, int32_t h, double *plane)
{
    const int64_t ntaps = 2 * (int64_t)h + 1;
#pragma omp parallel for collapse(2) schedule(static)
    for (int32_t iz = 0; iz < nz; ++iz) {
        for (int64_t k = 0; k < nb; ++k) {
            double yr, yi;
            corr_one(spec, nb, taps + 2 * ntaps * iz, h, k, &yr, &yi);
            plane[(int64_t)iz * nb + k] = yr * yr + yi * yi;
        }
    }
}

/* Selected cells (iz[c], k[c]) only: P and the complex Y. */
void oracle_correlate_cells(const double *spec, int64_t nb, const double *taps,
                            int32_t h, int64_t ncells, const int32_t *iz,
                            const int64_t *k, double *power, double *y)
{
    const int64_t ntaps = 2 * (int64_t)h + 1;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncells; ++c) {
        double yr, yi;
        corr_one(spec, nb, taps + 2 * ntaps * iz[c], h, k[c], &yr, &yi);
        power[c] = yr * yr + yi * yi;
        if (y) {
            y[2 * c] = yr;
            y[2 * c + 1] = yi;
        }
    }
}
