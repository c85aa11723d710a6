/*
 * Plain CPU oracle for the X-stage cross-multiply-accumulate.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this file: it is used by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, and nothing else.  It shares no code,
 * header, table or helper with the HIP library.
 *
 * What it computes (Sec. 1 and Sec. 2.4 of the paper): for every frequency
 * channel c the outer product of the vector of channelised voltages of all
 * inputs with its own conjugate, summed over the integration window,
 *
 *     V[c][i][j] = sum_t  x_i[c,t] * conj(x_j[c,t]),      i >= j,
 *
 * kept as the lower triangle including the autocorrelations (Sec. 2.4, the
 * output-size equation, reads the result as a lower-triangular matrix per
 * channel).  The paper integrates on the GPU and returns the integrated
 * matrix (Sec. 2.1, Sec. 4); the oracle returns exact integer sums.
 *
 * Arithmetic: plain int64, no blocking, no reordering beyond the definition.
 * Channels are independent, so the outer loop runs them in parallel (OpenMP).
 *
 * Input layout (one contiguous buffer, [channel][time][input]):
 *   fmt 0 (4+4 bit, Sec. 2.3): one byte per sample, high nibble = real part,
 *         low nibble = imaginary part, each a two's-complement 4-bit integer.
 *   fmt 1 (8+8 bit, the unpacked form of Sec. 2.4): two signed bytes per
 *         sample, real then imaginary.
 * Output layout: int64 pairs (re, im) at [channel][i*(i+1)/2 + j].
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Sign-extend a 4-bit two's-complement field. */
static int64_t xo_nibble(unsigned v)
{
    v &= 0xFu;
    return (v & 0x8u) ? (int64_t)v - 16 : (int64_t)v;
}

/* Decode sample number k of one time row into (re, im). */
static void xo_decode(const uint8_t* row, int fmt, int64_t k, int64_t* re, int64_t* im)
{
    if (fmt == 0) {
        unsigned b = row[k];
        *re = xo_nibble(b >> 4);
        *im = xo_nibble(b);
    } else {
        *re = (int64_t)(int8_t)row[2 * k];
        *im = (int64_t)(int8_t)row[2 * k + 1];
    }
}

int xo_version(void) { return 1; }

int xo_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Correlate channels [ch_begin, ch_begin + ch_count) of an input buffer that
 * holds n_ch channels of n_t samples of n_in inputs.  out receives ch_count
 * channels of n_in*(n_in+1)/2 (re, im) int64 pairs.  Returns 0, or -1 on a
 * bad argument.
 */
int xo_correlate(const void* in, int fmt, int64_t n_ch, int64_t n_t, int64_t n_in,
                 int64_t ch_begin, int64_t ch_count, int64_t* out)
{
    if (!in || !out || (fmt != 0 && fmt != 1) || n_ch < 0 || n_t < 0 || n_in <= 0 ||
        ch_begin < 0 || ch_count < 0 || ch_begin + ch_count > n_ch)
        return -1;
    const int64_t bps = (fmt == 0) ? 1 : 2;           /* bytes per sample */
    const int64_t n_b = n_in * (n_in + 1) / 2;         /* baselines incl. autos */
    const uint8_t* base = (const uint8_t*)in;

#pragma omp parallel
    {
        int64_t* re = (int64_t*)malloc((size_t)n_in * sizeof(int64_t));
        int64_t* im = (int64_t*)malloc((size_t)n_in * sizeof(int64_t));
#pragma omp for schedule(dynamic, 1)
        for (int64_t cc = 0; cc < ch_count; ++cc) {
            const int64_t c = ch_begin + cc;
            int64_t* acc = out + cc * n_b * 2;
            memset(acc, 0, (size_t)(n_b * 2) * sizeof(int64_t));
            for (int64_t t = 0; t < n_t; ++t) {
                const uint8_t* row = base + (c * n_t + t) * n_in * bps;
                for (int64_t k = 0; k < n_in; ++k)
                    xo_decode(row, fmt, k, &re[k], &im[k]);
                for (int64_t i = 0; i < n_in; ++i) {
                    int64_t* a = acc + (i * (i + 1) / 2) * 2;
                    const int64_t ar = re[i], ai = im[i];
                    for (int64_t j = 0; j <= i; ++j) {
                        /* (ar + i ai) * (re[j] - i im[j]) */
                        a[2 * j]     += ar * re[j] + ai * im[j];
                        a[2 * j + 1] += ai * re[j] - ar * im[j];
                    }
                }
            }
        }
        free(re);
        free(im);
    }
    return 0;
}

/*
 * Rows [row_begin, row_begin + row_count) of the triangle of one channel:
 * out receives, row after row, the entries (i, 0..i) as (re, im) int64 pairs
 * (sum over rows of (i + 1) pairs).  Same definition as xo_correlate, for
 * checking a sample of a channel too large to correlate whole; the rows are
 * shared out over the threads.  Returns 0, or -1 on a bad argument.
 */
int xo_correlate_rows(const void* in, int fmt, int64_t n_ch, int64_t n_t, int64_t n_in,
                      int64_t ch, int64_t row_begin, int64_t row_count, int64_t* out)
{
    if (!in || !out || (fmt != 0 && fmt != 1) || n_t < 0 || n_in <= 0 || ch < 0 || ch >= n_ch ||
        row_begin < 0 || row_count < 0 || row_begin + row_count > n_in)
        return -1;
    const int64_t bps = (fmt == 0) ? 1 : 2;
    const uint8_t* base = (const uint8_t*)in;
    /* first output pair of row i: sum_{r < i} (r + 1) - sum_{r < row_begin} (r + 1) */
    const int64_t first = row_begin * (row_begin + 1) / 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = row_begin; i < row_begin + row_count; ++i) {
        int64_t* acc = out + (i * (i + 1) / 2 - first) * 2;
        memset(acc, 0, (size_t)(i + 1) * 2 * sizeof(int64_t));
        for (int64_t t = 0; t < n_t; ++t) {
            const uint8_t* row = base + (ch * n_t + t) * n_in * bps;
            int64_t ar, ai;
            xo_decode(row, fmt, i, &ar, &ai);
            for (int64_t j = 0; j <= i; ++j) {
                int64_t br, bi;
                xo_decode(row, fmt, j, &br, &bi);
                acc[2 * j]     += ar * br + ai * bi;
                acc[2 * j + 1] += ai * br - ar * bi;
            }
        }
    }
    return 0;
}

/*
 * Beamformed power of every channel: for the complex integer weights w
 * (n_in (re, im) pairs, shared by all channels),
 *
 *     P[c] = sum_t | sum_i conj(w_i) * x_i[c,t] |^2 .
 *
 * Because V is the sum of outer products, P[c] equals the Hermitian form
 * w^H V[c] w; the tests use that identity to check a full-size visibility
 * set in O(n_in * n_t) work per channel.  Returns 0, or -1 on a bad argument.
 */
int xo_beam_power(const void* in, int fmt, int64_t n_ch, int64_t n_t, int64_t n_in,
                  const int64_t* w, int64_t* power)
{
    if (!in || !w || !power || (fmt != 0 && fmt != 1) || n_ch < 0 || n_t < 0 || n_in <= 0)
        return -1;
    const int64_t bps = (fmt == 0) ? 1 : 2;
    const uint8_t* base = (const uint8_t*)in;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < n_ch; ++c) {
        int64_t p = 0;
        for (int64_t t = 0; t < n_t; ++t) {
            const uint8_t* row = base + (c * n_t + t) * n_in * bps;
            int64_t yr = 0, yi = 0;
            for (int64_t k = 0; k < n_in; ++k) {
                int64_t a, b;
                xo_decode(row, fmt, k, &a, &b);
                const int64_t wr = w[2 * k], wi = w[2 * k + 1];
                /* (wr - i wi) * (a + i b) */
                yr += wr * a + wi * b;
                yi += wr * b - wi * a;
            }
            p += yr * yr + yi * yi;
        }
        power[c] = p;
    }
    return 0;
}
