/*
 * FP64 CPU oracle for batched complex discrete Fourier transforms.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
 * Python binding) may include, link, load or call this file.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg use it.  It
 * shares no code, header, table or constant with the GPU path.
 *
 * What it computes follows the paper's "FFT Basics" subsection (Background):
 *   X(k) = sum_{n=0}^{N-1} x(n) * w_N^{n k},  w_N = exp(-2 i pi / N)   (forward)
 * and the backward transform is the same sum with the sign of the exponent
 * flipped.  No normalisation is applied in either direction (the paper only
 * flips the sign; the unnormalised reading is the one the tests pin).
 *
 * Pieces:
 *   oracle_dft_naive   - the definition written out, O(N^2), any N >= 1.
 *   oracle_fft_radix2  - recursive radix-2 decimation in time, N a power of two.
 *   oracle_fft_mixed   - recursive smallest-prime-factor decimation in time,
 *                        any N >= 1 (prime lengths fall back to the definition).
 *   oracle_fft2d       - separable 2-D transform: every row, then every column.
 *   oracle_transpose   - out[b][c][r] = in[b][r][c].
 *   oracle_range_compress - the matched filter of SAR range compression: the
 *                        circular cross-correlation of every row with the
 *                        transmitted pulse replica (definition, O(n L)).
 *
 * Data: interleaved (re, im) doubles, batch-major [batch][n].  The `sign`
 * argument is the sign of the exponent: -1 forward, +1 backward.
 * `threads` <= 0 means one thread per online CPU.
 *
 * All arithmetic is IEEE double; build without -ffast-math.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

typedef struct { double re, im; } cplx;

static const double PI_QUARTER = 0.78539816339744830961566084581987572; /* pi/4 */

/*
 * exp(sign * 2 pi i * m / n), computed by octant reduction so that the angle
 * handed to cos/sin is at most pi/4 and the values at multiples of a quarter
 * turn are exact (1, +-i, -1).  m may be any integer; it is reduced mod n.
 * Used by the definition (O1) and the mixed-radix recursion.
 */
static cplx unit_root(int64_t m, int64_t n, int sign)
{
    int64_t r = m % n;
    if (r < 0) r += n;
    /* angle = 2 pi r / n = (pi/4) * (8 r / n).  a = 8 r; quarter h = a / (2n). */
    int64_t a = 8 * r;
    int64_t h = a / (2 * n);            /* 0..3 : completed quarter turns */
    int64_t u = a - h * 2 * n;          /* 0 <= u < 2n : position in the quarter, in units of (pi/4)/n */
    double c, s;
    if (u <= n) {
        double phi = PI_QUARTER * ((double)u / (double)n);
        c = cos(phi); s = sin(phi);
    } else {
        double phi = PI_QUARTER * ((double)(2 * n - u) / (double)n);
        c = sin(phi); s = cos(phi);
    }
    if (u == 0) { c = 1.0; s = 0.0; }
    double cr, sr;
    switch (h) {
        case 0: cr = c;  sr = s;  break;
        case 1: cr = -s; sr = c;  break;
        case 2: cr = -c; sr = -s; break;
        default: cr = s; sr = -c; break;
    }
    cplx w = { cr, sign < 0 ? -sr : sr };
    return w;
}

static inline cplx cmul(cplx a, cplx b)
{
    cplx r = { a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re };
    return r;
}

/* ---------------------------------------------------------------- O1 ---- */
/* The definition: X[k] = sum_n x[n] * W[(n k) mod N], summed in order n = 0..N-1. */
static void dft_one(const cplx* x, cplx* X, int64_t n, int sign, const cplx* W)
{
    for (int64_t k = 0; k < n; ++k) {
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            int64_t m = (int64_t)(((unsigned __int128)j * (unsigned __int128)k) % (unsigned __int128)n);
            cplx p = cmul(x[j], W[m]);
            sr += p.re; si += p.im;
        }
        X[k].re = sr; X[k].im = si;
    }
}

static cplx* root_table(int64_t n, int sign)
{
    cplx* W = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    if (!W) return NULL;
    for (int64_t m = 0; m < n; ++m) W[m] = unit_root(m, n, sign);
    return W;
}

/* --------------------------------------------------------------- O2 ---- */
/*
 * Radix-2 decimation in time.  The even samples and the odd samples are each
 * transformed (length n/2, written to out[0..n/2) and out[n/2..n)), then
 *   X[k]       = E[k] + w^k O[k]
 *   X[k + n/2] = E[k] - w^k O[k],   w = exp(sign 2 pi i / n).
 * The twiddle w^k is taken straight from cos/sin of 2 pi k / n, a different
 * route from unit_root(), so that agreement between O1 and O2 checks both.
 */
static void radix2_rec(const cplx* in, int64_t stride, int64_t n, cplx* out, int sign)
{
    if (n == 1) { out[0] = in[0]; return; }
    int64_t h = n / 2;
    radix2_rec(in, 2 * stride, h, out, sign);
    radix2_rec(in + stride, 2 * stride, h, out + h, sign);
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t k = 0; k < h; ++k) {
        double ang = two_pi * (double)k / (double)n;
        cplx w = { cos(ang), sign < 0 ? -sin(ang) : sin(ang) };
        cplx e = out[k];
        cplx o = cmul(w, out[k + h]);
        out[k].re = e.re + o.re;     out[k].im = e.im + o.im;
        out[k + h].re = e.re - o.re; out[k + h].im = e.im - o.im;
    }
}

/* --------------------------------------------------------------- O3 ---- */
static int64_t smallest_factor(int64_t n)
{
    if (n % 2 == 0) return 2;
    for (int64_t p = 3; p * p <= n; p += 2)
        if (n % p == 0) return p;
    return n;
}

/*
 * Smallest-prime-factor decimation in time: n = p * M,
 *   F_r = DFT_M(x[r], x[r+p], x[r+2p], ...),  r = 0..p-1
 *   X[k] = sum_r exp(sign 2 pi i r k / n) * F_r[k mod M].
 * A prime n is the definition itself.  `tmp` holds n values.
 */
static void mixed_rec(const cplx* in, int64_t stride, int64_t n, cplx* out, int sign, cplx* tmp)
{
    if (n == 1) { out[0] = in[0]; return; }
    int64_t p = smallest_factor(n);
    if (p == n) {
        /* prime length: the definition on a gathered copy */
        cplx* g = tmp;
        for (int64_t j = 0; j < n; ++j) g[j] = in[j * stride];
        for (int64_t k = 0; k < n; ++k) {
            double sr = 0.0, si = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                cplx w = unit_root((j * k) % n, n, sign);
                cplx q = cmul(g[j], w);
                sr += q.re; si += q.im;
            }
            out[k].re = sr; out[k].im = si;
        }
        return;
    }
    int64_t M = n / p;
    /* sub-transforms into tmp[r*M .. r*M+M), using out as their scratch */
    for (int64_t r = 0; r < p; ++r)
        mixed_rec(in + r * stride, stride * p, M, tmp + r * M, sign, out);
    for (int64_t k = 0; k < n; ++k) {
        double sr = 0.0, si = 0.0;
        for (int64_t r = 0; r < p; ++r) {
            cplx w = unit_root(r * k, n, sign);
            cplx q = cmul(w, tmp[r * M + (k % M)]);
            sr += q.re; si += q.im;
        }
        out[k].re = sr; out[k].im = si;
    }
}

/* ------------------------------------------------------- thread pool ---- */
typedef struct {
    int kind;               /* 0 naive, 1 radix2, 2 mixed */
    const cplx* in;
    cplx* out;
    int64_t n;
    int64_t first, last;    /* transform range [first, last) */
    int64_t in_stride;      /* element distance between samples of one transform */
    int64_t in_dist;        /* element distance between transforms (input) */
    int64_t out_stride;
    int64_t out_dist;
    int sign;
    const cplx* W;          /* naive only */
    int status;
} job_t;

static void* run_job(void* arg)
{
    job_t* j = (job_t*)arg;
    int64_t n = j->n;
    cplx* xin = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    cplx* xout = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    cplx* tmp = (cplx*)malloc(sizeof(cplx) * (size_t)n);
    if (!xin || !xout || !tmp) { j->status = 1; free(xin); free(xout); free(tmp); return NULL; }
    for (int64_t b = j->first; b < j->last; ++b) {
        const cplx* src = j->in + b * j->in_dist;
        for (int64_t i = 0; i < n; ++i) xin[i] = src[i * j->in_stride];
        if (j->kind == 0) dft_one(xin, xout, n, j->sign, j->W);
        else if (j->kind == 1) radix2_rec(xin, 1, n, xout, j->sign);
        else mixed_rec(xin, 1, n, xout, j->sign, tmp);
        cplx* dst = j->out + b * j->out_dist;
        for (int64_t i = 0; i < n; ++i) dst[i * j->out_stride] = xout[i];
    }
    free(xin); free(xout); free(tmp);
    j->status = 0;
    return NULL;
}

static int resolve_threads(int threads, int64_t work)
{
    if (threads <= 0) {
        long c = sysconf(_SC_NPROCESSORS_ONLN);
        threads = c > 0 ? (int)c : 1;
    }
    if (threads > 256) threads = 256;
    if ((int64_t)threads > work) threads = (int)(work > 0 ? work : 1);
    return threads;
}

static int run_batch(int kind, const cplx* in, cplx* out, int64_t n, int64_t count,
                     int64_t in_stride, int64_t in_dist, int64_t out_stride, int64_t out_dist,
                     int sign, int threads)
{
    if (n < 1 || count < 0 || (sign != -1 && sign != 1)) return 1;
    if (count == 0) return 0;
    cplx* W = NULL;
    if (kind == 0) { W = root_table(n, sign); if (!W) return 1; }
    int T = resolve_threads(threads, count);
    job_t* jobs = (job_t*)calloc((size_t)T, sizeof(job_t));
    pthread_t* tid = (pthread_t*)calloc((size_t)T, sizeof(pthread_t));
    if (!jobs || !tid) { free(jobs); free(tid); free(W); return 1; }
    int64_t per = count / T, extra = count % T, at = 0;
    for (int t = 0; t < T; ++t) {
        int64_t c = per + (t < extra ? 1 : 0);
        job_t jb = { kind, in, out, n, at, at + c, in_stride, in_dist, out_stride, out_dist, sign, W, 0 };
        jobs[t] = jb;
        at += c;
    }
    int rc = 0;
    for (int t = 1; t < T; ++t)
        if (pthread_create(&tid[t], NULL, run_job, &jobs[t]) != 0) { jobs[t].status = -1; run_job(&jobs[t]); }
    run_job(&jobs[0]);
    for (int t = 1; t < T; ++t) if (jobs[t].status != -1) pthread_join(tid[t], NULL);
    for (int t = 0; t < T; ++t) if (jobs[t].status > 0) rc = 1;
    free(jobs); free(tid); free(W);
    return rc;
}

static int is_pow2(int64_t n) { return n >= 1 && (n & (n - 1)) == 0; }

/* ------------------------------------------------------------ exports ---- */
int oracle_dft_naive(const double* in, double* out, int64_t n, int64_t batch, int sign, int threads)
{
    return run_batch(0, (const cplx*)in, (cplx*)out, n, batch, 1, n, 1, n, sign, threads);
}

int oracle_fft_radix2(const double* in, double* out, int64_t n, int64_t batch, int sign, int threads)
{
    if (!is_pow2(n)) return 2;
    return run_batch(1, (const cplx*)in, (cplx*)out, n, batch, 1, n, 1, n, sign, threads);
}

int oracle_fft_mixed(const double* in, double* out, int64_t n, int64_t batch, int sign, int threads)
{
    return run_batch(2, (const cplx*)in, (cplx*)out, n, batch, 1, n, 1, n, sign, threads);
}

/*
 * 2-D transform of `batch` matrices of rows x cols: the 1-D transform of
 * every row (length cols), then of every column (length rows).  Exact by
 * separability of the double sum.  Uses radix-2 for powers of two, the
 * mixed-radix recursion otherwise.  `out` may equal `in`.
 */
int oracle_fft2d(const double* in, double* out, int64_t rows, int64_t cols, int64_t batch,
                 int sign, int threads)
{
    if (rows < 1 || cols < 1 || batch < 1) return 1;
    const cplx* ci = (const cplx*)in;
    cplx* co = (cplx*)out;
    for (int64_t b = 0; b < batch; ++b) {
        const cplx* src = ci + b * rows * cols;
        cplx* dst = co + b * rows * cols;
        int kr = is_pow2(cols) ? 1 : 2, kc = is_pow2(rows) ? 1 : 2;
        if (run_batch(kr, src, dst, cols, rows, 1, cols, 1, cols, sign, threads)) return 1;
        if (run_batch(kc, dst, dst, rows, cols, cols, 1, cols, 1, sign, threads)) return 1;
    }
    return 0;
}

/* out[b][c][r] = in[b][r][c] on complex values; out must not overlap in. */
int oracle_transpose(const double* in, double* out, int64_t rows, int64_t cols, int64_t batch)
{
    if (rows < 1 || cols < 1 || batch < 1) return 1;
    const cplx* ci = (const cplx*)in;
    cplx* co = (cplx*)out;
    for (int64_t b = 0; b < batch; ++b)
        for (int64_t r = 0; r < rows; ++r)
            for (int64_t c = 0; c < cols; ++c)
                co[b * rows * cols + c * rows + r] = ci[b * rows * cols + r * cols + c];
    return 0;
}

/*
 * Range compression, the first step of the range-Doppler chain after the
 * range FFT (SAR application section, Fig. 3): each received row is
 * correlated with the transmitted pulse replica ref[0..L).  Done with
 * transforms it is B(F(x) .* conj(F(ref zero-padded to n))); with the
 * unnormalised backward transform that product reaches exactly
 *     y[m] = n * sum_{l<L} x[(m + l) mod n] * conj(ref[l]),   0 <= m < n,
 * (the n is the 1/n the backward transform leaves out), which is what this
 * evaluates, directly and in FP64, for `rows` rows of length n; rows are
 * split over threads.  `out` must not overlap `in`.
 */
typedef struct {
    const cplx* in;
    cplx* out;
    const cplx* ref;
    int64_t n, L, first, last;
} xc_job_t;

static void* xc_run(void* arg)
{
    xc_job_t* j = (xc_job_t*)arg;
    for (int64_t b = j->first; b < j->last; ++b) {
        const cplx* x = j->in + b * j->n;
        cplx* y = j->out + b * j->n;
        for (int64_t m = 0; m < j->n; ++m) {
            double re = 0.0, im = 0.0;
            for (int64_t l = 0; l < j->L; ++l) {
                const cplx a = x[(m + l) % j->n];
                const cplx r = j->ref[l];
                /* a * conj(r) */
                re += a.re * r.re + a.im * r.im;
                im += a.im * r.re - a.re * r.im;
            }
            y[m].re = (double)j->n * re;
            y[m].im = (double)j->n * im;
        }
    }
    return NULL;
}

int oracle_range_compress(const double* in, double* out, int64_t n, int64_t rows, const double* ref,
                          int64_t L, int threads)
{
    if (n < 1 || rows < 0 || L < 1 || L > n) return 1;
    if (rows == 0) return 0;
    int T = resolve_threads(threads, rows);
    xc_job_t* jobs = (xc_job_t*)calloc((size_t)T, sizeof(xc_job_t));
    pthread_t* tid = (pthread_t*)calloc((size_t)T, sizeof(pthread_t));
    int* started = (int*)calloc((size_t)T, sizeof(int));
    if (!jobs || !tid || !started) { free(jobs); free(tid); free(started); return 1; }
    int64_t per = rows / T, extra = rows % T, at = 0;
    for (int t = 0; t < T; ++t) {
        int64_t c = per + (t < extra ? 1 : 0);
        xc_job_t jb = { (const cplx*)in, (cplx*)out, (const cplx*)ref, n, L, at, at + c };
        jobs[t] = jb;
        at += c;
    }
    for (int t = 1; t < T; ++t) {
        started[t] = pthread_create(&tid[t], NULL, xc_run, &jobs[t]) == 0;
        if (!started[t]) xc_run(&jobs[t]);
    }
    xc_run(&jobs[0]);
    for (int t = 1; t < T; ++t) if (started[t]) pthread_join(tid[t], NULL);
    free(jobs); free(tid); free(started);
    return 0;
}

/* The root used by O1, exposed so tests can pin it against closed forms. */
void oracle_unit_root(int64_t m, int64_t n, int sign, double* re_im)
{
    cplx w = unit_root(m, n, sign);
    re_im[0] = w.re; re_im[1] = w.im;
}

int oracle_nthreads(void) { return resolve_threads(0, 1 << 30); }
