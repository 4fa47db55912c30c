/*
 * lbf_oracle.c -- plain, slow, FP64 reference of the tied-array beam former.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this code.  It shares no source, header,
 * helper or table with the GPU library, and the GPU library never calls it.
 *
 * What it computes follows Mol & Romein, "The LOFAR Beam Former: Implementation
 * and Performance Analysis":
 *
 *   delays     tau[b][s] = p_s . (u_b - u_ref) / c0 - delta_s  (Sec. 3, Sec. 4.3:
 *              weights depend on station location, channel frequency and
 *              tied-array beam coordinates; delta_s is the residual delay of
 *              station s left after its series was shifted by whole samples,
 *              Sec. 3, which the weights' phase compensates)
 *   weights    w[c][b][s] = exp(-2 pi i frac(f_c tau[b][s]))  (Sec. 3: the phase
 *              of each sample is shifted by a complex multiplication; the
 *              fractional turn is taken in FP64 because f*tau spans many turns)
 *   beam form  y[c][b][t][p] = sum_s w[c][b][s] x[s][c][t][p]  (Sec. 1, Sec. 3,
 *              Sec. 4.3: weighted addition of station signals, one weight set
 *              per beam, applied by complex multiply + add)
 *   Stokes     I = X conj X + Y conj Y, Q = X conj X - Y conj Y,
 *              U = 2 Re(X conj Y), V = 2 Im(X conj Y)           (Sec. 4.5)
 *   integrate  sum over t_int consecutive samples (Sec. 3, Sec. 5.1: integration
 *              factors 1..16) and over f_int adjacent channels
 *   reorder    out[b][k][t'][c'] -- one stream per beam and Stokes parameter
 *              (Sec. 4.6: beams split per polarisation / Stokes parameter and
 *              reordered into their final order)
 *   incoherent sum_s Stokes(x_s): unweighted accumulation of station powers
 *              (Sec. 3, incoherent beam)
 *
 * Every loop runs in the order written in the definitions above; the only
 * parallelism is independent channel groups handed to separate threads.
 * Complex numbers are stored as interleaved (re, im) doubles.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LBFO_C0 299792458.0
#define LBFO_PI 3.14159265358979323846

enum { LBFO_CI8 = 0, LBFO_CI16 = 1, LBFO_CF32 = 2 };

/* read x[s][c][t][p] as a complex double from the typed input array */
static void lbfo_sample(const void* x, int xtype, size_t idx, double* re, double* im)
{
    if (xtype == LBFO_CI8) {
        const int8_t* v = (const int8_t*)x;
        *re = (double)v[2 * idx];
        *im = (double)v[2 * idx + 1];
    } else if (xtype == LBFO_CI16) {
        const int16_t* v = (const int16_t*)x;
        *re = (double)v[2 * idx];
        *im = (double)v[2 * idx + 1];
    } else {
        const float* v = (const float*)x;
        *re = (double)v[2 * idx];
        *im = (double)v[2 * idx + 1];
    }
}

/* tau[b][s] = p_s . (u_b - u_ref) / c0 - resid[s] ; ref == NULL means u_ref = 0,
 * resid == NULL means no residual delays.  A station whose signal arrives
 * resid[s] seconds late needs its phase advanced by 2 pi f resid[s]: the
 * weight exp(-2 pi i f tau) does that with the residual subtracted. */
void lbfo_delays(const double* pos, int S, const double* dir, int B, const double* ref, const double* resid,
                 double* tau)
{
    for (int b = 0; b < B; ++b) {
        double d[3];
        for (int k = 0; k < 3; ++k)
            d[k] = dir[3 * b + k] - (ref ? ref[k] : 0.0);
        for (int s = 0; s < S; ++s) {
            double proj = pos[3 * s + 0] * d[0] + pos[3 * s + 1] * d[1] + pos[3 * s + 2] * d[2];
            tau[(size_t)b * S + s] = proj / LBFO_C0 - (resid ? resid[s] : 0.0);
        }
    }
}

/* w[c][b][s] = cos(2 pi r) - i sin(2 pi r), r = m - rint(m), m = f_c tau[b][s] */
void lbfo_weights(const double* tau, int B, int S, const double* freq, int C, double* w)
{
    for (int c = 0; c < C; ++c)
        for (int b = 0; b < B; ++b)
            for (int s = 0; s < S; ++s) {
                double m = freq[c] * tau[(size_t)b * S + s];
                double r = m - rint(m);
                size_t o = (((size_t)c * B + b) * S + s) * 2;
                w[o] = cos(2.0 * LBFO_PI * r);
                w[o + 1] = -sin(2.0 * LBFO_PI * r);
            }
}

/* y[c][b][t][p] = sum_{s=0}^{S-1} w[c][b][s] * x[s][c][t][p], in station order,
 * for the nc channels starting at c_lo of an input holding C channels.
 * w and y are indexed from channel c_lo: w[nc][B][S], y[nc][B][T][2]. */
void lbfo_beamform(const void* x, int xtype, int S, int C, int T, int c_lo, int nc,
                   const double* w, int B, double* y)
{
    for (int dc = 0; dc < nc; ++dc)
        for (int b = 0; b < B; ++b)
            for (int t = 0; t < T; ++t)
                for (int p = 0; p < 2; ++p) {
                    double yr = 0.0, yi = 0.0;
                    for (int s = 0; s < S; ++s) {
                        size_t wo = (((size_t)dc * B + b) * S + s) * 2;
                        double wr = w[wo], wi = w[wo + 1];
                        double xr, xi;
                        lbfo_sample(x, xtype, (((size_t)s * C + c_lo + dc) * T + t) * 2 + p, &xr, &xi);
                        yr += wr * xr - wi * xi;
                        yi += wr * xi + wi * xr;
                    }
                    size_t yo = ((((size_t)dc * B + b) * T + t) * 2 + p) * 2;
                    y[yo] = yr;
                    y[yo + 1] = yi;
                }
}

/* st[c][b][t][4] = (I, Q, U, V) from X = y[..][0], Y = y[..][1] */
void lbfo_stokes(const double* y, int C, int B, int T, double* st)
{
    size_t n = (size_t)C * B * T;
    for (size_t i = 0; i < n; ++i) {
        double xr = y[4 * i + 0], xi = y[4 * i + 1];
        double yr = y[4 * i + 2], yi = y[4 * i + 3];
        double xx = xr * xr + xi * xi;          /* X conj(X) */
        double yy = yr * yr + yi * yi;          /* Y conj(Y) */
        double xy_re = xr * yr + xi * yi;       /* Re(X conj(Y)) */
        double xy_im = xi * yr - xr * yi;       /* Im(X conj(Y)) */
        st[4 * i + 0] = xx + yy;
        st[4 * i + 1] = xx - yy;
        st[4 * i + 2] = 2.0 * xy_re;
        st[4 * i + 3] = 2.0 * xy_im;
    }
}

/* s[c'][b][t'][k] = sum_{c in group c'} sum_{t in group t'} st[c][b][t][k]
 * for the first K Stokes parameters (K = 1: I only; K = 4: IQUV). */
void lbfo_integrate(const double* st, int C, int B, int T, int K, int t_int, int f_int, double* s)
{
    int C2 = C / f_int, T2 = T / t_int;
    for (int c2 = 0; c2 < C2; ++c2)
        for (int b = 0; b < B; ++b)
            for (int t2 = 0; t2 < T2; ++t2)
                for (int k = 0; k < K; ++k) {
                    double acc = 0.0;
                    for (int dc = 0; dc < f_int; ++dc)
                        for (int dt = 0; dt < t_int; ++dt) {
                            int c = c2 * f_int + dc, t = t2 * t_int + dt;
                            acc += st[(((size_t)c * B + b) * T + t) * 4 + k];
                        }
                    s[(((size_t)c2 * B + b) * T2 + t2) * K + k] = acc;
                }
}

/* out[b][k][t'][c'] = s[c'][b][t'][k]; elem = 1 for real, 2 for complex values */
void lbfo_reorder(const double* s, int C2, int B, int T2, int K, int elem, double* out)
{
    for (int c2 = 0; c2 < C2; ++c2)
        for (int b = 0; b < B; ++b)
            for (int t2 = 0; t2 < T2; ++t2)
                for (int k = 0; k < K; ++k)
                    for (int e = 0; e < elem; ++e)
                        out[((((size_t)b * K + k) * T2 + t2) * C2 + c2) * elem + e] =
                            s[((((size_t)c2 * B + b) * T2 + t2) * K + k) * elem + e];
}

/* incoherent beam: inc[c'][t'][k] = sum over the groups of sum_s Stokes_k(x_s[c][t]) */
void lbfo_incoherent(const void* x, int xtype, int S, int C, int T, int K, int t_int, int f_int,
                     double* inc)
{
    int C2 = C / f_int, T2 = T / t_int;
    for (int c2 = 0; c2 < C2; ++c2)
        for (int t2 = 0; t2 < T2; ++t2)
            for (int k = 0; k < K; ++k) {
                double acc = 0.0;
                for (int dc = 0; dc < f_int; ++dc)
                    for (int dt = 0; dt < t_int; ++dt)
                        for (int s = 0; s < S; ++s) {
                            int c = c2 * f_int + dc, t = t2 * t_int + dt;
                            double xr, xi, yr, yi;
                            size_t base = (((size_t)s * C + c) * T + t) * 2;
                            lbfo_sample(x, xtype, base + 0, &xr, &xi);
                            lbfo_sample(x, xtype, base + 1, &yr, &yi);
                            double xx = xr * xr + xi * xi, yy = yr * yr + yi * yi;
                            double v;
                            if (k == 0) v = xx + yy;
                            else if (k == 1) v = xx - yy;
                            else if (k == 2) v = 2.0 * (xr * yr + xi * yi);
                            else v = 2.0 * (xi * yr - xr * yi);
                            acc += v;
                        }
                inc[((size_t)c2 * T2 + t2) * K + k] = acc;
            }
}

/* ------------------------------------------------------------------------ */
/* The whole chain over all channels, split into channel groups run on
 * separate threads: delays -> weights -> beam form -> Stokes -> integrate ->
 * reorder.  K = 0 returns voltages reordered to [b][p][t][c] (complex). */

typedef struct {
    const void* x; int xtype; int S, C, T, B, K, t_int, f_int;
    const double* tau; const double* freq;
    double* out; int g_lo, g_hi;
} lbfo_job;

static void* lbfo_worker(void* arg)
{
    lbfo_job* j = (lbfo_job*)arg;
    int S = j->S, C = j->C, T = j->T, B = j->B, f_int = j->f_int;
    int T2 = j->K ? T / j->t_int : T, C2 = C / f_int;
    double* w = (double*)malloc(sizeof(double) * 2 * (size_t)f_int * B * S);
    double* y = (double*)malloc(sizeof(double) * 4 * (size_t)f_int * B * T);
    double* st = (double*)malloc(sizeof(double) * 4 * (size_t)f_int * B * T);
    double* s = (double*)malloc(sizeof(double) * 4 * (size_t)B * T);
    for (int g = j->g_lo; g < j->g_hi; ++g) {
        int c0 = g * f_int;
        /* weights and voltages of this group's f_int channels, indexed from 0 */
        lbfo_weights(j->tau, B, S, j->freq + c0, f_int, w);
        lbfo_beamform(j->x, j->xtype, S, C, T, c0, f_int, w, B, y);
        if (j->K == 0) {
            for (int b = 0; b < B; ++b)
                for (int p = 0; p < 2; ++p)
                    for (int t = 0; t < T; ++t) {
                        size_t o = ((((size_t)b * 2 + p) * T + t) * C + c0) * 2;
                        size_t i = ((((size_t)0 * B + b) * T + t) * 2 + p) * 2;
                        j->out[o] = y[i];
                        j->out[o + 1] = y[i + 1];
                    }
            continue;
        }
        lbfo_stokes(y, f_int, B, T, st);
        lbfo_integrate(st, f_int, B, T, j->K, j->t_int, f_int, s);
        for (int b = 0; b < B; ++b)
            for (int k = 0; k < j->K; ++k)
                for (int t2 = 0; t2 < T2; ++t2)
                    j->out[(((size_t)b * j->K + k) * T2 + t2) * C2 + g] =
                        s[((size_t)b * T2 + t2) * j->K + k];
    }
    free(w); free(y); free(st); free(s);
    return NULL;
}

/* out: K > 0 -> [B][K][T/t_int][C/f_int] doubles; K == 0 -> voltages
 * [B][2][T][C] complex (f_int must then be 1).  Returns 0, or -1 on bad args. */
int lbfo_pipeline(const void* x, int xtype, int S, int C, int T, const double* pos,
                  const double* dir, int B, const double* ref, const double* resid, const double* freq,
                  int K, int t_int, int f_int, int nthreads, double* out)
{
    if (S < 1 || C < 1 || T < 1 || B < 1 || t_int < 1 || f_int < 1) return -1;
    if (C % f_int || (K && T % t_int) || (K == 0 && f_int != 1)) return -1;
    if (K != 0 && K != 1 && K != 4) return -1;
    double* tau = (double*)malloc(sizeof(double) * (size_t)B * S);
    lbfo_delays(pos, S, dir, B, ref, resid, tau);
    int G = C / f_int;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > G) nthreads = G;
    pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * nthreads);
    lbfo_job* jobs = (lbfo_job*)malloc(sizeof(lbfo_job) * nthreads);
    for (int i = 0; i < nthreads; ++i) {
        lbfo_job jb = { x, xtype, S, C, T, B, K, t_int, f_int, tau, freq, out,
                        (int)((long)G * i / nthreads), (int)((long)G * (i + 1) / nthreads) };
        jobs[i] = jb;
        pthread_create(&th[i], NULL, lbfo_worker, &jobs[i]);
    }
    for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
    free(th); free(jobs); free(tau);
    return 0;
}
