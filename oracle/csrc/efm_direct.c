/*
 * Plain FP64 evaluation of the entropic collision term in Fourier space.
 *
 * TEST INFRASTRUCTURE ONLY: called by tests/ and by the CPU-baseline leg of
 * bench.py, never by the product library.
 *
 * It writes out the definition of the entropic collision term, section 3.2.2,
 * eq. Qsk, split into gain and loss as in section 3.1.2:
 *
 *   G_k = sum_{l in K} B^s(l, k (-) l)            Fh_l Fh_{k (-) l}
 *   L_k = sum_{l in K} B^s(k (-) l, k (-) l)      Fh_l Fh_{k (-) l}
 *
 * where (-) is the difference taken modulo N in every component (the mode
 * arrays are stored in FFT index order, so an index difference mod N is the
 * symmetric-mod difference of the modes), and the filtered low-rank kernel of
 * section 4.1 (eq. fastAlg and the filtered form that follows it) is
 *
 *   B^s(l, m) = sig_l sig_m sum_t c_t U_t(l) V_t(m).
 *
 * Nothing is blocked, fused or reordered: one output mode per outer iteration
 * (OpenMP over k), one compensated (Neumaier) sum over l per output.
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>

typedef struct { double s, c; } nsum;

static inline void nadd(nsum* a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else                       a->c += (x - t) + a->s;
    a->s = t;
}

static inline int64_t sub_index(int64_t k, int64_t l, int d, int N)
{
    /* index of the mode (k - l) mod N, component-wise, C order, last axis fastest */
    int64_t out = 0, stride = 1;
    for (int i = 0; i < d; ++i) {
        int64_t kc = k % N, lc = l % N;
        k /= N; l /= N;
        int64_t m = (kc - lc) % N;
        if (m < 0) m += N;
        out += m * stride;
        stride *= N;
    }
    return out;
}

/* U, V: [n][T] row-major (all terms of one mode contiguous).
 * c: [T].  sig: [n].  Fr, Fi: [n] real/imag parts of Fh (normalised DFT).
 * Outputs Gr, Gi, Lr, Li: [n] gain and loss Fourier coefficients. */
void efm_direct_sum(int d, int N, int T,
                    const double* c, const double* U, const double* V,
                    const double* sig, const double* Fr, const double* Fi,
                    double* Gr, double* Gi, double* Lr, double* Li)
{
    int64_t n = 1;
    for (int i = 0; i < d; ++i) n *= N;

    /* B^s(m, m): the diagonal the loss term needs */
    double* diag = (double*)malloc(sizeof(double) * (size_t)n);
    if (!diag) return;
    for (int64_t m = 0; m < n; ++m) {
        double acc = 0.0;
        for (int t = 0; t < T; ++t) acc += c[t] * U[m * T + t] * V[m * T + t];
        diag[m] = sig[m] * sig[m] * acc;
    }

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n; ++k) {
        nsum gr = {0, 0}, gi = {0, 0}, lr = {0, 0}, li = {0, 0};
        for (int64_t l = 0; l < n; ++l) {
            int64_t m = sub_index(k, l, d, N);
            double b = 0.0;
            const double* ul = U + l * T;
            const double* vm = V + m * T;
            for (int t = 0; t < T; ++t) b += c[t] * ul[t] * vm[t];
            b *= sig[l] * sig[m];
            double pr = Fr[l] * Fr[m] - Fi[l] * Fi[m];
            double pi = Fr[l] * Fi[m] + Fi[l] * Fr[m];
            nadd(&gr, b * pr);       nadd(&gi, b * pi);
            nadd(&lr, diag[m] * pr); nadd(&li, diag[m] * pi);
        }
        Gr[k] = gr.s + gr.c; Gi[k] = gi.s + gi.c;
        Lr[k] = lr.s + lr.c; Li[k] = li.s + li.c;
    }
    free(diag);
}
