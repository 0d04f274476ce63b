/*
 * Plain float64 CPU oracle for the time-varying linear-prediction (all-pole)
 * filter and its adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the bench's CPU-baseline
 * leg do.  It shares no code with the HIP implementation.
 *
 * Every routine is the definition written out, sample by sample, in float64.
 * Inputs are float64 arrays: the Python wrapper promotes the float32 arrays the
 * GPU path reads exactly to float64 (finite-difference tests pass genuine
 * float64 perturbations instead).  IEEE round-to-nearest;
 * build without -ffast-math and with -ffp-contract=off.  OpenMP is used only
 * across independent sequences.
 *
 * Notation (paper, Sec. 3.2, time-varying LP):
 *   s(t) = e(t) - sum_{i=1..M} a_i(t) s(t-i),  e(t) = s(t) = 0 for t < 0,
 * with the coefficient row a(t) belonging to the OUTPUT time t.  Arrays are
 * row-major: e[b*T + t], a[(b*T + t)*M + (i-1)].  The optional initial state
 * zi[b*M + (j-1)] = s(-j), j = 1..M (most recent first) generalises the zero
 * initial conditions; zf has the same layout for s(T-j).
 */
#include <stddef.h>
#include <stdint.h>

/* Forward filter, Eq. (6): direct recursion over t = 0..T-1. */
void oracle_lp_forward(int64_t B, int64_t T, int M,
                       const double *e, const double *a, const double *zi,
                       double *s, double *zf)
{
    int64_t b;
#pragma omp parallel for schedule(dynamic, 1)
    for (b = 0; b < B; ++b) {
        const double *eb = e + b * T;
        const double *ab = a + b * T * (int64_t)M;
        double *sb = s + b * T;
        for (int64_t t = 0; t < T; ++t) {
            double acc = eb[t];
            for (int i = 1; i <= M; ++i) {
                double past;
                if (t - i >= 0)
                    past = sb[t - i];
                else
                    past = zi ? zi[b * M + (i - t - 1)] : 0.0;
                acc -= ab[t * M + (i - 1)] * past;
            }
            sb[t] = acc;
        }
        if (zf) {
            for (int j = 1; j <= M; ++j) {
                int64_t tt = T - j;
                zf[b * M + (j - 1)] = tt >= 0 ? sb[tt] : (zi ? zi[b * M + (j - T - 1)] : 0.0);
            }
        }
    }
}

/*
 * Adjoint, Eqs. (12)-(13).  With g(t) = dL/ds(t):
 *   ghat(t) = g(t) - sum_{i=1..M, t+i<T} a_i(t+i) ghat(t+i)    (t = T-1 .. 0)
 * i.e. the LP filter run backwards in time with the shifted coefficients
 * ahat_i(t) = a_i(t+i).  This is the "pull" form: each step reads the
 * diagonal a_1(t+1), a_2(t+2), ... .  Then
 *   dL/de(t)     = ghat(t)
 *   dL/da_i(t)   = -ghat(t) s(t-i)       (s(t-i) from zi, or 0, when t-i < 0)
 *   dL/dzi_j     = dL/ds(-j) = -sum_{i>=j} a_i(i-j) ghat(i-j)
 * s is the float64 forward output of oracle_lp_forward.  Any of grad_e,
 * grad_a, grad_zi may be NULL.  When grad_e is NULL, ghat_work (B*T doubles)
 * receives ghat instead; otherwise ghat_work may be NULL.
 */
void oracle_lp_backward(int64_t B, int64_t T, int M,
                        const double *g, const double *a, const double *zi,
                        const double *s, double *grad_e, double *grad_a,
                        double *grad_zi, double *ghat_work)
{
    int64_t b;
#pragma omp parallel for schedule(dynamic, 1)
    for (b = 0; b < B; ++b) {
        const double *gb = g + b * T;
        const double *ab = a + b * T * (int64_t)M;
        const double *sb = s + b * T;
        double *gh = grad_e ? grad_e + b * T : ghat_work + b * T;
        for (int64_t t = T - 1; t >= 0; --t) {
            double acc = gb[t];
            for (int i = 1; i <= M && t + i < T; ++i)
                acc -= ab[(t + i) * M + (i - 1)] * gh[t + i];
            gh[t] = acc;
        }
        if (grad_a) {
            double *gab = grad_a + b * T * (int64_t)M;
            for (int64_t t = 0; t < T; ++t) {
                for (int i = 1; i <= M; ++i) {
                    double past;
                    if (t - i >= 0)
                        past = sb[t - i];
                    else
                        past = zi ? zi[b * M + (i - t - 1)] : 0.0;
                    gab[t * M + (i - 1)] = -gh[t] * past;
                }
            }
        }
        if (grad_zi) {
            for (int j = 1; j <= M; ++j) {
                double acc = 0.0;
                for (int i = j; i <= M; ++i) {
                    int64_t t = i - j;
                    if (t < T)
                        acc -= ab[t * M + (i - 1)] * gh[t];
                }
                grad_zi[b * M + (j - 1)] = acc;
            }
        }
    }
}

/* Number of OpenMP threads the routines above use (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
