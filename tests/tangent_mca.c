/* Monte Carlo arithmetic evaluation of Milstein paths and their forward-mode
 * derivatives -- test infrastructure (see tangent_binary32.py).
 *
 * Evaluates, per path, the discounted payoff of a European or arithmetic-
 * average Asian option under the Heston model's Milstein scheme (full
 * truncation or absorption) and its derivatives with respect to
 * (S0, v0, r, kappa, theta, sigma, rho), in a working precision W (binary32
 * or binary64).  Each operation is evaluated in a wider type, its result
 * multiplied by (1 + xi u) with xi uniform in [-1, 1] and u the unit roundoff
 * of W (Monte Carlo arithmetic, Parker 1997), then rounded to W.  With
 * seed 0 nothing is perturbed: a plain round-to-nearest evaluation.
 *
 * The random inputs are the two normals of every step, passed in; the
 * perturbations come from a per-path splitmix64 stream of (seed, path), so the
 * result does not depend on the thread count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <string.h>

typedef struct {
    double S0, K, r, T, v0, kappa, theta, sigma, rho;
} tm_params;

#define SIN_COS_ABS 1.3e-7 /* absolute accuracy of binary32 sin/cos of an angle in revolutions */

static uint64_t splitmix(uint64_t *s)
{
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* uniform in [-1, 1) */
static double xi(uint64_t *s) { return (double)(splitmix(s) >> 11) * 0x1p-52 - 1.0; }

typedef struct {
    const tm_params *P;
    int type, absorb, single;
    uint32_t N;
    const uint8_t *fix;
    const double *za, *zb;
    uint64_t n, seed, lo, hi;
    double *out;
} tm_job;

/* One path in working type T with wide type X; R(x, ulps) rounds a wide
 * value (perturbed unless seed == 0).                                       */
#define TM_PATH(NAME, WT, XT, U, SINCOS, SQRT, EXP)                                                \
    static void NAME(const tm_job *jb, uint64_t i)                                                 \
    {                                                                                              \
        const tm_params *P = jb->P;                                                                \
        uint64_t st = jb->seed * 0xD1B54A32D192ED03ull ^ (i + 1) * 0x9E3779B97F4A7C15ull;          \
        const int mca = jb->seed != 0;                                                             \
        const uint32_t N = jb->N;                                                                  \
        const double dt = P->T / (double)N;                                                        \
        const double rbar = sqrt(1.0 - P->rho * P->rho);                                           \
        const WT c_dt = (WT)dt, c_rho = (WT)P->rho, c_rbar = (WT)rbar;                             \
        const WT c_drbar = (WT)(-P->rho / rbar), c_hdt = (WT)(0.5 * dt);                           \
        const WT c_mkdt = (WT)(-P->kappa * dt), c_kth = (WT)(P->kappa * P->theta * dt);            \
        const WT c_sig = (WT)P->sigma, c_qs2dt = (WT)(0.25 * P->sigma * P->sigma * dt);            \
        const WT c_hs2dt = (WT)(0.5 * P->sigma * P->sigma * dt), c_r = (WT)P->r;                   \
        const WT c_kdt = (WT)(P->kappa * dt), c_hsdt = (WT)(0.5 * P->sigma * dt);                  \
        const WT c_th = (WT)P->theta, c_mhdt = (WT)(-0.5) * c_dt;                                  \
        WT S = (WT)P->S0, V = (WT)P->v0, A = 0;                                                    \
        WT dS[7] = { 0 }, dV[7] = { 0 }, dA[7] = { 0 };                                            \
        double amp = 0.0;                                                                          \
        dS[0] = 1;                                                                                 \
        dV[1] = 1;                                                                                 \
        uint32_t n_fix = 0;                                                                        \
        for (uint32_t j = 0; j < N; ++j) {                                                         \
            WT z1, zb;                                                                             \
            {                                                                                      \
                double a = jb->za[i * N + j], b = jb->zb[i * N + j];                               \
                if (mca) {                                                                         \
                    a *= 1.0 + xi(&st) * 2.0 * (U);                                                \
                    if (SINCOS)                                                                    \
                        a += xi(&st) * SIN_COS_ABS * sqrt(a * a + 1.0);                            \
                    b *= 1.0 + xi(&st) * 2.0 * (U);                                                \
                    if (SINCOS)                                                                    \
                        b += xi(&st) * SIN_COS_ABS * sqrt(b * b + 1.0);                            \
                }                                                                                  \
                z1 = (WT)a;                                                                        \
                zb = (WT)b;                                                                        \
            }                                                                                      \
            WT z2 = R((XT)c_rho * z1 + R((XT)c_rbar * zb, 1), 1);                                  \
            WT dz2 = R((XT)c_drbar * zb + z1, 1);                                                  \
            int pos = V > 0;                                                                       \
            WT vp = pos ? V : (WT)0;                                                               \
            WT dvp[7];                                                                             \
            for (int k = 0; k < 7; ++k)                                                            \
                dvp[k] = pos ? dV[k] : (WT)0;                                                      \
            WT sq = R(SQRT((XT)R((XT)vp * c_dt, 1)), 1);                                           \
            WT dsq = (pos && sq > 0) ? R((XT)c_hdt / sq, 2) : (WT)0;                               \
            if ((double)dsq > amp)                                                                 \
                amp = (double)dsq;                                                                 \
            WT inc = R((XT)sq * z1 + R((XT)R((XT)(WT)(-0.5) * vp + c_r, 1) * c_dt, 1), 1);         \
            WT cin = R((XT)dsq * z1 + c_mhdt, 1);                                                  \
            WT dinc[7];                                                                            \
            for (int k = 0; k < 7; ++k)                                                            \
                dinc[k] = R((XT)dvp[k] * cin, 1);                                                  \
            dinc[2] = R((XT)dinc[2] + c_dt, 1);                                                    \
            WT g = R(EXP((XT)inc), 2);                                                             \
            WT Sn = R((XT)S * g, 1);                                                               \
            for (int k = 0; k < 7; ++k)                                                            \
                dS[k] = R((XT)g * dS[k] + R((XT)Sn * dinc[k], 1), 1);                              \
            S = Sn;                                                                                \
            WT vb = jb->absorb ? vp : V;                                                           \
            WT sz = R((XT)sq * z2, 1);                                                             \
            WT zz = R((XT)z2 * z2 - 1, 1);                                                         \
            WT mil = R((XT)c_qs2dt * zz, 1);                                                       \
            WT Vn = R((XT)vb + R((XT)c_mkdt * vp + c_kth, 1), 1);                                  \
            Vn = R((XT)Vn + R((XT)c_sig * sz, 1), 1);                                              \
            Vn = R((XT)Vn + mil, 1);                                                               \
            WT cv = R((XT)R((XT)c_sig * dsq, 1) * z2 + c_mkdt, 1);                                 \
            WT dVn[7];                                                                             \
            for (int k = 0; k < 7; ++k)                                                            \
                dVn[k] = R((XT)dvp[k] * cv + (jb->absorb ? dvp[k] : dV[k]), 1);                    \
            dVn[6] = R((XT)R((XT)c_sig * sq + R((XT)c_hs2dt * z2, 1), 1) * dz2 + dVn[6], 1);       \
            dVn[3] = R((XT)R((XT)c_th - vp, 1) * c_dt + dVn[3], 1);                                \
            dVn[4] = R((XT)dVn[4] + c_kdt, 1);                                                     \
            dVn[5] = R((XT)dVn[5] + R((XT)c_hsdt * zz + sz, 1), 1);                                \
            if (jb->absorb && Vn <= 0) {                                                           \
                Vn = 0;                                                                            \
                for (int k = 0; k < 7; ++k)                                                        \
                    dVn[k] = 0;                                                                    \
            }                                                                                      \
            V = Vn;                                                                                \
            memcpy(dV, dVn, sizeof dV);                                                            \
            if (jb->fix[j + 1]) {                                                                  \
                ++n_fix;                                                                           \
                A = R((XT)A + S, 1);                                                               \
                for (int k = 0; k < 7; ++k)                                                        \
                    dA[k] = R((XT)dA[k] + dS[k], 1);                                               \
            }                                                                                      \
        }                                                                                          \
        const int asian = jb->type == 2 || jb->type == 3;                                          \
        const double sgn = (jb->type == 0 || jb->type == 2) ? 1.0 : -1.0;                          \
        const double D = exp(-P->r * P->T);                                                        \
        double Xv, dX[7];                                                                          \
        if (asian) {                                                                               \
            Xv = (double)A / (double)n_fix;                                                        \
            for (int k = 0; k < 7; ++k)                                                            \
                dX[k] = (double)dA[k] / (double)n_fix;                                             \
        } else {                                                                                   \
            Xv = (double)S;                                                                        \
            for (int k = 0; k < 7; ++k)                                                            \
                dX[k] = (double)dS[k];                                                             \
        }                                                                                          \
        double intr = sgn * (Xv - P->K);                                                           \
        int itm = intr > 0.0;                                                                      \
        double *o = jb->out + i * 9;                                                               \
        o[0] = itm ? D * intr : 0.0;                                                               \
        for (int k = 0; k < 7; ++k)                                                                \
            o[1 + k] = itm ? D * sgn * dX[k] : 0.0;                                                \
        o[3] -= P->T * o[0];                                                                       \
        o[8] = amp;                                                                                \
    }

/* R(x, ulps): a wide value rounded to the working type, perturbed under MCA */
static inline float rnd_f(int mca, uint64_t *st, double x, double ulps)
{
    if (mca)
        x *= 1.0 + xi(st) * 0x1p-24 * ulps;
    return (float)x;
}

static inline double rnd_d(int mca, uint64_t *st, long double x, double ulps)
{
    if (mca)
        x *= 1.0L + (long double)(xi(st) * 0x1p-53 * ulps);
    return (double)x;
}

#define R(x, ulps) rnd_f(mca, &st, (x), (ulps))
TM_PATH(path_f32, float, double, 0x1p-24, 1, sqrt, exp)
#undef R
#define R(x, ulps) rnd_d(mca, &st, (x), (ulps))
TM_PATH(path_f64, double, long double, 0x1p-53, 0, sqrtl, expl)
#undef R

static void *tm_run(void *arg)
{
    const tm_job *jb = arg;
    for (uint64_t i = jb->lo; i < jb->hi; ++i) {
        if (jb->single)
            path_f32(jb, i);
        else
            path_f64(jb, i);
    }
    return NULL;
}

/* type 0..3: European call/put, Asian call/put; fix[0..N] marks fixing steps;
 * za, zb: [n][N] normals; single: binary32 (else binary64); seed 0: round to
 * nearest; out: [n][9].  Returns 0, or -1 on invalid arguments.             */
int tm_evaluate(const tm_params *P, int type, uint32_t N, const uint8_t *fix, int absorb,
                const double *za, const double *zb, uint64_t n, int single, uint64_t seed,
                int threads, double *out)
{
    if (type < 0 || type > 3 || N == 0 || !fix || !za || !zb || !out)
        return -1;
    if (threads < 1)
        threads = 1;
    if (threads > 64)
        threads = 64;
    if ((uint64_t)threads > n)
        threads = n ? (int)n : 1;
    pthread_t th[64];
    tm_job jobs[64];
    for (int t = 0; t < threads; ++t) {
        tm_job jb = { P, type, absorb, single, N, fix, za, zb, n, seed,
                      n * (uint64_t)t / (uint64_t)threads, n * (uint64_t)(t + 1) / (uint64_t)threads,
                      out };
        jobs[t] = jb;
    }
    for (int t = 1; t < threads; ++t)
        pthread_create(&th[t], NULL, tm_run, &jobs[t]);
    tm_run(&jobs[0]);
    for (int t = 1; t < threads; ++t)
        pthread_join(th[t], NULL);
    return 0;
}
