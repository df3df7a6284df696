/* Monte Carlo arithmetic evaluation of Milstein and QE paths and their
 * forward-mode derivatives -- test infrastructure (see tangent_binary32.py).
 *
 * Evaluates, per path, the discounted payoff of a European or arithmetic-
 * average Asian option under the Heston model's Milstein scheme (full
 * truncation or absorption) or Andersen's QE scheme, and its derivatives
 * with respect to (S0, v0, r, kappa, theta, sigma, rho), in a working
 * precision W (binary32 or binary64).  Each operation is evaluated in a wider type, its result
 * multiplied by (1 + xi u) with xi uniform in [-1, 1] and u the unit roundoff
 * of W (Monte Carlo arithmetic, Parker 1997), then rounded to W.  With
 * seed 0 nothing is perturbed: a plain round-to-nearest evaluation.
 *
 * The random inputs are the two normals of every step (QE: Zs, Zv, Uv),
 * passed in; the perturbations come from a per-path splitmix64 stream of
 * (seed, path), so the result does not depend on the thread count.
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
    int type, absorb, single, qe;
    uint32_t N;
    const uint8_t *fix;
    const double *za, *zb, *uv; /* Milstein: Za, Zb; QE: Zs, Zv, Uv */
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


/* Discounted payoff and its derivatives from S_T or the average (as the oracle). */
static void tm_finish_d(const tm_job *jb, uint64_t i, double S, double A, uint32_t n_fix,
                        const double dS[7], const double dA[7], double amp)
{
    const tm_params *P = jb->P;
    const int asian = jb->type == 2 || jb->type == 3;
    const double sgn = (jb->type == 0 || jb->type == 2) ? 1.0 : -1.0;
    const double D = exp(-P->r * P->T);
    double Xv, dX[7];
    if (asian) {
        Xv = A / (double)n_fix;
        for (int k = 0; k < 7; ++k)
            dX[k] = dA[k] / (double)n_fix;
    } else {
        Xv = S;
        for (int k = 0; k < 7; ++k)
            dX[k] = dS[k];
    }
    double intr = sgn * (Xv - P->K);
    int itm = intr > 0.0;
    double *o = jb->out + i * 9;
    o[0] = itm ? D * intr : 0.0;
    for (int k = 0; k < 7; ++k)
        o[1 + k] = itm ? D * sgn * dX[k] : 0.0;
    o[3] -= P->T * o[0];
    o[8] = amp;
}
#define tm_finish(jb, i, S, A, n_fix, dS, dA, amp)                                                 \
    do {                                                                                           \
        double dS_[7], dA_[7];                                                                     \
        for (int k_ = 0; k_ < 7; ++k_) {                                                           \
            dS_[k_] = (double)(dS)[k_];                                                            \
            dA_[k_] = (double)(dA)[k_];                                                            \
        }                                                                                          \
        tm_finish_d(jb, i, S, A, n_fix, dS_, dA_, amp);                                            \
    } while (0)

/* One QE path (Andersen's scheme, the oracle's forward-mode derivative of it):
 * the same quantities, every operation rounded as above; the branch decisions
 * are taken on the rounded values.  out[8]: 0.                              */
#define TM_PATH_QE(NAME, WT, XT, U, SINCOS, SQRT, EXP, LOG)                                       \
    static void NAME(const tm_job *jb, uint64_t i)                                                 \
    {                                                                                              \
        const tm_params *P = jb->P;                                                                \
        uint64_t st = jb->seed * 0xD1B54A32D192ED03ull ^ (i + 1) * 0x9E3779B97F4A7C15ull;          \
        const int mca = jb->seed != 0;                                                             \
        const uint32_t N = jb->N;                                                                  \
        const double dt = P->T / (double)N, kap = P->kappa, th = P->theta, sig = P->sigma;       \
        const double rho = P->rho;                                                                 \
        const double E = exp(-kap * dt), dE = -dt * E, s2s = sig * sig;                            \
        const double A1 = E * (1.0 - E) / kap, A0 = (1.0 - E) * (1.0 - E) / (2.0 * kap);          \
        const double dA1 = dE * (1.0 - 2.0 * E) / kap - A1 / kap;                                  \
        const double dA0 = -(1.0 - E) * dE / kap - A0 / kap;                                       \
        const double c = kap * rho / sig - 0.5;                                                    \
        const double dc[7] = {0, 0, 0, rho / sig, 0, -kap * rho / s2s, kap / sig};                 \
        const double dR[7] = {0, 0, 0, 0, 0, rho / s2s, -1.0 / sig};                               \
        const WT c_E = (WT)E, c_mth = (WT)(th * (1.0 - E)), c_cs1 = (WT)(s2s * A1);                \
        const WT c_cs0 = (WT)(th * s2s * A0), c_K0 = (WT)(-rho * kap * th * dt / sig);            \
        const WT c_K1 = (WT)(0.5 * dt * c - rho / sig), c_K2 = (WT)(0.5 * dt * c + rho / sig);    \
        const WT c_Kq = (WT)(0.5 * dt * (1.0 - rho * rho)), c_rdt = (WT)(P->r * dt);              \
        WT d_m[7] = {0}, d_s[7] = {0}, d_K0[7] = {0}, d_K1[7] = {0}, d_K2[7] = {0};               \
        WT d_Kq[7] = {0};                                                                          \
        d_m[3] = (WT)(-th * dE); /* d mth / dkappa; + V dE */                                      \
        d_m[4] = (WT)(1.0 - E);                                                                    \
        d_s[3] = (WT)(th * s2s * dA0);                                                             \
        d_s[4] = (WT)(s2s * A0);                                                                   \
        d_s[5] = (WT)(2.0 * sig * th * A0);                                                        \
        const WT c_dE = (WT)dE, c_dcs1_k = (WT)(s2s * dA1), c_dcs1_s = (WT)(2.0 * sig * A1);       \
        d_K0[3] = (WT)(-rho * th * dt / sig);                                                      \
        d_K0[4] = (WT)(-rho * kap * dt / sig);                                                     \
        d_K0[5] = (WT)(rho * kap * th * dt / s2s);                                                 \
        d_K0[6] = (WT)(-kap * th * dt / sig);                                                      \
        for (int k = 0; k < 7; ++k) {                                                              \
            d_K1[k] = (WT)(0.5 * dt * dc[k] + dR[k]);                                              \
            d_K2[k] = (WT)(0.5 * dt * dc[k] - dR[k]);                                              \
        }                                                                                          \
        d_Kq[6] = (WT)(-dt * rho);                                                                 \
        WT S = (WT)P->S0, V = (WT)P->v0, A = 0;                                                    \
        WT dS[7] = {0}, dV[7] = {0}, dA[7] = {0};                                                  \
        dS[0] = 1;                                                                                 \
        dV[1] = 1;                                                                                 \
        uint32_t n_fix = 0;                                                                        \
        for (uint32_t j = 0; j < N; ++j) {                                                         \
            double a = jb->za[i * N + j], b = jb->zb[i * N + j];                                   \
            if (mca) {                                                                             \
                a *= 1.0 + xi(&st) * 2.0 * (U);                                                    \
                if (SINCOS)                                                                        \
                    a += xi(&st) * SIN_COS_ABS * sqrt(a * a + b * b);                              \
                b *= 1.0 + xi(&st) * 2.0 * (U);                                                    \
                if (SINCOS)                                                                        \
                    b += xi(&st) * SIN_COS_ABS * sqrt(a * a + b * b);                              \
            }                                                                                      \
            const WT zs = (WT)a, zv = (WT)b, uv = (WT)jb->uv[i * N + j];                           \
            const WT m = R((XT)c_E * V + c_mth, 1), s2 = R((XT)c_cs1 * V + c_cs0, 1);              \
            const WT psi = R((XT)s2 / R((XT)m * m, 1), 2);                                         \
            WT dm[7], ds2[7], dpsi[7], dVn[7], Vn;                                                 \
            for (int k = 0; k < 7; ++k) {                                                          \
                dm[k] = R((XT)c_E * dV[k] + d_m[k], 1);                                            \
                ds2[k] = R((XT)c_cs1 * dV[k] + d_s[k], 1);                                         \
            }                                                                                      \
            dm[3] = R((XT)c_dE * V + dm[3], 1);                                                    \
            ds2[3] = R((XT)c_dcs1_k * V + ds2[3], 1);                                              \
            ds2[5] = R((XT)c_dcs1_s * V + ds2[5], 1);                                              \
            for (int k = 0; k < 7; ++k)                                                            \
                dpsi[k] = R(((XT)ds2[k] - (XT)2 * psi * m * dm[k]) / ((XT)m * m), 3);              \
            if (psi <= (WT)1.5) {                                                                  \
                const WT inv = R((XT)2 / psi, 2);                                                  \
                const WT r = R(SQRT((XT)R((XT)inv * (inv - 1), 2)), 1);                            \
                const WT b2 = R((XT)inv - 1 + r, 2);                                               \
                const WT bb = R(SQRT((XT)b2), 1);                                                  \
                const WT aa = R((XT)m / (1 + (XT)b2), 2);                                          \
                const WT g = R((XT)bb + zv, 1);                                                    \
                Vn = R((XT)aa * g * g, 2);                                                         \
                const WT db2_dinv = R(1 + ((XT)2 * inv - 1) / ((XT)2 * r), 3);                     \
                for (int k = 0; k < 7; ++k) {                                                      \
                    const WT dinv = R(-(XT)2 * dpsi[k] / ((XT)psi * psi), 3);                      \
                    const WT db2 = R((XT)db2_dinv * dinv, 1);                                      \
                    const WT da = R((XT)dm[k] / (1 + (XT)b2) - (XT)m * db2 / ((1 + (XT)b2) * (1 + (XT)b2)), 4); \
                    const WT db = R((XT)db2 / ((XT)2 * bb), 2);                                    \
                    dVn[k] = R((XT)da * g * g + (XT)2 * aa * g * db, 3);                           \
                }                                                                                  \
            } else {                                                                               \
                const WT p = R(((XT)psi - 1) / ((XT)psi + 1), 3);                                  \
                if (uv <= p) {                                                                     \
                    Vn = 0;                                                                        \
                    for (int k = 0; k < 7; ++k)                                                    \
                        dVn[k] = 0;                                                                \
                } else {                                                                           \
                    const WT L = R(LOG((XT)R((1 - (XT)p) / (1 - (XT)uv), 2)), 2);                  \
                    Vn = R((XT)m / (1 - (XT)p) * L, 2);                                            \
                    for (int k = 0; k < 7; ++k) {                                                  \
                        const WT dp = R((XT)2 * dpsi[k] / (((XT)psi + 1) * ((XT)psi + 1)), 3);     \
                        dVn[k] = R((XT)dm[k] * L / (1 - (XT)p) + (XT)m * (L - 1) * dp / ((1 - (XT)p) * (1 - (XT)p)), 4); \
                    }                                                                              \
                }                                                                                  \
            }                                                                                      \
            const WT q = R((XT)c_Kq * R((XT)V + Vn, 1), 1);                                        \
            const WT sq = R(SQRT((XT)q), 1);                                                       \
            WT inc = R((XT)c_rdt + c_K0, 1);                                                       \
            inc = R((XT)c_K1 * V + inc, 1);                                                        \
            inc = R((XT)c_K2 * Vn + inc, 1);                                                       \
            inc = R((XT)sq * zs + inc, 1);                                                         \
            WT dinc[7];                                                                            \
            for (int k = 0; k < 7; ++k) {                                                          \
                const WT dq = R((XT)c_Kq * R((XT)dV[k] + dVn[k], 1) + (XT)d_Kq[k] * ((XT)V + Vn), 2); \
                const WT dsq = q > 0 ? R((XT)dq / ((XT)2 * sq), 2) : (WT)0;                        \
                WT t = R((XT)d_K0[k] + (XT)d_K1[k] * V, 1);                                        \
                t = R((XT)c_K1 * dV[k] + t, 1);                                                    \
                t = R((XT)d_K2[k] * Vn + t, 1);                                                    \
                t = R((XT)c_K2 * dVn[k] + t, 1);                                                   \
                dinc[k] = R((XT)dsq * zs + t, 1);                                                  \
            }                                                                                      \
            dinc[2] = R((XT)dinc[2] + (WT)dt, 1);                                                  \
            const WT gg = R(EXP((XT)inc), 2);                                                      \
            const WT Sn = R((XT)S * gg, 1);                                                        \
            for (int k = 0; k < 7; ++k)                                                            \
                dS[k] = R((XT)gg * dS[k] + R((XT)Sn * dinc[k], 1), 1);                             \
            S = Sn;                                                                                \
            V = Vn;                                                                                \
            memcpy(dV, dVn, sizeof dV);                                                            \
            if (jb->fix[j + 1]) {                                                                  \
                ++n_fix;                                                                           \
                A = R((XT)A + S, 1);                                                               \
                for (int k = 0; k < 7; ++k)                                                        \
                    dA[k] = R((XT)dA[k] + dS[k], 1);                                               \
            }                                                                                      \
        }                                                                                          \
        tm_finish(jb, i, (double)S, (double)A, n_fix, dS, dA, 0.0);                                \
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
#define R(x, ulps) rnd_f(mca, &st, (x), (ulps))
TM_PATH_QE(path_qe_f32, float, double, 0x1p-24, 1, sqrt, exp, log)
#undef R
#define R(x, ulps) rnd_d(mca, &st, (x), (ulps))
TM_PATH_QE(path_qe_f64, double, long double, 0x1p-53, 0, sqrtl, expl, logl)
#undef R

static void *tm_run(void *arg)
{
    const tm_job *jb = arg;
    for (uint64_t i = jb->lo; i < jb->hi; ++i) {
        if (jb->qe)
            (jb->single ? path_qe_f32 : path_qe_f64)(jb, i);
        else if (jb->single)
            path_f32(jb, i);
        else
            path_f64(jb, i);
    }
    return NULL;
}

/* type 0..3: European call/put, Asian call/put; fix[0..N] marks fixing steps;
 * scheme 0 Milstein with full truncation, 1 with absorption, 2 QE;
 * za, zb (and uv for QE): [n][N] random inputs (Milstein: Za, Zb; QE: Zs, Zv,
 * Uv); single: binary32 (else binary64); seed 0: round to nearest;
 * out: [n][9].  Returns 0, or -1 on invalid arguments.                      */
int tm_evaluate(const tm_params *P, int type, uint32_t N, const uint8_t *fix, int scheme,
                const double *za, const double *zb, const double *uv, uint64_t n, int single,
                uint64_t seed, int threads, double *out)
{
    if (type < 0 || type > 3 || N == 0 || !fix || !za || !zb || !out || scheme < 0 ||
        scheme > 2 || (scheme == 2 && !uv))
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
        tm_job jb = { P, type, scheme == 1, single, scheme == 2, N, fix, za, zb, uv, n, seed,
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
