/*
 * heston_oracle.c -- plain FP64 reference for the Heston / Milstein Monte-Carlo
 * path. TEST INFRASTRUCTURE ONLY: it is called by the test-suite, by the smoke
 * check and by the benchmark's CPU-baseline leg, never by the product library.
 * It shares no code with the GPU path.
 *
 * What it computes (one path at a time, in double precision, no blocking and
 * no fusion):
 *   - the Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
 *     "Parallel Random Numbers: As Easy as 1, 2, 3", SC'11), used to draw the
 *     two independent normals of every step by the Box-Muller transform;
 *   - the correlated pair Z1 = Za, Z2 = rho Za + sqrt(1-rho^2) Zb
 *     (paper, Background: algorithm "Generation of two correlated Normal
 *     random variables");
 *   - the Milstein scheme of the paper (Background, algorithm "Milstein
 *     approximation under Heston model"): the log-price step carries no
 *     correction term and the variance step carries 1/4 sigma^2 dt (Z2^2-1);
 *     truncation either as the paper writes it (V <- max(V,0) after every step,
 *     "absorption") or as full truncation (V+ = max(V,0) used in drift and
 *     diffusion, the unclamped V carried);
 *   - the discounted payoffs of European and arithmetic-Asian calls and puts
 *     (Background, payoff definitions and risk-neutral pricing) and the
 *     pathwise Delta and Rho estimators (Background, "Pathwise method for
 *     greeks estimation": European estimators as printed, the Asian Rho with
 *     the exact derivative of the discrete average);
 *   - forward-mode (tangent) derivatives of each path's discounted payoff with
 *     respect to (S0, v0, r, kappa, theta, sigma, rho), by the chain rule
 *     carried step by step alongside the path, for the Milstein scheme and for
 *     the QE scheme below (its branch decisions held fixed);
 *   - the paper's Euler discretisation (Background, "Euler discretisation"):
 *     the same log-price and variance steps without the Milstein term, with
 *     either truncation;
 *   - two more fixes of negative variances from Lord, Koekkoek and van Dijk,
 *     "A comparison of biased simulation schemes for stochastic volatility
 *     models", Quantitative Finance 10(2), 2010: writing the variance step as
 *     V' = f1(V) + kappa (theta - f2(V)) dt + sigma sqrt(f3(V) dt) Z2 (+ the
 *     Milstein term) and using f3 in the log-price step, partial truncation
 *     takes f1 = f2 = identity, f3 = max(., 0), and reflection takes
 *     f1 = f2 = f3 = |.| (full truncation: f1 = identity, f2 = f3 = max(., 0);
 *     the paper's absorption: all max(., 0) and V' clamped);
 *   - Andersen's quadratic-exponential (QE) scheme (L. Andersen, "Simple and
 *     efficient simulation of the Heston stochastic volatility model", Journal
 *     of Computational Finance 11(3), 2008), the scheme the paper names as
 *     future work: the variance is drawn from a moment-matched squared normal
 *     or from a point mass at zero plus an exponential tail, and the log-price
 *     step uses the start and end variances of the step (central weights
 *     gamma1 = gamma2 = 1/2, switching level psi_c = 3/2, no martingale
 *     correction).
 *
 * Readings taken where the paper is silent (stated again in the design notes):
 *   - integer step loop j = 0..N-1 with dt = T/N;
 *   - the step uses the variance at the start of the step;
 *   - Za drives the price, Zb is mixed into the variance;
 *   - stream layout: key = (lo32 seed, hi32 seed); counter =
 *     (j>>1, lo32 path, hi32 path, 0); words 0,1 feed even steps and words 2,3
 *     odd steps; uniform u = ((w >> 9) + 1/2) 2^-23, which is exact in single
 *     and double precision and never 0 or 1;
 *   - Za = sqrt(-2 ln ua) cos(2 pi ub), Zb = sqrt(-2 ln ua) sin(2 pi ub).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_REC 6    /* S_T, V_T, Sbar, discounted payoff, pathwise Delta, pathwise Rho */
#define OR_TAN 9    /* discounted payoff, d/dS0, d/dv0, d/dr, d/dkappa, d/dtheta, d/dsigma, d/drho,
                       then (Milstein) the path's largest d sqrt(V+ dt) / dV+ =
                       max_j sqrt(dt / V+_j) / 2, or (QE) its smallest branch margin */

typedef struct {
    double S0, K, r, T, v0, kappa, theta, sigma, rho;
} or_params;

enum {
    OR_EURO_CALL = 0,
    OR_EURO_PUT = 1,
    OR_ASIAN_CALL = 2,
    OR_ASIAN_PUT = 3,
    OR_GEO_ASIAN_CALL = 4,
    OR_GEO_ASIAN_PUT = 5
};
enum {
    OR_FULL_TRUNC = 0,
    OR_ABSORB = 1,
    OR_QE = 2,
    OR_EULER_FULL_TRUNC = 3,
    OR_EULER_ABSORB = 4,
    OR_PARTIAL_TRUNC = 5,
    OR_REFLECT = 6
};
#define OR_REC_QE (OR_REC + 2) /* QE records add the path's smallest branch-decision margin and
                                   its amplification of variance errors (see sim_path_qe) */

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11): ten rounds of two 32x32->64 multiplies, with the
 * two-word key advanced by the Weyl constants between rounds.                */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t prod0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(prod1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)prod1;
        uint32_t n2 = (uint32_t)(prod0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)prod0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

double or_uniform(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * 0x1p-23;
}

/* The two independent standard normals of step `step` of path `path`. */
void or_normals(uint64_t seed, uint64_t path, uint32_t step, double *za, double *zb)
{
    uint32_t ctr[4] = { step >> 1, (uint32_t)path, (uint32_t)(path >> 32), 0u };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    uint32_t wa = (step & 1u) ? w[2] : w[0];
    uint32_t wb = (step & 1u) ? w[3] : w[1];
    double ua = or_uniform(wa);
    double ub = or_uniform(wb);
    double radius = sqrt(-2.0 * log(ua));
    double angle = 2.0 * M_PI * ub;
    *za = radius * cos(angle);
    *zb = radius * sin(angle);
}

/* ------------------------------------------------------------------------ */
/* Where the step's normals come from: the Philox stream, or caller arrays
 * (row-major [n_paths][n_steps], used for quasi-random normals).            */
typedef struct {
    uint64_t seed;
    const double *za; /* NULL -> Philox */
    const double *zb;
    uint32_t n_steps;
} or_source;

static void step_normals(const or_source *src, uint64_t path, uint64_t row, uint32_t j,
                         double *za, double *zb)
{
    if (src->za) {
        *za = src->za[row * src->n_steps + j];
        *zb = src->zb[row * src->n_steps + j];
    } else {
        or_normals(src->seed, path, j, za, zb);
    }
}

/* Averaging types: arithmetic (the paper's) or geometric average of S over the
 * fixing dates (the paper notes both are in use).                            */
static int is_geo(int type) { return type == OR_GEO_ASIAN_CALL || type == OR_GEO_ASIAN_PUT; }
static int is_asian(int type) { return type == OR_ASIAN_CALL || type == OR_ASIAN_PUT || is_geo(type); }
static int is_call(int type)
{
    return type == OR_EURO_CALL || type == OR_ASIAN_CALL || type == OR_GEO_ASIAN_CALL;
}

/* Fixing-date sums: A = sum S and B = sum t S (arithmetic), or A = sum ln S
 * and B = sum t (geometric).                                                 */
static void add_fixing(int type, double S, double t, double *A, double *B)
{
    if (is_geo(type)) {
        *A += log(S);
        *B += t;
    } else {
        *A += S;
        *B += t * S;
    }
}

/* Discounted payoff and pathwise Delta / Rho of a finished path (S_T, V_T and
 * the fixing sums A = sum S, B = sum t S); writes the first OR_REC values.    */
static void finish_path(const or_params *P, int type, uint32_t n_fix, double S, double V, double A,
                        double B, double *rec)
{
    const double D = exp(-P->r * P->T);
    const double nf = (double)n_fix;
    double Sbar = is_geo(type) ? exp(A / nf) : is_asian(type) ? A / nf : S;
    /* B / n_fix becomes dSbar/dr: the average of t S (arithmetic), or
     * G times the average fixing time (geometric).                           */
    if (is_geo(type))
        B = Sbar * B;
    double pay, dpw, rpw;
    if (is_call(type)) {
        int itm = Sbar > P->K;
        pay = D * (itm ? Sbar - P->K : 0.0);
        dpw = itm ? D * Sbar / P->S0 : 0.0;
        if (is_asian(type))
            rpw = itm ? D * (B / (double)n_fix - P->T * (Sbar - P->K)) : 0.0;
        else
            rpw = itm ? D * P->K * P->T : 0.0;
    } else {
        int itm = Sbar < P->K;
        pay = D * (itm ? P->K - Sbar : 0.0);
        dpw = itm ? -D * Sbar / P->S0 : 0.0;
        if (is_asian(type))
            rpw = itm ? D * (-B / (double)n_fix - P->T * (P->K - Sbar)) : 0.0;
        else
            rpw = itm ? -D * P->K * P->T : 0.0;
    }
    rec[0] = S;
    rec[1] = V;
    rec[2] = Sbar;
    rec[3] = pay;
    rec[4] = dpw;
    rec[5] = rpw;
}


/* One path of the Milstein scheme (or, in the Euler modes, of the Euler
 * scheme: the variance step without the Milstein term); writes the OR_REC
 * record.  fix[j] != 0 marks step j (1..N) as an Asian fixing date;
 * n_fix = |F|.                                                              */
static void sim_path(const or_params *P, int type, uint32_t N, const uint8_t *fix, uint32_t n_fix,
                     int mode, const or_source *src, uint64_t path, uint64_t row, double *rec)
{
    const int euler = mode == OR_EULER_FULL_TRUNC || mode == OR_EULER_ABSORB;
    const int absorb = mode == OR_ABSORB || mode == OR_EULER_ABSORB;
    const int partial = mode == OR_PARTIAL_TRUNC;
    const int reflect = mode == OR_REFLECT;
    const double dt = P->T / (double)N;
    const double rho_bar = sqrt(1.0 - P->rho * P->rho);
    double S = P->S0;
    double V = P->v0;
    double A = 0.0; /* sum of S at fixing dates        */
    double B = 0.0; /* sum of t_i S at fixing dates    */
    for (uint32_t j = 0; j < N; ++j) {
        double za, zb;
        step_normals(src, path, row, j, &za, &zb);
        double z1 = za;
        double z2 = P->rho * za + rho_bar * zb;
        double vp = V > 0.0 ? V : 0.0;
        double f1 = absorb ? vp : V, f2 = vp, f3 = vp;
        if (partial)
            f2 = V;
        if (reflect)
            f1 = f2 = f3 = fabs(V);
        S = S * exp((P->r - 0.5 * f3) * dt + sqrt(f3 * dt) * z1);
        V = f1 + P->kappa * (P->theta - f2) * dt + P->sigma * sqrt(f3 * dt) * z2;
        if (!euler)
            V += 0.25 * P->sigma * P->sigma * dt * (z2 * z2 - 1.0);
        if (absorb && V < 0.0)
            V = 0.0;
        if (fix[j + 1])
            add_fixing(type, S, (double)(j + 1) * dt, &A, &B);
    }
    finish_path(P, type, n_fix, S, V, A, B, rec);
}

/* ------------------------------------------------------------------------ */
/* Andersen's QE scheme.  Random inputs of step j: one Philox4x32-10 block
 * with counter (j, lo32 path, hi32 path, 4); words 0 and 1 give the
 * Box-Muller pair (Zs drives the log-price, Zv the quadratic branch of the
 * variance) and word 2 the uniform Uv of the exponential branch.            */
#define OR_QE_PSI_C 1.5
#define OR_QE_TAG 4u

void or_qe_draws(uint64_t seed, uint64_t path, uint32_t step, double *zs, double *zv, double *uv)
{
    uint32_t ctr[4] = { step, (uint32_t)path, (uint32_t)(path >> 32), OR_QE_TAG };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    double ua = or_uniform(w[0]);
    double ub = or_uniform(w[1]);
    double radius = sqrt(-2.0 * log(ua));
    double angle = 2.0 * M_PI * ub;
    *zs = radius * cos(angle);
    *zv = radius * sin(angle);
    *uv = or_uniform(w[2]);
}

/* One step of the variance: the CIR conditional mean m and variance s2 of
 * V(t+dt) given V(t) = V are matched either by a scaled squared normal
 * (psi = s2/m^2 <= psi_c) or by a point mass at 0 with an exponential tail.
 * *margin receives how close the step came to taking the other branch: the
 * relative distance of psi from psi_c and, in the exponential branch, the
 * distance of Uv from the mass p.                                            */
static double qe_variance(const or_params *P, double dt, double V, double zv, double uv,
                          double *margin)
{
    const double E = exp(-P->kappa * dt);
    const double s2s = P->sigma * P->sigma;
    const double m = P->theta + (V - P->theta) * E;
    const double s2 = V * s2s * E * (1.0 - E) / P->kappa
                      + P->theta * s2s * (1.0 - E) * (1.0 - E) / (2.0 * P->kappa);
    const double psi = s2 / (m * m);
    double mg = fabs(psi - OR_QE_PSI_C) / OR_QE_PSI_C;
    double Vn;
    if (psi <= OR_QE_PSI_C) {
        const double inv = 2.0 / psi;
        const double b2 = inv - 1.0 + sqrt(inv) * sqrt(inv - 1.0);
        const double a = m / (1.0 + b2);
        const double b = sqrt(b2);
        Vn = a * (b + zv) * (b + zv);
    } else {
        const double p = (psi - 1.0) / (psi + 1.0);
        const double beta = (1.0 - p) / m;
        Vn = (uv <= p) ? 0.0 : log((1.0 - p) / (1.0 - uv)) / beta;
        if (fabs(uv - p) < mg)
            mg = fabs(uv - p);
    }
    *margin = mg;
    return Vn;
}

/* One QE path; writes OR_REC values, at rec[OR_REC] the smallest
 * branch-decision margin of the path, and at rec[OR_REC + 1] its
 * amplification of relative variance errors,
 *   a = max(1, max_j Q_j / max(V_j, v0, theta)),  Q_j = max_{i<=j} V_i |dV_j/dV_i|
 * (Q_0 = V_0, Q_{j+1} = max(Q_j |D_j|, V_{j+1}), D_j = dV_{j+1}/dV_j by a
 * central difference of the one-step map at fixed random inputs): how much a
 * relative perturbation of the variance at one step can grow, in units of the
 * path's variance scale, by any later step.  Every later log-price increment
 * uses those variances, so rounding errors of a lower-precision evaluation of
 * the same path grow in proportion.                                          */
static void sim_path_qe(const or_params *P, int type, uint32_t N, const uint8_t *fix,
                        uint32_t n_fix, uint64_t seed, uint64_t path, double *rec)
{
    const double dt = P->T / (double)N;
    const double g1 = 0.5, g2 = 0.5;
    const double K0 = -P->rho * P->kappa * P->theta * dt / P->sigma;
    const double K1 = g1 * dt * (P->kappa * P->rho / P->sigma - 0.5) - P->rho / P->sigma;
    const double K2 = g2 * dt * (P->kappa * P->rho / P->sigma - 0.5) + P->rho / P->sigma;
    const double K3 = g1 * dt * (1.0 - P->rho * P->rho);
    const double K4 = g2 * dt * (1.0 - P->rho * P->rho);
    double S = P->S0;
    double V = P->v0;
    double A = 0.0, B = 0.0;
    double margin = INFINITY;
    double Q = V, amp = 1.0;
    const double vscale = fmax(P->v0, P->theta);
    for (uint32_t j = 0; j < N; ++j) {
        double zs, zv, uv, mg, unused;
        or_qe_draws(seed, path, j, &zs, &zv, &uv);
        const double Vn = qe_variance(P, dt, V, zv, uv, &mg);
        if (mg < margin)
            margin = mg;
        const double h = fmax(V * 1e-6, 1e-14);
        const double D = (qe_variance(P, dt, V + h, zv, uv, &unused)
                          - qe_variance(P, dt, fmax(V - h, 0.0), zv, uv, &unused))
                         / (V + h - fmax(V - h, 0.0));
        Q = fmax(Q * fabs(D), Vn);
        amp = fmax(amp, Q / fmax(Vn, vscale));
        S = S * exp(P->r * dt + K0 + K1 * V + K2 * Vn + sqrt(K3 * V + K4 * Vn) * zs);
        V = Vn;
        if (fix[j + 1])
            add_fixing(type, S, (double)(j + 1) * dt, &A, &B);
    }
    finish_path(P, type, n_fix, S, V, A, B, rec);
    rec[OR_REC] = margin;
    rec[OR_REC + 1] = amp;
}

/* Forward-mode derivatives of one path's discounted payoff with respect to
 * theta = (S0, v0, r, kappa, theta, sigma, rho).  Every state variable carries
 * its 7-vector of partial derivatives; each line differentiates the matching
 * line of sim_path by the chain rule.  Conventions at the non-smooth points:
 * d max(y,0)/dy = 1{y > 0}, and d sqrt(V+ dt)/dV = 0 where V+ = 0.          */
#define NP 7
static void tan_path(const or_params *P, int type, uint32_t N, const uint8_t *fix, uint32_t n_fix,
                     int mode, const or_source *src, uint64_t path, uint64_t row, double *out)
{
    enum { I_S0 = 0, I_V0, I_R, I_KAPPA, I_THETA, I_SIGMA, I_RHO };
    const double dt = P->T / (double)N;
    const double rho_bar = sqrt(1.0 - P->rho * P->rho);
    const double drho_bar = -P->rho / rho_bar; /* d rho_bar / d rho */
    double S = P->S0, dS[NP] = { 0 };
    double V = P->v0, dV[NP] = { 0 };
    double A = 0.0, dA[NP] = { 0 };
    double amp = 0.0;
    dS[I_S0] = 1.0;
    dV[I_V0] = 1.0;
    for (uint32_t j = 0; j < N; ++j) {
        double za, zb;
        step_normals(src, path, row, j, &za, &zb);
        double z1 = za;
        double z2 = P->rho * za + rho_bar * zb;
        double dz2[NP] = { 0 };
        dz2[I_RHO] = za + drho_bar * zb;

        int pos = V > 0.0;
        double vp = pos ? V : 0.0;
        double dvp[NP];
        for (int k = 0; k < NP; ++k)
            dvp[k] = pos ? dV[k] : 0.0;
        double sq = sqrt(vp * dt);                  /* sqrt(V+ dt)          */
        double dsq_dvp = pos ? dt / (2.0 * sq) : 0.0; /* d sqrt(V+ dt)/d V+   */
        if (dsq_dvp > amp)
            amp = dsq_dvp;

        /* log-price increment and its derivatives */
        double inc = (P->r - 0.5 * vp) * dt + sq * z1;
        double dinc[NP];
        for (int k = 0; k < NP; ++k)
            dinc[k] = -0.5 * dvp[k] * dt + dsq_dvp * dvp[k] * z1;
        dinc[I_R] += dt;
        double g = exp(inc);
        double Snew = S * g;
        for (int k = 0; k < NP; ++k)
            dS[k] = g * dS[k] + Snew * dinc[k];
        S = Snew;

        /* variance step and its derivatives */
        double vb = (mode == OR_FULL_TRUNC) ? V : vp;
        double Vnew = vb + P->kappa * (P->theta - vp) * dt + P->sigma * sq * z2
                      + 0.25 * P->sigma * P->sigma * dt * (z2 * z2 - 1.0);
        double dVnew[NP];
        for (int k = 0; k < NP; ++k) {
            double dvb = (mode == OR_FULL_TRUNC) ? dV[k] : dvp[k];
            dVnew[k] = dvb - P->kappa * dvp[k] * dt + P->sigma * dsq_dvp * dvp[k] * z2
                       + P->sigma * sq * dz2[k] + 0.5 * P->sigma * P->sigma * dt * z2 * dz2[k];
        }
        dVnew[I_KAPPA] += (P->theta - vp) * dt;
        dVnew[I_THETA] += P->kappa * dt;
        dVnew[I_SIGMA] += sq * z2 + 0.5 * P->sigma * dt * (z2 * z2 - 1.0);
        if (mode == OR_ABSORB && Vnew <= 0.0) {
            Vnew = 0.0;
            for (int k = 0; k < NP; ++k)
                dVnew[k] = 0.0;
        }
        V = Vnew;
        for (int k = 0; k < NP; ++k)
            dV[k] = dVnew[k];

        if (fix[j + 1]) {
            A += S;
            for (int k = 0; k < NP; ++k)
                dA[k] += dS[k];
        }
    }
    const double D = exp(-P->r * P->T);
    double X, dX[NP];
    if (is_asian(type)) {
        X = A / (double)n_fix;
        for (int k = 0; k < NP; ++k)
            dX[k] = dA[k] / (double)n_fix;
    } else {
        X = S;
        for (int k = 0; k < NP; ++k)
            dX[k] = dS[k];
    }
    double sgn = is_call(type) ? 1.0 : -1.0;
    double intrinsic = sgn * (X - P->K);
    int itm = intrinsic > 0.0;
    double pay = D * (itm ? intrinsic : 0.0);
    out[0] = pay;
    for (int k = 0; k < NP; ++k)
        out[1 + k] = itm ? D * sgn * dX[k] : 0.0;
    out[1 + I_R] += -P->T * pay; /* the discount factor depends on r */
    out[1 + NP] = amp;
}

/* Forward-mode derivatives of one QE path's discounted payoff with respect to
 * (S0, v0, r, kappa, theta, sigma, rho): Andersen's step (qe_variance, the
 * log-price update of sim_path_qe) differentiated by the chain rule through
 * E = e^{-kappa dt}, the conditional moments m and s2, psi = s2 / m^2 and the
 * branch the step takes; the branch decisions themselves (psi against psi_c,
 * Uv against p) are held fixed, and the point mass at zero has derivative 0.
 * The derivative of sqrt(K3 V + K4 V') is taken as 0 where its argument is 0.
 * out[0..7] as tan_path; out[8] = the path's smallest branch margin (as
 * sim_path_qe reports it), below which a bump can switch a branch.          */
static void tan_path_qe(const or_params *P, int type, uint32_t N, const uint8_t *fix,
                        uint32_t n_fix, uint64_t seed, uint64_t path, double *out)
{
    enum { I_S0 = 0, I_V0, I_R, I_KAPPA, I_THETA, I_SIGMA, I_RHO };
    const double dt = P->T / (double)N;
    const double kap = P->kappa, th = P->theta, sig = P->sigma, rho = P->rho;
    const double g1 = 0.5, g2 = 0.5;
    /* log-price coefficients (as sim_path_qe) and their partials */
    const double c = kap * rho / sig - 0.5;
    const double K0 = -rho * kap * th * dt / sig;
    const double K1 = g1 * dt * c - rho / sig;
    const double K2 = g2 * dt * c + rho / sig;
    const double K3 = g1 * dt * (1.0 - rho * rho);
    const double K4 = g2 * dt * (1.0 - rho * rho);
    double dK0[NP] = { 0 }, dK1[NP] = { 0 }, dK2[NP] = { 0 }, dK34[NP] = { 0 };
    dK0[I_KAPPA] = -rho * th * dt / sig;
    dK0[I_THETA] = -rho * kap * dt / sig;
    dK0[I_SIGMA] = rho * kap * th * dt / (sig * sig);
    dK0[I_RHO] = -kap * th * dt / sig;
    const double dc_dk = rho / sig, dc_ds = -kap * rho / (sig * sig), dc_dr = kap / sig;
    dK1[I_KAPPA] = g1 * dt * dc_dk;
    dK1[I_SIGMA] = g1 * dt * dc_ds + rho / (sig * sig);
    dK1[I_RHO] = g1 * dt * dc_dr - 1.0 / sig;
    dK2[I_KAPPA] = g2 * dt * dc_dk;
    dK2[I_SIGMA] = g2 * dt * dc_ds - rho / (sig * sig);
    dK2[I_RHO] = g2 * dt * dc_dr + 1.0 / sig;
    dK34[I_RHO] = -2.0 * g1 * dt * rho; /* K3 = K4 */
    /* variance-step constants: m = theta + (V - theta) E,
     * s2 = sigma^2 (V A1 + theta A0), A1 = E (1-E) / kappa, A0 = (1-E)^2 / (2 kappa) */
    const double E = exp(-kap * dt), dE = -dt * E; /* dE / dkappa */
    const double s2s = sig * sig;
    const double A1 = E * (1.0 - E) / kap, A0 = (1.0 - E) * (1.0 - E) / (2.0 * kap);
    const double dA1 = dE * (1.0 - 2.0 * E) / kap - A1 / kap;
    const double dA0 = -(1.0 - E) * dE / kap - A0 / kap;

    double S = P->S0, dS[NP] = { 0 };
    double V = P->v0, dV[NP] = { 0 };
    double A = 0.0, dA[NP] = { 0 };
    double margin = INFINITY;
    dS[I_S0] = 1.0;
    dV[I_V0] = 1.0;
    for (uint32_t j = 0; j < N; ++j) {
        double zs, zv, uv, mg;
        or_qe_draws(seed, path, j, &zs, &zv, &uv);
        const double Vn = qe_variance(P, dt, V, zv, uv, &mg);
        if (mg < margin)
            margin = mg;
        /* the moments and psi, with derivatives */
        const double m = th + (V - th) * E;
        const double s2 = s2s * (V * A1 + th * A0);
        const double psi = s2 / (m * m);
        double dm[NP], ds2[NP], dpsi[NP], dVn[NP];
        for (int k = 0; k < NP; ++k) {
            dm[k] = E * dV[k];
            ds2[k] = s2s * A1 * dV[k];
        }
        dm[I_KAPPA] += (V - th) * dE;
        dm[I_THETA] += 1.0 - E;
        ds2[I_KAPPA] += s2s * (V * dA1 + th * dA0);
        ds2[I_THETA] += s2s * A0;
        ds2[I_SIGMA] += 2.0 * sig * (V * A1 + th * A0);
        for (int k = 0; k < NP; ++k)
            dpsi[k] = ds2[k] / (m * m) - 2.0 * s2 * dm[k] / (m * m * m);
        if (psi <= OR_QE_PSI_C) {
            /* Vn = a (b + Zv)^2, b^2 = 2/psi - 1 + sqrt(2/psi) sqrt(2/psi - 1), a = m / (1 + b^2) */
            const double inv = 2.0 / psi;
            const double r = sqrt(inv) * sqrt(inv - 1.0);
            const double b2 = inv - 1.0 + r;
            const double a = m / (1.0 + b2);
            const double b = sqrt(b2);
            const double db2_dinv = 1.0 + (2.0 * inv - 1.0) / (2.0 * r);
            for (int k = 0; k < NP; ++k) {
                const double dinv = -2.0 * dpsi[k] / (psi * psi);
                const double db2 = db2_dinv * dinv;
                const double da = dm[k] / (1.0 + b2) - m * db2 / ((1.0 + b2) * (1.0 + b2));
                const double db = db2 / (2.0 * b);
                dVn[k] = da * (b + zv) * (b + zv) + 2.0 * a * (b + zv) * db;
            }
        } else {
            /* point mass at 0 with probability p, else Vn = m / (1-p) ln((1-p) / (1-Uv)) */
            const double p = (psi - 1.0) / (psi + 1.0);
            if (uv <= p) {
                for (int k = 0; k < NP; ++k)
                    dVn[k] = 0.0;
            } else {
                const double L = log((1.0 - p) / (1.0 - uv));
                for (int k = 0; k < NP; ++k) {
                    const double dp = 2.0 * dpsi[k] / ((psi + 1.0) * (psi + 1.0));
                    dVn[k] = dm[k] * L / (1.0 - p) + m * (L - 1.0) * dp / ((1.0 - p) * (1.0 - p));
                }
            }
        }
        /* log-price step */
        const double q = K3 * V + K4 * Vn;
        const double sq = sqrt(q);
        const double inc = P->r * dt + K0 + K1 * V + K2 * Vn + sq * zs;
        double dinc[NP];
        for (int k = 0; k < NP; ++k) {
            const double dq = K3 * dV[k] + K4 * dVn[k] + dK34[k] * (V + Vn);
            const double dsq = q > 0.0 ? dq / (2.0 * sq) : 0.0;
            dinc[k] = dK0[k] + dK1[k] * V + K1 * dV[k] + dK2[k] * Vn + K2 * dVn[k] + dsq * zs;
        }
        dinc[I_R] += dt;
        const double g = exp(inc);
        const double Snew = S * g;
        for (int k = 0; k < NP; ++k)
            dS[k] = g * dS[k] + Snew * dinc[k];
        S = Snew;
        V = Vn;
        for (int k = 0; k < NP; ++k)
            dV[k] = dVn[k];
        if (fix[j + 1]) {
            A += S;
            for (int k = 0; k < NP; ++k)
                dA[k] += dS[k];
        }
    }
    const double D = exp(-P->r * P->T);
    double X, dX[NP];
    if (is_asian(type)) {
        X = A / (double)n_fix;
        for (int k = 0; k < NP; ++k)
            dX[k] = dA[k] / (double)n_fix;
    } else {
        X = S;
        for (int k = 0; k < NP; ++k)
            dX[k] = dS[k];
    }
    const double sgn = is_call(type) ? 1.0 : -1.0;
    const double intrinsic = sgn * (X - P->K);
    const int itm = intrinsic > 0.0;
    const double pay = D * (itm ? intrinsic : 0.0);
    out[0] = pay;
    for (int k = 0; k < NP; ++k)
        out[1 + k] = itm ? D * sgn * dX[k] : 0.0;
    out[1 + I_R] += -P->T * pay;
    out[1 + NP] = margin;
}

/* ------------------------------------------------------------------------ */
typedef struct {
    const or_params *P;
    int type, mode, tangent;
    uint32_t N, n_fix;
    const uint8_t *fix;
    const or_source *src;
    uint64_t first, lo, hi;
    double *out;
} or_job;

static void *run_job(void *arg)
{
    or_job *jb = (or_job *)arg;
    for (uint64_t row = jb->lo; row < jb->hi; ++row) {
        uint64_t path = jb->first + row;
        if (jb->tangent && jb->mode == OR_QE)
            tan_path_qe(jb->P, jb->type, jb->N, jb->fix, jb->n_fix, jb->src->seed, path,
                        jb->out + row * OR_TAN);
        else if (jb->tangent)
            tan_path(jb->P, jb->type, jb->N, jb->fix, jb->n_fix, jb->mode, jb->src, path, row,
                     jb->out + row * OR_TAN);
        else if (jb->mode == OR_QE)
            sim_path_qe(jb->P, jb->type, jb->N, jb->fix, jb->n_fix, jb->src->seed, path,
                        jb->out + row * OR_REC_QE);
        else
            sim_path(jb->P, jb->type, jb->N, jb->fix, jb->n_fix, jb->mode, jb->src, path, row,
                     jb->out + row * OR_REC);
    }
    return NULL;
}

/* Runs paths first .. first+n_paths-1.  fix_steps lists the Asian fixing
 * steps (values in 1..N, strictly increasing); NULL means every step for an
 * Asian and is ignored for a European.  za/zb: NULL for the Philox stream,
 * else caller normals [n_paths][N].  Returns 0, or -1 on a bad argument.    */
static int run(const or_params *P, int type, uint32_t N, const uint32_t *fix_steps, uint32_t n_fix,
               int mode, uint64_t seed, uint64_t first, uint64_t n_paths, const double *za,
               const double *zb, int n_threads, int tangent, double *out)
{
    if (N == 0 || type < 0 || type > OR_GEO_ASIAN_PUT || mode < OR_FULL_TRUNC || mode > OR_REFLECT)
        return -1;
    if (tangent && is_geo(type))
        return -1; /* the tangent path covers the European and arithmetic payoffs */
    if (tangent && mode != OR_FULL_TRUNC && mode != OR_ABSORB && mode != OR_QE)
        return -1; /* the tangent paths follow the Milstein and QE schemes */
    /* QE draws its own Philox inputs (no caller normals) and needs sigma > 0
     * and theta > 0. */
    if (mode == OR_QE && (za || zb || !(P->sigma > 0.0) || !(P->theta > 0.0)))
        return -1;
    uint8_t *fix = (uint8_t *)calloc((size_t)N + 1, 1);
    if (!fix)
        return -1;
    uint32_t nf = 0;
    if (is_asian(type) && fix_steps) {
        for (uint32_t i = 0; i < n_fix; ++i) {
            if (fix_steps[i] < 1 || fix_steps[i] > N || fix[fix_steps[i]]) {
                free(fix);
                return -1;
            }
            fix[fix_steps[i]] = 1;
            ++nf;
        }
    } else if (is_asian(type)) {
        for (uint32_t j = 1; j <= N; ++j)
            fix[j] = 1;
        nf = N;
    } else {
        fix[N] = 1;
        nf = 1;
    }
    if (nf == 0) {
        free(fix);
        return -1;
    }
    or_source src = { seed, za, zb, N };
    if (n_threads < 1)
        n_threads = 1;
    if ((uint64_t)n_threads > n_paths)
        n_threads = n_paths > 0 ? (int)n_paths : 1;
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    or_job *jobs = (or_job *)calloc((size_t)n_threads, sizeof(or_job));
    for (int t = 0; t < n_threads; ++t) {
        or_job jb = { P, type, mode, tangent, N, nf, fix, &src, first,
                      n_paths * (uint64_t)t / (uint64_t)n_threads,
                      n_paths * (uint64_t)(t + 1) / (uint64_t)n_threads, out };
        jobs[t] = jb;
        if (n_threads == 1)
            run_job(&jobs[t]);
        else
            pthread_create(&th[t], NULL, run_job, &jobs[t]);
    }
    if (n_threads > 1)
        for (int t = 0; t < n_threads; ++t)
            pthread_join(th[t], NULL);
    free(jobs);
    free(th);
    free(fix);
    return 0;
}

int or_simulate(const or_params *P, int type, uint32_t N, const uint32_t *fix_steps, uint32_t n_fix,
                int mode, uint64_t seed, uint64_t first, uint64_t n_paths, const double *za,
                const double *zb, int n_threads, double *rec_out)
{
    return run(P, type, N, fix_steps, n_fix, mode, seed, first, n_paths, za, zb, n_threads, 0,
               rec_out);
}

int or_tangent(const or_params *P, int type, uint32_t N, const uint32_t *fix_steps, uint32_t n_fix,
               int mode, uint64_t seed, uint64_t first, uint64_t n_paths, const double *za,
               const double *zb, int n_threads, double *tan_out)
{
    return run(P, type, N, fix_steps, n_fix, mode, seed, first, n_paths, za, zb, n_threads, 1,
               tan_out);
}

/* Bulk Philox normals for tests: za/zb [n_paths][N] for paths first.. */
void or_normals_block(uint64_t seed, uint64_t first, uint64_t n_paths, uint32_t N, double *za,
                      double *zb)
{
    for (uint64_t p = 0; p < n_paths; ++p)
        for (uint32_t j = 0; j < N; ++j)
            or_normals(seed, first + p, j, &za[p * N + j], &zb[p * N + j]);
}

/* Bulk QE inputs for tests: zs/zv/uv [n_paths][N] for paths first.. */
void or_qe_draws_block(uint64_t seed, uint64_t first, uint64_t n_paths, uint32_t N, double *zs,
                       double *zv, double *uv)
{
    for (uint64_t p = 0; p < n_paths; ++p)
        for (uint32_t j = 0; j < N; ++j)
            or_qe_draws(seed, first + p, j, &zs[p * N + j], &zv[p * N + j], &uv[p * N + j]);
}

void or_philox_block(const uint32_t *ctr, const uint32_t *key, uint64_t n, uint32_t *out)
{
    for (uint64_t i = 0; i < n; ++i)
        or_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}
