/*
 * FP64 CPU oracle for the Markovian engine's tau-leap step (FlashSpread,
 * arXiv 2604.22092, Section "Markovian engine", Algorithm "Markovian
 * Engine: One Tau-Leaping Step").
 *
 * TEST INFRASTRUCTURE: only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this.  It shares no code with the HIP
 * path (it has its own Philox).
 *
 * Rates are piecewise constant: a susceptible node i has rate beta * I_i,
 * I_i = sum over its incoming CSR row of 1{X_j = I} (the influence, unit
 * weights); an exposed node sigma; an infectious node gamma; a removed node
 * 0.  One step, in the algorithm's order:
 *   1. Lambda = sum_i lambda_i over all nodes
 *   2. tau = min(theta N / Lambda, p_max / max_i lambda_i, tau_max)
 *      (a zero denominator gives +inf, so with no positive rate tau = tau_max)
 *   3. p_i = 1 - exp(-lambda_i tau), evaluated as -expm1(-lambda_i tau)
 *   4. u_i from Philox4x32-10(ctr = (i, k mod 2^32, 0, 0), key = seed): word 0,
 *      top 24 bits times 2^-24; node i fires when u_i < p_i; no draw when
 *      lambda_i = 0
 *   5. transitions: SEIR  S->E->I->R;  SIR  S->I->R;  SIS  S->I->S
 *   6. the influence of every node is recomputed from the new states by its
 *      definition (the engine's two update modes must both give this value)
 *   7. exact counts after the step; the elapsed time advances by tau
 * The influence is recomputed from scratch (step 6), never updated
 * incrementally: that is the definition the GPU's sparse pushes and dense
 * recounts are checked against.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

enum { MK_S = 0, MK_E = 1, MK_I = 2, MK_R = 3 };
enum { MK_SEIR = 0, MK_SIR = 1, MK_SIS = 2 };

typedef struct {
    int32_t model; /* MK_SEIR, MK_SIR, MK_SIS */
    int32_t pad;
    double beta, sigma, gamma; /* per-edge infection rate, E->I rate, I->R (or I->S) rate */
    double theta, p_max, tau_max;
    uint64_t seed;
} mk_params;

/* Philox4x32-10 as in oracle.c (kept separate: this file shares nothing). */
static void mk_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static double mk_uniform(uint64_t seed, int64_t node, uint64_t step)
{
    uint32_t ctr[4] = {(uint32_t)node, (uint32_t)step, 0u, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    mk_philox(ctr, key, out);
    return (double)(out[0] >> 8) * (1.0 / 16777216.0);
}

/* Influence by definition: the infectious in-neighbours of every node. */
void mk_influence(int64_t n, const int32_t* row_ptr, const int32_t* col_ind, const int32_t* state, int32_t* infl)
{
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = 0;
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) c += state[col_ind[e]] == MK_I;
        infl[i] = c;
    }
}

static double mk_rate(const mk_params* p, int32_t x, int32_t infl)
{
    switch (x) {
    case MK_S: return p->beta * (double)infl;
    case MK_E: return p->sigma;
    case MK_I: return p->gamma;
    default: return 0.0;
    }
}

static int32_t mk_next(const mk_params* p, int32_t x)
{
    switch (x) {
    case MK_S: return p->model == MK_SEIR ? MK_E : MK_I;
    case MK_E: return MK_I;
    case MK_I: return p->model == MK_SIS ? MK_S : MK_R;
    default: return x;
    }
}

/* The step size of Algorithm "Markovian Engine" from the current rates. */
double mk_tau(const mk_params* p, int64_t n, const int32_t* state, const int32_t* infl, double* lam_sum,
              double* lam_max)
{
    double L = 0.0, M = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double l = mk_rate(p, state[i], infl[i]);
        L += l;
        if (l > M) M = l;
    }
    double tau = p->tau_max;
    if (L > 0.0) {
        double a = p->theta * (double)n / L;
        if (a < tau) tau = a;
    }
    if (M > 0.0) {
        double b = p->p_max / M;
        if (b < tau) tau = b;
    }
    if (lam_sum) *lam_sum = L;
    if (lam_max) *lam_max = M;
    return tau;
}

/*
 * One step k from `state` (updated in place) with `infl` the influence of
 * the current state (updated to that of the new state).  Returns tau;
 * counts[4] receives the counts after the step, *events the number of
 * nodes that fired.  Optional per-node logs (NULL to skip): lambda, p, u
 * (u = -1 where no draw was made).
 */
double mk_step(int64_t n, const int32_t* row_ptr, const int32_t* col_ind, const mk_params* p, uint64_t k,
               int32_t* state, int32_t* infl, int64_t counts[4], int64_t* events, double* log_lam,
               double* log_p, double* log_u)
{
    double tau = mk_tau(p, n, state, infl, NULL, NULL);
    int64_t ev = 0;
    for (int64_t i = 0; i < n; ++i) {
        double l = mk_rate(p, state[i], infl[i]);
        double q = -expm1(-l * tau);
        double u = -1.0;
        if (l > 0.0) {
            u = mk_uniform(p->seed, i, k);
            if (u < q) {
                state[i] = mk_next(p, state[i]);
                ev += 1;
            }
        }
        if (log_lam) log_lam[i] = l;
        if (log_p) log_p[i] = q;
        if (log_u) log_u[i] = u;
    }
    mk_influence(n, row_ptr, col_ind, state, infl);
    counts[0] = counts[1] = counts[2] = counts[3] = 0;
    for (int64_t i = 0; i < n; ++i) counts[state[i]] += 1;
    if (events) *events = ev;
    return tau;
}

/* n_steps steps from step index k0; history (n_steps x 4), taus (n_steps),
 * events (n_steps) may be NULL.  scratch: n int32 (the influence). */
void mk_run(int64_t n, const int32_t* row_ptr, const int32_t* col_ind, const mk_params* p, uint64_t k0,
            int64_t n_steps, int32_t* state, int32_t* scratch, int64_t* history, double* taus, int64_t* events)
{
    mk_influence(n, row_ptr, col_ind, state, scratch);
    for (int64_t s = 0; s < n_steps; ++s) {
        int64_t c[4], ev;
        double tau = mk_step(n, row_ptr, col_ind, p, k0 + (uint64_t)s, state, scratch, c, &ev, NULL, NULL, NULL);
        if (history) memcpy(history + 4 * s, c, sizeof c);
        if (taus) taus[s] = tau;
        if (events) events[s] = ev;
    }
}
