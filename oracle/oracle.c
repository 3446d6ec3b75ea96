/*
 * FP64 CPU oracle for the renewal tau-leap SEIR step (FlashSpread, arXiv 2604.22092).
 *
 * TEST INFRASTRUCTURE.  This file is the reference that the HIP library is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the library never does.  It shares no code,
 * header, table or constant generator with the HIP path.
 *
 * It is deliberately plain: one node after another, arithmetic in double,
 * no blocking, no fusion, no reordering beyond what the paper's definitions
 * state.  Every function cites the passage it follows.
 *
 * What one step computes (Algorithm 3 "per-call replay of b fused steps",
 * Eq. (influence), Eq. (infectivity), Proposition 1, Section "Bernoulli
 * tau-leaping"), for every node i of one replica r at step k, reading only
 * values from the start of the step:
 *   1. pressure  P_i = sum over incoming CSR row i of w_e * iota[col_e]
 *   2. rate      lambda_i = beta*P_i (S), h_EI(tau_i) (E), h_IR(tau_i) (I), 0 (R)
 *   3. prob.     q_i = 1 - exp(-lambda_i * dt), evaluated as -expm1(-lambda_i*dt)
 *   4. draw      u = (Philox4x32-10(ctr=(i, k mod 2^32, r, 0), key=seed)[0] >> 8) * 2^-24,
 *                fire = (u < q_i); no draw when lambda_i == 0
 *   5. state     X' = successor(X) when fire (S->E->I->R, R absorbing)
 *   6. age       reset to 0 on a transition, else advanced by dt (renewal property)
 *   7. infectivity for the next step  iota'_i = s(tau'_i) * 1{X'_i = I}, with the
 *      shedding profile s of Eq. (infectivity): s == 1 (constant shedding,
 *      Markovian edges), a scaled density A*f(tau) of a holding-time law, or a
 *      scaled hazard A*h(tau) (the in-kernel age-dependent form of the
 *      overhead study, Table "agedep_overhead")
 *   8. exact integer counts of S, E, I, R after the step
 *
 * Readings taken where the paper leaves a choice (each also listed in the
 * design notes of the repository):
 *   - beta is applied to the pressure, not folded into iota; iota is
 *     s(tau) 1{X = I} (mathematically the same product, Eq. (infectivity)).
 *   - the infectivity read by step k is that of the state and age at the
 *     start of step k (the pre-pass of Algorithm 3); writing it at the end of
 *     step k-1 from the new state and age, as the fused kernel does, is the
 *     same value.
 *   - the hazard is evaluated at the age at the start of the step.
 *   - the step size is fixed (the adaptive rule is not on this path).
 *   - FP32-storage ages advance as (float)((float)tau + (float)dt), mirroring
 *     the single-precision storage the method keeps; compact ages are integer
 *     step counts n with tau = n*dt, saturating at 65535.
 *   - compact storage keeps the infectivity in IEEE binary16 (Section
 *     "Mixed-precision storage with an fp32 accumulator", Table
 *     "mixed_precision_dtypes"): with an age-dependent profile the stored
 *     value is s(tau) rounded to the nearest binary16 (ties to even); the
 *     constant profile's 1 is exact.
 */
#define _DEFAULT_SOURCE 1 /* M_PI, M_SQRT2 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox counter-based generator (Salmon, Moraes, Dror & Shaw, "Parallel     */
/* Random Numbers: As Easy as 1, 2, 3", SC'11).  One round maps the counter   */
/* (x0, x1, x2, x3) under round key (k0, k1) to                               */
/*   (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),  hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0))      */
/* and the key is bumped by the Weyl constants (W0, W1) between rounds.       */
/* Ten rounds.  The 4x64 instance exists only so the round structure can be   */
/* checked against an independent library implementation.                    */
/* ------------------------------------------------------------------------ */

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        unsigned __int128 p0 = (unsigned __int128)M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Vector helpers for the test harness: n independent counters. */
void or_philox4x32_10_many(int64_t n, const uint32_t* ctr, const uint32_t key[2], uint32_t* out)
{
    for (int64_t j = 0; j < n; ++j) or_philox4x32_10(ctr + 4 * j, key, out + 4 * j);
}

void or_philox4x64_10_many(int64_t n, const uint64_t* ctr, const uint64_t key[2], uint64_t* out)
{
    for (int64_t j = 0; j < n; ++j) or_philox4x64_10(ctr + 4 * j, key, out + 4 * j);
}

/* The per-node uniform of step 4: word 0 of Philox4x32-10 at counter        */
/* (node, step mod 2^32, replica, 0) under key (seed low, seed high), top 24  */
/* bits scaled by 2^-24, so u lies on the grid {0, 2^-24, ..., 1 - 2^-24}.    */
double or_uniform(uint64_t seed, int64_t node, uint64_t step, uint32_t replica)
{
    uint32_t ctr[4] = {(uint32_t)node, (uint32_t)step, replica, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    or_philox4x32_10(ctr, key, out);
    return (double)(out[0] >> 8) * (1.0 / 16777216.0);
}

/* ------------------------------------------------------------------------ */
/* Scaled complementary error function erfcx(z) = exp(z^2) erfc(z), double.   */
/* Written out from its definition where that is accurate in double, with     */
/* the standard large-argument asymptotic series and the reflection identity  */
/* erfcx(-z) = 2 exp(z^2) - erfcx(z) elsewhere (the same identities the       */
/* paper's appendix on erfcx lists; here evaluated in double).                */
/* ------------------------------------------------------------------------ */

static double exp_of_square(double z)
{
    /* exp(z*z) with the rounding error of the square carried explicitly:     */
    /* z*z = s + e exactly, exp(s + e) = exp(s) * (1 + e + ...).              */
    double s = z * z;
    double e = fma(z, z, -s);
    return exp(s) * (1.0 + e);
}

double or_erfcx(double z)
{
    if (isnan(z)) return z;
    if (z < 0.0) {
        if (z < -26.7) return INFINITY; /* exp(z^2) beyond double range */
        return 2.0 * exp_of_square(z) - or_erfcx(-z);
    }
    if (z < 25.0) return exp_of_square(z) * erfc(z);
    /* asymptotic series: erfcx(z) ~ 1/(z sqrt(pi)) * sum_n (-1)^n (2n-1)!! / (2 z^2)^n; */
    /* at z >= 25 the eighth term is below 1e-20 relative.                        */
    double t = 1.0 / (2.0 * z * z);
    double term = 1.0, sum = 1.0;
    for (int n = 1; n <= 8; ++n) {
        term *= -(2.0 * n - 1.0) * t;
        sum += term;
    }
    return sum / (z * sqrt(M_PI));
}

void or_erfcx_many(int64_t n, const double* z, double* out)
{
    for (int64_t j = 0; j < n; ++j) out[j] = or_erfcx(z[j]);
}

/* ------------------------------------------------------------------------ */
/* Hazards h(tau) = f(tau) / S(tau) of the holding-time laws.                */
/* ------------------------------------------------------------------------ */

enum { OR_DIST_EXP = 0, OR_DIST_LOGNORMAL = 1, OR_DIST_WEIBULL = 2, OR_DIST_ERLANG = 3 };

typedef struct {
    int32_t kind; /* OR_DIST_* */
    int32_t k;    /* Erlang: integer shape >= 1 */
    double a;     /* EXP: rate; LOGNORMAL: mu of ln tau; WEIBULL: shape; ERLANG: rate */
    double b;     /* LOGNORMAL: sigma of ln tau; WEIBULL: scale */
} or_dist;

/* Proposition 1 (stable log-normal hazard):                                 */
/*   h(tau) = sqrt(2/pi) / (tau * sigma * erfcx(z)),  z = (ln tau - mu)/(sigma sqrt 2) */
/* with h(0) = 0 (the limit tau -> 0, where erfcx(z) -> infinity).             */
double or_hazard_lognormal(double tau, double mu, double sigma)
{
    if (!(tau > 0.0)) return 0.0;
    double z = (log(tau) - mu) / (sigma * M_SQRT2);
    double ex = or_erfcx(z);
    if (isinf(ex)) return 0.0;
    return sqrt(2.0 / M_PI) / (tau * sigma * ex);
}

/* Weibull(shape kk, scale lam): h(tau) = (kk/lam) (tau/lam)^(kk-1). */
double or_hazard_weibull(double tau, double shape, double scale)
{
    if (tau < 0.0) return 0.0;
    if (shape == 1.0) return 1.0 / scale;
    if (tau == 0.0) return 0.0; /* shape > 1 */
    return (shape / scale) * pow(tau / scale, shape - 1.0);
}

/* Erlang(k, rate theta): density theta (theta t)^(k-1) e^(-theta t) / (k-1)!,  */
/* survival e^(-theta t) sum_{n<k} (theta t)^n / n!; the exponentials cancel:   */
/*   h(tau) = theta * x^(k-1)/(k-1)!  /  sum_{n=0}^{k-1} x^n/n!,   x = theta*tau  */
double or_hazard_erlang(double tau, int32_t k, double rate)
{
    if (tau < 0.0) return 0.0;
    double x = rate * tau;
    double term = 1.0, sum = 1.0; /* term_n = x^n / n! */
    for (int32_t n = 1; n <= k - 1; ++n) {
        term = term * x / (double)n;
        sum += term;
    }
    return rate * term / sum;
}

double or_hazard(const or_dist* d, double tau)
{
    switch (d->kind) {
    case OR_DIST_EXP: return d->a;
    case OR_DIST_LOGNORMAL: return or_hazard_lognormal(tau, d->a, d->b);
    case OR_DIST_WEIBULL: return or_hazard_weibull(tau, d->a, d->b);
    case OR_DIST_ERLANG: return or_hazard_erlang(tau, d->k, d->a);
    default: return NAN;
    }
}

void or_hazard_many(const or_dist* d, int64_t n, const double* tau, double* out)
{
    for (int64_t j = 0; j < n; ++j) out[j] = or_hazard(d, tau[j]);
}

/* ------------------------------------------------------------------------ */
/* Densities f(tau) of the same laws, for shedding profiles s = A*f          */
/* (Eq. (infectivity): a log-normal density is the paper's example).          */
/* At tau = 0 they take their right limit (0 except for the exponential law,  */
/* Weibull shape 1 and Erlang k = 1, whose density starts at the rate).       */
/* ------------------------------------------------------------------------ */

/* log-normal: f = exp(-(ln tau - mu)^2 / (2 sigma^2)) / (tau sigma sqrt(2 pi)) */
double or_density_lognormal(double tau, double mu, double sigma)
{
    if (!(tau > 0.0)) return 0.0;
    double z = (log(tau) - mu) / sigma;
    return exp(-0.5 * z * z) / (tau * sigma * sqrt(2.0 * M_PI));
}

/* Weibull(shape kk, scale lam): f = (kk/lam) (tau/lam)^(kk-1) exp(-(tau/lam)^kk) */
double or_density_weibull(double tau, double shape, double scale)
{
    if (tau < 0.0) return 0.0;
    if (tau == 0.0) return shape == 1.0 ? 1.0 / scale : 0.0;
    double x = tau / scale;
    return (shape / scale) * pow(x, shape - 1.0) * exp(-pow(x, shape));
}

/* Erlang(k, rate theta): f = theta (theta tau)^(k-1) exp(-theta tau) / (k-1)! */
double or_density_erlang(double tau, int32_t k, double rate)
{
    if (tau < 0.0) return 0.0;
    if (tau == 0.0) return k == 1 ? rate : 0.0;
    double x = rate * tau;
    return rate * exp((double)(k - 1) * log(x) - x - lgamma((double)k));
}

double or_density(const or_dist* d, double tau)
{
    switch (d->kind) {
    case OR_DIST_EXP: return tau < 0.0 ? 0.0 : d->a * exp(-d->a * tau);
    case OR_DIST_LOGNORMAL: return or_density_lognormal(tau, d->a, d->b);
    case OR_DIST_WEIBULL: return or_density_weibull(tau, d->a, d->b);
    case OR_DIST_ERLANG: return or_density_erlang(tau, d->k, d->a);
    default: return NAN;
    }
}

void or_density_many(const or_dist* d, int64_t n, const double* tau, double* out)
{
    for (int64_t j = 0; j < n; ++j) out[j] = or_density(d, tau[j]);
}

/* ------------------------------------------------------------------------ */
/* One tau-leap step (Algorithm 3), FP64 arithmetic, node by node.           */
/* ------------------------------------------------------------------------ */

enum { OR_S = 0, OR_E = 1, OR_I = 2, OR_R = 3 };
enum { OR_AGE_DAYS_F32 = 0, OR_AGE_STEPS_U16 = 1 };

enum { OR_SHED_CONST = 0, OR_SHED_DENSITY = 1, OR_SHED_HAZARD = 2 };

typedef struct {
    or_dist ei, ir;
    double beta; /* per-edge transmission rate (per day) */
    double dt;   /* step size (days) */
    uint64_t seed;
    int32_t age_mode; /* OR_AGE_* */
    int32_t shed_mode; /* OR_SHED_*: s == 1, s = shed_scale*f, s = shed_scale*h of law `shed` */
    or_dist shed;
    double shed_scale;
} or_params;

/* Shedding profile s(tau) of an infectious node of age tau (Eq. (infectivity)). */
double or_shed(const or_params* p, double tau)
{
    switch (p->shed_mode) {
    case OR_SHED_CONST: return 1.0;
    case OR_SHED_DENSITY: return p->shed_scale * or_density(&p->shed, tau);
    case OR_SHED_HAZARD: return p->shed_scale * or_hazard(&p->shed, tau);
    default: return NAN;
    }
}

/* x rounded to the nearest IEEE 754 binary16 value, ties to even, returned as
 * a double.  binary16 keeps 11 significant bits: a value in [2^e, 2^(e+1)),
 * e >= -14, is a multiple of 2^(e-10); below 2^-14 (subnormals) every value
 * is a multiple of 2^-24.  The largest finite value is 65504; magnitudes from
 * 65520 up (the midpoint towards 2^16) round to infinity. */
double or_binary16(double x)
{
    if (isnan(x) || isinf(x) || x == 0.0) return x;
    const double a = fabs(x);
    if (a >= 65520.0) return copysign(INFINITY, x);
    int e2;
    (void)frexp(a, &e2);   /* a in [2^(e2-1), 2^e2) */
    int e = e2 - 1;
    if (e < -14) e = -14;
    const double quantum = ldexp(1.0, e - 10);
    return copysign(rint(a / quantum) * quantum, x); /* rint: ties to even */
}

void or_binary16_many(int64_t n, const double* x, double* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = or_binary16(x[i]);
}

/* The stored infectivity value of an infectious node: s(tau), in binary16
 * under compact storage. */
static double stored_shed(const or_params* p, double tau)
{
    const double v = or_shed(p, tau);
    return p->age_mode == OR_AGE_STEPS_U16 ? or_binary16(v) : v;
}

/* Infectivity of every node from its state and age: s(tau_i) 1{X_i = I}. */
void or_infectivity(int64_t n, const or_params* p, const int32_t* state, const float* age_days,
                    const uint16_t* age_steps, double* out)
{
    for (int64_t i = 0; i < n; ++i) {
        double tau = (p->age_mode == OR_AGE_DAYS_F32) ? (double)age_days[i] : (double)age_steps[i] * p->dt;
        out[i] = state[i] == OR_I ? stored_shed(p, tau) : 0.0;
    }
}

/* Per-node outcome, used both by the full step and by the sampled-node form. */
typedef struct {
    int32_t state;    /* X' */
    int32_t fired;
    float age_days;   /* tau' (age_mode DAYS) */
    uint16_t age_steps; /* n' (age_mode STEPS) */
    uint16_t pad;
    double pressure, lambda, q, u; /* u = -1 when no draw was made */
} or_node_out;

static void node_update(int64_t i, const int32_t* row_ptr, const int32_t* col_ind,
                        const float* weights, const or_params* p, uint64_t step,
                        uint32_t replica, int32_t x, float age_days, uint16_t age_steps,
                        const double* iota, or_node_out* o)
{
    /* 1. pressure over the incoming row, in CSR order (Eq. (influence)) */
    double P = 0.0;
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        double w = weights ? (double)weights[e] : 1.0;
        P += w * iota[col_ind[e]];
    }
    /* 2. rate from the state */
    double tau = (p->age_mode == OR_AGE_DAYS_F32) ? (double)age_days
                                                  : (double)age_steps * p->dt;
    double lam = 0.0;
    if (x == OR_S) lam = p->beta * P;
    else if (x == OR_E) lam = or_hazard(&p->ei, tau);
    else if (x == OR_I) lam = or_hazard(&p->ir, tau);
    /* 3. transition probability of the Bernoulli tau-leap */
    double q = -expm1(-lam * p->dt);
    /* 4. draw */
    int fire = 0;
    double u = -1.0;
    if (lam > 0.0) {
        u = or_uniform(p->seed, i, step, replica);
        fire = (u < q);
    }
    /* 5.-6. transition and renewal age */
    int32_t xn = fire ? x + 1 : x;
    o->state = xn;
    o->fired = fire;
    if (fire) {
        o->age_days = 0.0f;
        o->age_steps = 0;
    } else {
        o->age_days = (float)(age_days + (float)p->dt);
        o->age_steps = (uint16_t)(age_steps < 65535 ? age_steps + 1 : 65535);
    }
    o->pressure = P;
    o->lambda = lam;
    o->q = q;
    o->u = u;
}

/*
 * Full step over all n nodes of one replica.  state/age are updated in place
 * (each node owns its slot and no node reads another's state or age);
 * iota_in is the start-of-step infectivity, iota_out receives the next one.
 * Optional per-node logs (may be NULL): lambda, q, u (u = -1 when not drawn).
 * counts[4] receives the exact S, E, I, R tallies after the step.
 */
void or_step(int64_t n, const int32_t* row_ptr, const int32_t* col_ind, const float* weights,
             const or_params* p, uint64_t step, uint32_t replica, int32_t* state,
             float* age_days, uint16_t* age_steps, const double* iota_in, double* iota_out,
             int64_t counts[4], double* log_lambda, double* log_q, double* log_u)
{
    counts[0] = counts[1] = counts[2] = counts[3] = 0;
    for (int64_t i = 0; i < n; ++i) {
        or_node_out o;
        float ad = age_days ? age_days[i] : 0.0f;
        uint16_t as = age_steps ? age_steps[i] : 0;
        node_update(i, row_ptr, col_ind, weights, p, step, replica, state[i], ad, as, iota_in, &o);
        state[i] = o.state;
        if (age_days) age_days[i] = o.age_days;
        if (age_steps) age_steps[i] = o.age_steps;
        /* 7. next-step infectivity (Eq. (infectivity)) from the new state and age */
        double tau_new = (p->age_mode == OR_AGE_DAYS_F32) ? (double)o.age_days : (double)o.age_steps * p->dt;
        iota_out[i] = (o.state == OR_I) ? stored_shed(p, tau_new) : 0.0;
        counts[o.state] += 1;
        if (log_lambda) log_lambda[i] = o.lambda;
        if (log_q) log_q[i] = o.q;
        if (log_u) log_u[i] = o.u;
    }
}

/*
 * The same update evaluated for a list of nodes only, from a full snapshot of
 * the start-of-step state (used to check very large instances node by node).
 * Outputs are per listed node; nothing is written back.
 */
void or_step_nodes(int64_t n, const int32_t* row_ptr, const int32_t* col_ind, const float* weights,
                   const or_params* p, uint64_t step, uint32_t replica, const int32_t* state,
                   const float* age_days, const uint16_t* age_steps, const double* iota,
                   int64_t m, const int64_t* nodes, int32_t* out_state, float* out_age_days,
                   uint16_t* out_age_steps, double* out_lambda, double* out_q, double* out_u)
{
    (void)n;
    for (int64_t j = 0; j < m; ++j) {
        int64_t i = nodes[j];
        or_node_out o;
        node_update(i, row_ptr, col_ind, weights, p, step, replica, state[i],
                    age_days ? age_days[i] : 0.0f, age_steps ? age_steps[i] : 0, iota, &o);
        out_state[j] = o.state;
        if (out_age_days) out_age_days[j] = o.age_days;
        if (out_age_steps) out_age_steps[j] = o.age_steps;
        if (out_lambda) out_lambda[j] = o.lambda;
        if (out_q) out_q[j] = o.q;
        if (out_u) out_u[j] = o.u;
    }
}

/*
 * A whole trajectory of n_steps steps for one replica, starting at step index
 * step0 with the given state/age (iota is built from the state and age).
 * history (n_steps x 4, may be NULL) receives the counts after every step.
 * scratch must hold 2*n doubles (the two infectivity buffers).
 */
void or_run(int64_t n, const int32_t* row_ptr, const int32_t* col_ind, const float* weights,
            const or_params* p, uint64_t step0, int64_t n_steps, uint32_t replica,
            int32_t* state, float* age_days, uint16_t* age_steps, double* scratch,
            int64_t* history)
{
    double* cur = scratch;
    double* nxt = scratch + n;
    or_infectivity(n, p, state, age_days, age_steps, cur);
    int64_t counts[4];
    for (int64_t s = 0; s < n_steps; ++s) {
        or_step(n, row_ptr, col_ind, weights, p, step0 + (uint64_t)s, replica, state, age_days,
                age_steps, cur, nxt, counts, NULL, NULL, NULL);
        if (history) memcpy(history + 4 * s, counts, sizeof counts);
        double* t = cur; cur = nxt; nxt = t;
    }
}

/* ------------------------------------------------------------------------ */
/* Adaptive step size (Section "Bernoulli tau-leaping", adaptive step        */
/* selection; the tau update that closes each fused step of Algorithm 3).    */
/* ------------------------------------------------------------------------ */

/* The step that follows a step whose largest rate over all nodes was
 * lam_max: min(dt_max, eps / (lam_max + delta)).  With lam_max + delta = 0
 * the quotient is +inf and the cap applies. */
double or_next_dt(double lam_max, double eps, double dt_max, double delta)
{
    double d = eps / (lam_max + delta);
    return d < dt_max ? d : dt_max;
}

/*
 * An adaptive trajectory of n_steps steps for one replica (ages in days):
 * the first step uses dt_max; every later step uses or_next_dt of the
 * largest rate lambda_i of the step before it, over all nodes.  dts
 * (n_steps, may be NULL) receives the step sizes used, history (n_steps x 4,
 * may be NULL) the counts.  scratch must hold 3*n doubles.  p->dt is ignored.
 */
void or_run_adaptive(int64_t n, const int32_t* row_ptr, const int32_t* col_ind, const float* weights,
                     const or_params* p, double eps, double dt_max, double delta, uint64_t step0,
                     int64_t n_steps, uint32_t replica, int32_t* state, float* age_days, double* scratch,
                     int64_t* history, double* dts)
{
    double* cur = scratch;
    double* nxt = scratch + n;
    double* lam = scratch + 2 * n;
    or_params q = *p;
    q.age_mode = OR_AGE_DAYS_F32;
    q.dt = dt_max;
    or_infectivity(n, &q, state, age_days, NULL, cur);
    int64_t counts[4];
    for (int64_t s = 0; s < n_steps; ++s) {
        or_step(n, row_ptr, col_ind, weights, &q, step0 + (uint64_t)s, replica, state, age_days, NULL,
                cur, nxt, counts, lam, NULL, NULL);
        if (history) memcpy(history + 4 * s, counts, sizeof counts);
        if (dts) dts[s] = q.dt;
        double lam_max = 0.0;
        for (int64_t i = 0; i < n; ++i)
            if (lam[i] > lam_max) lam_max = lam[i];
        q.dt = or_next_dt(lam_max, eps, dt_max, delta);
        double* t = cur; cur = nxt; nxt = t;
    }
}
