/*
 * Exact event-driven simulation of the continuous-time SEIR renewal process on
 * a small contact graph.  TEST INFRASTRUCTURE: it exists only to pin the
 * tau-leap oracle against the true process it approximates; nothing else
 * uses it, and it shares no function with the oracle (holding times are
 * sampled directly from their laws, never through the hazard functions).
 *
 * The process (Section "Problem formulation", Fig. SEIR):
 *   S -> E  at rate beta * sum_{j in N_in(i)} w_ji 1{X_j = I}   (edge-driven, Markovian)
 *   E -> I  after a holding time drawn at entry from the E law   (renewal)
 *   I -> R  after a holding time drawn at entry from the I law   (renewal)
 *   R absorbing.
 * With constant shedding the infection rates are piecewise constant between
 * events, so the next infection is exponential with the total rate, redrawn
 * after every event (memorylessness); nodal transitions are scheduled times.
 * The paper cites this exact scheme family for non-Markovian networks
 * (Boguna et al. 2014) as the reference its tau-leaping approximates.
 */
#define _DEFAULT_SOURCE 1 /* M_PI, M_SQRT2 */
#include <math.h>
#include <stdint.h>

typedef struct {
    int32_t kind; /* 0 exp(rate a), 1 lognormal(mu a, sigma b), 2 weibull(shape a, scale b), 3 erlang(k, rate a) */
    int32_t k;
    double a, b;
} gx_dist;

typedef struct { uint64_t s; } gx_rng;

static uint64_t gx_next(gx_rng* r)
{
    /* splitmix64 (Steele, Lea & Flood 2014) */
    uint64_t z = (r->s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double gx_unif_open(gx_rng* r) /* uniform on (0, 1) */
{
    return ((double)(gx_next(r) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

static double gx_normal(gx_rng* r) /* Box-Muller */
{
    double u1 = gx_unif_open(r), u2 = gx_unif_open(r);
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

static double gx_holding(const gx_dist* d, gx_rng* r)
{
    switch (d->kind) {
    case 0: return d->a > 0.0 ? -log(gx_unif_open(r)) / d->a : INFINITY;
    case 1: return exp(d->a + d->b * gx_normal(r));
    case 2: return d->b * pow(-log(gx_unif_open(r)), 1.0 / d->a);
    case 3: {
        double s = 0.0;
        for (int32_t j = 0; j < d->k; ++j) s += -log(gx_unif_open(r));
        return s / d->a;
    }
    default: return NAN;
    }
}

/*
 * One realisation on [0, t_end].  init_state: 0=S 1=E 2=I 3=R at t = 0; nodes
 * that start in E or I draw a fresh holding time at t = 0 (age 0).
 * out_peak_I: max over [0, t_end] of the number of I nodes.
 * out_counts[4]: S, E, I, R at t_end.
 * Optional grid (n_grid times, ascending): out_grid (n_grid x 4) counts at each time.
 * Returns the number of events processed, or -1 when n exceeds the local limit.
 */
int64_t gx_run(int64_t n, const int32_t* row_ptr, const int32_t* col_ind, const float* weights,
               const gx_dist* ei, const gx_dist* ir, double beta, double t_end,
               const int32_t* init_state, uint64_t rng_seed, int64_t* out_peak_I,
               int64_t* out_counts, int64_t n_grid, const double* grid, int64_t* out_grid)
{
    enum { NMAX = 4096 };
    if (n > NMAX) return -1;
    int32_t x[NMAX];
    double t_next[NMAX];
    gx_rng rng = {rng_seed * 0xD1B54A32D192ED03ull + 0x632BE59BD9B4E019ull};
    int64_t cnt[4] = {0, 0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        x[i] = init_state[i];
        cnt[x[i]]++;
        if (x[i] == 1) t_next[i] = gx_holding(ei, &rng);
        else if (x[i] == 2) t_next[i] = gx_holding(ir, &rng);
        else t_next[i] = INFINITY;
    }
    int64_t peak = cnt[2];
    int64_t g = 0, events = 0;
    double t = 0.0;
    for (;;) {
        /* infection rates of susceptible nodes */
        double total = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (x[i] != 0) continue;
            double p = 0.0;
            for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
                if (x[col_ind[e]] == 2) p += weights ? (double)weights[e] : 1.0;
            total += beta * p;
        }
        double t_inf = total > 0.0 ? t - log(gx_unif_open(&rng)) / total : INFINITY;
        int64_t jn = -1;
        double t_nod = INFINITY;
        for (int64_t i = 0; i < n; ++i)
            if (t_next[i] < t_nod) { t_nod = t_next[i]; jn = i; }
        double t_ev = t_inf < t_nod ? t_inf : t_nod;
        /* report grid points passed before this event */
        while (g < n_grid && grid[g] < t_ev && grid[g] <= t_end) {
            for (int c = 0; c < 4; ++c) out_grid[4 * g + c] = cnt[c];
            ++g;
        }
        if (!(t_ev <= t_end)) break;
        t = t_ev;
        ++events;
        if (t_inf < t_nod) {
            /* choose the susceptible node proportionally to its rate */
            double target = gx_unif_open(&rng) * total, acc = 0.0;
            int64_t pick = -1, last = -1;
            for (int64_t i = 0; i < n; ++i) {
                if (x[i] != 0) continue;
                double p = 0.0;
                for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
                    if (x[col_ind[e]] == 2) p += weights ? (double)weights[e] : 1.0;
                if (p <= 0.0) continue;
                last = i;
                acc += beta * p;
                if (acc >= target) { pick = i; break; }
            }
            if (pick < 0) pick = last;
            cnt[0]--; cnt[1]++;
            x[pick] = 1;
            t_next[pick] = t + gx_holding(ei, &rng);
        } else {
            int32_t s = x[jn];
            cnt[s]--; cnt[s + 1]++;
            x[jn] = s + 1;
            if (s + 1 == 2) t_next[jn] = t + gx_holding(ir, &rng);
            else t_next[jn] = INFINITY;
        }
        if (cnt[2] > peak) peak = cnt[2];
    }
    while (g < n_grid) {
        for (int c = 0; c < 4; ++c) out_grid[4 * g + c] = cnt[c];
        ++g;
    }
    *out_peak_I = peak;
    for (int c = 0; c < 4; ++c) out_counts[c] = cnt[c];
    return events;
}

/* Many independent realisations (seed + rep) from the same initial state. */
void gx_run_many(int64_t reps, int64_t n, const int32_t* row_ptr, const int32_t* col_ind,
                 const float* weights, const gx_dist* ei, const gx_dist* ir, double beta,
                 double t_end, const int32_t* init_state, uint64_t rng_seed,
                 int64_t* out_peak_I /* reps */, int64_t* out_counts /* reps x 4 */)
{
    for (int64_t r = 0; r < reps; ++r)
        gx_run(n, row_ptr, col_ind, weights, ei, ir, beta, t_end, init_state,
               rng_seed + (uint64_t)r * 0x9E3779B97F4A7C15ull, out_peak_I + r,
               out_counts + 4 * r, 0, 0, 0);
}
