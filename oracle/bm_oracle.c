/*
 * bm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU oracle for the Monte Carlo integration of the
 * Brownian-motor Langevin equation (24) with the jump-adapted simplified
 * weak order 2.0 predictor-corrector scheme (Algorithms 1-4 of Spiechowicz,
 * Kostur & Machura, "GPU accelerated Monte Carlo simulation of Brownian motors
 * dynamics with CUDA").  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library; the product path never does.
 * It shares no code, header, table or constant generator with the HIP path.
 *
 * Everything is written out step by step in the order of the paper:
 *   - counter-based random numbers: Philox4x32-10 / Philox4x64-10
 *     (Salmon, Moraes, Dror & Shaw, SC'11, "Parallel random numbers: as easy
 *     as 1, 2, 3"), restated from that paper's definition;
 *   - Algorithm 2 / eq. (25): three-point Gaussian increment (and, for
 *     comparison, the normal increments it replaces);
 *   - Algorithm 3 / eqs. (3)-(6), (26)-(27): white Poissonian increment;
 *   - Algorithm 4 / eqs. (13)-(14), (29)-(30): dichotomous increment;
 *   - Algorithm 1: predictor-corrector step for eq. (24) (and the inertial
 *     extension x'' + gamma x' = ... used by the benchmark workloads);
 *   - Sec. 5 "Instruction optimization": folding of x modulo L;
 *   - eq. (31): time-averaged velocity estimator per path.
 *
 * Readings where the paper is silent (all shared with the HIP path and listed
 * in the design notes):
 *   R1  Within a step the constant forcing (Poisson bias -lambda*zeta,
 *       dichotomous level, periodic drive, tilt) is part of the drift and enters
 *       all three drift evaluations (eqs. 26, 30 say the equation *reduces* to
 *       one with that forcing between jumps); only the kick amplitude z is added
 *       once, in the corrector.  `literal_alg1` selects the as-printed variant
 *       (increments added in the corrector only) for tests.
 *   R2  [.] in Algorithms 3/4 is floor.
 *   R3  Jumps fall on the fixed dt grid through the integer countdown s.
 *   R4  Initial countdown/state: Poisson s0 = floor(E/(lambda dt)); the
 *       dichotomous state is drawn from its stationary law and entered through
 *       a flip at step 0 (d set to the opposite state, s = 0).
 *   R5  Random streams: key = (seed_lo, seed_hi), counter = (index, path,
 *       point, tag); tag 0 three-point draws, 1 Poisson kicks (two kicks per
 *       block, indexed by kick number), 2 initial conditions, 3 dichotomous
 *       dwell times (four flips per block, indexed by flip number).
 *   R6  The uniform phi of Algorithm 2 is consumed as base-6 digits: each
 *       32-bit word yields four digits (most significant first); digit 0 gives
 *       -G sqrt(3 dt), digit 1 gives +G sqrt(3 dt), digits 2..5 give 0.  For
 *       the jump draws phi = w * 2^-32, so 1 - phi > 0.
 *   R8  Inertial model: state (x, v), noise, kicks and forcing act on v.
 *   R9  F1 is evaluated at t_n and both F2 at t_{n+1}; the drive phase is the
 *       integer n mod spp.
 *   R10 x is folded into [0, L) after every step, w counts the periods.
 *
 * Build:  gcc -O2 -ffp-contract=off -fPIC -shared bm_oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox (Salmon et al., SC'11): N=4 words of width W, R rounds.            */
/* One round on (c0,c1,c2,c3) with key (k0,k1):                              */
/*   (hi0,lo0) = M0*c0, (hi1,lo1) = M1*c2   (full double-width products)     */
/*   out = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)                          */
/* and the key is bumped by the Weyl constants between rounds.               */
/* ------------------------------------------------------------------------ */

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 64-bit words: the full 128-bit product of two 64-bit words. */
static void mul64_full(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mul64_full(M0, c0, &hi0, &lo0);
        mul64_full(M1, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Model description (oracle's own types; not shared with the library).     */
/* ------------------------------------------------------------------------ */

enum { OR_OVERDAMPED = 0, OR_INERTIAL = 1 };
enum { OR_POT_SIN = 0,      /* V = sin(2 pi x), L = 1                    */
       OR_POT_RATCHET = 1,  /* V = -sin(2 pi x) - sin(4 pi x)/4, L = 1   */
       OR_POT_TENT = 2,     /* eq. (2): V = 1+x on [-1,0), 1-x on [0,1], L = 2 */
       OR_POT_FREE = 3,     /* V = 0 (test potential), L = 1             */
       OR_POT_HARMONIC = 4  /* V = k x^2/2 (test potential), no folding  */ };
enum { OR_GAUSS = 1, OR_POISSON = 2, OR_DICH = 4,
       OR_NORMAL = 8,      /* Gaussian noise with normal increments (non-simplified scheme) */
       OR_JUMP_GRID = 16   /* Poisson kicks at their exact times (jump-adapted grid)        */ };

typedef struct {
    int32_t dyn, pot, noise, literal_alg1;
    double gamma;              /* friction (inertial model)                     */
    double a, omega, F;        /* drive a cos(omega t) and constant tilt F       */
    double k_harm;             /* stiffness of the harmonic test potential       */
    double D;                  /* Gaussian intensity: G = sqrt(2D) or sqrt(2 gamma D) */
    double lambda, zeta;       /* eqs. (3)-(6): shot rate and mean amplitude     */
    double Fa, Fb, mua, mub;   /* eqs. (13)-(14): levels -Fa, +Fb; leaving rates */
    double dt;                 /* time step                                      */
    int64_t spp;               /* steps per drive period (0: no periodic drive)  */
    int64_t n_window;          /* eq. (31): step index of t_i                    */
    uint64_t seed;
    uint32_t point;
    uint32_t pad;
    double x0_lo, x0_hi, v0_lo, v0_hi;
    double step_tol;           /* step control on chi (0: fixed step dt)          */
    int32_t max_halvings;      /* step control: smallest step dt / 2^max_halvings */
    int32_t pad2;
} or_params;

typedef struct {
    double x;       /* position folded into [0, L)                     */
    int64_t w;      /* folded periods: unwrapped position = w*L + x    */
    double v;       /* velocity (inertial model)                       */
    double xi;      /* folded position at the window start             */
    int64_t wi;     /* folded periods at the window start              */
    int64_t sP;     /* Algorithm 3 countdown                           */
    double thP;     /* jump-adapted grid: fraction of its step at which the next kick falls */
    uint64_t kP;    /* Poisson kicks drawn so far                      */
    int64_t sD;     /* Algorithm 4 countdown                           */
    uint64_t mD;    /* dichotomous flips so far                        */
    int32_t d;      /* Algorithm 4 state: 0 -> -Fa, 1 -> +Fb           */
    int32_t lev;    /* step control: current step is dt / 2^lev        */
    uint64_t kA;    /* step control: steps taken (index of the Algorithm 2 draw) */
} or_path;

static const double PI = 3.14159265358979323846;

static double period_of(const or_params *P)
{
    return P->pot == OR_POT_TENT ? 2.0 : 1.0;
}

static void draw(const or_params *P, uint32_t index, uint64_t path, uint32_t tag, uint32_t out[4])
{
    uint32_t ctr[4] = { index, (uint32_t)path, P->point, tag };
    uint32_t key[2] = { (uint32_t)P->seed, (uint32_t)(P->seed >> 32) };
    or_philox4x32_10(ctr, key, out);
}

/* phi = w 2^-32 in [0,1); the exponential variate -ln(1 - phi) of eq. (27). */
static double expo_from_word(uint32_t w)
{
    double phi = (double)w * 0x1p-32;
    return -log(1.0 - phi);
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2 with eq. (25): the three-point increment at step n.           */
/* Returns -1, +1 or 0 (to be multiplied by G sqrt(3 dt)).                   */
/* ------------------------------------------------------------------------ */
int or_three_point(const or_params *P, uint64_t path, int64_t n)
{
    /* the n-th draw of the path's tag-0 stream */
    uint32_t w[4];
    draw(P, (uint32_t)(n / 16), path, 0u, w);
    uint32_t u = w[(n % 16) / 4];
    int digit_pos = (int)(n % 4);
    /* digit j of u (most significant first) = floor(6 * (6^j u mod 2^32) / 2^32) */
    for (int j = 0; j < digit_pos; ++j)
        u = (uint32_t)((uint64_t)u * 6u);          /* keep the fraction */
    int digit = (int)(((uint64_t)u * 6u) >> 32);
    if (digit == 0) return -1;      /* phi <= 1/6          */
    if (digit == 1) return +1;      /* 1/6 < phi <= 1/3    */
    return 0;                       /* otherwise           */
}

/* ------------------------------------------------------------------------ */
/* Non-simplified scheme (the Gaussian increments that eq. (25) replaces):   */
/* Delta xi ~ N(0, G^2 dt).  Standard normal z at step n by the Box-Muller   */
/* transform of words (2j, 2j+1) of block n/4, j = (n mod 4)/2:              */
/*   r = sqrt(-2 ln(1 - phi_1)), z = r cos(2 pi phi_2) (n even),             */
/*   z = r sin(2 pi phi_2) (n odd),  phi = w 2^-32.                          */
/* ------------------------------------------------------------------------ */
double or_normal(const or_params *P, uint64_t path, int64_t n)
{
    uint32_t w[4];
    draw(P, (uint32_t)(n / 4), path, 0u, w);
    int j = (int)((n % 4) / 2);
    double phi1 = (double)w[2 * j] * 0x1p-32;
    double phi2 = (double)w[2 * j + 1] * 0x1p-32;
    double r = sqrt(-2.0 * log(1.0 - phi1));
    return (n % 2 == 0) ? r * cos(2.0 * PI * phi2) : r * sin(2.0 * PI * phi2);
}

/* ------------------------------------------------------------------------ */
/* Potential force -V'(x).                                                   */
/* ------------------------------------------------------------------------ */
static double minus_dV(const or_params *P, double x)
{
    switch (P->pot) {
    case OR_POT_SIN:      /* V = sin(2 pi x) */
        return -2.0 * PI * cos(2.0 * PI * x);
    case OR_POT_RATCHET:  /* V = -sin(2 pi x) - sin(4 pi x)/4 */
        return 2.0 * PI * cos(2.0 * PI * x) + PI * cos(4.0 * PI * x);
    case OR_POT_TENT: {   /* eq. (2), period 2 */
        double y = x - 2.0 * floor(x / 2.0);       /* y in [0, 2) ~ x mod L */
        return (y <= 1.0) ? 1.0 : -1.0;           /* [0,1]: V=1-x; [-1,0): V=1+x */
    }
    case OR_POT_FREE:
        return 0.0;
    case OR_POT_HARMONIC:
        return -P->k_harm * x;
    }
    return 0.0;
}

/* Periodic drive plus tilt at step index j: a cos(omega t_j) + F with the
 * phase kept as the integer j mod spp (R9). */
static double drive(const or_params *P, int64_t j)
{
    if (P->spp <= 0) return P->F;
    int64_t k = j % P->spp;
    return P->a * cos(2.0 * PI * (double)k / (double)P->spp) + P->F;
}

/* Periodic drive plus tilt at the time t_j + theta dt inside step j (0 < theta < 1),
 * needed only on the jump-adapted grid. */
static double drive_at(const or_params *P, int64_t j, double theta)
{
    if (P->spp <= 0) return P->F;
    int64_t k = j % P->spp;
    return P->a * cos(2.0 * PI * ((double)k + theta) / (double)P->spp) + P->F;
}

/* Drift of eq. (24) (overdamped) or of the inertial extension, with the drive
 * value A and the constant-within-step forcing `c` (R1). */
static void drift(const or_params *P, double x, double v, double A, double c,
                  double *fx, double *fv)
{
    double f = minus_dV(P, x) + A + c;
    if (P->dyn == OR_INERTIAL) {
        *fx = v;
        *fv = -P->gamma * v + f;
    } else {
        *fx = f;
        *fv = 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Initial conditions (R4, tag 2).                                           */
/* ------------------------------------------------------------------------ */
static void fold(const or_params *P, or_path *s)
{
    if (P->pot == OR_POT_HARMONIC) return;
    double L = period_of(P);
    double k = floor(s->x / L);
    s->x = s->x - k * L;
    s->w = s->w + (int64_t)k;
}

void or_init(const or_params *P, uint64_t first_path, uint64_t count, or_path *out)
{
    for (uint64_t i = 0; i < count; ++i) {
        uint64_t p = first_path + i;
        or_path *s = &out[i];
        memset(s, 0, sizeof(*s));
        uint32_t I[4];
        draw(P, 0u, p, 2u, I);
        s->x = P->x0_lo + (P->x0_hi - P->x0_lo) * ((double)I[0] * 0x1p-32);
        s->v = (P->dyn == OR_INERTIAL)
             ? P->v0_lo + (P->v0_hi - P->v0_lo) * ((double)I[1] * 0x1p-32) : 0.0;
        s->w = 0;
        fold(P, s);
        if (P->noise & OR_POISSON) {
            if (P->noise & OR_JUMP_GRID) {
                /* first kick time in steps: whole steps before its step, fraction within it */
                double T = expo_from_word(I[2]) / (P->lambda * P->dt);
                s->sP = (int64_t)floor(T);
                s->thP = T - (double)s->sP;
            } else {
                s->sP = (int64_t)floor(expo_from_word(I[2]) / (P->lambda * P->dt));
            }
        }
        if (P->noise & OR_DICH) {
            /* stationary law: Pr{+Fb} = mu_a / (mu_a + mu_b) (rate into +Fb over total) */
            int dstar = ((double)I[3] * 0x1p-32 < P->mua / (P->mua + P->mub)) ? 1 : 0;
            s->d = 1 - dstar;     /* step 0 flips into dstar and draws its dwell */
            s->sD = 0;
        }
        /* step control starts from the smallest step and lets chi coarsen it */
        if (P->step_tol > 0) s->lev = P->max_halvings;
        if (P->n_window == 0) { s->xi = s->x; s->wi = s->w; }
    }
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 over one interval of length h: predictor-corrector with the   */
/* drive value A0 at its start and A1 at its end, constant forcing c, noise  */
/* increment dxi and kick z (added once, in the corrector).  `lit` is the    */
/* as-printed variant's extra forcing increment (R1).                         */
/* ------------------------------------------------------------------------ */
static void predictor_corrector(const or_params *P, double *px, double *pv, double h, double dxi,
                                double z, double c, double lit, double A0, double A1, double *chi)
{
    double x = *px, v = *pv;
    double F1x, F1v, F2x, F2v;
    double xb, vb;
    drift(P, x, v, A0, c, &F1x, &F1v);
    if (P->dyn == OR_INERTIAL) {
        xb = x + F1x * h;
        vb = v + F1v * h + dxi;
        drift(P, xb, vb, A1, c, &F2x, &F2v);
        xb = x + 0.5 * (F1x + F2x) * h;               /* predictor */
        vb = v + 0.5 * (F1v + F2v) * h + dxi;
        drift(P, xb, vb, A1, c, &F2x, &F2v);
        double xn = x + 0.5 * (F1x + F2x) * h;        /* corrector */
        double vn = v + 0.5 * (F1v + F2v) * h + dxi + z;
        /* local error estimate: predictor minus corrector (before the kick) */
        if (chi) *chi = fmax(fabs(xb - xn), fabs(vb - (vn - z)));
        vn += lit * h;
        *px = xn; *pv = vn;
    } else {
        xb = x + F1x * h + dxi;
        drift(P, xb, v, A1, c, &F2x, &F2v);
        xb = x + 0.5 * (F1x + F2x) * h + dxi;         /* predictor */
        drift(P, xb, v, A1, c, &F2x, &F2v);
        double xn = x + 0.5 * (F1x + F2x) * h + dxi + z; /* corrector */
        if (chi) *chi = fabs(xb - (xn - z));
        xn += lit * h;
        *px = xn;
    }
}

/* Gaussian noise intensity factor G of the component receiving the noise. */
static double noise_G(const or_params *P)
{
    return (P->dyn == OR_INERTIAL) ? sqrt(2.0 * P->gamma * P->D) : sqrt(2.0 * P->D);
}

/* Unit Gaussian increment of the interval that follows kick k on the
 * jump-adapted grid (tag 5, indexed by kick number like tag 0 by step):
 * three-point value in {-1, 0, +1} (to be scaled by G sqrt(3 h_sub)) or a
 * standard normal (to be scaled by G sqrt(h_sub)). */
static double kick_interval_noise(const or_params *P, uint64_t path, uint64_t k)
{
    uint32_t w[4];
    if (P->noise & OR_GAUSS) {
        draw(P, (uint32_t)(k / 16), path, 5u, w);
        uint32_t u = w[(k % 16) / 4];
        for (uint64_t j = 0; j < k % 4; ++j) u = (uint32_t)((uint64_t)u * 6u);
        int digit = (int)(((uint64_t)u * 6u) >> 32);
        return digit == 0 ? -1.0 : (digit == 1 ? 1.0 : 0.0);
    }
    if (P->noise & OR_NORMAL) {
        draw(P, (uint32_t)(k / 4), path, 5u, w);
        int j = (int)((k % 4) / 2);
        double phi1 = (double)w[2 * j] * 0x1p-32;
        double phi2 = (double)w[2 * j + 1] * 0x1p-32;
        double r = sqrt(-2.0 * log(1.0 - phi1));
        return (k % 2 == 0) ? r * cos(2.0 * PI * phi2) : r * sin(2.0 * PI * phi2);
    }
    return 0.0;
}

/* Algorithm 4 at one step of dt: flip and draw the new dwell when the countdown
 * has run out, else count down.  Returns the level Gamma over the step. */
static double dichotomous_step(const or_params *P, uint64_t path, or_path *s)
{
    if (!(P->noise & OR_DICH)) return 0.0;
    const double h = P->dt;
    if (s->sD <= 0) {
        uint32_t K[4];
        draw(P, (uint32_t)(s->mD / 4), path, 3u, K);
        s->d = 1 - s->d;
        double mu = s->d ? P->mub : P->mua;   /* rate of leaving the new state */
        s->sD = (int64_t)floor(expo_from_word(K[s->mD % 4]) / (mu * h));
        s->mD += 1;
    } else {
        s->sD -= 1;
    }
    return s->d ? P->Fb : -P->Fa;
}

/* Algorithm 3 on the fixed grid (R3) at one step of dt: when the countdown has run
 * out, the kick amplitude z (added at the end of the step) and the next countdown;
 * else count down and z = 0. */
static double poisson_fixed_step(const or_params *P, uint64_t path, or_path *s)
{
    if (!(P->noise & OR_POISSON)) return 0.0;
    const double h = P->dt;
    double z = 0.0;
    if (s->sP <= 0) {
        uint32_t J[4];
        draw(P, (uint32_t)(s->kP / 2), path, 1u, J);
        int half = (int)(s->kP % 2);
        s->sP = (int64_t)floor(expo_from_word(J[2 * half]) / (P->lambda * h));
        z = P->zeta * expo_from_word(J[2 * half + 1]);
        s->kP += 1;
    } else {
        s->sP -= 1;
    }
    return z;
}

/* ------------------------------------------------------------------------ */
/* One step n -> n+1 of one path.                                            */
/* ------------------------------------------------------------------------ */
static void step(const or_params *P, uint64_t path, int64_t n, or_path *s)
{
    const double h = P->dt;

    /* Algorithm 2: Gaussian increment, G = sqrt(2 D_G) (inertial: sqrt(2 gamma D)).
     * unit = the draw before its scale (three-point value or standard normal). */
    double dxi = 0.0, unit = 0.0;
    if (P->noise & OR_GAUSS) {
        unit = (double)or_three_point(P, path, n);
        dxi = unit * noise_G(P) * sqrt(3.0 * h);
    } else if (P->noise & OR_NORMAL) {
        unit = or_normal(P, path, n);
        dxi = unit * noise_G(P) * sqrt(h);
    }

    /* Algorithm 4: dichotomous increment (constant over the step). */
    double Gam = dichotomous_step(P, path, s);

    double bias = (P->noise & OR_POISSON) ? P->lambda * P->zeta : 0.0;

    if ((P->noise & OR_POISSON) && (P->noise & OR_JUMP_GRID)) {
        /* Jump-adapted grid: the kicks of this step fall at fractions theta of it;
         * the step is split at each, every piece integrated by Algorithm 1 with
         * its own length and Gaussian increment, the kick added at its end. */
        double c = Gam - bias;
        if (s->sP > 0) {
            s->sP -= 1;
            predictor_corrector(P, &s->x, &s->v, h, dxi, 0.0, c, 0.0, drive(P, n), drive(P, n + 1), NULL);
        } else {
            double from = 0.0, u = unit;
            double A_from = drive(P, n);
            for (;;) {
                double th = s->thP;                  /* next kick inside this step */
                double hs = (th - from) * h;
                double scale = (P->noise & OR_GAUSS) ? noise_G(P) * sqrt(3.0 * hs)
                                                     : noise_G(P) * sqrt(hs);
                double A_th = drive_at(P, n, th);
                uint32_t J[4];
                draw(P, (uint32_t)(s->kP / 2), path, 1u, J);
                int half = (int)(s->kP % 2);
                double z = P->zeta * expo_from_word(J[2 * half + 1]);
                predictor_corrector(P, &s->x, &s->v, hs, u * scale, z, c, 0.0, A_from, A_th, NULL);
                /* next kick time, counted from this one */
                double T = th + expo_from_word(J[2 * half]) / (P->lambda * h);
                u = kick_interval_noise(P, path, s->kP);
                s->kP += 1;
                s->sP = (int64_t)floor(T);
                s->thP = T - (double)s->sP;
                from = th;
                A_from = A_th;
                if (s->sP > 0) break;
            }
            /* last piece, to the end of the step */
            double hs = (1.0 - from) * h;
            double scale = (P->noise & OR_GAUSS) ? noise_G(P) * sqrt(3.0 * hs) : noise_G(P) * sqrt(hs);
            predictor_corrector(P, &s->x, &s->v, hs, u * scale, 0.0, c, 0.0, A_from, drive(P, n + 1), NULL);
            s->sP -= 1;
        }
    } else {
        /* Algorithm 3: Poissonian increment on the fixed grid (R3). */
        double z = poisson_fixed_step(P, path, s);
        /* Algorithm 1: predictor-corrector. */
        double c = P->literal_alg1 ? 0.0 : (Gam - bias);
        double lit = P->literal_alg1 ? (Gam - bias) : 0.0;
        predictor_corrector(P, &s->x, &s->v, h, dxi, z, c, lit, drive(P, n), drive(P, n + 1), NULL);
    }

    fold(P, s);                                     /* x mod L (Sec. 5) */
    if (n + 1 == P->n_window) { s->xi = s->x; s->wi = s->w; }
}

/* Advance `count` paths (first index first_path) from step n_from to n_to. */
void or_advance(const or_params *P, uint64_t first_path, uint64_t count,
                int64_t n_from, int64_t n_to, or_path *st)
{
    for (uint64_t i = 0; i < count; ++i)
        for (int64_t n = n_from; n < n_to; ++n)
            step(P, first_path + i, n, &st[i]);
}

/* ------------------------------------------------------------------------ */
/* Step-size control on chi (the paragraph after Algorithm 1: the difference  */
/* chi between predictor and corrector estimates the local error and may      */
/* steer the step size).  Our reading (the paper gives no controller):        */
/*  - steps are dt / 2^lev, 0 <= lev <= max_halvings (starting from the      */
/*    smallest), so every time reached                                         */
/*    lies on the grid of dt / 2^max_halvings and no step straddles a          */
/*    multiple of dt (a step may double only where the doubled step starts on  */
/*    its own grid);                                                           */
/*  - one controller serves a group of 64 consecutive paths (64 g ..          */
/*    64 g + 63, those below n_paths): after each step e = the largest         */
/*    max(|chi_x|, |chi_v|) over the group; e > tol halves the next step,     */
/*    e < tol / 16 doubles it (where allowed), otherwise it is kept;          */
/*  - every step is accepted (no rejection, so no sampling bias from           */
/*    redrawing), and step k of a path (counting steps of any size) takes      */
/*    the k-th three-point draw of its tag-0 stream scaled by G sqrt(3 h);     */
/*    without refinement this is the fixed-step scheme draw for draw;          */
/*  - the drive at t = (n + u / 2^J) dt is a cos(2 pi ((n mod spp) 2^J + u) /  */
/*    (spp 2^J)) + F, J = max_halvings;                                        */
/*  - the jump processes stay on the dt grid (Algorithms 3 and 4 as in the    */
/*    fixed-step scheme): the dichotomous level and the Poisson bias are       */
/*    drift over the whole interval [n dt, (n+1) dt), whatever its sub-steps,  */
/*    and a kick drawn at step n is added after its last sub-step; chi never   */
/*    includes the kick.  Normal increments and the jump-adapted grid are not  */
/*    combined with step control.                                              */
/* ------------------------------------------------------------------------ */
static double drive_sub(const or_params *P, int64_t n, int64_t u, int J)
{
    if (P->spp <= 0) return P->F;
    double scale = ldexp(1.0, J);
    double k = (double)(n % P->spp) * scale + (double)u;
    return P->a * cos(2.0 * PI * k / ((double)P->spp * scale)) + P->F;
}

/* Advance the group of paths st[0 .. count-1] (paths first_path .., one control
 * group: count <= 64) over the steps n_from .. n_to of length dt. */
static void advance_group(const or_params *P, uint64_t first_path, uint64_t count,
                          int64_t n_from, int64_t n_to, or_path *st)
{
    const int J = P->max_halvings;
    const int64_t full = (int64_t)1 << J;              /* one dt in grid units */
    const double G = noise_G(P);
    const double bias = (P->noise & OR_POISSON) ? P->lambda * P->zeta : 0.0;
    double chi[64], c[64], z[64];
    for (int64_t n = n_from; n < n_to; ++n) {
        for (uint64_t i = 0; i < count; ++i) {           /* jumps of this step of dt */
            double Gam = dichotomous_step(P, first_path + i, &st[i]);
            z[i] = poisson_fixed_step(P, first_path + i, &st[i]);
            c[i] = Gam - bias;
        }
        int64_t u = 0;                                 /* position inside [n, n+1) */
        while (u < full) {
            const int lev = st[0].lev;                 /* shared by the group */
            const int64_t hu = (int64_t)1 << (J - lev);
            const double h = P->dt * ldexp(1.0, -lev);
            const double A0 = drive_sub(P, n, u, J), A1 = drive_sub(P, n, u + hu, J);
            double e = 0.0;
            for (uint64_t i = 0; i < count; ++i) {
                or_path *s = &st[i];
                double dxi = 0.0;
                if (P->noise & OR_GAUSS)
                    dxi = (double)or_three_point(P, first_path + i, (int64_t)s->kA) * G * sqrt(3.0 * h);
                predictor_corrector(P, &s->x, &s->v, h, dxi, 0.0, c[i], 0.0, A0, A1, &chi[i]);
                s->kA += 1;
                if (chi[i] > e || chi[i] != chi[i]) e = chi[i] != chi[i] ? INFINITY : chi[i];
            }
            u += hu;
            int next = lev;
            if (e > P->step_tol) {
                if (lev < J) next = lev + 1;
            } else if (e < P->step_tol / 16.0 && lev > 0 && u % (2 * hu) == 0) {
                next = lev - 1;
            }
            for (uint64_t i = 0; i < count; ++i) st[i].lev = next;
        }
        for (uint64_t i = 0; i < count; ++i) {
            if (P->dyn == OR_INERTIAL) st[i].v += z[i];
            else st[i].x += z[i];
            fold(P, &st[i]);
            if (n + 1 == P->n_window) { st[i].xi = st[i].x; st[i].wi = st[i].w; }
        }
    }
}

/* Advance paths first_path .. first_path + count - 1 of an ensemble of n_paths
 * with step control from step n_from to n_to (in units of dt).  first_path must
 * start a group (a multiple of 64), and the paths must cover whole groups (count a
 * multiple of 64, or reaching n_paths).  Returns 0, or -1 for a misaligned range. */
int or_advance_adaptive(const or_params *P, uint64_t first_path, uint64_t count, uint64_t n_paths,
                        int64_t n_from, int64_t n_to, or_path *st)
{
    if (first_path % 64 != 0 || first_path + count > n_paths) return -1;
    if (count % 64 != 0 && first_path + count != n_paths) return -1;
    if (P->max_halvings < 0 || P->max_halvings > 20) return -1;
    if (P->noise & (OR_NORMAL | OR_JUMP_GRID)) return -1;
    for (uint64_t g = 0; g < count; g += 64) {
        uint64_t c = count - g < 64 ? count - g : 64;
        advance_group(P, first_path + g, c, n_from, n_to, st + g);
    }
    return 0;
}

/* eq. (31): per-path velocity ((x(t_f) - x(t_i)) / (t_f - t_i)), t_f = n_now dt. */
void or_velocity(const or_params *P, uint64_t count, const or_path *st, int64_t n_now, double *vp)
{
    double L = period_of(P);
    double T = (double)(n_now - P->n_window) * P->dt;
    for (uint64_t i = 0; i < count; ++i) {
        double dx = (double)(st[i].w - st[i].wi) * L + (st[i].x - st[i].xi);
        vp[i] = dx / T;
    }
}

/* Unwrapped position w*L + x. */
void or_unwrapped(const or_params *P, uint64_t count, const or_path *st, double *xu)
{
    double L = period_of(P);
    for (uint64_t i = 0; i < count; ++i)
        xu[i] = (double)st[i].w * L + st[i].x;
}

uint32_t or_sizeof_path(void) { return (uint32_t)sizeof(or_path); }
uint32_t or_sizeof_params(void) { return (uint32_t)sizeof(or_params); }
