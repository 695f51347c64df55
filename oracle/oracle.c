/*
 * FP64 CPU ORACLE for population-annealing molecular dynamics (PAMD).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it (through oracle/oracle.py).  It shares no code,
 * header, table or constant generator with the HIP path.
 *
 * Follows Christiansen, Weigel & Janke, "Accelerating molecular dynamics
 * simulations with population annealing" (arXiv:1806.06016):
 *   - PAMD scheme, step 1: R independent copies at T0         -> ora_init_velocities
 *   - PAMD scheme, step 3: theta NVT MD steps per copy         -> ora_md_steps
 *     (velocity Verlet; stochastic thermostat required so that copies made by
 *      resampling decorrelate -- paragraph after Fig. 1; Andersen collisions)
 *   - PAMD scheme, step 2: weights tau_j = exp(-(beta_i - beta_{i-1}) E_j) / Q,
 *     Q = (1/R) sum_j exp(-(beta_i - beta_{i-1}) E_j)          -> ora_lse / ora_counts
 *   - free energy from the recorded normalisers Q (paragraph before Fig. 2)
 * Force-field form (the paper uses AMBER ff94 for met-enkephalin; parameters
 * here are synthetic): harmonic bonds and angles, Fourier dihedrals,
 * all-pairs Lennard-Jones + Coulomb with 1-2/1-3 exclusions and scaled 1-4 pairs.
 *
 * Everything is double precision, straightforward loops, OpenMP over replicas
 * only.  Random numbers: Philox-4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC'11), written from that definition.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox-4x32-10 (SC'11): 10 rounds of the 4-word S-box, key bumped by the  */
/* Weyl constants between rounds.                                             */
/* ------------------------------------------------------------------------ */
#define PH_M0 0xD2511F53u
#define PH_M1 0xCD9E8D57u
#define PH_W0 0x9E3779B9u
#define PH_W1 0xBB67AE85u

void ora_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PH_W0;
            k1 += PH_W1;
        }
        uint64_t p0 = (uint64_t)PH_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PH_M1 * (uint64_t)c2;
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

/* stream identities of the counter's fourth word */
enum { ST_COLLIDE = 0, ST_VELOCITY = 1, ST_RESAMPLE = 2, ST_INIT = 3, ST_MULTINOMIAL = 4, ST_LANGEVIN = 5 };

typedef struct {
    uint32_t seed_lo, seed_hi, run, pad;
} ora_rng;

static void draw(const ora_rng* g, uint32_t slot, uint32_t step, uint32_t block,
                 uint32_t stream, uint32_t out[4])
{
    uint32_t ctr[4] = {slot, step, block, stream};
    uint32_t key[2] = {g->seed_lo, g->seed_hi + g->run};
    ora_philox4x32_10(ctr, key, out);
}

/* 24-bit uniform in (0,1): ((w >> 8) + 1/2) 2^-24 */
static double u24(uint32_t w) { return ((double)(w >> 8) + 0.5) * (1.0 / 16777216.0); }

/* Box-Muller: three standard normals from one 4-word draw */
static void normals3(const uint32_t w[4], double z[3])
{
    const double two_pi = 6.283185307179586476925286766559;
    double r0 = sqrt(-2.0 * log(u24(w[0])));
    double a0 = two_pi * u24(w[1]);
    double r1 = sqrt(-2.0 * log(u24(w[2])));
    double a1 = two_pi * u24(w[3]);
    z[0] = r0 * cos(a0);
    z[1] = r0 * sin(a0);
    z[2] = r1 * cos(a1);
}

/* Collision test word for atom a: block (a mod 16) + 16 floor(a / 64),
 * word floor(a / 16) mod 4 of that block. */
static uint32_t collide_block(int a) { return (uint32_t)((a & 15) + 16 * (a >> 6)); }
static int collide_word(int a) { return (a >> 4) & 3; }

/* ------------------------------------------------------------------------ */
/* system description                                                        */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n;                 /* atoms */
    const double* mass;        /* [n] */
    const double* charge;      /* [n] */
    const double* sigma;       /* [n] */
    const double* eps;         /* [n] */
    int32_t nb;
    const int32_t* bidx;       /* [nb][2] */
    const double* bk;
    const double* br0;
    int32_t na;
    const int32_t* aidx;       /* [na][3], centre in the middle */
    const double* ak;
    const double* at0;
    int32_t nd;
    const int32_t* didx;       /* [nd][4] */
    const double* dk;
    const int32_t* dn;
    const double* ddelta;
    int32_t np;                /* non-excluded pairs i<j */
    const int32_t* pidx;       /* [np][2] */
    const double* ps_lj;       /* [np] scale of the LJ term */
    const double* ps_c;        /* [np] scale of the Coulomb term */
    double coulomb_k;
    int32_t dielectric;        /* 0: k q q / r   1: k q q / (4 r^2) */
    int32_t pad;
} ora_sys;

enum { T_BOND = 1, T_ANGLE = 2, T_DIHEDRAL = 4, T_LJ = 8, T_COUL = 16, T_ALL = 31 };

static inline void sub3(const double* a, const double* b, double* o)
{
    o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static inline double dot3(const double* a, const double* b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static inline void cross3(const double* a, const double* b, double* o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/*
 * Potential energy and (optionally) forces F = -grad U of one configuration.
 * x, f: [n][3].  eterm (optional): per-term energies {bond, angle, dihedral, LJ, Coulomb}.
 *
 *   bonds      U = 1/2 k (|r_ij| - r0)^2
 *   angles     U = 1/2 k (theta - theta0)^2, theta = atan2(|u x w|, u.w)
 *   dihedrals  U = k (1 + cos(n phi - delta)), phi = atan2(|b2| b1.n2, n1.n2),
 *              b1 = x_j - x_i, b2 = x_k - x_j, b3 = x_l - x_k, n1 = b1 x b2, n2 = b2 x b3
 *   LJ         U = s 4 eps_ij ((sigma_ij/r)^12 - (sigma_ij/r)^6),
 *              sigma_ij = (sigma_i + sigma_j)/2, eps_ij = sqrt(eps_i eps_j)
 *   Coulomb    U = s k_e q_i q_j / r          (vacuum)
 *              U = s k_e q_i q_j / (4 r^2)    (dielectric eps(r) = 4 r)
 */
double ora_energy_forces(const ora_sys* s, const double* x, double* f, double* eterm, int32_t mask)
{
    const int n = s->n;
    double eb = 0, ea = 0, ed = 0, elj = 0, ec = 0;
    if (f)
        memset(f, 0, sizeof(double) * 3 * n);

    if (mask & T_BOND) {
        for (int t = 0; t < s->nb; ++t) {
            int i = s->bidx[2 * t], j = s->bidx[2 * t + 1];
            double d[3];
            sub3(&x[3 * i], &x[3 * j], d);
            double r = sqrt(dot3(d, d));
            double dr = r - s->br0[t];
            eb += 0.5 * s->bk[t] * dr * dr;
            if (f) {
                /* dU/dx_i = k (r - r0) d / r ; at r = 0 the zero-rest-length
                 * spring has the smooth gradient k d */
                double g = (s->br0[t] == 0.0) ? s->bk[t] : s->bk[t] * dr / r;
                for (int c = 0; c < 3; ++c) {
                    f[3 * i + c] -= g * d[c];
                    f[3 * j + c] += g * d[c];
                }
            }
        }
    }

    if (mask & T_ANGLE) {
        for (int t = 0; t < s->na; ++t) {
            int i = s->aidx[3 * t], j = s->aidx[3 * t + 1], k = s->aidx[3 * t + 2];
            double u[3], w[3], cx[3];
            sub3(&x[3 * i], &x[3 * j], u);
            sub3(&x[3 * k], &x[3 * j], w);
            cross3(u, w, cx);
            double sn = sqrt(dot3(cx, cx));
            double cs = dot3(u, w);
            double theta = atan2(sn, cs);
            double dth = theta - s->at0[t];
            ea += 0.5 * s->ak[t] * dth * dth;
            if (f) {
                double lu = sqrt(dot3(u, u)), lw = sqrt(dot3(w, w));
                double cost = cs / (lu * lw);
                double sint = sn / (lu * lw);
                if (sint < 1e-8)
                    sint = 1e-8;
                double dUdth = s->ak[t] * dth;
                /* d theta / d x_i = (cos theta u^ - w^) / (|u| sin theta) */
                for (int c = 0; c < 3; ++c) {
                    double gi = (cost * u[c] / lu - w[c] / lw) / (lu * sint);
                    double gk = (cost * w[c] / lw - u[c] / lu) / (lw * sint);
                    f[3 * i + c] -= dUdth * gi;
                    f[3 * k + c] -= dUdth * gk;
                    f[3 * j + c] += dUdth * (gi + gk);
                }
            }
        }
    }

    if (mask & T_DIHEDRAL) {
        for (int t = 0; t < s->nd; ++t) {
            int i = s->didx[4 * t], j = s->didx[4 * t + 1], k = s->didx[4 * t + 2], l = s->didx[4 * t + 3];
            double b1[3], b2[3], b3[3], n1[3], n2[3];
            sub3(&x[3 * j], &x[3 * i], b1);
            sub3(&x[3 * k], &x[3 * j], b2);
            sub3(&x[3 * l], &x[3 * k], b3);
            cross3(b1, b2, n1);
            cross3(b2, b3, n2);
            double lb2 = sqrt(dot3(b2, b2));
            /* phi = atan2(|b2| b1.(b2 x b3), (b1 x b2).(b2 x b3)) */
            double phi = atan2(lb2 * dot3(b1, n2), dot3(n1, n2));
            double nn = (double)s->dn[t];
            ed += s->dk[t] * (1.0 + cos(nn * phi - s->ddelta[t]));
            if (f) {
                double dUdphi = -s->dk[t] * nn * sin(nn * phi - s->ddelta[t]);
                double n1sq = dot3(n1, n1), n2sq = dot3(n2, n2);
                if (n1sq < 1e-24) n1sq = 1e-24;
                if (n2sq < 1e-24) n2sq = 1e-24;
                /* gradient of phi (Blondel & Karplus 1996 form) */
                double gi[3], gl[3];
                for (int c = 0; c < 3; ++c) {
                    gi[c] = -lb2 / n1sq * n1[c];
                    gl[c] = lb2 / n2sq * n2[c];
                }
                double p = dot3(b1, b2) / (lb2 * lb2);
                double q = dot3(b3, b2) / (lb2 * lb2);
                for (int c = 0; c < 3; ++c) {
                    double gj = (-1.0 - p) * gi[c] + q * gl[c];
                    double gk = p * gi[c] + (-1.0 - q) * gl[c];
                    f[3 * i + c] -= dUdphi * gi[c];
                    f[3 * j + c] -= dUdphi * gj;
                    f[3 * k + c] -= dUdphi * gk;
                    f[3 * l + c] -= dUdphi * gl[c];
                }
            }
        }
    }

    if (mask & (T_LJ | T_COUL)) {
        for (int t = 0; t < s->np; ++t) {
            int i = s->pidx[2 * t], j = s->pidx[2 * t + 1];
            double d[3];
            sub3(&x[3 * i], &x[3 * j], d);
            double r2 = dot3(d, d);
            double r = sqrt(r2);
            double g = 0.0; /* -dU/dr / r : force on i = g d */
            if (mask & T_LJ) {
                double sig = 0.5 * (s->sigma[i] + s->sigma[j]);
                double ep = sqrt(s->eps[i] * s->eps[j]);
                double sr6 = pow(sig / r, 6.0);
                double sr12 = sr6 * sr6;
                double sc = s->ps_lj[t];
                elj += sc * 4.0 * ep * (sr12 - sr6);
                g += sc * 24.0 * ep * (2.0 * sr12 - sr6) / r2;
            }
            if (mask & T_COUL) {
                double qq = s->coulomb_k * s->charge[i] * s->charge[j] * s->ps_c[t];
                if (s->dielectric == 0) {
                    ec += qq / r;
                    g += qq / (r2 * r);
                } else {
                    ec += qq / (4.0 * r2);
                    g += 2.0 * qq / (4.0 * r2 * r2);
                }
            }
            if (f) {
                for (int c = 0; c < 3; ++c) {
                    f[3 * i + c] += g * d[c];
                    f[3 * j + c] -= g * d[c];
                }
            }
        }
    }

    if (eterm) {
        eterm[0] = eb; eterm[1] = ea; eterm[2] = ed; eterm[3] = elj; eterm[4] = ec;
    }
    return eb + ea + ed + elj + ec;
}

/* batched energy/forces over R configurations x[R][n][3] */
void ora_energy_forces_batch(const ora_sys* s, int32_t R, const double* x, double* f, double* E,
                             double* eterm, int32_t mask)
{
    const int n = s->n;
#pragma omp parallel for schedule(dynamic, 4)
    for (int r = 0; r < R; ++r)
        E[r] = ora_energy_forces(s, x + (size_t)r * 3 * n, f ? f + (size_t)r * 3 * n : NULL,
                                 eterm ? eterm + (size_t)5 * r : NULL, mask);
}

/* ------------------------------------------------------------------------ */
/* PAMD step 1: Maxwell-Boltzmann velocities at T (stream 3)                 */
/* ------------------------------------------------------------------------ */
void ora_init_velocities(const ora_sys* s, const ora_rng* g, int32_t R, const uint32_t* slot,
                         double kB, double T, double* v)
{
    const int n = s->n;
#pragma omp parallel for schedule(static)
    for (int r = 0; r < R; ++r) {
        uint32_t sl = slot ? slot[r] : (uint32_t)r;
        for (int a = 0; a < n; ++a) {
            uint32_t w[4];
            double z[3];
            draw(g, sl, 0u, (uint32_t)a, ST_INIT, w);
            normals3(w, z);
            double sd = sqrt(kB * T / s->mass[a]);
            for (int c = 0; c < 3; ++c)
                v[(size_t)r * 3 * n + 3 * a + c] = sd * z[c];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* PAMD step 3: theta NVT velocity-Verlet steps, Andersen or Langevin bath  */
/* ------------------------------------------------------------------------ */
typedef struct {
    double dt;
    double kB;
    double T;                /* bath temperature of this block */
    uint32_t p24;            /* collide iff (w >> 8) < p24 ; p24 = round((1 - e^{-nu dt}) 2^24) */
    uint32_t step0;          /* global step counter of the first step */
    int32_t n_steps;
    int32_t mask;            /* force-field terms (T_ALL normally) */
    double gamma;            /* Langevin friction (1/time); used when langevin != 0 */
    int32_t langevin;        /* 0: Andersen collisions (p24), 1: Langevin bath */
    int32_t pad;
} ora_md;

/*
 * x, v: [R][n][3] (in/out).  For every replica independently:
 *   F = F(x)
 *   Andersen (velocity Verlet + collisions), repeat n_steps:
 *     v += dt/2 F/m ; x += dt v ; F = F(x) ; v += dt/2 F/m ;
 *     each atom collides with probability p: v_a ~ N(0, kB T / m_a)
 *   Langevin (the B-A-O-A-B splitting of Leimkuhler & Matthews, 2013: velocity
 *   Verlet whose drift is split around an exact Ornstein-Uhlenbeck step),
 *   repeat n_steps:
 *     v += dt/2 F/m ; x += dt/2 v ;
 *     v = c1 v + c2 sqrt(kB T / m) xi,  c1 = exp(-gamma dt), c2 = sqrt(1 - c1^2),
 *         xi: three normals of stream 5, counter (slot, step, atom, 5) ;
 *     x += dt/2 v ; F = F(x) ; v += dt/2 F/m
 *   E_pot = U(x), E_kin = sum 1/2 m v^2 at the end.
 * collisions (optional) counts collided atoms per replica (Andersen).
 */
void ora_md_steps(const ora_sys* s, const ora_rng* g, const ora_md* p, int32_t R,
                  const uint32_t* slot, double* x, double* v, double* Epot, double* Ekin,
                  int64_t* collisions)
{
    const int n = s->n;
#pragma omp parallel
    {
        double* F = (double*)malloc(sizeof(double) * 3 * n);
#pragma omp for schedule(dynamic, 2)
        for (int r = 0; r < R; ++r) {
            double* xr = x + (size_t)r * 3 * n;
            double* vr = v + (size_t)r * 3 * n;
            uint32_t sl = slot ? slot[r] : (uint32_t)r;
            int64_t ncol = 0;
            ora_energy_forces(s, xr, F, NULL, p->mask);
            const double c1 = exp(-p->gamma * p->dt);
            const double c2 = sqrt(1.0 - c1 * c1);
            for (int st = 0; st < p->n_steps; ++st) {
                uint32_t step = p->step0 + (uint32_t)st;
                if (p->langevin) {
                    for (int a = 0; a < n; ++a) {
                        double h = 0.5 * p->dt / s->mass[a];
                        double sd = sqrt(p->kB * p->T / s->mass[a]);
                        uint32_t w[4];
                        double z[3];
                        for (int c = 0; c < 3; ++c) {
                            vr[3 * a + c] += h * F[3 * a + c];
                            xr[3 * a + c] += 0.5 * p->dt * vr[3 * a + c];
                        }
                        draw(g, sl, step, (uint32_t)a, ST_LANGEVIN, w);
                        normals3(w, z);
                        for (int c = 0; c < 3; ++c) {
                            vr[3 * a + c] = c1 * vr[3 * a + c] + c2 * sd * z[c];
                            xr[3 * a + c] += 0.5 * p->dt * vr[3 * a + c];
                        }
                    }
                } else {
                    for (int a = 0; a < n; ++a) {
                        double h = 0.5 * p->dt / s->mass[a];
                        for (int c = 0; c < 3; ++c) {
                            vr[3 * a + c] += h * F[3 * a + c];
                            xr[3 * a + c] += p->dt * vr[3 * a + c];
                        }
                    }
                }
                ora_energy_forces(s, xr, F, NULL, p->mask);
                for (int a = 0; a < n; ++a) {
                    double h = 0.5 * p->dt / s->mass[a];
                    for (int c = 0; c < 3; ++c)
                        vr[3 * a + c] += h * F[3 * a + c];
                }
                if (p->langevin || p->p24 == 0)
                    continue;
                for (int a = 0; a < n; ++a) {
                    uint32_t w[4];
                    draw(g, sl, step, collide_block(a), ST_COLLIDE, w);
                    if ((w[collide_word(a)] >> 8) < p->p24) {
                        uint32_t wv[4];
                        double z[3];
                        draw(g, sl, step, (uint32_t)a, ST_VELOCITY, wv);
                        normals3(wv, z);
                        double sd = sqrt(p->kB * p->T / s->mass[a]);
                        for (int c = 0; c < 3; ++c)
                            vr[3 * a + c] = sd * z[c];
                        ++ncol;
                    }
                }
            }
            if (Epot)
                Epot[r] = ora_energy_forces(s, xr, NULL, NULL, p->mask);
            if (Ekin) {
                double k = 0;
                for (int a = 0; a < n; ++a)
                    k += 0.5 * s->mass[a] * dot3(&vr[3 * a], &vr[3 * a]);
                Ekin[r] = k;
            }
            if (collisions)
                collisions[r] = ncol;
        }
        free(F);
    }
}

/* ------------------------------------------------------------------------ */
/* PAMD step 2: weights, normaliser Q, copy numbers                          */
/* ------------------------------------------------------------------------ */

/*
 * For energies E[R] and dbeta = 1/(kB T_i) - 1/(kB T_{i-1}):
 *   m  = min_j E_j
 *   S  = sum_j exp(-dbeta (E_j - m))          (plain left-to-right sum)
 *   S2 = sum_j exp(-2 dbeta (E_j - m))
 *   ln Q = -dbeta m + ln S - ln R             (Q = (1/R) sum_j e^{-dbeta E_j})
 * returns 0, or 4 if an energy is not finite.
 */
int32_t ora_lse(int64_t R, const double* E, double dbeta, double* m_out, double* S_out,
                double* S2_out, double* lnQ_out)
{
    double m = INFINITY;
    for (int64_t j = 0; j < R; ++j) {
        if (!isfinite(E[j]))
            return 4;
        if (E[j] < m)
            m = E[j];
    }
    double S = 0.0, S2 = 0.0;
    for (int64_t j = 0; j < R; ++j) {
        double w = exp(-dbeta * (E[j] - m));
        S += w;
        S2 += w * w;
    }
    *m_out = m;
    *S_out = S;
    *S2_out = S2;
    *lnQ_out = -dbeta * m + log(S) - log((double)R);
    return 0;
}

/* 53-bit uniform in [0,1) from two words: ((w0 >> 5) 2^26 + (w1 >> 6)) 2^-53 */
static double u53(uint32_t w0, uint32_t w1)
{
    return ((double)(w0 >> 5) * 67108864.0 + (double)(w1 >> 6)) * (1.0 / 9007199254740992.0);
}

/* resampling uniforms of stream 2: counter (slot j, temperature index, 0, 2) */
void ora_resample_uniforms(const ora_rng* g, int64_t R, uint32_t temp_index, double* u)
{
    for (int64_t j = 0; j < R; ++j) {
        uint32_t w[4];
        draw(g, (uint32_t)j, temp_index, 0u, ST_RESAMPLE, w);
        u[j] = u53(w[0], w[1]);
    }
}

/* multinomial draws of stream 4: counter (draw k, temperature index, 0, 4) */
void ora_multinomial_uniforms(const ora_rng* g, int64_t n_draws, uint32_t temp_index, double* u)
{
    for (int64_t k = 0; k < n_draws; ++k) {
        uint32_t w[4];
        draw(g, (uint32_t)k, temp_index, 0u, ST_MULTINOMIAL, w);
        u[k] = u53(w[0], w[1]);
    }
}

/*
 * Nearest-integer resampling with random rounding:
 *   tau_j = R_target exp(-dbeta (E_j - m)) / S      (sum_j tau_j = R_target)
 *   c_j   = floor(tau_j) + [u_j < tau_j - floor(tau_j)]
 * tau_out (optional) receives tau_j.  Returns sum_j c_j.
 */
int64_t ora_counts(int64_t R, const double* E, double dbeta, double m, double S, int64_t R_target,
                   const double* u, int32_t* c, double* tau_out)
{
    int64_t tot = 0;
    for (int64_t j = 0; j < R; ++j) {
        double tau = (double)R_target * exp(-dbeta * (E[j] - m)) / S;
        double fl = floor(tau);
        int32_t cj = (int32_t)fl + ((u[j] < tau - fl) ? 1 : 0);
        c[j] = cj;
        tot += cj;
        if (tau_out)
            tau_out[j] = tau;
    }
    return tot;
}

/* normalised weight variance V = R sum p_j^2 - 1, p_j = w_j / sum w */
double ora_weight_variance(int64_t R, const double* E, double dbeta)
{
    double m, S, S2, lnQ;
    if (ora_lse(R, E, dbeta, &m, &S, &S2, &lnQ) != 0)
        return NAN;
    return (double)R * S2 / (S * S) - 1.0;
}
