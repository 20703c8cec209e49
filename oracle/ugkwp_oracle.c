/*
 * ugkwp_oracle.c -- plain, slow, double-precision CPU reference for one time step of the
 * three-dimensional unified gas-kinetic wave-particle (UGKWP) method of Chen, Zhu and Xu,
 * "A three-dimensional unified gas-kinetic wave-particle solver for flow computation in all
 * regimes" (arXiv 2007.13091).
 *
 * TEST INFRASTRUCTURE ONLY.  The product never links, loads or calls this file: only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark do.  It shares no code
 * with the GPU library.  It has its own mesh preparation, Philox generator, Maxwellian
 * moments, interface flux, sampling, tracking and update, written from the paper's
 * equations and the readings of the paper written down in the design notes.
 *
 * The phases run in the plain order of the scheme (paper Sec. 2.2-2.4):
 *   primitives and the time step (Sec. 2.4(a)), hydro/particle split (Eq. of W^p),
 *   wave flux per face (Eqs. of F^eq and F^{fr,wave}), sampling of hydro particles
 *   (Sec. 2.4(b)), free-flight times (Eq. sampling_of_free_transport_time), free transport
 *   (Sec. 2.3), particle sums and the conservative update (Eq. update_macro_variables),
 *   deletion of collided particles (the four-step particle procedure of Sec. 2.3).
 * Optionally, time averaging of W for steady states (Sec. 2.4(c)).
 * Every sum runs sequentially in that plain order.  Built with OpenMP (a second library,
 * for timing on many cores only), the loops whose items are independent -- the faces'
 * fluxes, the cells' gradients and samples, the particles' flights -- run in parallel, each
 * item writing only its own outputs; the results are the same bit for bit.
 * All arithmetic is IEEE double with libm transcendental functions; it must be compiled
 * with -ffp-contract=off and without -ffast-math.
 *
 * Pins (what fixes this code independently of itself) live in tests/test_oracle_*.py:
 * Philox against numpy, moments and q-coefficients against quadrature, the uniform-state
 * flux against the Euler flux, conservation in closed boxes, the free-molecular limit,
 * brute-force tracking on two-cell meshes, exact sampling counts and masses, and the
 * Euler-limit shock tube against an exact Riemann solver; for the Shakhov model, Gauss-Hermite
 * moments of its correction and the homogeneous relaxation of the heat flux.  The complete
 * multi-step trajectory at finite Knudsen number has no printed values in the paper: beyond
 * those invariants it is "parity unpinned".
 */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_ARG 1
#define ORC_E_MESH 2
#define ORC_E_CAPACITY 3
#define ORC_E_LOST 4
#define ORC_E_NONPHYS 5

/* BC_PERIODIC is test support, not a condition of the paper: a tagged face leads to the
   face at x + shift, which makes every face interior and all five totals exact invariants */
enum { BC_SPECULAR = 0, BC_DIFFUSE = 1, BC_FARFIELD = 2, BC_PERIODIC = 3 };

/* relative floor of the hydro density rho^h = rho - rho^p (see phase_cells) */
#define RHOH_EPS 1e-12
enum { TAG_TF = 1, TAG_POS = 2, TAG_VEL = 3, TAG_WALL = 4, TAG_INJECT = 5, TAG_INT = 6, TAG_WALLINT = 7, TAG_GP = 8 };
#define KMAX 8 /* internal degrees of freedom supported (gamma = (K + 5) / (K + 3)) */

/* ------------------------------------------------------------------------------------ */
/* Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), counter based.       */
/* ------------------------------------------------------------------------------------ */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ULL * c0;
        unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ULL * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* eta in (0,1): the top 52 bits plus one half, times 2^-52 (never 0 or 1). */
static double u01(uint64_t r) { return ((double)(r >> 12) + 0.5) * 0x1p-52; }

/* Four uniforms keyed by (particle id, step, tag, sub-index, instance); key = (seed, 0). */
static void draw4(uint64_t seed, uint64_t uid, int64_t step, int tag, uint32_t sub,
                  int64_t inst, double eta[4])
{
    uint64_t ctr[4] = {uid, (uint64_t)step, ((uint64_t)tag << 32) | sub, (uint64_t)inst};
    uint64_t key[2] = {seed, 0};
    uint64_t r[4];
    orc_philox4x64_10(ctr, key, r);
    for (int i = 0; i < 4; ++i) eta[i] = u01(r[i]);
}

/* Particle id: bit 63 born at a far-field face, bits 62..44 birth step, bits 43..20 birth
 * cell (or face), bits 19..0 index within that cell and step. */
uint64_t orc_make_uid(int ghost, int64_t step, int64_t where, int64_t k)
{
    return ((uint64_t)(ghost & 1) << 63) | (((uint64_t)step & 0x7FFFFULL) << 44) |
           (((uint64_t)where & 0xFFFFFFULL) << 20) | ((uint64_t)k & 0xFFFFFULL);
}

/* ------------------------------------------------------------------------------------ */
/* Maxwellian moments (R = 1, K = 0).  <u^k> of a normalised 1D Maxwellian with mean U and  */
/* lambda = 1/(2T); full range, u > 0 and u < 0.  Recursion                               */
/*   <u^{k+2}> = U <u^{k+1}> + (k+1)/(2 lambda) <u^k>   (holds on each half line too).     */
/* ------------------------------------------------------------------------------------ */
#define NMOM 7
void orc_moments(int range, double U, double lam, double m[NMOM])
{
    if (range == 0) {
        m[0] = 1.0;
        m[1] = U;
    } else if (range > 0) {
        m[0] = 0.5 * erfc(-sqrt(lam) * U);
        m[1] = U * m[0] + 0.5 * exp(-lam * U * U) / sqrt(M_PI * lam);
    } else {
        m[0] = 0.5 * erfc(sqrt(lam) * U);
        m[1] = U * m[0] - 0.5 * exp(-lam * U * U) / sqrt(M_PI * lam);
    }
    for (int k = 0; k + 2 < NMOM; ++k) m[k + 2] = U * m[k + 1] + (k + 1) / (2.0 * lam) * m[k];
}

/* Face frame: n, t1 = normalise(e_a x n) with a the axis of smallest |n_a| (lowest index on a
 * tie), t2 = n x t1. */
static void face_frame(const double n[3], double t1[3], double t2[3])
{
    int a = 0;
    if (fabs(n[1]) < fabs(n[a])) a = 1;
    if (fabs(n[2]) < fabs(n[a])) a = 2;
    double e[3] = {0, 0, 0};
    e[a] = 1.0;
    double c[3] = {e[1] * n[2] - e[2] * n[1], e[2] * n[0] - e[0] * n[2], e[0] * n[1] - e[1] * n[0]};
    double l = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
    t1[0] = c[0] / l; t1[1] = c[1] / l; t1[2] = c[2] / l;
    t2[0] = n[1] * t1[2] - n[2] * t1[1];
    t2[1] = n[2] * t1[0] - n[0] * t1[2];
    t2[2] = n[0] * t1[1] - n[1] * t1[0];
}

/* Primitive state in a face frame; K internal degrees of freedom (Sec. 2.1: the Maxwellian
 * carries exp(-lambda xi^2) over K components of xi, and rho E = rho |U|^2 / 2 + (3 + K) rho T / 2). */
typedef struct { double rho, un, v, w, lam, T; int K; } prim_t;

/* temperature of a conservative state (R = 1, N = 3 + K) */
static double temp_k(const double W[5], int K)
{
    return (2.0 / (3.0 + K)) * (W[4] - 0.5 * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]) / W[0]) / W[0];
}

static prim_t to_frame(const double W[5], const double n[3], const double t1[3], const double t2[3], int K)
{
    prim_t p;
    p.rho = W[0];
    double U = W[1] / W[0], V = W[2] / W[0], Wz = W[3] / W[0];
    p.un = U * n[0] + V * n[1] + Wz * n[2];
    p.v = U * t1[0] + V * t1[1] + Wz * t1[2];
    p.w = U * t2[0] + V * t2[1] + Wz * t2[2];
    p.T = temp_k(W, K);
    p.lam = 1.0 / (2.0 * p.T);
    p.K = K;
    return p;
}

/* <psi> and <u_n psi> of a unit-density Maxwellian in the face frame, with the normal
 * moments m[] taken over the chosen range of u_n; psi = (1, u_n, v, w, (u_n^2+v^2+w^2+xi^2)/2),
 * <xi^2> = K / (2 lambda). */
static void psi_moments(const prim_t *p, const double m[NMOM], double H[5], double G[5])
{
    double tr = p->v * p->v + p->w * p->w + 1.0 / p->lam + p->K / (2.0 * p->lam); /* <v^2 + w^2 + xi^2> */
    H[0] = m[0];
    H[1] = m[1];
    H[2] = m[0] * p->v;
    H[3] = m[0] * p->w;
    H[4] = 0.5 * (m[2] + m[0] * tr);
    G[0] = m[1];
    G[1] = m[2];
    G[2] = m[1] * p->v;
    G[3] = m[1] * p->w;
    G[4] = 0.5 * (m[3] + m[1] * tr);
}

/* ------------------------------------------------------------------------------------ */
/* Time-integrated coefficients, Eq. of q1..q5, with x = dt/tau and e = exp(-x).  Only the */
/* combinations the first-order flux needs are formed here:                               */
/*   q1 = tau (x - 1 + e),   q4 - dt e = tau (1 - (1 + x) e).                              */
/* For x < 1 both are summed as their Taylor series (terms x^2 .. x^24, Horner order):     */
/*   q1/tau        = sum_{k>=2} (-1)^k x^k / k!                                            */
/*   (q4-dt e)/tau = sum_{k>=2} (-1)^k (k-1) x^k / k!                                      */
/* ------------------------------------------------------------------------------------ */
#define QSER_X 1.0
#define QSER_K 24
void orc_qcoef(double dt, double tau, double out[5])
{
    double x = dt / tau;
    double e = exp(-x);
    double q1, q4m, q2, q3, q5p;
    if (x < QSER_X) {
        double fact[QSER_K + 1];
        fact[0] = 1.0;
        for (int k = 1; k <= QSER_K; ++k) fact[k] = fact[k - 1] * k;
        double s1 = 0, s4 = 0, s2 = 0, s3 = 0, s5 = 0;
        for (int k = QSER_K; k >= 2; --k) {
            double sg = (k % 2 == 0) ? 1.0 : -1.0;
            s1 = s1 * x + sg / fact[k];
            s4 = s4 * x + sg * (k - 1) / fact[k];
            if (k >= 3) {
                s2 = s2 * x + sg * (k - 2) / fact[k];
                s3 = s3 * x - sg / fact[k];
                s5 = s5 * x + sg * (double)((k - 1) * (k - 2)) / (2.0 * fact[k]);
            }
        }
        q1 = tau * (s1 * x * x);
        q4m = tau * (s4 * x * x);
        q2 = tau * tau * (s2 * x * x * x);
        q3 = tau * tau * (s3 * x * x * x);
        q5p = tau * tau * (s5 * x * x * x);
    } else {
        q1 = tau * (x - 1.0 + e);
        q4m = tau * (1.0 - (1.0 + x) * e);
        q2 = tau * tau * (2.0 * (1.0 - e) - x * (1.0 + e));
        q3 = tau * tau * (0.5 * x * x - x + 1.0 - e);
        q5p = tau * tau * ((1.0 + x + 0.5 * x * x) * e - 1.0);
    }
    out[0] = q1; out[1] = q2; out[2] = q3; out[3] = q4m; out[4] = q5p;
}

/* The wave-only (gas-kinetic) phase that starts a run (the continuum start of Sec. 4.3 and
 * Sec. 4.4): no particle is sampled, so the waves carry the whole free transport of W^h,
 * F^{fr,UGKS} = int u_n (q4 g0^h + q5 u.g_x^h) psi, i.e. the wave flux of Sec. 2.4 with the
 * terms of the sampled collisionless particles (-dt e and + dt^2 e / 2) left out:
 * q4 = (q4 - dt e) + dt e and q5 = (q5 + dt^2 e / 2) - dt^2 e / 2. */
static void wave_only_coef(double dt, double tau, double q[5])
{
    double e = exp(-dt / tau);
    q[3] = q[3] + dt * e;
    q[4] = q[4] - 0.5 * dt * dt * e;
}

static void rotate_back(const double Ff[5], const double n[3], const double t1[3], const double t2[3],
                        double F[5])
{
    F[0] = Ff[0];
    for (int d = 0; d < 3; ++d) F[1 + d] = Ff[1] * n[d] + Ff[2] * t1[d] + Ff[3] * t2[d];
    F[4] = Ff[4];
}

/* ------------------------------------------------------------------------------------ */
/* Shakhov model (Pr != 1).  The state the particles relax to is                           */
/*   g^+ = g [1 + (1 - Pr) c.q (|c|^2 / T - 5) / (5 p T)],  c = u - U, p = rho T (R = 1, K = 0), */
/* q the heat flux of the gas.  Reading: in the interface distribution the g0 term becomes    */
/* g0^+ (the slope and time-derivative terms keep the Maxwellian).  Over all velocities the    */
/* correction carries no mass and no momentum (its weight is odd in c and <c_i c_j (|c|^2/T -  */
/* 5)> = 0) and the energy flux (1 - Pr) q.n (from <c_n^2 |c|^2> = 5 T^2 and <c_n^2 |c|^4> =   */
/* 35 T^3 per unit density), whatever rho0, U0 and T0 are.  So F^eq gains q1 qsh in its        */
/* energy component, qsh = (1 - Pr) q_f.n with q_f the heat flux at the face (see orc_step).  */
/* qsh = 0 leaves the BGK flux untouched.                                                    */
/* ------------------------------------------------------------------------------------ */

/* ------------------------------------------------------------------------------------ */
/* First-order interface flux of the wave part over dt, per unit area, global frame:      */
/*   F = F^eq + F^{fr,wave}                                                               */
/*   F^eq      = rho0 q1 <u_n psi>_0           (g0 from the upwind moments of both sides)  */
/*   F^{fr,wave} = sum_s rhoh_s (q4 - dt e) <u_n psi>_{s, half}                            */
/* tau at the face = mu_ref T0^omega / p0 + C2 |pl - pr| / (pl + pr) dt (Sec. 2.4(d)).     */
/* rhoh_l, rhoh_r: density of the hydro Maxwellian (U and T of the total state).           */
/* ------------------------------------------------------------------------------------ */
static void flux_pair(const prim_t *l, const prim_t *r, double rhohl, double rhohr, double dt,
                      double mu_ref, double omega, double c2, int gks, double qsh, double Ff[5])
{
    double ml[NMOM], mr[NMOM], Hl[5], Gl[5], Hr[5], Gr[5];
    orc_moments(+1, l->un, l->lam, ml);
    orc_moments(-1, r->un, r->lam, mr);
    psi_moments(l, ml, Hl, Gl);
    psi_moments(r, mr, Hr, Gr);
    double W0[5];
    for (int k = 0; k < 5; ++k) W0[k] = l->rho * Hl[k] + r->rho * Hr[k];
    prim_t z;
    z.rho = W0[0];
    z.un = W0[1] / W0[0];
    z.v = W0[2] / W0[0];
    z.w = W0[3] / W0[0];
    z.K = l->K;
    z.T = temp_k(W0, z.K);
    z.lam = 1.0 / (2.0 * z.T);
    double pl = l->rho * l->T, pr = r->rho * r->T;
    double tau = mu_ref * pow(z.T, omega) / (z.rho * z.T) + c2 * (fabs(pl - pr) / (pl + pr)) * dt;
    double q[5];
    orc_qcoef(dt, tau, q);
    if (gks) wave_only_coef(dt, tau, q);
    double m0[NMOM], H0[5], G0[5];
    orc_moments(0, z.un, z.lam, m0);
    psi_moments(&z, m0, H0, G0);
    for (int k = 0; k < 5; ++k)
        Ff[k] = q[0] * z.rho * G0[k] + q[3] * (rhohl * Gl[k] + rhohr * Gr[k]);
    if (qsh != 0.0) Ff[4] = Ff[4] + q[0] * qsh;
}

void orc_flux_interior(const double Wl[5], const double Wr[5], double rhohl, double rhohr,
                       const double n[3], double dt, double mu_ref, double omega, double c2, int gks, int K,
                       double qsh, double F[5])
{
    double t1[3], t2[3], Ff[5];
    face_frame(n, t1, t2);
    prim_t l = to_frame(Wl, n, t1, t2, K), r = to_frame(Wr, n, t1, t2, K);
    flux_pair(&l, &r, rhohl, rhohr, dt, mu_ref, omega, c2, gks, qsh, Ff);
    rotate_back(Ff, n, t1, t2, F);
}

/* Specular (symmetry) wall: interior flux against the mirror state (u_n -> -u_n), then only
 * the normal-momentum component is kept; n points out of the domain. */
void orc_flux_specular(const double W[5], double rhoh, const double n[3], double dt,
                       double mu_ref, double omega, double c2, int gks, int K, double F[5])
{
    double t1[3], t2[3], Ff[5];
    face_frame(n, t1, t2);
    prim_t l = to_frame(W, n, t1, t2, K);
    prim_t g = l;
    g.un = -l.un;
    flux_pair(&l, &g, rhoh, rhoh, dt, mu_ref, omega, c2, gks, 0.0, Ff);
    Ff[0] = 0.0; Ff[2] = 0.0; Ff[3] = 0.0; Ff[4] = 0.0;
    rotate_back(Ff, n, t1, t2, F);
}

/* Diffuse isothermal wall (Sec. 2.4(e)), first order, n out of the domain.  Incoming part
 * (u_n > 0): q1 g + (q4 - dt e) g^h at the cell state with the cell's tau; the wall emits
 * rho_w M(T_w, U_w) over u_n < 0 for the whole step, rho_w fixed by zero net mass flux. */
void orc_flux_diffuse(const double W[5], double rhoh, double tau_c, const double n[3], double dt,
                      double Tw, const double Uw[3], int gks, int K, double F[5])
{
    double t1[3], t2[3], Ff[5];
    face_frame(n, t1, t2);
    prim_t l = to_frame(W, n, t1, t2, K);
    double q[5];
    orc_qcoef(dt, tau_c, q);
    if (gks) wave_only_coef(dt, tau_c, q);
    double ml[NMOM], Hl[5], Gl[5];
    orc_moments(+1, l.un, l.lam, ml);
    psi_moments(&l, ml, Hl, Gl);
    double Fin[5];
    for (int k = 0; k < 5; ++k) Fin[k] = q[0] * l.rho * Gl[k] + q[3] * rhoh * Gl[k];
    prim_t w;
    w.rho = 1.0;
    w.un = Uw[0] * n[0] + Uw[1] * n[1] + Uw[2] * n[2];
    w.v = Uw[0] * t1[0] + Uw[1] * t1[1] + Uw[2] * t1[2];
    w.w = Uw[0] * t2[0] + Uw[1] * t2[1] + Uw[2] * t2[2];
    w.T = Tw;
    w.lam = 1.0 / (2.0 * Tw);
    w.K = K;
    double mw[NMOM], Hw[5], Gw[5];
    orc_moments(-1, w.un, w.lam, mw);
    psi_moments(&w, mw, Hw, Gw);
    double rhow = -Fin[0] / (dt * Gw[0]);
    for (int k = 0; k < 5; ++k) Ff[k] = Fin[k] + dt * rhow * Gw[k];
    Ff[0] = 0.0;
    rotate_back(Ff, n, t1, t2, F);
}

/* ------------------------------------------------------------------------------------ */
/* Second order (Sec. 2.2: the initial distribution with slopes, the equilibrium state    */
/* with its slopes and time derivative; Sec. 2.4 for the wave part).                       */
/*                                                                                          */
/* Moments of polynomials in (u, v, w, z = xi^2) (face frame) over a Maxwellian: degree < 7 */
/* in each velocity and < 3 in z, as dense coefficients, multiplied out and integrated term  */
/* by term with <u^a v^b w^c z^d> = <u^a>_range <v^b> <w^c> <z^d>, where for K internal      */
/* components <z> = K/(2 lambda) and <z^2> = K (K + 2) / (4 lambda^2).                      */
/* ------------------------------------------------------------------------------------ */
#define PD 7
#define PZ 3
typedef struct { double c[PD][PD][PD][PZ]; } poly_t;

static void poly_clear(poly_t *p) { memset(p, 0, sizeof(*p)); }

static void poly_mono(int a, int b, int c, poly_t *p)
{
    poly_clear(p);
    p->c[a][b][c][0] = 1.0;
}

/* psi_k: 1, u, v, w, (u^2 + v^2 + w^2 + xi^2)/2 (xi: 0 leaves the xi^2 term out, for K = 0,
   where all its moments vanish) */
static void poly_psi(int k, int xi, poly_t *p)
{
    poly_clear(p);
    if (k == 0) p->c[0][0][0][0] = 1.0;
    else if (k == 1) p->c[1][0][0][0] = 1.0;
    else if (k == 2) p->c[0][1][0][0] = 1.0;
    else if (k == 3) p->c[0][0][1][0] = 1.0;
    else {
        p->c[2][0][0][0] = 0.5; p->c[0][2][0][0] = 0.5; p->c[0][0][2][0] = 0.5;
        if (xi) p->c[0][0][0][1] = 0.5;
    }
}

/* a . psi */
static void poly_apsi(const double a[5], int xi, poly_t *p)
{
    poly_clear(p);
    p->c[0][0][0][0] = a[0];
    p->c[1][0][0][0] = a[1];
    p->c[0][1][0][0] = a[2];
    p->c[0][0][1][0] = a[3];
    p->c[2][0][0][0] = 0.5 * a[4];
    p->c[0][2][0][0] = 0.5 * a[4];
    p->c[0][0][2][0] = 0.5 * a[4];
    if (xi) p->c[0][0][0][1] = 0.5 * a[4];
}

static int g_poly_overflow = 0;

/* the nonzero terms of a polynomial: exponents and coefficients */
typedef struct { int n; int e[PD * PD * PD * PZ][4]; double c[PD * PD * PD * PZ]; } terms_t;

static void poly_terms(const poly_t *p, int nz, terms_t *t)
{
    t->n = 0;
    for (int i = 0; i < PD; ++i)
        for (int j = 0; j < PD; ++j)
            for (int k = 0; k < PD; ++k)
                for (int q = 0; q < nz; ++q)
                    if (p->c[i][j][k][q] != 0.0) {
                        t->e[t->n][0] = i; t->e[t->n][1] = j; t->e[t->n][2] = k; t->e[t->n][3] = q;
                        t->c[t->n] = p->c[i][j][k][q];
                        ++t->n;
                    }
}

/* z = x y, term by term (the products of x's terms in order, each with y's terms in order);
   nz: how many powers of xi^2 the factors may hold (1 for K = 0) */
static void poly_mul(const poly_t *x, const poly_t *y, int nz, poly_t *z)
{
    terms_t tx, ty;
    poly_terms(x, nz, &tx);
    poly_terms(y, nz, &ty);
    poly_clear(z);
    for (int a = 0; a < tx.n; ++a)
        for (int b = 0; b < ty.n; ++b) {
            const int i = tx.e[a][0] + ty.e[b][0], j = tx.e[a][1] + ty.e[b][1];
            const int k = tx.e[a][2] + ty.e[b][2], q = tx.e[a][3] + ty.e[b][3];
            if (i >= PD || j >= PD || k >= PD || q >= PZ) {
#pragma omp atomic write
                g_poly_overflow = 1;
                continue;
            }
            z->c[i][j][k][q] += tx.c[a] * ty.c[b];
        }
}

/* <p> over a unit-density Maxwellian g in the face frame, u over range (0 all, +1 u > 0,
 * -1 u < 0), v, w and xi over the full space */
static double poly_moment(const poly_t *p, int range, const prim_t *g)
{
    double mu[NMOM], mv[NMOM], mw[NMOM];
    orc_moments(range, g->un, g->lam, mu);
    orc_moments(0, g->v, g->lam, mv);
    orc_moments(0, g->w, g->lam, mw);
    const double mz[PZ] = {1.0, g->K / (2.0 * g->lam), g->K * (g->K + 2.0) / (4.0 * g->lam * g->lam)};
    const int nz = g->K > 0 ? PZ : 1;
    double s = 0.0;
    for (int i = 0; i < PD; ++i)
        for (int j = 0; j < PD; ++j)
            for (int k = 0; k < PD; ++k)
                for (int q = 0; q < nz; ++q)
                    if (p->c[i][j][k][q] != 0.0) s += p->c[i][j][k][q] * mu[i] * mv[j] * mw[k] * mz[q];
    return s;
}

/* out_k = < pre (a . psi) psi_k > (a == NULL: < pre psi_k >) */
static void mvec(const poly_t *pre, const double *a, int range, const prim_t *g, double out[5])
{
    poly_t t, ap, pk, r;
    const int xi = g->K > 0;
    const int nz = xi ? PZ : 1;
    if (a) {
        poly_apsi(a, xi, &ap);
        poly_mul(pre, &ap, nz, &t);
    } else {
        t = *pre;
    }
    for (int k = 0; k < 5; ++k) {
        poly_psi(k, xi, &pk);
        poly_mul(&t, &pk, nz, &r);
        out[k] = poly_moment(&r, range, g);
    }
}

/* Micro slope from a macro derivative (Sec. 2.2): a with < (a . psi) psi > = b over the full
 * Maxwellian g (b = derivative of W divided by the density), N = 3 + K.  With c = u - U, the
 * moments <c^2> = T = 1/(2 lambda) per direction and <xi^2> = K T give
 *   R = 2 b5 - (|U|^2 + N/(2 lambda)) b1,  R_i = b_{i+1} - U_i b1 (i = 1..3)
 *   a5 = (4 lambda^2 / N) (R - 2 sum_i U_i R_i),  a_{i+1} = 2 lambda R_i - U_i a5,
 *   a1 = b1 - sum_i U_i a_{i+1} - a5 (|U|^2 + N/(2 lambda)) / 2. */
void orc_slope(double un, double v, double w, double lam, int K, const double b[5], double a[5])
{
    double U[3] = {un, v, w};
    double N = 3.0 + K;
    double q2 = un * un + v * v + w * w;
    double R = 2.0 * b[4] - (q2 + N / (2.0 * lam)) * b[0];
    double Ri[3];
    for (int i = 0; i < 3; ++i) Ri[i] = b[1 + i] - U[i] * b[0];
    a[4] = (4.0 * lam * lam / N) * (R - 2.0 * (U[0] * Ri[0] + U[1] * Ri[1] + U[2] * Ri[2]));
    for (int i = 0; i < 3; ++i) a[1 + i] = 2.0 * lam * Ri[i] - U[i] * a[4];
    a[0] = b[0] - (U[0] * a[1] + U[1] * a[2] + U[2] * a[3]) - 0.5 * a[4] * (q2 + N / (2.0 * lam));
}

static void slope_of(const prim_t *g, const double dW[5], double a[5])
{
    double b[5];
    for (int k = 0; k < 5; ++k) b[k] = dW[k] / g->rho;
    orc_slope(g->un, g->v, g->w, g->lam, g->K, b, a);
}

/* test hook: <u^p v^q w^r (a . psi) psi> over a Maxwellian in the frame */
void orc_mvec(int p, int q, int r, const double *a, int range, double un, double v, double w, double lam, int K,
              double out[5])
{
    poly_t pre;
    poly_mono(p, q, r, &pre);
    prim_t g;
    g.rho = 1.0; g.un = un; g.v = v; g.w = w; g.lam = lam; g.T = 1.0 / (2.0 * lam); g.K = K;
    mvec(&pre, a, range, &g, out);
}

/* One side of a face for the second-order flux, in the face frame: the reconstructed state
 * (total W) with its derivatives along n, t1, t2, and the reconstructed hydro state W~^h with
 * its derivatives (hydro density 0: no hydro part). */
typedef struct {
    prim_t g;
    double dW[3][5];
    prim_t h;
    double dWh[3][5];
} side_t;

/* Second-order interface flux over dt, per unit area, face frame (SURVEY-style steps):
 *   W0 from the upwind half moments of the two reconstructed states;
 *   side slopes a_{s,d} from their derivatives; the equilibrium slope abar_d from
 *   W_x = rho_l <(a_l,d . psi) psi>_{>0} + rho_r <(a_r,d . psi) psi>_{<0} (W_x = int f_x psi);
 *   Abar from the compatibility condition <(u abar_n + v abar_t1 + w abar_t2 + Abar) . psi psi> = 0;
 *   F^eq = rho0 [q1 <u psi> + q2 <u (u abar_n + v abar_t1 + w abar_t2) . psi psi> + q3 <u (Abar . psi) psi>];
 *   F^wave = sum_s rho^h_s [(q4 - dt e) <u psi>_s + (q5 + dt^2 e / 2) <u (u a~_n + v a~_t1 + w a~_t2) . psi psi>_s]
 *   over the half spaces, with a~ the slopes of W~^h. */
static void flux2_pair(const side_t *L, const side_t *R, double dt, double mu_ref, double omega, double c2,
                       int gks, double qsh, double Ff[5])
{
    poly_t one, pu, pv, pw, puu, puv, puw;
    poly_mono(0, 0, 0, &one);
    poly_mono(1, 0, 0, &pu);
    poly_mono(0, 1, 0, &pv);
    poly_mono(0, 0, 1, &pw);
    poly_mono(2, 0, 0, &puu);
    poly_mono(1, 1, 0, &puv);
    poly_mono(1, 0, 1, &puw);
    double Hl[5], Hr[5], W0[5];
    mvec(&one, NULL, +1, &L->g, Hl);
    mvec(&one, NULL, -1, &R->g, Hr);
    for (int k = 0; k < 5; ++k) W0[k] = L->g.rho * Hl[k] + R->g.rho * Hr[k];
    prim_t z;
    z.rho = W0[0];
    z.un = W0[1] / W0[0];
    z.v = W0[2] / W0[0];
    z.w = W0[3] / W0[0];
    z.K = L->g.K;
    z.T = temp_k(W0, z.K);
    z.lam = 1.0 / (2.0 * z.T);
    double abar[3][5];
    for (int d = 0; d < 3; ++d) {
        double al[5], ar[5], Sl[5], Sr[5], Wx[5];
        slope_of(&L->g, L->dW[d], al);
        slope_of(&R->g, R->dW[d], ar);
        mvec(&one, al, +1, &L->g, Sl);
        mvec(&one, ar, -1, &R->g, Sr);
        for (int k = 0; k < 5; ++k) Wx[k] = L->g.rho * Sl[k] + R->g.rho * Sr[k];
        slope_of(&z, Wx, abar[d]);
    }
    double t0[5], t1[5], t2[5], bt[5], At[5];
    mvec(&pu, abar[0], 0, &z, t0);
    mvec(&pv, abar[1], 0, &z, t1);
    mvec(&pw, abar[2], 0, &z, t2);
    for (int k = 0; k < 5; ++k) bt[k] = -(t0[k] + t1[k] + t2[k]);
    orc_slope(z.un, z.v, z.w, z.lam, z.K, bt, At);
    double pl = L->g.rho * L->g.T, pr = R->g.rho * R->g.T;
    double tau = mu_ref * pow(z.T, omega) / (z.rho * z.T) + c2 * (fabs(pl - pr) / (pl + pr)) * dt;
    double q[5];
    orc_qcoef(dt, tau, q);
    if (gks) wave_only_coef(dt, tau, q);
    double G0[5], X0[5], X1[5], X2[5], GA[5];
    mvec(&pu, NULL, 0, &z, G0);
    mvec(&puu, abar[0], 0, &z, X0);
    mvec(&puv, abar[1], 0, &z, X1);
    mvec(&puw, abar[2], 0, &z, X2);
    mvec(&pu, At, 0, &z, GA);
    for (int k = 0; k < 5; ++k)
        Ff[k] = z.rho * (q[0] * G0[k] + q[1] * (X0[k] + X1[k] + X2[k]) + q[2] * GA[k]);
    const side_t *S[2] = {L, R};
    for (int s = 0; s < 2; ++s) {
        const prim_t *h = &S[s]->h;
        if (!(h->rho > 0.0)) continue;
        int range = s == 0 ? +1 : -1;
        double ah[3][5], Gh[5], Y0[5], Y1[5], Y2[5];
        for (int d = 0; d < 3; ++d) slope_of(h, S[s]->dWh[d], ah[d]);
        mvec(&pu, NULL, range, h, Gh);
        mvec(&puu, ah[0], range, h, Y0);
        mvec(&puv, ah[1], range, h, Y1);
        mvec(&puw, ah[2], range, h, Y2);
        for (int k = 0; k < 5; ++k) Ff[k] += h->rho * (q[3] * Gh[k] + q[4] * (Y0[k] + Y1[k] + Y2[k]));
    }
    if (qsh != 0.0) Ff[4] = Ff[4] + q[0] * qsh;
}

/* derivatives of a conservative state along n, t1, t2 from its gradient G[k][d] (global
 * frame), in frame components */
static void frame_derivs(const double G[15], const double n[3], const double t1[3], const double t2[3],
                         double out[3][5])
{
    const double *e[3] = {n, t1, t2};
    for (int d = 0; d < 3; ++d) {
        double dk[5];
        for (int k = 0; k < 5; ++k) dk[k] = G[3 * k] * e[d][0] + G[3 * k + 1] * e[d][1] + G[3 * k + 2] * e[d][2];
        out[d][0] = dk[0];
        out[d][1] = dk[1] * n[0] + dk[2] * n[1] + dk[3] * n[2];
        out[d][2] = dk[1] * t1[0] + dk[2] * t1[1] + dk[3] * t1[2];
        out[d][3] = dk[1] * t2[0] + dk[2] * t2[1] + dk[3] * t2[2];
        out[d][4] = dk[4];
    }
}

static void make_side(const double W[5], const double G[15], const double Wh[5], const double Gh[15],
                      const double n[3], const double t1[3], const double t2[3], int K, side_t *s)
{
    s->g = to_frame(W, n, t1, t2, K);
    frame_derivs(G, n, t1, t2, s->dW);
    /* a face hydro density within 1e-12 of the face density of zero is roundoff of an empty
       hydro part (the limiter can pin it exactly to a neighbour's zero) and counts as zero */
    if (Wh[0] > RHOH_EPS * W[0]) {
        s->h = to_frame(Wh, n, t1, t2, K);
        frame_derivs(Gh, n, t1, t2, s->dWh);
    } else {
        memset(&s->h, 0, sizeof(s->h));
        s->h.K = K;
        memset(s->dWh, 0, sizeof(s->dWh));
    }
}

/* Second-order interior flux (global frame): reconstructed face states Wl, Wr and hydro
 * states Whl, Whr (conservative), gradients G[k][d] = dW_k/dx_d of each. */
void orc_flux2_interior(const double Wl[5], const double Wr[5], const double Whl[5], const double Whr[5],
                        const double Gl[15], const double Gr[15], const double Ghl[15], const double Ghr[15],
                        const double n[3], double dt, double mu_ref, double omega, double c2, int gks, int K,
                        double qsh, double F[5])
{
    double t1[3], t2[3], Ff[5];
    face_frame(n, t1, t2);
    side_t L, R;
    make_side(Wl, Gl, Whl, Ghl, n, t1, t2, K, &L);
    make_side(Wr, Gr, Whr, Ghr, n, t1, t2, K, &R);
    flux2_pair(&L, &R, dt, mu_ref, omega, c2, gks, qsh, Ff);
    rotate_back(Ff, n, t1, t2, F);
}

/* Specular wall at second order: the mirror image of the reconstructed field (normal
 * momentum and normal derivatives flip sign, twice for the normal momentum's normal
 * derivative), then only the normal-momentum component is kept. */
void orc_flux2_specular(const double W[5], const double Wh[5], const double G[15], const double Gh[15],
                        const double n[3], double dt, double mu_ref, double omega, double c2, int gks, int K, double F[5])
{
    double t1[3], t2[3], Ff[5];
    face_frame(n, t1, t2);
    side_t L, R;
    make_side(W, G, Wh, Gh, n, t1, t2, K, &L);
    R = L;
    R.g.un = -L.g.un;
    R.h.un = -L.h.un;
    for (int d = 0; d < 3; ++d) {
        double sd = d == 0 ? -1.0 : 1.0; /* derivative along n flips */
        for (int k = 0; k < 5; ++k) {
            double sk = k == 1 ? -1.0 : 1.0; /* normal momentum flips */
            R.dW[d][k] = sd * sk * L.dW[d][k];
            R.dWh[d][k] = sd * sk * L.dWh[d][k];
        }
    }
    flux2_pair(&L, &R, dt, mu_ref, omega, c2, gks, 0.0, Ff);
    Ff[0] = 0.0; Ff[2] = 0.0; Ff[3] = 0.0; Ff[4] = 0.0;
    rotate_back(Ff, n, t1, t2, F);
}

/* Far field at second order: the free stream with zero gradients as the right side. */
void orc_flux2_farfield(const double W[5], const double Wh[5], const double G[15], const double Gh[15],
                        const double Winf[5], const double n[3], double dt, double mu_ref, double omega,
                        double c2, int gks, int K, double qsh, double F[5])
{
    double t1[3], t2[3], Ff[5], zero[15];
    memset(zero, 0, sizeof(zero));
    face_frame(n, t1, t2);
    side_t L, R;
    make_side(W, G, Wh, Gh, n, t1, t2, K, &L);
    make_side(Winf, zero, Winf, zero, n, t1, t2, K, &R);
    flux2_pair(&L, &R, dt, mu_ref, omega, c2, gks, qsh, Ff);
    rotate_back(Ff, n, t1, t2, F);
}

/* ------------------------------------------------------------------------------------ */
/* Mesh: cells (4-node tetrahedra, 8-node axis-aligned boxes in VTK node order), faces     */
/* found by matching sorted node sets.                                                    */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    int type;
    double Tw, Uw[3], Winf[5];
    double shift[3];  /* periodic */
} obc_t;

typedef struct {
    int64_t key[4];
    int64_t cell;
    int lf;
} fkey_t;

typedef struct oracle {
    /* parameters */
    double mu_ref, omega, cfl, c2;
    int n_ref, n_min, max_cross;
    uint64_t seed;
    int64_t inst;
    /* mesh */
    int64_t nc, nf;
    int *ctype, *cnf;
    double *vol, *xc, *dS;
    int64_t *cface;   /* [nc][6] global face id */
    int *csign;       /* [nc][6] +1 when the cell owns the face */
    double *pn, *pd;  /* [nc][6][3], [nc][6]: outward plane n.x = d */
    int64_t *cnb;     /* [nc][6] neighbour cell, or -1 - bc index */
    int64_t *cbf;     /* [nc][6] input index of the boundary face, or -1 */
    double *bo, *be1, *be2, *barea; /* per input boundary face: corner, two edges, area */
    int *btri;                       /* triangle (1) or parallelogram (0) */
    int *cnblf;       /* [nc][6] local face index in the neighbour */
    int *cper;        /* [nc][6] periodic face: 1 + its bc index (crossing adds that bc's shift) */
    int64_t nper;     /* periodic face pairs */
    double *orig, *edge; /* sampling frame: [nc][3], [nc][3][3] */
    double *lfx;         /* [nc][6][3] centre of each local face */
    double *fx;          /* [nf][3] face centre (the owner's) */
    int recon;           /* 0 first order, 1 LSQ + Barth-Jespersen, 2 LSQ + Venkatakrishnan */
    double venkat_k;     /* Venkatakrishnan constant K in eps^2 = (K h)^3 */
    int K;               /* internal degrees of freedom (Sec. 2.1), gamma = (K + 5)/(K + 3) */
    int64_t gks_steps;   /* the steps n < gks_steps (counted from orc_set_state) are wave-only:
                            no particle is sampled or enters, the waves carry all of W^h */
    int sampling;        /* hydro-particle velocities: 0 the pairs U +- sqrt(T) X of Sec. 2.4(b);
                            1 the energy-exact variant (one factor per cell on the deviations);
                            2 the first-order g_p; 3 independent draws from the equilibrium of
                            the collision model (see phase_sample) */
    double pr;           /* Prandtl number of the collision model: 1 the BGK model of the paper,
                            otherwise the Shakhov model (see shakhov_setup) */
    int64_t *fown, *fnb; /* fnb: neighbour cell or -1 - bc index */
    double *fn, *farea;
    int nbc;
    obc_t *bc;
    /* state */
    double *W, *P;    /* [nc][5] */
    int64_t *nleft;
    int64_t step;
    double t;
    /* particles */
    int64_t np, cap;
    double *px, *pu, *pm;
    double *pe;          /* internal energy variable xi^2 of each particle (K > 0), phi_4 = m (|u|^2 + e) / 2 */
    int64_t *pc;
    uint64_t *pid;
    /* time averaging (Sec. 2.4(c)): steps n > avg_from are averaged (avg_from < 0: off) */
    int64_t avg_from;
    double *avgA;      /* [nc][5] sum of dt^n W^n */
    /* terms of the last update per cell (test hook): -sum_f s_f Phi_f, E and S, raw */
    double *tflux, *tE, *tS;
    double avg_D;      /* sum of dt^n */
    int64_t avg_n;     /* steps averaged */
    double avg_res;    /* relative change of the average in the last averaged step */
    /* last step statistics */
    double st_dt;
    int64_t st_sampled, st_collided, st_escaped, st_alive, st_cross, st_wallhits, st_injected;
    int64_t st_floored, st_rhoh_neg; /* cells whose rho - rho^p was in (0, 1e-12 rho], or below 0 */
    int64_t st_maxcross;             /* the most face crossings of one particle */
} oracle_t;

static int cmp_fkey(const void *a, const void *b)
{
    const fkey_t *x = (const fkey_t *)a, *y = (const fkey_t *)b;
    for (int i = 0; i < 4; ++i) {
        if (x->key[i] < y->key[i]) return -1;
        if (x->key[i] > y->key[i]) return 1;
    }
    if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
    return x->lf - y->lf;
}

static void sort_key(int64_t k[4], int nn)
{
    for (int i = 0; i < nn; ++i)
        for (int j = i + 1; j < nn; ++j)
            if (k[j] < k[i]) { int64_t t = k[i]; k[i] = k[j]; k[j] = t; }
    for (int i = nn; i < 4; ++i) k[i] = -1;
}

/* local faces of a box hex (VTK order): x-, x+, y-, y+, z-, z+ */
static const int HEXF[6][4] = {{0, 3, 7, 4}, {1, 2, 6, 5}, {0, 1, 5, 4}, {3, 2, 6, 7}, {0, 1, 2, 3}, {4, 5, 6, 7}};
/* local faces of a tetrahedron: face i is opposite node i */
static const int TETF[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

void orc_destroy(oracle_t *o);
static int reserve(oracle_t *o, int64_t n);

static void *xcalloc(size_t n, size_t s) { return calloc(n ? n : 1, s); }

oracle_t *orc_create(int64_t n_nodes, const double *xyz, int64_t n_cells, const uint8_t *cell_type,
                     const int64_t *cell_node_off, const int64_t *cell_nodes, int64_t n_bfaces,
                     const int64_t *bface_nodes, const int32_t *bface_bc, int32_t n_bc,
                     const int32_t *bc_type, const double *bc_Tw, const double *bc_Uw,
                     const double *bc_Winf, const double *bc_shift, double mu_ref, double omega, double cfl,
                     double c2,
                     int32_t n_ref, int32_t n_min, int32_t max_cross, uint64_t seed, int64_t inst,
                     int32_t *status)
{
    *status = ORC_E_MESH;
    if (n_cells <= 0 || n_nodes <= 0) { *status = ORC_E_ARG; return NULL; }
    oracle_t *o = (oracle_t *)xcalloc(1, sizeof(oracle_t));
    o->mu_ref = mu_ref; o->omega = omega; o->cfl = cfl; o->c2 = c2;
    o->n_ref = n_ref; o->n_min = n_min; o->max_cross = max_cross;
    o->seed = seed; o->inst = inst;
    int64_t nc = n_cells;
    o->nc = nc;
    o->ctype = (int *)xcalloc(nc, sizeof(int));
    o->cnf = (int *)xcalloc(nc, sizeof(int));
    o->vol = (double *)xcalloc(nc, sizeof(double));
    o->xc = (double *)xcalloc(3 * nc, sizeof(double));
    o->dS = (double *)xcalloc(3 * nc, sizeof(double));
    o->cface = (int64_t *)xcalloc(6 * nc, sizeof(int64_t));
    o->csign = (int *)xcalloc(6 * nc, sizeof(int));
    o->pn = (double *)xcalloc(18 * nc, sizeof(double));
    o->pd = (double *)xcalloc(6 * nc, sizeof(double));
    o->cnb = (int64_t *)xcalloc(6 * nc, sizeof(int64_t));
    o->cbf = (int64_t *)xcalloc(6 * nc, sizeof(int64_t));
    for (int64_t i = 0; i < 6 * nc; ++i) o->cbf[i] = -1;
    o->cnblf = (int *)xcalloc(6 * nc, sizeof(int));
    o->cper = (int *)xcalloc(6 * nc, sizeof(int));
    o->orig = (double *)xcalloc(3 * nc, sizeof(double));
    o->lfx = (double *)xcalloc(18 * nc, sizeof(double));
    o->venkat_k = 1.0;
    o->edge = (double *)xcalloc(9 * nc, sizeof(double));
    o->W = (double *)xcalloc(5 * nc, sizeof(double));
    o->P = (double *)xcalloc(5 * nc, sizeof(double));
    o->avgA = (double *)xcalloc(5 * nc, sizeof(double));
    o->tflux = (double *)xcalloc(5 * nc, sizeof(double));
    o->tE = (double *)xcalloc(5 * nc, sizeof(double));
    o->tS = (double *)xcalloc(5 * nc, sizeof(double));
    o->avg_from = -1;
    o->pr = 1.0;
    o->avg_res = INFINITY;
    o->nleft = (int64_t *)xcalloc(nc, sizeof(int64_t));
    o->nbc = n_bc;
    o->bc = (obc_t *)xcalloc(n_bc, sizeof(obc_t));
    for (int b = 0; b < n_bc; ++b) {
        o->bc[b].type = bc_type[b];
        o->bc[b].Tw = bc_Tw[b];
        for (int d = 0; d < 3; ++d) o->bc[b].Uw[d] = bc_Uw[3 * b + d];
        for (int k = 0; k < 5; ++k) o->bc[b].Winf[k] = bc_Winf[5 * b + k];
        for (int d = 0; d < 3; ++d) o->bc[b].shift[d] = bc_shift[3 * b + d];
    }

    /* per-cell local geometry: outward plane, area and face centre of each local face */
    double *larea = (double *)xcalloc(6 * nc, sizeof(double));
    int64_t nkeys = 0;
    for (int64_t c = 0; c < nc; ++c) {
        int64_t off = cell_node_off[c];
        int nn = (int)(cell_node_off[c + 1] - off);
        const int64_t *cn = cell_nodes + off;
        for (int i = 0; i < nn; ++i)
            if (cn[i] < 0 || cn[i] >= n_nodes) goto fail;
        if (cell_type[c] == 8 && nn == 8) {
            o->ctype[c] = 8;
            o->cnf[c] = 6;
            double x0 = xyz[3 * cn[0]], y0 = xyz[3 * cn[0] + 1], z0 = xyz[3 * cn[0] + 2];
            double x1 = xyz[3 * cn[6]], y1 = xyz[3 * cn[6] + 1], z1 = xyz[3 * cn[6] + 2];
            if (!(x1 > x0 && y1 > y0 && z1 > z0)) goto fail;
            /* every node must sit on its corner of the box */
            for (int i = 0; i < 8; ++i) {
                int bx = (i == 1 || i == 2 || i == 5 || i == 6);
                int by = (i == 2 || i == 3 || i == 6 || i == 7);
                int bz = (i >= 4);
                const double *p = xyz + 3 * cn[i];
                if (p[0] != (bx ? x1 : x0) || p[1] != (by ? y1 : y0) || p[2] != (bz ? z1 : z0)) goto fail;
            }
            double dx = x1 - x0, dy = y1 - y0, dz = z1 - z0;
            o->vol[c] = dx * dy * dz;
            o->xc[3 * c] = 0.5 * (x0 + x1);
            o->xc[3 * c + 1] = 0.5 * (y0 + y1);
            o->xc[3 * c + 2] = 0.5 * (z0 + z1);
            double lo[3] = {x0, y0, z0}, hi[3] = {x1, y1, z1}, ar[3] = {dy * dz, dx * dz, dx * dy};
            for (int a = 0; a < 3; ++a) {
                for (int s = 0; s < 2; ++s) {
                    int lf = 2 * a + s;
                    double *n = o->pn + 18 * c + 3 * lf;
                    n[0] = n[1] = n[2] = 0.0;
                    n[a] = s ? 1.0 : -1.0;
                    o->pd[6 * c + lf] = s ? hi[a] : -lo[a];
                    larea[6 * c + lf] = ar[a];
                    for (int d = 0; d < 3; ++d)
                        o->lfx[18 * c + 3 * lf + d] = d == a ? (s ? hi[a] : lo[a]) : o->xc[3 * c + d];
                }
            }
            o->orig[3 * c] = x0; o->orig[3 * c + 1] = y0; o->orig[3 * c + 2] = z0;
            double *E = o->edge + 9 * c;
            for (int i = 0; i < 9; ++i) E[i] = 0.0;
            E[0] = dx; E[4] = dy; E[8] = dz;
        } else if (cell_type[c] == 4 && nn == 4) {
            o->ctype[c] = 4;
            o->cnf[c] = 4;
            const double *A = xyz + 3 * cn[0], *B = xyz + 3 * cn[1], *C = xyz + 3 * cn[2], *D = xyz + 3 * cn[3];
            double e1[3], e2[3], e3[3];
            for (int d = 0; d < 3; ++d) { e1[d] = B[d] - A[d]; e2[d] = C[d] - A[d]; e3[d] = D[d] - A[d]; }
            double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e1[1] * (e2[0] * e3[2] - e2[2] * e3[0]) +
                         e1[2] * (e2[0] * e3[1] - e2[1] * e3[0]);
            if (!(fabs(det) > 0.0)) goto fail;
            o->vol[c] = fabs(det) / 6.0;
            for (int d = 0; d < 3; ++d) {
                o->xc[3 * c + d] = 0.25 * (A[d] + B[d] + C[d] + D[d]);
                o->orig[3 * c + d] = A[d];
                o->edge[9 * c + d] = e1[d];
                o->edge[9 * c + 3 + d] = e2[d];
                o->edge[9 * c + 6 + d] = e3[d];
            }
            for (int lf = 0; lf < 4; ++lf) {
                const double *p = xyz + 3 * cn[TETF[lf][0]], *q = xyz + 3 * cn[TETF[lf][1]],
                             *r = xyz + 3 * cn[TETF[lf][2]], *opp = xyz + 3 * cn[lf];
                double a[3], b[3], N[3];
                for (int d = 0; d < 3; ++d) { a[d] = q[d] - p[d]; b[d] = r[d] - p[d]; }
                N[0] = a[1] * b[2] - a[2] * b[1];
                N[1] = a[2] * b[0] - a[0] * b[2];
                N[2] = a[0] * b[1] - a[1] * b[0];
                double side = N[0] * (opp[0] - p[0]) + N[1] * (opp[1] - p[1]) + N[2] * (opp[2] - p[2]);
                if (side > 0) { N[0] = -N[0]; N[1] = -N[1]; N[2] = -N[2]; }
                double len = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
                double *n = o->pn + 18 * c + 3 * lf;
                double fc[3];
                for (int d = 0; d < 3; ++d) { n[d] = N[d] / len; fc[d] = (p[d] + q[d] + r[d]) / 3.0; }
                o->pd[6 * c + lf] = n[0] * fc[0] + n[1] * fc[1] + n[2] * fc[2];
                larea[6 * c + lf] = 0.5 * len;
                for (int d = 0; d < 3; ++d) o->lfx[18 * c + 3 * lf + d] = fc[d];
            }
        } else {
            goto fail;
        }
        nkeys += o->cnf[c];
    }

    /* face matching */
    {
        fkey_t *keys = (fkey_t *)xcalloc(nkeys, sizeof(fkey_t));
        int64_t q = 0;
        for (int64_t c = 0; c < nc; ++c) {
            const int64_t *cn = cell_nodes + cell_node_off[c];
            for (int lf = 0; lf < o->cnf[c]; ++lf) {
                fkey_t *k = keys + q++;
                int nn = o->ctype[c] == 8 ? 4 : 3;
                for (int i = 0; i < nn; ++i) k->key[i] = o->ctype[c] == 8 ? cn[HEXF[lf][i]] : cn[TETF[lf][i]];
                sort_key(k->key, nn);
                k->cell = c;
                k->lf = lf;
            }
        }
        qsort(keys, nkeys, sizeof(fkey_t), cmp_fkey);
        fkey_t *bk = (fkey_t *)xcalloc(n_bfaces, sizeof(fkey_t));
        for (int64_t b = 0; b < n_bfaces; ++b) {
            int nn = bface_nodes[4 * b + 3] < 0 ? 3 : 4;
            for (int i = 0; i < 4; ++i) bk[b].key[i] = bface_nodes[4 * b + i];
            sort_key(bk[b].key, nn);
            bk[b].cell = bface_bc[b];
            bk[b].lf = (int)b;
            if (bface_bc[b] < 0 || bface_bc[b] >= n_bc) { free(keys); free(bk); goto fail; }
        }
        qsort(bk, n_bfaces, sizeof(fkey_t), cmp_fkey);
        o->fown = (int64_t *)xcalloc(nkeys, sizeof(int64_t));
        o->fnb = (int64_t *)xcalloc(nkeys, sizeof(int64_t));
        o->fn = (double *)xcalloc(3 * nkeys, sizeof(double));
        o->farea = (double *)xcalloc(nkeys, sizeof(double));
        o->fx = (double *)xcalloc(3 * nkeys, sizeof(double));
        int64_t nf = 0;
        int bad = 0;
        for (int64_t i = 0; i < nkeys && !bad;) {
            int64_t j = i + 1;
            while (j < nkeys && memcmp(keys[j].key, keys[i].key, sizeof(keys[i].key)) == 0) ++j;
            int64_t c = keys[i].cell;
            int lf = keys[i].lf;
            if (j - i == 2) {
                int64_t c2 = keys[i + 1].cell;
                int lf2 = keys[i + 1].lf;
                /* owner: the first cell in sorted order (lower index) */
                o->fown[nf] = c;
                o->fnb[nf] = c2;
                for (int d = 0; d < 3; ++d) o->fn[3 * nf + d] = o->pn[18 * c + 3 * lf + d];
                for (int d = 0; d < 3; ++d) o->fx[3 * nf + d] = o->lfx[18 * c + 3 * lf + d];
                o->farea[nf] = larea[6 * c + lf];
                o->cface[6 * c + lf] = nf; o->csign[6 * c + lf] = 1;
                o->cface[6 * c2 + lf2] = nf; o->csign[6 * c2 + lf2] = -1;
                o->cnb[6 * c + lf] = c2; o->cnblf[6 * c + lf] = lf2;
                o->cnb[6 * c2 + lf2] = c; o->cnblf[6 * c2 + lf2] = lf;
                /* the neighbour uses exactly the reversed plane of the owner */
                for (int d = 0; d < 3; ++d) o->pn[18 * c2 + 3 * lf2 + d] = -o->pn[18 * c + 3 * lf + d];
                o->pd[6 * c2 + lf2] = -o->pd[6 * c + lf];
                ++nf;
            } else if (j - i == 1) {
                fkey_t probe = keys[i];
                int64_t lo = 0, hi = n_bfaces - 1, found = -1;
                while (lo <= hi) {
                    int64_t mid = (lo + hi) / 2;
                    int cm = 0;
                    for (int t = 0; t < 4 && cm == 0; ++t)
                        cm = bk[mid].key[t] < probe.key[t] ? -1 : (bk[mid].key[t] > probe.key[t] ? 1 : 0);
                    if (cm == 0) { found = mid; break; }
                    if (cm < 0) lo = mid + 1; else hi = mid - 1;
                }
                if (found < 0) { bad = 1; break; }
                int b = (int)bk[found].cell;
                if (o->bc[b].type == BC_PERIODIC) {
                    /* paired after this loop; mark the slot with its bc for now */
                    o->cper[6 * c + lf] = 1 + b;
                    o->cbf[6 * c + lf] = bk[found].lf;
                    i = j;
                    continue;
                }
                o->fown[nf] = c;
                o->fnb[nf] = -1 - b;
                for (int d = 0; d < 3; ++d) o->fn[3 * nf + d] = o->pn[18 * c + 3 * lf + d];
                for (int d = 0; d < 3; ++d) o->fx[3 * nf + d] = o->lfx[18 * c + 3 * lf + d];
                o->farea[nf] = larea[6 * c + lf];
                o->cface[6 * c + lf] = nf; o->csign[6 * c + lf] = 1;
                o->cnb[6 * c + lf] = -1 - b; o->cnblf[6 * c + lf] = -1;
                o->cbf[6 * c + lf] = bk[found].lf;
                ++nf;
            } else {
                bad = 1;
            }
            i = j;
        }
        free(keys);
        free(bk);
        if (bad) goto fail;
        /* periodic pairs: face A of bc b leads to the face B whose centre is A's centre plus
           b's shift, tagged with the opposite shift; they become one face owned by A's cell */
        char *paired = (char *)xcalloc(6 * nc, 1);
        for (int64_t c = 0; c < nc && !bad; ++c) {
            for (int lf = 0; lf < o->cnf[c] && !bad; ++lf) {
                int ba = o->cper[6 * c + lf] - 1;
                if (ba < 0 || paired[6 * c + lf]) continue;
                const double *s = o->bc[ba].shift, *xa = o->lfx + 18 * c + 3 * lf;
                double tx[3];
                for (int d = 0; d < 3; ++d) tx[d] = xa[d] + s[d];
                double scale = 1.0 + fabs(tx[0]) + fabs(tx[1]) + fabs(tx[2]);
                int64_t c2 = -1;
                int lf2 = -1;
                for (int64_t q = 0; q < nc && c2 < 0; ++q) {
                    for (int l2 = 0; l2 < o->cnf[q]; ++l2) {
                        int bb = o->cper[6 * q + l2] - 1;
                        if (bb < 0 || (q == c && l2 == lf) || paired[6 * q + l2]) continue;
                        const double *sb = o->bc[bb].shift, *xb = o->lfx + 18 * q + 3 * l2;
                        if (fabs(sb[0] + s[0]) + fabs(sb[1] + s[1]) + fabs(sb[2] + s[2]) > 1e-12 * scale) continue;
                        if (fabs(xb[0] - tx[0]) + fabs(xb[1] - tx[1]) + fabs(xb[2] - tx[2]) > 1e-9 * scale) continue;
                        c2 = q;
                        lf2 = l2;
                        break;
                    }
                }
                if (c2 < 0) { bad = 1; break; }
                o->fown[nf] = c;
                o->fnb[nf] = c2;
                for (int d = 0; d < 3; ++d) o->fn[3 * nf + d] = o->pn[18 * c + 3 * lf + d];
                for (int d = 0; d < 3; ++d) o->fx[3 * nf + d] = xa[d];
                o->farea[nf] = larea[6 * c + lf];
                o->cface[6 * c + lf] = nf; o->csign[6 * c + lf] = 1;
                o->cface[6 * c2 + lf2] = nf; o->csign[6 * c2 + lf2] = -1;
                o->cnb[6 * c + lf] = c2; o->cnblf[6 * c + lf] = lf2;
                o->cnb[6 * c2 + lf2] = c; o->cnblf[6 * c2 + lf2] = lf;
                paired[6 * c + lf] = paired[6 * c2 + lf2] = 1;
                ++o->nper;
                ++nf;
            }
        }
        free(paired);
        if (bad) goto fail;
        o->nf = nf;
    }
    for (int64_t c = 0; c < nc; ++c) {
        for (int lf = 0; lf < o->cnf[c]; ++lf) {
            const double *n = o->pn + 18 * c + 3 * lf;
            double a = larea[6 * c + lf];
            for (int d = 0; d < 3; ++d) o->dS[3 * c + d] += 0.5 * fabs(a * n[d]);
        }
    }
    free(larea);
    /* boundary faces in input order: p0, edges p1 - p0 and (p2 or p3) - p0, area */
    o->bo = (double *)xcalloc(3 * n_bfaces, sizeof(double));
    o->be1 = (double *)xcalloc(3 * n_bfaces, sizeof(double));
    o->be2 = (double *)xcalloc(3 * n_bfaces, sizeof(double));
    o->barea = (double *)xcalloc(n_bfaces, sizeof(double));
    o->btri = (int *)xcalloc(n_bfaces, sizeof(int));
    for (int64_t b = 0; b < n_bfaces; ++b) {
        const int64_t *bn = bface_nodes + 4 * b;
        int tri = bn[3] < 0;
        const double *p0 = xyz + 3 * bn[0], *p1 = xyz + 3 * bn[1], *pq = xyz + 3 * (tri ? bn[2] : bn[3]);
        double e1[3], e2[3];
        for (int d = 0; d < 3; ++d) {
            o->bo[3 * b + d] = p0[d];
            e1[d] = p1[d] - p0[d];
            e2[d] = pq[d] - p0[d];
            o->be1[3 * b + d] = e1[d];
            o->be2[3 * b + d] = e2[d];
        }
        double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2], cz = e1[0] * e2[1] - e1[1] * e2[0];
        double cr = sqrt(cx * cx + cy * cy + cz * cz);
        o->barea[b] = tri ? 0.5 * cr : cr;
        o->btri[b] = tri;
    }
    o->cap = 0;
    *status = ORC_OK;
    return o;
fail:
    free(larea);
    orc_destroy(o);
    return NULL;
}

void orc_destroy(oracle_t *o)
{
    if (!o) return;
    free(o->ctype); free(o->cnf); free(o->vol); free(o->xc); free(o->dS);
    free(o->cface); free(o->csign); free(o->pn); free(o->pd); free(o->cnb); free(o->cnblf); free(o->cbf);
    free(o->cper);
    free(o->bo); free(o->be1); free(o->be2); free(o->barea); free(o->btri);
    free(o->orig); free(o->edge); free(o->fown); free(o->fnb); free(o->fn); free(o->farea);
    free(o->lfx); free(o->fx);
    free(o->bc); free(o->W); free(o->P); free(o->avgA); free(o->nleft);
    free(o->tflux); free(o->tE); free(o->tS);
    free(o->px); free(o->pu); free(o->pm); free(o->pe); free(o->pc); free(o->pid);
    free(o);
}

int64_t orc_n_cells(const oracle_t *o) { return o->nc; }
int64_t orc_n_faces(const oracle_t *o) { return o->nf; }
int64_t orc_n_particles(const oracle_t *o) { return o->np; }
int64_t orc_step_index(const oracle_t *o) { return o->step; }

/* Threads of the OpenMP build (n > 0 sets them first); the serial build always runs one. */
int orc_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
double orc_time(const oracle_t *o) { return o->t; }

/* reconstruction: 0 first order, 1 LSQ + Barth-Jespersen, 2 LSQ + Venkatakrishnan (K) */
int orc_set_recon(oracle_t *o, int recon, double venkat_k)
{
    if (recon < 0 || recon > 2 || !(venkat_k > 0.0)) return ORC_E_ARG;
    /* the gradients use neighbour centres, which a periodic face would need shifted */
    if (recon != 0 && o->nper > 0) return ORC_E_ARG;
    o->recon = recon;
    o->venkat_k = venkat_k;
    return ORC_OK;
}

/* Wave-only start (the continuum start of the paper's hypersonic cases, Sec. 4.3 and 4.4: the
   flow field is first computed by the gas-kinetic scheme alone): the steps n < gks_steps,
   counted from orc_set_state, sample no particle and inject none, and their wave flux carries
   the whole free transport of W^h (see wave_only_coef). */
int orc_set_gks_steps(oracle_t *o, int64_t gks_steps)
{
    if (gks_steps < 0) return ORC_E_ARG;
    o->gks_steps = gks_steps;
    return ORC_OK;
}

/* Internal degrees of freedom (Sec. 2.1): K components of xi in the Maxwellian, so that
   rho E = rho |U|^2 / 2 + (3 + K) rho T / 2 and gamma = (K + 5)/(K + 3) (K = 2: a diatomic gas,
   gamma = 7/5).  A particle carries its internal energy variable e = |xi|^2, sampled like xi
   (Sec. 2.3: sampled from the temperature and K, as in DSMC); 0 <= K <= KMAX. */
int orc_set_internal_dof(oracle_t *o, int K)
{
    if (K < 0 || K > KMAX) return ORC_E_ARG;
    o->K = K;
    return ORC_OK;
}

/* sampling of the hydro particles' velocities: 0 as printed in Sec. 2.4(b) (default), 1 the
   energy-exact variant (a departure from the paper), 2 the first-order g_p, 3 independent
   draws from the equilibrium of the collision model (see phase_sample) */
int orc_set_sampling(oracle_t *o, int mode)
{
    if (mode < 0 || mode > 3) return ORC_E_ARG;
    /* the first-order g_p needs the cell gradients of the reconstruction */
    if (mode == 2 && o->recon == 0) return ORC_E_ARG;
    o->sampling = mode;
    return ORC_OK;
}

/* Collision model: Pr = 1 is the BGK model the paper builds the method on (Sec. 2.1); any other
   0 < Pr < 2 selects the Shakhov model, one of the relaxation models the paper names in its
   place (Sec. 2.1, Sec. 5), for a monatomic gas only (K = 0) and with the hydro particles drawn
   one by one (sampling 2 or 3: pairs U +- sqrt(T) X carry no heat flux); checked by orc_step. */
int orc_set_prandtl(oracle_t *o, double pr)
{
    if (!(pr > 0.0 && pr < 2.0)) return ORC_E_ARG;
    o->pr = pr;
    return ORC_OK;
}

void orc_geometry(const oracle_t *o, double *vol, double *xc, double *dS)
{
    memcpy(vol, o->vol, sizeof(double) * o->nc);
    memcpy(xc, o->xc, sizeof(double) * 3 * o->nc);
    memcpy(dS, o->dS, sizeof(double) * 3 * o->nc);
}

void orc_stats(const oracle_t *o, double *dt, int64_t out[10])
{
    *dt = o->st_dt;
    out[0] = o->st_alive; out[1] = o->st_sampled; out[2] = o->st_collided;
    out[3] = o->st_escaped; out[4] = o->st_cross; out[5] = o->st_wallhits; out[6] = o->st_injected;
    out[7] = o->st_floored; out[8] = o->st_rhoh_neg; out[9] = o->st_maxcross;
}

int orc_set_state(oracle_t *o, const double *W)
{
    memcpy(o->W, W, sizeof(double) * 5 * o->nc);
    memset(o->P, 0, sizeof(double) * 5 * o->nc);
    memset(o->nleft, 0, sizeof(int64_t) * o->nc);
    o->np = 0;
    o->step = 0;
    o->t = 0.0;
    memset(o->avgA, 0, sizeof(double) * 5 * o->nc);
    o->avg_D = 0.0;
    o->avg_n = 0;
    o->avg_res = INFINITY;
    return ORC_OK;
}

/* Replace the state between steps: W and the raw sums P ([nc][5]) of the n particles that
   remain (x, u, m, cell, uid), the step counter and the time.  The particles become the old
   particles of the next step (any order); N_left of a cell is its count.  The averaging sums
   are cleared and its setting kept. */
int orc_import_state(oracle_t *o, const double *W, const double *P, int64_t n, const double *x, const double *u,
                     const double *m, const int64_t *cell, const uint64_t *uid, const double *e, int64_t step,
                     double t)
{
    if (n < 0 || step < 0) return ORC_E_ARG;
    for (int64_t i = 0; i < n; ++i)
        if (cell[i] < 0 || cell[i] >= o->nc) return ORC_E_ARG;
    if (reserve(o, n)) return ORC_E_CAPACITY;
    memcpy(o->W, W, sizeof(double) * 5 * o->nc);
    memcpy(o->P, P, sizeof(double) * 5 * o->nc);
    memset(o->nleft, 0, sizeof(int64_t) * o->nc);
    for (int64_t i = 0; i < n; ++i) {
        for (int d = 0; d < 3; ++d) { o->px[3 * i + d] = x[3 * i + d]; o->pu[3 * i + d] = u[3 * i + d]; }
        o->pm[i] = m[i];
        o->pe[i] = e ? e[i] : 0.0;
        o->pc[i] = cell[i];
        o->pid[i] = uid[i];
        o->nleft[cell[i]] += 1;
    }
    o->np = n;
    o->step = step;
    o->t = t;
    memset(o->avgA, 0, sizeof(double) * 5 * o->nc);
    o->avg_D = 0.0;
    o->avg_n = 0;
    o->avg_res = INFINITY;
    return ORC_OK;
}

/* Average the steps n > n_avg (counted from orc_set_state) from now on; n_avg < 0 turns
   averaging off.  Clears what was accumulated. */
void orc_set_averaging(oracle_t *o, int64_t n_avg)
{
    o->avg_from = n_avg < 0 ? -1 : n_avg;
    memset(o->avgA, 0, sizeof(double) * 5 * o->nc);
    o->avg_D = 0.0;
    o->avg_n = 0;
    o->avg_res = INFINITY;
}

/* Wbar ([nc][5], may be NULL), the relative change of the last averaged step and the number
   of steps averaged; ORC_E_ARG while nothing has been averaged. */
int orc_average(const oracle_t *o, double *Wbar, double *residual, int64_t *n_averaged)
{
    if (o->avg_n == 0) return ORC_E_ARG;
    if (Wbar)
        for (int64_t i = 0; i < 5 * o->nc; ++i) Wbar[i] = o->avgA[i] / o->avg_D;
    if (residual) *residual = o->avg_res;
    if (n_averaged) *n_averaged = o->avg_n;
    return ORC_OK;
}

void orc_get_state(const oracle_t *o, double *W, double *P, int64_t *nleft)
{
    memcpy(W, o->W, sizeof(double) * 5 * o->nc);
    memcpy(P, o->P, sizeof(double) * 5 * o->nc);
    memcpy(nleft, o->nleft, sizeof(int64_t) * o->nc);
}

/* Test hook: the terms of the last update of every cell, raw (times Omega): the wave flux
   -sum_f s_f Phi_f, the sums E over the particles that ended the step in the cell and S over
   those that started it there ([nc][5] each). */
void orc_last_terms(const oracle_t *o, double *flux, double *E, double *S)
{
    memcpy(flux, o->tflux, sizeof(double) * 5 * o->nc);
    memcpy(E, o->tE, sizeof(double) * 5 * o->nc);
    memcpy(S, o->tS, sizeof(double) * 5 * o->nc);
}

void orc_get_particles(const oracle_t *o, double *x, double *u, double *m, int64_t *cell, uint64_t *uid, double *e)
{
    memcpy(x, o->px, sizeof(double) * 3 * o->np);
    memcpy(u, o->pu, sizeof(double) * 3 * o->np);
    memcpy(m, o->pm, sizeof(double) * o->np);
    if (e) memcpy(e, o->pe, sizeof(double) * o->np);
    memcpy(cell, o->pc, sizeof(int64_t) * o->np);
    memcpy(uid, o->pid, sizeof(uint64_t) * o->np);
}

static int reserve(oracle_t *o, int64_t n)
{
    if (n <= o->cap) return 0;
    int64_t cap = o->cap ? o->cap : 1024;
    while (cap < n) cap *= 2;
    double *px = (double *)realloc(o->px, sizeof(double) * 3 * cap);
    if (px) o->px = px;
    double *pu = (double *)realloc(o->pu, sizeof(double) * 3 * cap);
    if (pu) o->pu = pu;
    double *pm = (double *)realloc(o->pm, sizeof(double) * cap);
    if (pm) o->pm = pm;
    double *pe = (double *)realloc(o->pe, sizeof(double) * cap);
    if (pe) o->pe = pe;
    int64_t *pc = (int64_t *)realloc(o->pc, sizeof(int64_t) * cap);
    if (pc) o->pc = pc;
    uint64_t *pid = (uint64_t *)realloc(o->pid, sizeof(uint64_t) * cap);
    if (pid) o->pid = pid;
    if (!px || !pu || !pm || !pe || !pc || !pid) return -1;
    o->cap = cap;
    return 0;
}

/* phi = m (1, u, (|u|^2 + e) / 2): mass, momentum and energy carried by a particle (Sec. 2.3),
   e its internal energy variable (0 for K = 0). */
static void add_phi(double S[5], double m, const double u[3], double e)
{
    S[0] += m;
    S[1] += m * u[0];
    S[2] += m * u[1];
    S[3] += m * u[2];
    S[4] += m * (0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2] + e));
}

/* e = T |X|^2 with X the first K of standard normals drawn by Box-Muller from the draws
   (seed, uid, step, tag, sub0 + j, inst), j = 0, 1: the internal energy variable of a particle
   in equilibrium at temperature T (a chi-squared law with K degrees of freedom, times T) */
static double internal_energy(uint64_t seed, uint64_t uid, int64_t step, int tag, uint32_t sub0, int64_t inst,
                              int K, double T)
{
    double acc = 0.0;
    for (int j = 0; 4 * j < K; ++j) {
        double ev[4];
        draw4(seed, uid, step, tag, sub0 + (uint32_t)j, inst, ev);
        double r1 = sqrt(-2.0 * log(ev[0])), r2 = sqrt(-2.0 * log(ev[2]));
        double X[4] = {r1 * cos(2.0 * M_PI * ev[1]), r1 * sin(2.0 * M_PI * ev[1]), r2 * cos(2.0 * M_PI * ev[3]),
                       r2 * sin(2.0 * M_PI * ev[3])};
        for (int i = 0; i < 4 && 4 * j + i < K; ++i) acc = acc + X[i] * X[i];
    }
    return T * acc;
}

/* ------------------------------------------------------------------------------------ */
/* Free transport of one particle for time ts through the mesh (Sec. 2.3), face to face:  */
/* exit time over the faces with n.u > 0 other than the entry face, clamped at 0, lowest  */
/* local index on a tie; t_exit >= t_rem stays in the cell.  Walls: specular mirrors u;    */
/* diffuse re-emits from the wall Maxwellian (flux-weighted normal component); far-field  */
/* removes the particle.  Returns 0 (inside), 1 (escaped) or -1 (too many crossings).      */
/* ------------------------------------------------------------------------------------ */
int orc_track(const oracle_t *o, double x[3], double u[3], double *e, int64_t *cell, double ts, int entry0,
              uint64_t uid, int64_t step, int64_t *ncross, int64_t *nwall)
{
    int64_t c = *cell;
    int entry = entry0;
    double trem = ts;
    int bounce = 0;
    *ncross = 0;
    for (;;) {
        double best = INFINITY;
        int bf = -1;
        for (int lf = 0; lf < o->cnf[c]; ++lf) {
            if (lf == entry) continue;
            const double *n = o->pn + 18 * c + 3 * lf;
            double un = n[0] * u[0] + n[1] * u[1] + n[2] * u[2];
            if (un > 0.0) {
                double tt = (o->pd[6 * c + lf] - (n[0] * x[0] + n[1] * x[1] + n[2] * x[2])) / un;
                if (tt < 0.0) tt = 0.0;
                if (tt < best) { best = tt; bf = lf; }
            }
        }
        if (bf < 0 || best >= trem) {
            for (int d = 0; d < 3; ++d) x[d] = x[d] + u[d] * trem;
            *cell = c;
            return 0;
        }
        for (int d = 0; d < 3; ++d) x[d] = x[d] + u[d] * best;
        trem = trem - best;
        if (++*ncross > o->max_cross) { *cell = c; return -1; }
        int64_t nb = o->cnb[6 * c + bf];
        if (nb >= 0) {
            int per = o->cper[6 * c + bf];
            if (per) {
                /* periodic face: the particle goes on from the partner face */
                const double *s = o->bc[per - 1].shift;
                for (int d = 0; d < 3; ++d) x[d] = x[d] + s[d];
            }
            entry = o->cnblf[6 * c + bf];
            c = nb;
            continue;
        }
        const obc_t *b = o->bc + (-1 - nb);
        const double *n = o->pn + 18 * c + 3 * bf;
        if (b->type == BC_SPECULAR) {
            double un = n[0] * u[0] + n[1] * u[1] + n[2] * u[2];
            for (int d = 0; d < 3; ++d) u[d] = u[d] - 2.0 * un * n[d];
            entry = bf;
        } else if (b->type == BC_DIFFUSE) {
            double eta[4], t1[3], t2[3];
            draw4(o->seed, uid, step, TAG_WALL, (uint32_t)bounce, o->inst, eta);
            ++bounce;
            ++*nwall;
            face_frame(n, t1, t2);
            double sq = sqrt(b->Tw);
            double vn = sqrt(-2.0 * b->Tw * log(eta[0]));
            double r = sqrt(-2.0 * log(eta[1]));
            double X1 = r * cos(2.0 * M_PI * eta[2]), X2 = r * sin(2.0 * M_PI * eta[2]);
            for (int d = 0; d < 3; ++d) u[d] = b->Uw[d] - vn * n[d] + sq * (X1 * t1[d] + X2 * t2[d]);
            /* full accommodation: the internal energy leaves in equilibrium at T_w too */
            if (o->K > 0 && e)
                *e = internal_energy(o->seed, uid, step, TAG_WALLINT, 2u * (uint32_t)(bounce - 1), o->inst, o->K, b->Tw);
            entry = bf;
        } else {
            *cell = c;
            return 1;
        }
    }
}

/* ------------------------------------------------------------------------------------ */
/* One time step.                                                                          */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    double dt;
    double *tau, *ec, *rhoh, *U, *T;
    double *Wh;      /* [nc][5] hydro state (rho^h / rho) W (second order) */
    double *gW, *gH; /* [nc][5][3] limited gradients of W and of the hydro state */
    double *qh;      /* [nc][3] heat flux of the gas (Shakhov model only) */
} cellq_t;

static void cellq_free(cellq_t *q)
{
    free(q->tau); free(q->ec); free(q->rhoh); free(q->U); free(q->T);
    free(q->Wh); free(q->gW); free(q->gH); free(q->qh);
}

/* Heat flux of the gas in each cell at the start of a step (Shakhov model):
 *   q = (1/Omega) sum_k m_k c_k |c_k|^2 / 2,  c_k = u_k - U,
 * over the particles in the cell, U = (W_1, W_2, W_3) / W_0 the cell's velocity (K = 0).
 * Reading: the hydro part is a Maxwellian at the cell's U and T (the law it is sampled from)
 * and carries none.  Summed in particle order. */
static void cell_heat_flux(const oracle_t *o, double *qh)
{
    memset(qh, 0, sizeof(double) * 3 * o->nc);
    for (int64_t i = 0; i < o->np; ++i) {
        const int64_t c = o->pc[i];
        const double *W = o->W + 5 * c;
        double cv[3];
        for (int d = 0; d < 3; ++d) cv[d] = o->pu[3 * i + d] - W[1 + d] / W[0];
        const double h = 0.5 * o->pm[i] * (cv[0] * cv[0] + cv[1] * cv[1] + cv[2] * cv[2]);
        for (int d = 0; d < 3; ++d) qh[3 * c + d] += h * cv[d];
    }
    for (int64_t c = 0; c < o->nc; ++c)
        for (int d = 0; d < 3; ++d) qh[3 * c + d] = qh[3 * c + d] / o->vol[c];
}

/* the cells' heat fluxes for the current state (test hook) */
void orc_heat_flux(const oracle_t *o, double *qh) { cell_heat_flux(o, qh); }

/* Primitives, relaxation time tau = mu_ref T^omega / p (Eq. tau_via_T_ref, T_ref = 1), the
 * time step dt = CFL min Omega / sum_d (|U_d| + 3 sqrt(T)) dS_d (Sec. 2.4(a)), the hydro
 * density rho^h = rho - rho^p clamped at 0, and the collisionless fraction exp(-dt/tau). */
static int phase_cells(oracle_t *o, cellq_t *q)
{
    const int64_t nc = o->nc;
    q->tau = (double *)xcalloc(nc, sizeof(double));
    q->ec = (double *)xcalloc(nc, sizeof(double));
    q->rhoh = (double *)xcalloc(nc, sizeof(double));
    q->U = (double *)xcalloc(3 * nc, sizeof(double));
    q->T = (double *)xcalloc(nc, sizeof(double));
    double dtmin = INFINITY;
    for (int64_t c = 0; c < nc; ++c) {
        const double *W = o->W + 5 * c;
        double rho = W[0];
        if (!(rho > 0.0) || !isfinite(rho)) return ORC_E_NONPHYS;
        double U = W[1] / rho, V = W[2] / rho, Z = W[3] / rho;
        double T = temp_k(W, o->K);
        if (!(T > 0.0) || !isfinite(T)) return ORC_E_NONPHYS;
        q->U[3 * c] = U; q->U[3 * c + 1] = V; q->U[3 * c + 2] = Z;
        q->T[c] = T;
        q->tau[c] = o->mu_ref * pow(T, o->omega) / (rho * T);
        double cs = 3.0 * sqrt(T);
        double lam = (fabs(U) + cs) * o->dS[3 * c] + (fabs(V) + cs) * o->dS[3 * c + 1] +
                     (fabs(Z) + cs) * o->dS[3 * c + 2];
        double r = o->vol[c] / lam;
        if (r < dtmin) dtmin = r;
    }
    q->dt = o->cfl * dtmin;
    o->st_floored = 0;
    o->st_rhoh_neg = 0;
    for (int64_t c = 0; c < nc; ++c) {
        /* rho^h = rho - rho^p is a difference of two sums; below 1e-12 rho it is roundoff of
           that subtraction (e.g. free-molecular cells where the particles hold all the mass)
           and counts as an empty hydro part */
        double rh = o->W[5 * c] - o->P[5 * c] / o->vol[c];
        q->rhoh[c] = rh > RHOH_EPS * o->W[5 * c] ? rh : 0.0;
        if (rh > 0.0 && q->rhoh[c] == 0.0) ++o->st_floored;
        if (rh < 0.0) ++o->st_rhoh_neg;
        q->ec[c] = o->step < o->gks_steps ? 0.0 : exp(-q->dt / q->tau[c]);
    }
    return ORC_OK;
}

/* Temperature of a conservative state of this gas (R = 1). */
static double temp_of(const oracle_t *o, const double W[5]) { return temp_k(W, o->K); }

/* The state seen across local face lf of cell c for the gradient: the neighbour's (at its
 * centre) or, at a boundary, a ghost at the centre mirrored in the face plane: specular, the
 * mirror state (normal momentum reversed); diffuse, density and temperature of the cell with
 * the velocity reflected about the wall's (2 U_w - U); far field, the free stream.  The
 * ghost's hydro state is (rho^h / rho) times its state (the free stream: all of it). */
static void across(const oracle_t *o, const cellq_t *q, int64_t c, int lf, double xj[3], double Wj[5],
                   double Whj[5])
{
    int64_t nb = o->cnb[6 * c + lf];
    const double *xc = o->xc + 3 * c, *Wc = o->W + 5 * c;
    if (nb >= 0) {
        for (int d = 0; d < 3; ++d) xj[d] = o->xc[3 * nb + d];
        for (int k = 0; k < 5; ++k) { Wj[k] = o->W[5 * nb + k]; Whj[k] = q->Wh[5 * nb + k]; }
        return;
    }
    const double *n = o->pn + 18 * c + 3 * lf;
    double dist = o->pd[6 * c + lf] - (n[0] * xc[0] + n[1] * xc[1] + n[2] * xc[2]);
    for (int d = 0; d < 3; ++d) xj[d] = xc[d] + 2.0 * dist * n[d];
    const obc_t *b = o->bc + (-1 - nb);
    if (b->type == BC_FARFIELD) {
        for (int k = 0; k < 5; ++k) { Wj[k] = b->Winf[k]; Whj[k] = b->Winf[k]; }
        return;
    }
    double rho = Wc[0], U[3] = {Wc[1] / rho, Wc[2] / rho, Wc[3] / rho}, T = temp_of(o, Wc), Ug[3];
    if (b->type == BC_SPECULAR) {
        double un = U[0] * n[0] + U[1] * n[1] + U[2] * n[2];
        for (int d = 0; d < 3; ++d) Ug[d] = U[d] - 2.0 * un * n[d];
    } else {
        for (int d = 0; d < 3; ++d) Ug[d] = 2.0 * b->Uw[d] - U[d];
    }
    Wj[0] = rho;
    for (int d = 0; d < 3; ++d) Wj[1 + d] = rho * Ug[d];
    Wj[4] = 0.5 * rho * (Ug[0] * Ug[0] + Ug[1] * Ug[1] + Ug[2] * Ug[2]) + 0.5 * (3.0 + o->K) * rho * T;
    double f = q->rhoh[c] / rho;
    for (int k = 0; k < 5; ++k) Whj[k] = f * Wj[k];
}

/* Gradients for second order (Sec. 2.2, reconstruction): the unweighted least-squares
 * gradient over the face neighbours, g = (sum d d^T)^-1 sum d (W_j - W_c) with d = x_j - x_c,
 * of the 5 components of W and of the hydro state W~^h = (rho^h / rho) W; then per component
 * a limiter phi = min over the faces of
 *   Barth-Jespersen:  min(1, (W_max - W_c) / D) for D > 0, min(1, (W_min - W_c) / D) for D < 0
 *   Venkatakrishnan:  ((M^2 + eps^2) D + 2 D^2 M) / (D (M^2 + 2 D^2 + M D + eps^2)), M the same
 *                     bound minus W_c, eps^2 = (K h)^3, h = Omega^(1/3)
 * with D = g . (x_f - x_c) (1 where D = 0), W_max and W_min over the cell and its neighbours.
 * A cell whose limited face states include rho <= 0, T <= 0 or a negative hydro density
 * (or a hydro temperature <= 0) falls back to first order (all its gradients zero).  A face
 * hydro density within 1e-12 of the face density of zero is roundoff of an empty hydro part
 * (the limiter pins it exactly to a neighbour's zero, and rounding picks the sign): it counts
 * as zero, here and in the flux. */
static void phase_grad(oracle_t *o, cellq_t *q)
{
    const int64_t nc = o->nc;
    q->Wh = (double *)xcalloc(5 * nc, sizeof(double));
    q->gW = (double *)xcalloc(15 * nc, sizeof(double));
    q->gH = (double *)xcalloc(15 * nc, sizeof(double));
    for (int64_t c = 0; c < nc; ++c) {
        double f = q->rhoh[c] / o->W[5 * c];
        for (int k = 0; k < 5; ++k) q->Wh[5 * c + k] = f * o->W[5 * c + k];
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t c = 0; c < nc; ++c) {
        const double *xc = o->xc + 3 * c;
        double A[3][3] = {{0}}, r[10][3] = {{0}}, vmax[10], vmin[10], vc[10];
        for (int k = 0; k < 5; ++k) { vc[k] = o->W[5 * c + k]; vc[5 + k] = q->Wh[5 * c + k]; }
        for (int k = 0; k < 10; ++k) vmax[k] = vmin[k] = vc[k];
        for (int lf = 0; lf < o->cnf[c]; ++lf) {
            double xj[3], Wj[5], Whj[5], dx[3], vj[10];
            across(o, q, c, lf, xj, Wj, Whj);
            for (int d = 0; d < 3; ++d) dx[d] = xj[d] - xc[d];
            for (int k = 0; k < 5; ++k) { vj[k] = Wj[k]; vj[5 + k] = Whj[k]; }
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) A[a][b] += dx[a] * dx[b];
            for (int k = 0; k < 10; ++k) {
                for (int a = 0; a < 3; ++a) r[k][a] += dx[a] * (vj[k] - vc[k]);
                if (vj[k] > vmax[k]) vmax[k] = vj[k];
                if (vj[k] < vmin[k]) vmin[k] = vj[k];
            }
        }
        /* inverse of the symmetric 3x3 normal matrix by cofactors */
        double C[3][3];
        C[0][0] = A[1][1] * A[2][2] - A[1][2] * A[2][1];
        C[0][1] = A[0][2] * A[2][1] - A[0][1] * A[2][2];
        C[0][2] = A[0][1] * A[1][2] - A[0][2] * A[1][1];
        C[1][0] = A[1][2] * A[2][0] - A[1][0] * A[2][2];
        C[1][1] = A[0][0] * A[2][2] - A[0][2] * A[2][0];
        C[1][2] = A[0][2] * A[1][0] - A[0][0] * A[1][2];
        C[2][0] = A[1][0] * A[2][1] - A[1][1] * A[2][0];
        C[2][1] = A[0][1] * A[2][0] - A[0][0] * A[2][1];
        C[2][2] = A[0][0] * A[1][1] - A[0][1] * A[1][0];
        double det = A[0][0] * C[0][0] + A[0][1] * C[1][0] + A[0][2] * C[2][0];
        double g[10][3];
        for (int k = 0; k < 10; ++k)
            for (int a = 0; a < 3; ++a)
                g[k][a] = (C[a][0] * r[k][0] + C[a][1] * r[k][1] + C[a][2] * r[k][2]) / det;
        if (o->recon == 1 || o->recon == 2) {
            double h = cbrt(o->vol[c]);
            double eps2 = pow(o->venkat_k * h, 3.0);
            for (int k = 0; k < 10; ++k) {
                double phi = 1.0;
                for (int lf = 0; lf < o->cnf[c]; ++lf) {
                    const double *xf = o->lfx + 18 * c + 3 * lf;
                    double D = g[k][0] * (xf[0] - xc[0]) + g[k][1] * (xf[1] - xc[1]) + g[k][2] * (xf[2] - xc[2]);
                    double pf = 1.0;
                    if (D != 0.0) {
                        double M = D > 0.0 ? vmax[k] - vc[k] : vmin[k] - vc[k];
                        if (o->recon == 1) {
                            pf = M / D;
                            if (pf > 1.0) pf = 1.0;
                        } else {
                            pf = ((M * M + eps2) * D + 2.0 * D * D * M) / (D * (M * M + 2.0 * D * D + M * D + eps2));
                        }
                    }
                    if (pf < phi) phi = pf;
                }
                for (int a = 0; a < 3; ++a) g[k][a] *= phi;
            }
        }
        int ok = 1;
        for (int lf = 0; lf < o->cnf[c] && ok; ++lf) {
            const double *xf = o->lfx + 18 * c + 3 * lf;
            double Wf[10];
            for (int k = 0; k < 10; ++k)
                Wf[k] = vc[k] + g[k][0] * (xf[0] - xc[0]) + g[k][1] * (xf[1] - xc[1]) + g[k][2] * (xf[2] - xc[2]);
            if (!(Wf[0] > 0.0) || !(temp_of(o, Wf) > 0.0)) ok = 0;
            if (!(Wf[5] >= -RHOH_EPS * Wf[0])) ok = 0;
            if (Wf[5] > RHOH_EPS * Wf[0] && !(temp_of(o, Wf + 5) > 0.0)) ok = 0;
        }
        for (int k = 0; k < 5; ++k)
            for (int a = 0; a < 3; ++a) {
                q->gW[15 * c + 3 * k + a] = ok ? g[k][a] : 0.0;
                q->gH[15 * c + 3 * k + a] = ok ? g[5 + k][a] : 0.0;
            }
    }
}

/* a cell's state extrapolated to a point: V_c + g . (x - x_c) */
static void extrap(const double *Vc, const double *g, const double *xc, const double *x, double out[5])
{
    for (int k = 0; k < 5; ++k)
        out[k] = Vc[k] + g[3 * k] * (x[0] - xc[0]) + g[3 * k + 1] * (x[1] - xc[1]) + g[3 * k + 2] * (x[2] - xc[2]);
}

/* a uniform point in cell c from the draw (uid, step, TAG_POS): per axis in a box; in a
 * tetrahedron the unit cube folded onto it (Rocchini & Cignoni 2000) */
static void place_in_cell(const oracle_t *o, int64_t c, uint64_t uid, double x[3])
{
    double ep[4];
    draw4(o->seed, uid, o->step, TAG_POS, 0, o->inst, ep);
    const double *org = o->orig + 3 * c, *Ed = o->edge + 9 * c;
    double s = ep[0], t = ep[1], w = ep[2];
    if (o->ctype[c] == 4) {
        if (s + t > 1.0) { s = 1.0 - s; t = 1.0 - t; }
        if (t + w > 1.0) {
            double tmp = w;
            w = 1.0 - s - t;
            t = 1.0 - tmp;
        } else if (s + t + w > 1.0) {
            double tmp = w;
            w = s + t + w - 1.0;
            s = 1.0 - t - tmp;
        }
    }
    for (int d = 0; d < 3; ++d) x[d] = org[d] + s * Ed[d] + t * Ed[3 + d] + w * Ed[6 + d];
}

/* First-order g_p (Sec. 2.3), the law of the hydro particles with sampling = 2.  The particles
 * that collided by time t follow the modified equilibrium
 *   g_p = g_0 + (t e/(1 - e) - tau) u . grad g + (t/(1 - e) - tau) d_t g,   e = exp(-t/tau).
 * Reading: at t = dt, with g expanded to first order about the end of that interval, which is
 * the state W^n the step starts from (g_0 + dt d_t g = g(W^n)), this is
 *   g_p = g(W^n) [1 + alpha (sum_d u_d (a_d . psi) + A . psi)],
 *   alpha = dt e/(1 - e) - tau = dt / expm1(dt/tau) - tau,
 * where a_d is the micro slope of the cell's limited gradient of W along x_d (the slope solve
 * of dW/dx_d / rho) and A the time slope from the compatibility condition
 * <(sum_d u_d (a_d . psi) + A . psi) psi g> = 0; the correction carries no mass, momentum or
 * energy.  alpha tends to -tau in the continuum limit (the Chapman-Enskog distribution) and
 * to -dt/2 in the free-molecular one.
 * Sampling by acceptance-rejection from one stream of proposals per cell (see
 * sample_one_by_one): proposal p is u = U + sqrt(T) X (X ~ N(0, I) by Box-Muller on the draw
 * (uid_p, step, TAG_GP, 0), uid_p the id a particle p of the cell would have; with K > 0 the
 * internal energy T chi^2_K from the draws (uid_p, TAG_INT, 0 and 1)), accepted when
 * eta B < 1 + alpha (...) with eta the first uniform of (uid_p, step, TAG_GP, 1).  B bounds
 * |1 + alpha (...)| where every normal of the proposal is at most R = 4 in size
 * (Chapman-Enskog form of the correction, below); beyond that box, and where 1 + alpha (...)
 * < 0, the law is clipped.
 * The bound: with the correction written as (X = (u - U)/sqrt(T), z = e/T)
 *   X_i X_j d_j U_i - (|X|^2 + z)/(3 + K) div U + ((|X|^2 + z)/2 - (5 + K)/2) sqrt(T) X . grad ln T,
 *   B = 1 + |alpha| (R^2 (sum_ij |d_j U_i| + |div U|)
 *                    + ((3 + K) R^2 + 5 + K)/2 R sqrt(T) sum_j |d_j T| / T). */
typedef struct { double a[3][5], A[5], alpha, B; } gp_t;

/* g_p of a cell of state W with limited gradient gW ([5][3], d W_k / d x_d), tau and dt */
static void gp_setup(const double W[5], const double gW[15], double tau, double dt, int Kdof, gp_t *gp)
{
    const double rho = W[0], U[3] = {W[1] / rho, W[2] / rho, W[3] / rho}, T = temp_k(W, Kdof), lam = 0.5 / T;
    const prim_t g = {1.0, U[0], U[1], U[2], lam, T, Kdof};
    double bt[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int d = 0; d < 3; ++d) {
        double b[5], m[5];
        for (int k = 0; k < 5; ++k) b[k] = gW[3 * k + d] / rho;
        orc_slope(U[0], U[1], U[2], lam, Kdof, b, gp->a[d]);
        poly_t pre;
        poly_mono(d == 0, d == 1, d == 2, &pre);
        mvec(&pre, gp->a[d], 0, &g, m);
        for (int k = 0; k < 5; ++k) bt[k] -= m[k];
    }
    orc_slope(U[0], U[1], U[2], lam, Kdof, bt, gp->A);
    gp->alpha = dt / expm1(dt / tau) - tau;
    /* primitive gradients for the bound: d_j U_i and d_j T */
    double sU = 0.0, divU = 0.0, sT = 0.0;
    for (int j = 0; j < 3; ++j) {
        double dU[3], dT;
        for (int i = 0; i < 3; ++i) dU[i] = (gW[3 * (1 + i) + j] - U[i] * gW[j]) / rho;
        dT = (gW[12 + j] - W[4] / rho * gW[j]) / rho - (U[0] * dU[0] + U[1] * dU[1] + U[2] * dU[2]);
        dT = 2.0 / (3.0 + Kdof) * dT;
        for (int i = 0; i < 3; ++i) sU += fabs(dU[i]);
        divU += dU[j];
        sT += fabs(dT);
    }
    const double R = 4.0, K = (double)Kdof;
    gp->B = 1.0 + fabs(gp->alpha) * (R * R * (sU + fabs(divU)) + 0.5 * ((3.0 + K) * R * R + 5.0 + K) * R * sqrt(T) * sT / T);
}

/* 1 + alpha (sum_d u_d (a_d . psi) + A . psi) at velocity u and internal energy e */
static double gp_weight(const gp_t *gp, const double u[3], double e)
{
    const double psi[5] = {1.0, u[0], u[1], u[2], 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2] + e)};
    double s = 0.0;
    for (int k = 0; k < 5; ++k) s += gp->A[k] * psi[k];
    for (int d = 0; d < 3; ++d) {
        double ad = 0.0;
        for (int k = 0; k < 5; ++k) ad += gp->a[d][k] * psi[k];
        s += u[d] * ad;
    }
    return 1.0 + gp->alpha * s;
}

/* The first-order g_p of one cell, for the tests: alpha, B, and 1 + alpha (...) at n points
 * (u[n][3], e[n]). */
void orc_gp_eval(const double W[5], const double gW[15], double tau, double dt, int K, int64_t n, const double *u,
                 const double *e, double *alpha, double *B, double *w)
{
    gp_t gp;
    gp_setup(W, gW, tau, dt, K, &gp);
    *alpha = gp.alpha;
    *B = gp.B;
    for (int64_t i = 0; i < n; ++i) w[i] = gp_weight(&gp, u + 3 * i, e[i]);
}

/* Shakhov weight of a hydro particle (Pr != 1): with X = (u - U)/sqrt(T) the equilibrium g^+
 * of the Shakhov model (see flux_pair) is g [1 + (a.X)(|X|^2 - 5)], a = (1 - Pr) q / (5 rho
 * T^(3/2)), q the cell's heat flux, rho and T the cell's.  Reading: the hydro part is drawn from
 * it with the cell's U and T, like the Maxwellian it replaces (sampling 3), or with the
 * correction added to that of g_p (sampling 2).  B bounds |(a.X)(|X|^2 - 5)| on |X| <= 4, where
 * the largest value is 4 (16 - 5) |a|; beyond, the law is clipped (P(|X| > 4) = 1.1e-3). */
typedef struct { double a[3], B; } sh_t;

static void shakhov_setup(const double W[5], double T, const double q[3], double pr, sh_t *s)
{
    const double f = (1.0 - pr) / (5.0 * W[0] * T * sqrt(T));
    for (int d = 0; d < 3; ++d) s->a[d] = f * q[d];
    s->B = 44.0 * sqrt(s->a[0] * s->a[0] + s->a[1] * s->a[1] + s->a[2] * s->a[2]);
}

static double shakhov_term(const sh_t *s, const double X[3])
{
    return (s->a[0] * X[0] + s->a[1] * X[1] + s->a[2] * X[2]) * ((X[0] * X[0] + X[1] * X[1] + X[2] * X[2]) - 5.0);
}

/* proposal p of a cell for the hydro particles drawn one by one (sampling 2: gp, else NULL;
 * the Shakhov model: sh, else NULL): u = U + sqrt(T) X and e from the draws of uid_p (see
 * gp_setup's comment); returns its weight w = (1 + alpha (...) of g_p, or 1) + (a.X)(|X|^2 - 5)
 * and the acceptance uniform eta */
static double hydro_proposal(const oracle_t *o, const gp_t *gp, const sh_t *sh, uint64_t uidp, const double U[3],
                             double T, double u[3], double *e, double *eta)
{
    double ev[4], ea[4];
    draw4(o->seed, uidp, o->step, TAG_GP, 0u, o->inst, ev);
    double r1 = sqrt(-2.0 * log(ev[0])), r2 = sqrt(-2.0 * log(ev[2]));
    double X[3] = {r1 * cos(2.0 * M_PI * ev[1]), r1 * sin(2.0 * M_PI * ev[1]), r2 * cos(2.0 * M_PI * ev[3])};
    for (int d = 0; d < 3; ++d) u[d] = U[d] + sqrt(T) * X[d];
    *e = o->K > 0 ? internal_energy(o->seed, uidp, o->step, TAG_INT, 0u, o->inst, o->K, T) : 0.0;
    draw4(o->seed, uidp, o->step, TAG_GP, 1u, o->inst, ea);
    *eta = ea[0];
    double w = gp ? gp_weight(gp, u, *e) : 1.0;
    if (sh) w = w + shakhov_term(sh, X);
    return w;
}

/* The ns hydro particles of cell c drawn one by one (sampling 2 and 3), stored from index i0:
 * the proposals p = 0, 1, 2, ... of the cell are tried in order, B = (B of g_p, or 1) + (B of
 * sh, or 0), and the k-th accepted one becomes particle k (id uid_k, its own uniform position),
 * until ns are accepted or P = min(64 ns, 2^20) proposals are spent; a particle k still
 * missing then takes proposal k whether accepted or not.  (One stream per cell rather than
 * per particle: a wave of 64 lanes then tries 64 proposals at once and keeps every lane busy.)
 * S (if given) receives the sums of phi. */
static void sample_one_by_one(oracle_t *o, int64_t c, int64_t ns, int64_t i0, double msam, const gp_t *gp,
                              const sh_t *sh, const double U[3], double T, double *S)
{
    const double B = (gp ? gp->B : 1.0) + (sh ? sh->B : 0.0);
    const int64_t pmax = 64 * ns < ((int64_t)1 << 20) ? 64 * ns : ((int64_t)1 << 20);
    int64_t k = 0;
    for (int64_t p = 0; p < pmax + ns && k < ns; ++p) {
        const int fill = p >= pmax; /* the proposals are spent: particle k takes proposal k */
        const int64_t pp = fill ? k : p;
        const int64_t i = i0 + k;
        double e = 0.0, eta = 0.0;
        const double w = hydro_proposal(o, gp, sh, orc_make_uid(0, o->step, c, pp), U, T, o->pu + 3 * i, &e, &eta);
        if (!fill && !(eta * B < w)) continue;
        const uint64_t uid = orc_make_uid(0, o->step, c, k);
        place_in_cell(o, c, uid, o->px + 3 * i);
        o->pm[i] = msam;
        o->pc[i] = c;
        o->pid[i] = uid;
        o->pe[i] = e;
        if (S) add_phi(S + 5 * c, msam, o->pu + 3 * i, e);
        ++k;
    }
}

/* the Shakhov weight of one cell, for the tests: a, B, and (a.X)(|X|^2 - 5) at n points X[n][3] */
void orc_shakhov_eval(const double W[5], double T, const double q[3], double pr, int64_t n, const double *X,
                      double *a, double *B, double *w)
{
    sh_t s;
    shakhov_setup(W, T, q, pr, &s);
    for (int d = 0; d < 3; ++d) a[d] = s.a[d];
    *B = s.B;
    for (int64_t i = 0; i < n; ++i) w[i] = shakhov_term(&s, X + 3 * i);
}

/* Hydro particles sampled at the start of the step (Sec. 2.4(b)), appended after the old
 * ones.  With K > 0 each particle also gets its internal energy variable e = T |X'|^2 from
 * K standard normals of its own (Sec. 2.3: sampled from the temperature and K).
 * Per cell: rho^hp = exp(-dt/tau) rho^h, m_ref = (rho^p + rho^hp) Omega / N_ref,
 * N_sam = 2 ceil(rho^hp Omega / (2 m_ref)) raised to cover N_min - N_left (rounded up to
 * even), m_sam = rho^hp Omega / N_sam.  Pair j: X_j ~ N(0, I) by Box-Muller; the partners
 * get the velocities U + sqrt(T) X_j and U - sqrt(T) X_j (the pair of Sec. 2.4(b): the sample
 * carries exactly the mass rho^hp Omega and the momentum rho^hp Omega U of the Maxwellian, its
 * thermal energy is random); each partner its own uniform position in the cell.
 * sampling = 1 (a departure from the paper): every deviation is multiplied by one factor per
 * cell, s = sqrt(3 N_sam/2 / sum_j |X_j|^2), so that the sample also carries exactly the
 * energy rho^hp Omega (|U|^2/2 + 3T/2).
 * S (if given) receives the sums of phi over the new particles. */
static int phase_sample(oracle_t *o, const cellq_t *q, double *S, int64_t *nsampled)
{
    /* the counts first, so that every cell knows where its particles go; the cells are then
       sampled independently (in parallel in the OpenMP build) */
    const int64_t nc = o->nc, np0 = o->np;
    int64_t *first = (int64_t *)xcalloc(nc + 1, sizeof(int64_t));
    first[0] = np0;
    for (int64_t c = 0; c < nc; ++c) {
        double rhohp = q->ec[c] * q->rhoh[c];
        double rhop = o->P[5 * c] / o->vol[c];
        int64_t ns = 0;
        if (rhohp > 0.0 && rhop + rhohp > 0.0) {
            double r = (0.5 * o->n_ref) * (rhohp / (rhop + rhohp));
            ns = 2 * (int64_t)ceil(r);
            int64_t need = (int64_t)o->n_min - o->nleft[c];
            if (need > 0) {
                int64_t ne = 2 * ((need + 1) / 2);
                if (ne > ns) ns = ne;
            }
            if (ns > (1 << 20)) { free(first); return ORC_E_CAPACITY; }
        }
        first[c + 1] = first[c] + ns;
    }
    if (reserve(o, first[nc])) { free(first); return ORC_E_CAPACITY; }
    o->np = first[nc];
    *nsampled = first[nc] - np0;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t c = 0; c < nc; ++c) {
        const int64_t ns = first[c + 1] - first[c];
        if (ns == 0) continue;
        double rhohp = q->ec[c] * q->rhoh[c];
        double msam = rhohp * o->vol[c] / ns;
        double sT = sqrt(q->T[c]);
        if (o->sampling >= 2) {
            gp_t gp;
            sh_t sh;
            if (o->sampling == 2) gp_setup(o->W + 5 * c, q->gW + 15 * c, q->tau[c], q->dt, o->K, &gp);
            if (o->pr != 1.0) shakhov_setup(o->W + 5 * c, q->T[c], q->qh + 3 * c, o->pr, &sh);
            sample_one_by_one(o, c, ns, first[c], msam, o->sampling == 2 ? &gp : NULL, o->pr != 1.0 ? &sh : NULL,
                              q->U + 3 * c, q->T[c], S);
            continue;
        }
        if (o->sampling == 1) {
            /* energy-exact pairs: the pairs already carry the momentum rho^hp U exactly; one
               factor on every thermal deviation of the cell, sqrt(3 N_pairs / sum_j |X_j|^2),
               makes their energy rho^hp (|U|^2/2 + 3T/2) exact as well */
            double sx2 = 0.0;
            for (int64_t j = 0; j < ns; j += 2) {
                uint64_t puid = orc_make_uid(0, o->step, c, j);
                double ev[4];
                draw4(o->seed, puid, o->step, TAG_VEL, 0, o->inst, ev);
                double r1 = sqrt(-2.0 * log(ev[0])), r2 = sqrt(-2.0 * log(ev[2]));
                double X[3] = {r1 * cos(2.0 * M_PI * ev[1]), r1 * sin(2.0 * M_PI * ev[1]), r2 * cos(2.0 * M_PI * ev[3])};
                sx2 += X[0] * X[0] + X[1] * X[1] + X[2] * X[2];
            }
            sT = sT * sqrt(3.0 * (double)(ns / 2) / sx2);
        }
        double fint = 1.0;
        if (o->sampling == 1 && o->K > 0) {
            /* energy-exact internal energies: one factor K N_sam / sum_k |X_k|^2 on every particle's
               e, so that the sample carries exactly rho^hp Omega K T / 2 of internal energy */
            double se = 0.0;
            for (int64_t k = 0; k < ns; ++k)
                se += internal_energy(o->seed, orc_make_uid(0, o->step, c, k), o->step, TAG_INT, 0, o->inst, o->K, 1.0);
            fint = (double)o->K * (double)ns / se;
        }
        for (int64_t k = 0; k < ns; ++k) {
            int64_t i = first[c] + k;
            uint64_t uid = orc_make_uid(0, o->step, c, k);
            uint64_t puid = orc_make_uid(0, o->step, c, k & ~(int64_t)1);
            double ev[4];
            draw4(o->seed, puid, o->step, TAG_VEL, 0, o->inst, ev);
            double r1 = sqrt(-2.0 * log(ev[0])), r2 = sqrt(-2.0 * log(ev[2]));
            double X[3] = {r1 * cos(2.0 * M_PI * ev[1]), r1 * sin(2.0 * M_PI * ev[1]), r2 * cos(2.0 * M_PI * ev[3])};
            double sg = (k & 1) ? -1.0 : 1.0;
            for (int d = 0; d < 3; ++d) o->pu[3 * i + d] = q->U[3 * c + d] + sg * (sT * X[d]);
            place_in_cell(o, c, uid, o->px + 3 * i);
            o->pm[i] = msam;
            o->pc[i] = c;
            o->pid[i] = uid;
            double e = 0.0;
            if (o->K > 0) {
                e = internal_energy(o->seed, uid, o->step, TAG_INT, 0, o->inst, o->K, q->T[c]);
                if (o->sampling == 1) e = e * fint;
            }
            o->pe[i] = e;
            if (S) add_phi(S + 5 * c, msam, o->pu + 3 * i, e);
        }
    }
    free(first);
    return ORC_OK;
}

/* Normal speed of a particle entering from a Maxwellian reservoir: z = v_n / sigma has the
 * flux-weighted density z phi(z - a) / Z(a) on z > 0 (a = drift / sigma, phi the standard
 * normal density, Z(a) = phi(a) + a Phi(a)); its distribution function is
 *   G(z) = (phi(a) - phi(z - a) + a (Phi(z - a) - Phi(-a))) / Z(a).
 * G(z) = eta is solved by 60 bisections of [0, max(a, 0) + 40]. */
static double npdf(double t) { return exp(-0.5 * t * t) / sqrt(2.0 * M_PI); }
static double ncdf(double t) { return 0.5 * erfc(-t / sqrt(2.0)); }
double orc_flux_speed(double a, double eta)
{
    double Z = npdf(a) + a * ncdf(a);
    double lo = 0.0, hi = (a > 0.0 ? a : 0.0) + 40.0;
    for (int it = 0; it < 60; ++it) {
        double z = 0.5 * (lo + hi);
        double G = (npdf(a) - npdf(z - a) + a * (ncdf(z - a) - ncdf(-a))) / Z;
        if (G < eta) lo = z; else hi = z;
    }
    return 0.5 * (lo + hi);
}

/* Free-stream particles entering through far-field faces (a reading of the far-field
 * boundary for the particle part): the outside is a reservoir of the free stream W_inf, whose
 * collisionless hydro part exp(-dt/tau_inf) rho_inf crosses each face with the one-sided
 * number flux Gamma = s Phi(s/sigma) + sigma phi(s/sigma) (s = U_inf . n_in, sigma =
 * sqrt(T_inf)).  Face of area A on cell Omega: mass M = exp(-dt/tau_inf) rho_inf Gamma A dt,
 * N = ceil(Gamma A dt N_ref / Omega) particles of mass M / N (the reference mass of the cell
 * in the free stream); none when that ratio is below 1e-9.  Particle k: normal speed from the
 * flux-weighted half-Maxwellian, tangential components N(U_inf.t, T_inf) in the face frame,
 * entry uniform in time over the step and uniform on the face; it then flies for the rest of
 * the step with the face as entry face.  Appended after the sampled particles; tin[] and ein[]
 * receive their flight time and entry face. */
static int phase_inject(oracle_t *o, double dt, double **tin, int **ein, int64_t *ninj)
{
    *ninj = 0;
    if (o->step < o->gks_steps) return ORC_OK; /* wave-only phase: the free stream enters as waves */
    int64_t cap = 0;
    for (int64_t c = 0; c < o->nc; ++c) {
        for (int lf = 0; lf < o->cnf[c]; ++lf) {
            int64_t nb = o->cnb[6 * c + lf];
            if (nb >= 0 || o->bc[-1 - nb].type != BC_FARFIELD) continue;
            const obc_t *b = o->bc + (-1 - nb);
            const double *Wi = b->Winf;
            double rho = Wi[0];
            double Ui[3] = {Wi[1] / rho, Wi[2] / rho, Wi[3] / rho};
            double T = temp_k(Wi, o->K);
            double tau = o->mu_ref * pow(T, o->omega) / (rho * T);
            double e = exp(-dt / tau);
            int64_t bf = o->cbf[6 * c + lf];
            const double *n = o->pn + 18 * c + 3 * lf; /* out of the domain */
            double nin[3] = {-n[0], -n[1], -n[2]};
            double t1[3], t2[3];
            face_frame(nin, t1, t2);
            double sig = sqrt(T);
            double sd = Ui[0] * nin[0] + Ui[1] * nin[1] + Ui[2] * nin[2];
            double a = sd / sig;
            double Gam = sig * (npdf(a) + a * ncdf(a));
            double area = o->barea[bf];
            double r = Gam * area * dt * o->n_ref / o->vol[c];
            if (!(e * rho > 0.0) || !(r >= 1e-9)) continue;
            int64_t N = (int64_t)ceil(r);
            if (N > (1 << 20)) return ORC_E_CAPACITY;
            double msam = (e * rho * Gam * area * dt) / N;
            double vt1 = Ui[0] * t1[0] + Ui[1] * t1[1] + Ui[2] * t1[2];
            double vt2 = Ui[0] * t2[0] + Ui[1] * t2[1] + Ui[2] * t2[2];
            const double *fo = o->bo + 3 * bf, *f1 = o->be1 + 3 * bf, *f2 = o->be2 + 3 * bf;
            for (int64_t k = 0; k < N; ++k) {
                uint64_t uid = orc_make_uid(1, o->step, bf, k);
                double ev[4], ep[4];
                draw4(o->seed, uid, o->step, TAG_INJECT, 0, o->inst, ev);
                draw4(o->seed, uid, o->step, TAG_POS, 0, o->inst, ep);
                double vn = sig * orc_flux_speed(a, ev[0]);
                double rr = sqrt(-2.0 * log(ev[1]));
                double X1 = rr * cos(2.0 * M_PI * ev[2]), X2 = rr * sin(2.0 * M_PI * ev[2]);
                double w1 = vt1 + sig * X1, w2 = vt2 + sig * X2;
                double u[3], xs[3];
                for (int d = 0; d < 3; ++d) u[d] = vn * nin[d] + w1 * t1[d] + w2 * t2[d];
                double p1 = ep[0], p2 = ep[1];
                if (o->btri[bf] && p1 + p2 > 1.0) { p1 = 1.0 - p1; p2 = 1.0 - p2; }
                for (int d = 0; d < 3; ++d) xs[d] = fo[d] + p1 * f1[d] + p2 * f2[d];
                if (reserve(o, o->np + 1)) return ORC_E_CAPACITY;
                if (*ninj + 1 > cap) {
                    cap = cap ? 2 * cap : 1024;
                    double *tn = (double *)realloc(*tin, sizeof(double) * cap);
                    if (tn) *tin = tn;
                    int *en = (int *)realloc(*ein, sizeof(int) * cap);
                    if (en) *ein = en;
                    if (!tn || !en) return ORC_E_CAPACITY;
                }
                int64_t i = o->np++;
                for (int d = 0; d < 3; ++d) { o->px[3 * i + d] = xs[d]; o->pu[3 * i + d] = u[d]; }
                o->pm[i] = msam;
                o->pe[i] = o->K > 0 ? internal_energy(o->seed, uid, o->step, TAG_INT, 0, o->inst, o->K, T) : 0.0;
                o->pc[i] = c;
                o->pid[i] = uid;
                (*tin)[*ninj] = ev[3] * dt;
                (*ein)[*ninj] = lf;
                ++*ninj;
            }
        }
    }
    return ORC_OK;
}

/* Test hook: the limited gradients of W and of the hydro state for the current state
 * ([nc][5][3] each) and the hydro state ([nc][5]); nothing advances. */
int orc_gradients(oracle_t *o, double *gW, double *gH, double *Wh)
{
    cellq_t q;
    memset(&q, 0, sizeof(q));
    int st = phase_cells(o, &q);
    if (st == ORC_OK) {
        phase_grad(o, &q);
        memcpy(gW, q.gW, sizeof(double) * 15 * o->nc);
        memcpy(gH, q.gH, sizeof(double) * 15 * o->nc);
        memcpy(Wh, q.Wh, sizeof(double) * 5 * o->nc);
    }
    cellq_free(&q);
    return st;
}

/* Test hook: the cell phase and the sampling of the current step only (the new particles are
 * appended at their sampled positions; nothing streams and the step does not advance). */
int orc_sample_only(oracle_t *o, double *dt)
{
    cellq_t q = {0};
    int st = phase_cells(o, &q);
    int64_t ns = 0;
    if (st == ORC_OK && o->recon) phase_grad(o, &q);
    if (st == ORC_OK && o->pr != 1.0) {
        q.qh = (double *)xcalloc(3 * o->nc, sizeof(double));
        cell_heat_flux(o, q.qh);
    }
    if (st == ORC_OK) st = phase_sample(o, &q, NULL, &ns);
    *dt = q.dt;
    o->st_sampled = ns;
    cellq_free(&q);
    return st;
}

/* Time averaging for steady states (Sec. 2.4(c)): the average over the steps n > N_avg,
   each weighted by the step dt^n that produced W^n,
       Wbar^n = sum_{m > N_avg} dt^m W^m / sum_{m > N_avg} dt^m,
   kept as the running sums A = sum dt^m W^m and D = sum dt^m.  Its relative change from
   Wbar^{n-1} (the paper leaves the norm open) in the volume-weighted L1 norm of the whole
   field, sum_c Omega_c sum_k |Wbar^n_ck - Wbar^{n-1}_ck| / sum_c Omega_c sum_k |Wbar^n_ck|
   (+infinity until two steps are averaged). */
static void phase_average(oracle_t *o, double dt)
{
    double diff = 0.0, mag = 0.0;
    const double d0 = o->avg_D, d1 = d0 + dt;
    const int prev = o->avg_n > 0;
    for (int64_t c = 0; c < o->nc; ++c) {
        double dc = 0.0, mc = 0.0;
        for (int k = 0; k < 5; ++k) {
            const double a0 = o->avgA[5 * c + k];
            const double a1 = a0 + dt * o->W[5 * c + k];
            o->avgA[5 * c + k] = a1;
            const double wb1 = a1 / d1;
            mc = mc + fabs(wb1);
            if (prev) dc = dc + fabs(wb1 - a0 / d0);
        }
        mag = mag + o->vol[c] * mc;
        diff = diff + o->vol[c] * dc;
    }
    o->avg_res = prev ? diff / mag : INFINITY;
    o->avg_D = d1;
    o->avg_n += 1;
}

int orc_step(oracle_t *o)
{
    const int64_t nc = o->nc, nf = o->nf;
    cellq_t q = {0};
    double *Phi = (double *)xcalloc(5 * nf, sizeof(double));
    double *S = (double *)xcalloc(5 * nc, sizeof(double));
    double *E = (double *)xcalloc(5 * nc, sizeof(double));
    double *Pn = (double *)xcalloc(5 * nc, sizeof(double));
    int64_t *nl = (int64_t *)xcalloc(nc, sizeof(int64_t));
    double *tin = NULL;
    int *ein = NULL;
    int status = ORC_OK;
    /* the Shakhov model is built for a monatomic gas and drawn particle by particle */
    if (o->pr != 1.0 && (o->K != 0 || o->sampling < 2)) status = ORC_E_ARG;
    if (status == ORC_OK) status = phase_cells(o, &q);
    if (status != ORC_OK) goto done;
    const double dt = q.dt;
    o->st_dt = dt;
    const double pr = o->pr;
    if (pr != 1.0) {
        q.qh = (double *)xcalloc(3 * nc, sizeof(double));
        cell_heat_flux(o, q.qh);
    }

    if (o->recon) phase_grad(o, &q);
    const int gks = o->step < o->gks_steps;

    /* wave flux over every face, oriented owner -> neighbour, times the face area */
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t f = 0; f < nf; ++f) {
        int64_t c = o->fown[f], nb = o->fnb[f];
        const double *n = o->fn + 3 * f;
        double F[5];
        /* Shakhov model: the heat flux at the face is the mean of the two cells' (a far-field
           face: the free stream's is zero); walls keep the BGK flux (reading) */
        double qsh = 0.0;
        if (pr != 1.0 && (nb >= 0 || o->bc[-1 - nb].type == BC_FARFIELD)) {
            const double *qa = q.qh + 3 * c, zero[3] = {0.0, 0.0, 0.0};
            const double *qb = nb >= 0 ? q.qh + 3 * nb : zero;
            const double qn = (0.5 * (qa[0] + qb[0])) * n[0] + (0.5 * (qa[1] + qb[1])) * n[1] +
                              (0.5 * (qa[2] + qb[2])) * n[2];
            qsh = (1.0 - pr) * qn;
        }
        if (o->recon) {
            /* second order: states extrapolated to the face centre from both sides */
            const double *xf = o->fx + 3 * f;
            double Wl[5], Whl[5];
            extrap(o->W + 5 * c, q.gW + 15 * c, o->xc + 3 * c, xf, Wl);
            extrap(q.Wh + 5 * c, q.gH + 15 * c, o->xc + 3 * c, xf, Whl);
            if (nb >= 0) {
                double Wr[5], Whr[5];
                extrap(o->W + 5 * nb, q.gW + 15 * nb, o->xc + 3 * nb, xf, Wr);
                extrap(q.Wh + 5 * nb, q.gH + 15 * nb, o->xc + 3 * nb, xf, Whr);
                orc_flux2_interior(Wl, Wr, Whl, Whr, q.gW + 15 * c, q.gW + 15 * nb, q.gH + 15 * c, q.gH + 15 * nb, n,
                                   dt, o->mu_ref, o->omega, o->c2, gks, o->K, qsh, F);
            } else {
                const obc_t *b = o->bc + (-1 - nb);
                if (b->type == BC_SPECULAR)
                    orc_flux2_specular(Wl, Whl, q.gW + 15 * c, q.gH + 15 * c, n, dt, o->mu_ref, o->omega, o->c2, gks,
                                       o->K, F);
                else if (b->type == BC_DIFFUSE)
                    orc_flux_diffuse(Wl, Whl[0] > RHOH_EPS * Wl[0] ? Whl[0] : 0.0, q.tau[c], n, dt, b->Tw, b->Uw,
                                     gks, o->K, F);
                else
                    orc_flux2_farfield(Wl, Whl, q.gW + 15 * c, q.gH + 15 * c, b->Winf, n, dt, o->mu_ref, o->omega,
                                       o->c2, gks, o->K, qsh, F);
            }
        } else if (nb >= 0) {
            orc_flux_interior(o->W + 5 * c, o->W + 5 * nb, q.rhoh[c], q.rhoh[nb], n, dt, o->mu_ref, o->omega,
                              o->c2, gks, o->K, qsh, F);
        } else {
            const obc_t *b = o->bc + (-1 - nb);
            if (b->type == BC_SPECULAR)
                orc_flux_specular(o->W + 5 * c, q.rhoh[c], n, dt, o->mu_ref, o->omega, o->c2, gks, o->K, F);
            else if (b->type == BC_DIFFUSE)
                orc_flux_diffuse(o->W + 5 * c, q.rhoh[c], q.tau[c], n, dt, b->Tw, b->Uw, gks, o->K, F);
            else
                orc_flux_interior(o->W + 5 * c, b->Winf, q.rhoh[c], b->Winf[0], n, dt, o->mu_ref, o->omega,
                                  o->c2, gks, o->K, qsh, F);
        }
        for (int k = 0; k < 5; ++k) Phi[5 * f + k] = F[k] * o->farea[f];
    }

    /* particle sums at the start of the step: the particles left from the last step plus the
       hydro particles sampled now */
    for (int64_t c = 0; c < nc; ++c)
        for (int k = 0; k < 5; ++k) S[5 * c + k] = o->P[5 * c + k];
    int64_t nold = o->np;
    int64_t nsampled = 0;
    status = phase_sample(o, &q, S, &nsampled);
    if (status != ORC_OK) goto done;
    o->st_sampled = nsampled;
    int64_t ninj_start = o->np, ninj = 0;
    status = phase_inject(o, dt, &tin, &ein, &ninj);
    if (status != ORC_OK) goto done;
    o->st_injected = ninj;

    /* free-flight time of every old particle t_f = min(-tau ln eta, dt), with tau of the cell it
       starts in; new particles fly for dt.  Stream, sum, and delete the collided and escaped. */
    /* each particle's flight is independent of the others: tracked first (in parallel in the
       OpenMP build), then summed and compacted in particle order */
    const int64_t np = o->np;
    int8_t *prc = (int8_t *)xcalloc(np > 0 ? np : 1, sizeof(int8_t));
    int8_t *pcol = (int8_t *)xcalloc(np > 0 ? np : 1, sizeof(int8_t));
    int64_t *pcross = (int64_t *)xcalloc(np > 0 ? np : 1, sizeof(int64_t));
    int64_t *pwall = (int64_t *)xcalloc(np > 0 ? np : 1, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < np; ++i) {
        double ts = dt;
        int entry0 = -1;
        if (i >= ninj_start) {
            ts = tin[i - ninj_start];
            entry0 = ein[i - ninj_start];
        }
        if (i < nold) {
            double eta[4];
            draw4(o->seed, o->pid[i], o->step, TAG_TF, 0, o->inst, eta);
            double tf = -q.tau[o->pc[i]] * log(eta[0]);
            if (tf < dt) { ts = tf; pcol[i] = 1; }
        }
        prc[i] = (int8_t)orc_track(o, o->px + 3 * i, o->pu + 3 * i, o->pe + i, o->pc + i, ts, entry0, o->pid[i],
                                   o->step, pcross + i, pwall + i);
    }
    int64_t ncoll = 0, nesc = 0, ncross_tot = 0, nwall = 0, keep = 0, maxcross = 0;
    for (int64_t i = 0; i < np; ++i) {
        ncross_tot += pcross[i];
        if (pcross[i] > maxcross) maxcross = pcross[i];
        nwall += pwall[i];
        if (prc[i] < 0) status = ORC_E_LOST;
    }
    for (int64_t i = 0; i < np && status == ORC_OK; ++i) {
        if (prc[i] == 1) { ++nesc; continue; }
        int64_t c = o->pc[i];
        add_phi(E + 5 * c, o->pm[i], o->pu + 3 * i, o->pe[i]);
        if (pcol[i]) { ++ncoll; continue; }
        add_phi(Pn + 5 * c, o->pm[i], o->pu + 3 * i, o->pe[i]);
        nl[c] += 1;
        if (keep != i) {
            for (int d = 0; d < 3; ++d) { o->px[3 * keep + d] = o->px[3 * i + d]; o->pu[3 * keep + d] = o->pu[3 * i + d]; }
            o->pm[keep] = o->pm[i];
            o->pe[keep] = o->pe[i];
            o->pc[keep] = o->pc[i];
            o->pid[keep] = o->pid[i];
        }
        ++keep;
    }
    free(prc); free(pcol); free(pcross); free(pwall);
    if (status != ORC_OK) goto done;
    o->np = keep;

    /* conservative update: W^{n+1} = W^n + (-sum_f s_f Phi_f + E - S) / Omega, where E sums phi
       over every particle that ends the step in the cell (collided ones where they collided)
       and S over every particle that started it there (the net particle flux) */
    for (int64_t c = 0; c < nc; ++c) {
        double acc[5] = {0, 0, 0, 0, 0};
        for (int lf = 0; lf < o->cnf[c]; ++lf) {
            int64_t f = o->cface[6 * c + lf];
            double s = (double)o->csign[6 * c + lf];
            for (int k = 0; k < 5; ++k) acc[k] = acc[k] - s * Phi[5 * f + k];
        }
        for (int k = 0; k < 5; ++k) {
            o->tflux[5 * c + k] = acc[k];
            o->tE[5 * c + k] = E[5 * c + k];
            o->tS[5 * c + k] = S[5 * c + k];
            acc[k] = acc[k] + (E[5 * c + k] - S[5 * c + k]);
            o->W[5 * c + k] = o->W[5 * c + k] + acc[k] / o->vol[c];
            o->P[5 * c + k] = Pn[5 * c + k];
        }
        o->nleft[c] = nl[c];
    }
    o->st_collided = ncoll;
    o->st_escaped = nesc;
    o->st_alive = keep;
    o->st_cross = ncross_tot;
    o->st_maxcross = maxcross;
    o->st_wallhits = nwall;
    o->step += 1;
    o->t += dt;
    if (o->avg_from >= 0 && o->step > o->avg_from) phase_average(o, dt);
done:
    cellq_free(&q);
    free(Phi); free(S); free(E); free(Pn); free(nl); free(tin); free(ein);
    return status;
}
