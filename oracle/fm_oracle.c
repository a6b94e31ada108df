/*
 * fm_oracle.c -- plain, slow, double-precision CPU oracle for the one-loop flow of the
 * N-patch coupling function V(k1,k2,k3) of the two-dimensional Hubbard model, following
 * D. Rohe and C. Honerkamp, "Quasi-particle functional Renormalisation Group calculations
 * in the two-dimensional half-filled Hubbard model at finite temperatures"
 * (arXiv:2005.00827).
 *
 * TEST INFRASTRUCTURE. This file is the checker for the HIP library, not part of it. Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg load it. It shares
 * no source, header, table, constant or generator with the HIP library; the two sides see
 * only the same seeded inputs.
 *
 * What it computes, in the order the method states it:
 *   - the dispersion of Sec. 2.1 (Eq. free_dispersion_xi) on a half-shifted L x L loop grid;
 *   - angular Fermi-surface patches (Sec. 3.2 text on angular resolutions; App. A, Step 2 on
 *     projecting onto the patch), or "identity" patching where every loop point is its own
 *     patch and all momenta are exact (a test mode);
 *   - the one-loop vertex flow (App. A, Eqs. vertex_flow_general, vertex_flow_simple,
 *     vertex_flow_feedback_Z) written out for a spin-rotation-invariant static vertex with
 *     the particle-particle, crossed and direct particle-hole terms, in a temperature flow
 *     with scale s = ln T, each internal line weighted by the Z of its patch;
 *   - fixed-step RK4 and Dormand-Prince 5(4) integration in ln T, with the stop rule
 *     "largest |V| above a threshold" (Sec. 3.2, definition of U*(T));
 *   - the paper's own interaction flow (Sec. 2.2; App. A, Steps 1 and 2): the same channel
 *     formula at fixed T with flow parameter g, internal lines G_g = g Z G0 and
 *     S_g = Z^2 G0, integrated from g = 0, giving the crossover coupling U* = g*^2 U where
 *     the stop rule fires.
 * The paper states the vertex flow only in shorthand and for the interaction flow; the
 * explicit channel formula and the temperature-flow weight used here are readings that
 * the tests pin against second-order perturbation theory, closed forms and a generic
 * spin-resolved flow.
 *
 * Conventions (shared only as definitions, not as code):
 *   loop point index j = jx + L*jy, k = -pi + 2 pi (j + 1/2) / L per axis;
 *   transfers live on the unshifted grid q = 2 pi m / L, stored as (mx, my) mod L;
 *   V is row-major V[(a*N + b)*N + c] with a, b the patches of the incoming k1, k2 and c
 *   the patch of the outgoing k3 (spin of k1); k4 = k1 + k2 - k3 is implicit.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------------------ */
/* Public structs (mirrored by ctypes in oracle.py).                                    */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    double t, tp, mu;   /* Eq. free_dispersion_xi: hopping t, next-nearest t', chem. potential */
    int N, L;           /* patch count, loop grid side */
    int identity;       /* 1: patch = loop point (N = L*L), exact momenta */
    unsigned channels;  /* bit 1: particle-particle, bit 2: crossed ph, bit 4: direct ph */
    int n_shells;       /* > 1 (odd): energy shells, N = n_shells x angular sectors */
    const double *shell_edges; /* [(n_shells-1)/2] ascending |xi| edges, or NULL (default) */
} orc_model;

typedef struct {
    double T0, T_end;   /* temperature flow: from T0 down to T_end; interaction flow: T0 is
                           the fixed temperature, T_end unused */
    int integrator;     /* 0: classical RK4, fixed steps in s; 1: Dormand-Prince 5(4) */
    int n_steps;        /* RK4 step count */
    double rtol, atol, h0, h_min;
    double v_max;       /* stop when max |V| exceeds this */
    int n_z;            /* 0: Z = 1 on every line */
    const double *z_lnT; /* [n_z] ascending nodes in the flow parameter (ln T, or g) */
    const double *z_tab; /* [n_z][N] */
    int gflow;          /* 0: temperature flow, s = ln T; 1: interaction flow, s = g */
    double g_end;       /* interaction flow: from g = 0 to g_end */
    double v_rel;       /* interaction flow: stop when max |V| exceeds v_rel |U| (0: 100) */
    int rhs_binned;     /* evaluate every right-hand side in the binned form (the same sums
                           in another order; measures how a flow amplifies rounding-order
                           differences) */
    int progress;       /* 1: one line per step attempt on stderr (long flows) */
    const double *k_tab; /* interaction flow only: [n_z][N] Katanin factors K on the same
                           nodes as z_tab (NULL: K = 1, no Katanin correction) */
} orc_flowcfg;

typedef struct {
    double T_c, T_final, max_abs_V;
    int status, n_accepted, n_rejected, n_rhs;
    double g_c, U_star, g_final;   /* interaction flow: crossing g*, U* = g*^2 U, last g */
} orc_result;

enum { ORC_RUNNING = 0, ORC_DIVERGED = 1, ORC_NONFINITE = 2, ORC_REACHED_TEND = 3,
       ORC_STEPFAIL = 4 };

/* ------------------------------------------------------------------------------------ */
/* Lattice, dispersion and patches.                                                    */
/* ------------------------------------------------------------------------------------ */

/* Eq. free_dispersion_xi: xi(k) = -2t(cos kx + cos ky) - 4t' cos kx cos ky - mu. */
static double disp(const orc_model *m, double kx, double ky)
{
    return -2.0 * m->t * (cos(kx) + cos(ky)) - 4.0 * m->tp * cos(kx) * cos(ky) - m->mu;
}

/* Half-shifted loop grid: no point on the zone boundary or at Gamma. */
static double grid_k(int j, int L) { return -M_PI + 2.0 * M_PI * (j + 0.5) / L; }

/* Sector centres theta_a = theta_off + 2 pi a / N.  With N % 8 == 0 the centres contain the
 * antinodal (theta = 0) and nodal (theta = pi/4) directions, as in the paper's count of
 * seven patches from antinode to node giving 48 in total (Sec. 3.2). */
static double theta_off(int N)
{
    if (N == 1 || N % 8 == 0) return 0.0;
    if (N % 8 == 4) return M_PI / N;
    return NAN;
}

static int patch_of(double kx, double ky, int N, double *margin)
{
    double x = (atan2(ky, kx) - theta_off(N)) * N / (2.0 * M_PI);
    double r = (double)lround(x);
    if (margin) *margin = 0.5 - fabs(x - r);
    long p = ((long)r) % N;
    if (p < 0) p += N;
    return (int)p;
}

/* Point on the ray at angle th where xi equals `level` (0: the Fermi surface): the first
 * sign change of xi - level between Gamma and the zone edge, found by a 4096-sample scan and
 * bisection; no sign change means the sample of smallest |xi - level| is used. */
static double disp_at(const orc_model *m, double kx, double ky, double level)
{
    return disp(m, kx, ky) - level;
}

static void fs_point(const orc_model *m, double th, double level, double *kx, double *ky)
{
    const int ns = 4096;
    double c = cos(th), s = sin(th);
    double rmax = M_PI / fmax(fabs(c), fabs(s));
    double f0 = disp_at(m, 0.0, 0.0, level);
    double r_best = 0.0, f_best = fabs(f0);
    if (f0 == 0.0) { *kx = 0.0; *ky = 0.0; return; }
    double r_prev = 0.0, f_prev = f0;
    for (int i = 1; i <= ns; ++i) {
        double r = rmax * i / ns;
        double f = disp_at(m, r * c, r * s, level);
        if ((f_prev < 0.0 && f >= 0.0) || (f_prev > 0.0 && f <= 0.0)) {
            double lo = r_prev, hi = r;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                double fm = disp_at(m, mid * c, mid * s, level);
                if ((f_prev < 0.0 && fm < 0.0) || (f_prev > 0.0 && fm > 0.0)) lo = mid;
                else hi = mid;
            }
            *kx = hi * c; *ky = hi * s;
            return;
        }
        if (fabs(f) < f_best) { f_best = fabs(f); r_best = r; }
        r_prev = r; f_prev = f;
    }
    *kx = r_best * c; *ky = r_best * s;
}

static int mod_l(long x, int L) { long r = x % L; return (int)(r < 0 ? r + L : r); }

typedef struct {
    int N, L, np, identity;
    double *xi;      /* [np] */
    int *patch;      /* [np] */
    int *anchor;     /* [N][2]: snapped k_F index (angular) or the loop index (identity) */
    int pp_shift;    /* k_a + k_b on the index grid: anchor sum + pp_shift */
    double margin;   /* smallest distance of a loop point to a sector boundary, in sectors */
} geom;

static void geom_free(geom *g)
{
    free(g->xi); free(g->patch); free(g->anchor);
    memset(g, 0, sizeof(*g));
}

/* Energy shells (Sec. 3.2: the angular patches subdivided in energy, 7 shells x 32 sectors =
 * 224 patches).  With S = n_shells (odd) and M = (S - 1)/2, the shells meet at the energies
 * +-E_1 < ... < +-E_M (given, or by default E_k = 2|t| (2^k - 1)/(2^M - 1), finest at the
 * Fermi surface).  A loop point of energy x lies in shell M - k below the Fermi surface and
 * M + k above it, k being the number of edges below |x|; patch = shell * (N/S) + sector.
 * A patch is represented by the point of its sector's centre ray at the shell's energy: 0 for
 * the Fermi-surface shell, the middle of an inner shell, and for the outermost shell its edge
 * plus half the width of the shell inside it. */
static double shell_edge(const orc_model *m, int k)
{
    int M = (m->n_shells - 1) / 2;
    if (m->shell_edges) return m->shell_edges[k - 1];
    return 2.0 * fabs(m->t) * (pow(2.0, k) - 1.0) / (pow(2.0, M) - 1.0);
}

static int n_shells_of(const orc_model *m) { return m->n_shells > 1 ? m->n_shells : 1; }

static int shell_of(const orc_model *m, double x)
{
    int M = (n_shells_of(m) - 1) / 2, k = 0;
    while (k < M && fabs(x) > shell_edge(m, k + 1)) ++k;
    return x < 0.0 ? M - k : M + k;
}

static double shell_energy(const orc_model *m, int e)
{
    int M = (n_shells_of(m) - 1) / 2, k = abs(e - M);
    if (k == 0) return 0.0;
    double lo = shell_edge(m, k);
    double mag = k < M ? 0.5 * (lo + shell_edge(m, k + 1))
                       : lo + 0.5 * (lo - (k > 1 ? shell_edge(m, k - 1) : 0.0));
    return e < M ? -mag : mag;
}

static int geom_build(const orc_model *m, geom *g)
{
    memset(g, 0, sizeof(*g));
    int L = m->L, N = m->N;
    int S = n_shells_of(m), Ns = N / (S > 0 ? S : 1);
    if (L < 2 || (L & 1)) return -1;
    if (m->identity) { if (N != L * L) return -1; }
    else if (S % 2 == 0 || N % S || Ns < 1 || isnan(theta_off(Ns)) || (L % 4)) return -1;
    for (int k = 1; k <= (S - 1) / 2; ++k)
        if (!(shell_edge(m, k) > (k > 1 ? shell_edge(m, k - 1) : 0.0))) return -1;
    g->N = N; g->L = L; g->np = L * L; g->identity = m->identity;
    g->xi = (double *)malloc(sizeof(double) * g->np);
    g->patch = (int *)malloc(sizeof(int) * g->np);
    g->anchor = (int *)malloc(sizeof(int) * 2 * N);
    g->margin = 0.5;
    for (int jy = 0; jy < L; ++jy)
        for (int jx = 0; jx < L; ++jx) {
            int j = jx + L * jy;
            double kx = grid_k(jx, L), ky = grid_k(jy, L);
            g->xi[j] = disp(m, kx, ky);
            if (m->identity) {
                g->patch[j] = j;
            } else {
                double mg;
                g->patch[j] = shell_of(m, g->xi[j]) * Ns + patch_of(kx, ky, Ns, &mg);
                if (mg < g->margin) g->margin = mg;
                for (int k = 1; k <= (S - 1) / 2; ++k)     /* no point on a shell edge */
                    if (fabs(fabs(g->xi[j]) - shell_edge(m, k)) < 1e-9) { geom_free(g); return -1; }
            }
        }
    if (m->identity) {
        for (int a = 0; a < N; ++a) { g->anchor[2 * a] = a % L; g->anchor[2 * a + 1] = a / L; }
        g->pp_shift = 1;
    } else {
        for (int a = 0; a < N; ++a) {
            double kx, ky;
            fs_point(m, theta_off(Ns) + 2.0 * M_PI * (a % Ns) / Ns, shell_energy(m, a / Ns),
                     &kx, &ky);
            g->anchor[2 * a] = mod_l(lround(kx * L / (2.0 * M_PI)), L);
            g->anchor[2 * a + 1] = mod_l(lround(ky * L / (2.0 * M_PI)), L);
        }
        g->pp_shift = 0;
    }
    return 0;
}

/* Transfers as flat indices mx + L*my. */
static int q_pp(const geom *g, int a, int b)
{
    int L = g->L;
    int mx = mod_l(g->anchor[2 * a] + g->anchor[2 * b] + g->pp_shift, L);
    int my = mod_l(g->anchor[2 * a + 1] + g->anchor[2 * b + 1] + g->pp_shift, L);
    return mx + L * my;
}
static int q_diff(const geom *g, int x, int y) /* k_x - k_y */
{
    int L = g->L;
    int mx = mod_l(g->anchor[2 * x] - g->anchor[2 * y], L);
    int my = mod_l(g->anchor[2 * x + 1] - g->anchor[2 * y + 1], L);
    return mx + L * my;
}
/* Partner of loop point j: pp: q - k_j;  ph: k_j + q. */
static int partner_pp(int L, int q, int j)
{
    return mod_l((q % L) - (j % L) - 1, L) + L * mod_l((q / L) - (j / L) - 1, L);
}
static int partner_ph(int L, int q, int j)
{
    return mod_l((q % L) + (j % L), L) + L * mod_l((q / L) + (j / L), L);
}

/* ------------------------------------------------------------------------------------ */
/* Bubble weights.                                                                      */
/*                                                                                      */
/* chi(x,y;T) = -(f(x) - f(y))/(x - y) with the Fermi function f, i.e. the static         */
/* particle-hole bubble of two bare lines (App. A, Step 1: bare lines (i w - xi)^-1); the   */
/* particle-particle bubble is chi(x,-y).  With a = x/2T, b = y/2T,                        */
/*   chi = (tanh a - tanh b) / (4T (a - b)),                                             */
/*   T d/dT chi = -phi[a,b] / (4T),  phi(u) = u sech^2 u,  phi[a,b] its divided difference.*/
/* The divided difference is evaluated through the exact identity                        */
/*   phi[a,b] = sech^2 a - b * sinh(a+b) sech a sech b * (tanh a - tanh b)/(a-b),          */
/* (from a sech^2 a - b sech^2 b = (a-b) sech^2 a + b (sech^2 a - sech^2 b) and            */
/*  sech^2 a - sech^2 b = -sinh(a+b) sinh(a-b) sech^2 a sech^2 b), with every sinh*sech*sech */
/* product formed from exponentials of non-positive arguments.                           */
/* ------------------------------------------------------------------------------------ */

/* sinh(s) sech(a) sech(b) for |s| <= |a| + |b|. */
static double sh_sech_sech(double s, double a, double b)
{
    double as = fabs(s), aa = fabs(a), ab = fabs(b);
    if (as == 0.0) return 0.0;
    double num = -2.0 * expm1(-2.0 * as) * exp(as - aa - ab);
    double den = (1.0 + exp(-2.0 * aa)) * (1.0 + exp(-2.0 * ab));
    return copysign(num / den, s);
}

static double sech2(double a)
{
    double e = exp(-2.0 * fabs(a));
    return 4.0 * e / ((1.0 + e) * (1.0 + e));
}

/* (tanh a - tanh b)/(a - b) = sinh(a-b)/(a-b) sech a sech b. */
static double tanh_dd(double a, double b)
{
    double d = a - b;
    if (d == 0.0) return sech2(a);
    return sh_sech_sech(d, a, b) / d;
}

/* phi[a,b] is symmetric; the identity is used with |a| >= |b|: its second term equals
 * b (sech^2 b - sech^2 a)/(a - b), which for |b| > |a| would nearly cancel sech^2 a. */
double orc_phi_dd(double a, double b)
{
    if (fabs(a) < fabs(b)) { double t = a; a = b; b = t; }
    return sech2(a) - b * sh_sech_sech(a + b, a, b) * tanh_dd(a, b);
}

double orc_chi_ph(double x, double y, double T) { return tanh_dd(x / (2 * T), y / (2 * T)) / (4 * T); }
double orc_chi_pp(double x, double y, double T) { return orc_chi_ph(x, -y, T); }
double orc_chidot_ph(double x, double y, double T) { return -orc_phi_dd(x / (2 * T), y / (2 * T)) / (4 * T); }
double orc_chidot_pp(double x, double y, double T) { return orc_chidot_ph(x, -y, T); }

/* ------------------------------------------------------------------------------------ */
/* Geometry query (for host-side tests).                                                */
/* ------------------------------------------------------------------------------------ */
int orc_geometry(const orc_model *m, double *xi_out, int *patch_out, int *anchor_out,
                 double *margin_out)
{
    geom g;
    if (geom_build(m, &g)) return -1;
    if (xi_out) memcpy(xi_out, g.xi, sizeof(double) * g.np);
    if (patch_out) memcpy(patch_out, g.patch, sizeof(int) * g.np);
    if (anchor_out) memcpy(anchor_out, g.anchor, sizeof(int) * 2 * g.N);
    if (margin_out) *margin_out = g.margin;
    geom_free(&g);
    return 0;
}

/* Distinct transfers: counts of {q_pp(a,b)} and {k_x - k_y}. */
int orc_transfer_counts(const orc_model *m, int *n_pp, int *n_ph)
{
    geom g;
    if (geom_build(m, &g)) return -1;
    char *s1 = (char *)calloc(g.np, 1), *s2 = (char *)calloc(g.np, 1);
    int c1 = 0, c2 = 0;
    for (int a = 0; a < g.N; ++a)
        for (int b = 0; b < g.N; ++b) {
            int q = q_pp(&g, a, b);
            if (!s1[q]) { s1[q] = 1; ++c1; }
            q = q_diff(&g, a, b);
            if (!s2[q]) { s2[q] = 1; ++c2; }
        }
    *n_pp = c1; *n_ph = c2;
    free(s1); free(s2); geom_free(&g);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Right-hand side, direct form.                                                        */
/*                                                                                      */
/* With W_X(j) = Z[pi(j)] Z[pi(j')] T d/dT chi_X(xi_j, xi_j') and sum_j = (1/L^2) sum over  */
/* the loop grid, the temperature-flow derivative dV/d ln T (a,b,c) is                   */
/*   - sum_j W_pp(j; q_pp)  V(a,b,pj) V(pj,pj',c)                j' = q_pp - j            */
/*   + sum_j W_ph(j; q_cr)  V(a,pj,pj') V(pj',b,c)               j' = j + q_cr            */
/*   + sum_j W_ph(j; q_d) [-2 V(a,pj,c) V(pj',b,pj)                                        */
/*                         + V(pj,a,c) V(pj',b,pj) + V(a,pj,c) V(b,pj',pj)]  j' = j + q_d  */
/* where pj = pi(j), q_pp = k1 + k2, q_cr = k3 - k2, q_d = k1 - k3.  This is the one-loop   */
/* diagram of Eq. vertex_flow_general with the particle-particle, crossed and direct        */
/* particle-hole terms written out for the spin-rotation-invariant coupling function       */
/* (App. A: separating spin and momentum dependence), Z inserted on internal lines as in   */
/* Eq. vertex_flow_feedback_Z with Z projected onto the patch of each line.               */
/* ------------------------------------------------------------------------------------ */

#define VIX(N, a, b, c) ((((size_t)(a)) * (N) + (b)) * (N) + (c))

/* Weight of the internal line pair (j, j') with Z_x = Z of the patch of line x:
 *   temperature flow, d/d ln T of the bubble with Z on both lines:
 *     W = Z_j Z_j' T d/dT chi_X(xi_j, xi_j');
 *   interaction flow (App. A, Step 2, Eqs. both_propagators_Z, vertex_flow_feedback_Z):
 *   the line pair S_g G_g + G_g S_g with G_g = g Z G0, S_g = Z^2 G0, i.e.
 *     W = g Z_j Z_j' (Z_j + Z_j') chi_X(xi_j, xi_j')   (2 g chi_X without Z, Step 1). */
/* K: interaction flow with the Katanin correction (App. A, Step 3): the single-scale line
 * S_g = Z^2 G0 becomes dG_g/dg = K Z^2 G0, so the line pair (j, j') carries
 * g Z_j Z_j' (K_j Z_j + K_j' Z_j') chi (Eq. vertex_flow_feedback_Z_with_Katanin); NULL: K = 1. */
typedef struct { int gflow; double T, g; const double *K; } wkind;

static void fill_weights(const geom *g, wkind wk, const double *Z, int pp, int q, double *w)
{
    int L = g->L;
    for (int j = 0; j < g->np; ++j) {
        int jp = pp ? partner_pp(L, q, j) : partner_ph(L, q, j);
        double za = Z ? Z[g->patch[j]] : 1.0, zb = Z ? Z[g->patch[jp]] : 1.0;
        if (wk.gflow) {
            double chi = pp ? orc_chi_pp(g->xi[j], g->xi[jp], wk.T)
                            : orc_chi_ph(g->xi[j], g->xi[jp], wk.T);
            double ka = wk.K ? wk.K[g->patch[j]] : 1.0, kb = wk.K ? wk.K[g->patch[jp]] : 1.0;
            w[j] = wk.g * za * zb * (ka * za + kb * zb) * chi;
        } else {
            double chid = pp ? orc_chidot_pp(g->xi[j], g->xi[jp], wk.T)
                             : orc_chidot_ph(g->xi[j], g->xi[jp], wk.T);
            w[j] = za * zb * chid;
        }
    }
}

static double rhs_one(const geom *g, unsigned ch, const double *V, int a, int b, int c,
                      const double *wpp, int qpp, const double *wcr, int qcr,
                      const double *wd, int qd)
{
    int N = g->N, L = g->L;
    double s = 0.0;
    if (ch & 1u)
        for (int j = 0; j < g->np; ++j) {
            int pj = g->patch[j], pq = g->patch[partner_pp(L, qpp, j)];
            s -= wpp[j] * V[VIX(N, a, b, pj)] * V[VIX(N, pj, pq, c)];
        }
    if (ch & 2u)
        for (int j = 0; j < g->np; ++j) {
            int pj = g->patch[j], pq = g->patch[partner_ph(L, qcr, j)];
            s += wcr[j] * V[VIX(N, a, pj, pq)] * V[VIX(N, pq, b, c)];
        }
    if (ch & 4u)
        for (int j = 0; j < g->np; ++j) {
            int pj = g->patch[j], pq = g->patch[partner_ph(L, qd, j)];
            s += wd[j] * (-2.0 * V[VIX(N, a, pj, c)] * V[VIX(N, pq, b, pj)]
                          + V[VIX(N, pj, a, c)] * V[VIX(N, pq, b, pj)]
                          + V[VIX(N, a, pj, c)] * V[VIX(N, b, pq, pj)]);
        }
    return s / (double)g->np;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Weight tables for every transfer that occurs, keyed by the flat transfer index. */
typedef struct { double **pp, **ph; } wcache;

static void wcache_build(const geom *g, unsigned ch, wkind wk, const double *Z, wcache *wc)
{
    int np = g->np, N = g->N;
    wc->pp = (double **)calloc(np, sizeof(double *));
    wc->ph = (double **)calloc(np, sizeof(double *));
    char *need_pp = (char *)calloc(np, 1), *need_ph = (char *)calloc(np, 1);
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            if (ch & 1u) need_pp[q_pp(g, a, b)] = 1;
            if (ch & 6u) need_ph[q_diff(g, a, b)] = 1;
        }
    int *list = (int *)malloc(sizeof(int) * 2 * np);
    int n = 0;
    for (int q = 0; q < np; ++q) {
        if (need_pp[q]) { wc->pp[q] = (double *)malloc(sizeof(double) * np); list[n++] = q; }
        if (need_ph[q]) { wc->ph[q] = (double *)malloc(sizeof(double) * np); list[n++] = -1 - q; }
    }
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < n; ++i) {
        int q = list[i] >= 0 ? list[i] : -1 - list[i];
        int pp = list[i] >= 0;
        fill_weights(g, wk, Z, pp, q, pp ? wc->pp[q] : wc->ph[q]);
    }
    free(list); free(need_pp); free(need_ph);
}

static void wcache_free(const geom *g, wcache *wc)
{
    for (int q = 0; q < g->np; ++q) { free(wc->pp[q]); free(wc->ph[q]); }
    free(wc->pp); free(wc->ph);
}

static void rhs_geom(const geom *g, unsigned ch, wkind wk, const double *Z, const double *V,
                     double *dV)
{
    int N = g->N;
    wcache wc;
    wcache_build(g, ch, wk, Z, &wc);
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b)
            for (int c = 0; c < N; ++c) {
                int qpp = q_pp(g, a, b), qcr = q_diff(g, c, b), qd = q_diff(g, a, c);
                dV[VIX(N, a, b, c)] = rhs_one(g, ch, V, a, b, c, wc.pp[qpp], qpp,
                                              wc.ph[qcr], qcr, wc.ph[qd], qd);
            }
    wcache_free(g, &wc);
}

int orc_rhs(const orc_model *m, double T, const double *Z, const double *V, double *dV,
            int nthreads)
{
    geom g;
    if (!(T > 0.0) || geom_build(m, &g)) return -1;
    set_threads(nthreads);
    wkind wk = {0, T, 0.0};
    rhs_geom(&g, m->channels, wk, Z, V, dV);
    geom_free(&g);
    return 0;
}

/* Interaction flow: dV/dg at temperature T and scale g. */
int orc_rhs_g(const orc_model *m, double T, double gval, const double *Z, const double *V,
              double *dV, int nthreads)
{
    geom g;
    if (!(T > 0.0) || geom_build(m, &g)) return -1;
    set_threads(nthreads);
    wkind wk = {1, T, gval, NULL};
    rhs_geom(&g, m->channels, wk, Z, V, dV);
    geom_free(&g);
    return 0;
}

/* The same with the Katanin factors K[N] on the single-scale line (K NULL: K = 1). */
int orc_rhs_gk(const orc_model *m, double T, double gval, const double *Z, const double *K,
               const double *V, double *dV, int nthreads)
{
    geom g;
    if (!(T > 0.0) || geom_build(m, &g)) return -1;
    set_threads(nthreads);
    wkind wk = {1, T, gval, K};
    rhs_geom(&g, m->channels, wk, Z, V, dV);
    geom_free(&g);
    return 0;
}

/* Sampled outputs: weights computed per output, nothing cached. */
static int rhs_points_wk(const orc_model *m, wkind wk, const double *Z, const double *V, int n,
                         const int *abc, double *out, int nthreads)
{
    geom g;
    if (!(wk.T > 0.0) || geom_build(m, &g)) return -1;
    set_threads(nthreads);
#pragma omp parallel
    {
        double *wpp = (double *)malloc(sizeof(double) * g.np);
        double *wcr = (double *)malloc(sizeof(double) * g.np);
        double *wd = (double *)malloc(sizeof(double) * g.np);
#pragma omp for schedule(dynamic)
        for (int i = 0; i < n; ++i) {
            int a = abc[3 * i], b = abc[3 * i + 1], c = abc[3 * i + 2];
            int qpp = q_pp(&g, a, b), qcr = q_diff(&g, c, b), qd = q_diff(&g, a, c);
            fill_weights(&g, wk, Z, 1, qpp, wpp);
            fill_weights(&g, wk, Z, 0, qcr, wcr);
            fill_weights(&g, wk, Z, 0, qd, wd);
            out[i] = rhs_one(&g, m->channels, V, a, b, c, wpp, qpp, wcr, qcr, wd, qd);
        }
        free(wpp); free(wcr); free(wd);
    }
    geom_free(&g);
    return 0;
}

int orc_rhs_points(const orc_model *m, double T, const double *Z, const double *V, int n,
                   const int *abc, double *out, int nthreads)
{
    wkind wk = {0, T, 0.0};
    return rhs_points_wk(m, wk, Z, V, n, abc, out, nthreads);
}

int orc_rhs_points_g(const orc_model *m, double T, double gval, const double *Z,
                     const double *V, int n, const int *abc, double *out, int nthreads)
{
    wkind wk = {1, T, gval};
    return rhs_points_wk(m, wk, Z, V, n, abc, out, nthreads);
}

/* ------------------------------------------------------------------------------------ */
/* Right-hand side, binned form: the same sums regrouped by the patch pair (a',b') of the  */
/* two internal lines, B_q(a',b') = sum over j with pi(j)=a', pi(j')=b' of T d/dT chi     */
/* (chi itself for the interaction flow, whose Z factor depends on the pair's patches     */
/* only).  Exists to check that regrouping against the direct form, and to measure how a   */
/* flow amplifies a change of summation order.                                            */
/* ------------------------------------------------------------------------------------ */
static void rhs_binned_geom(const geom *gp, unsigned ch, wkind wk, const double *Z,
                            const double *V, double *dV)
{
    const double T = wk.T;
    const geom g = *gp;
    int N = g.N, L = g.L, np = g.np;
    size_t NN = (size_t)N * N;
    double **bpp = (double **)calloc(np, sizeof(double *));
    double **bph = (double **)calloc(np, sizeof(double *));
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            int q = q_pp(&g, a, b);
            if (!bpp[q]) bpp[q] = (double *)calloc(NN, sizeof(double));
            q = q_diff(&g, a, b);
            if (!bph[q]) bph[q] = (double *)calloc(NN, sizeof(double));
        }
#pragma omp parallel for schedule(dynamic)
    for (int q = 0; q < np; ++q) {
        for (int j = 0; j < np; ++j) {
            if (bpp[q]) {
                int jp = partner_pp(L, q, j);
                bpp[q][(size_t)g.patch[j] * N + g.patch[jp]] +=
                    wk.gflow ? orc_chi_pp(g.xi[j], g.xi[jp], T) : orc_chidot_pp(g.xi[j], g.xi[jp], T);
            }
            if (bph[q]) {
                int jp = partner_ph(L, q, j);
                bph[q][(size_t)g.patch[j] * N + g.patch[jp]] +=
                    wk.gflow ? orc_chi_ph(g.xi[j], g.xi[jp], T) : orc_chidot_ph(g.xi[j], g.xi[jp], T);
            }
        }
    }
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b)
            for (int c = 0; c < N; ++c) {
                const double *Bp = bpp[q_pp(&g, a, b)];
                const double *Bc = bph[q_diff(&g, c, b)];
                const double *Bd = bph[q_diff(&g, a, c)];
                double s = 0.0;
                for (int x = 0; x < N; ++x)
                    for (int y = 0; y < N; ++y) {
                        double zx = Z ? Z[x] : 1.0, zy = Z ? Z[y] : 1.0;
                        double kx = wk.K ? wk.K[x] : 1.0, ky = wk.K ? wk.K[y] : 1.0;
                        double zz = wk.gflow ? wk.g * zx * zy * (kx * zx + ky * zy) : zx * zy;
                        size_t xy = (size_t)x * N + y;
                        if (ch & 1u) s -= zz * Bp[xy] * V[VIX(N, a, b, x)] * V[VIX(N, x, y, c)];
                        if (ch & 2u) s += zz * Bc[xy] * V[VIX(N, a, x, y)] * V[VIX(N, y, b, c)];
                        if (ch & 4u)
                            s += zz * Bd[xy] * (-2.0 * V[VIX(N, a, x, c)] * V[VIX(N, y, b, x)]
                                                + V[VIX(N, x, a, c)] * V[VIX(N, y, b, x)]
                                                + V[VIX(N, a, x, c)] * V[VIX(N, b, y, x)]);
                    }
                dV[VIX(N, a, b, c)] = s / (double)np;
            }
    for (int q = 0; q < np; ++q) { free(bpp[q]); free(bph[q]); }
    free(bpp); free(bph);
}

int orc_rhs_binned(const orc_model *m, double T, const double *Z, const double *V, double *dV,
                   int nthreads)
{
    geom g;
    if (!(T > 0.0) || geom_build(m, &g)) return -1;
    set_threads(nthreads);
    wkind wk = {0, T, 0.0};
    rhs_binned_geom(&g, m->channels, wk, Z, V, dV);
    geom_free(&g);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* The quasi-particle weight from the self-energy on the real axis (Sec. 3.1: Im Sigma as   */
/* raw data on a frequency grid, Re Sigma by Kramers-Kronig, Z from the slope of Re Sigma  */
/* taken outside the window of inverted slope; App. A, Eq. definition_Z).                  */
/*                                                                                      */
/* The self-energy is the two-loop (second-order) diagram of a static vertex: for an      */
/* external point k (the patch's representative point, not snapped) and loop points p1   */
/* (hole), p3 (particle), with p2 = k + p1 - p3 (particle) taken off the grid exactly,     */
/*   Im Sigma(w, k) = -pi (1/L^4) sum_{p1,p3} W F delta(w + xi1 - xi2 - xi3),              */
/*   F = f1 (1 - f2)(1 - f3) + (1 - f1) f2 f3,                                            */
/* and W the squared vertex summed over spins: U^2 for the bare coupling (second-order    */
/* perturbation theory), else with V at the patches a of k, b of p1, c of p3,             */
/*   W = V(a,b,c)^2 + (V(a,b,c) - V(b,a,c))^2 / 2                                         */
/* (the opposite-spin pair with both assignments of its outgoing lines, and the            */
/* antisymmetrised same-spin pair), which is U^2 for V = U.  The delta function is spread  */
/* over the two nearest nodes of a uniform grid of n_w frequencies on [-W0, W0],          */
/* W0 = 3.0001 (4|t| + 4|t'| + |mu|), linearly (every term's weight kept exactly).         */
/* Re Sigma(w) = -(1/pi) P int Im Sigma(w') / (w - w') dw' with Im Sigma linear between    */
/* nodes, integrated in closed form per interval.                                          */
/* Z = 1 / (1 - s), s the least-squares slope of Re Sigma over the nodes with              */
/* 2T <= |w| <= 4T (a margin of 2T around the Fermi level, where the slope inverts); NaN  */
/* when fewer than 8 nodes fall there, a slope the frequency grid does not resolve.       */
/* ------------------------------------------------------------------------------------ */
static double fermi(double x, double T) { return 0.5 * (1.0 - tanh(0.5 * x / T)); }

/* Representative point of patch a: the loop point itself under identity patching, else  */
/* the unsnapped point on the patch's centre ray at its shell's representative energy.    */
static void patch_point(const orc_model *m, int a, double *kx, double *ky)
{
    if (m->identity) { *kx = grid_k(a % m->L, m->L); *ky = grid_k(a / m->L, m->L); return; }
    int S = n_shells_of(m), Ns = m->N / S;
    fs_point(m, theta_off(Ns) + 2.0 * M_PI * (a % Ns) / Ns, shell_energy(m, a / Ns), kx, ky);
}

double orc_sigma_wmax(const orc_model *m)
{
    return 3.0001 * (4.0 * fabs(m->t) + 4.0 * fabs(m->tp) + fabs(m->mu));
}

/* Principal-value Kramers-Kronig of a piecewise-linear Im on a uniform grid (re = Re). */
void orc_kramers_kronig(int n_w, double w0, double dw, const double *im, double *re)
{
    for (int i = 0; i < n_w; ++i) {
        double w = w0 + dw * i, acc = 0.0;
        for (int j = 0; j + 1 < n_w; ++j) {
            double x0 = w0 + dw * j, x1 = x0 + dw;
            double slope = (im[j + 1] - im[j]) / dw;
            double at_w = im[j] + slope * (w - x0);      /* the interval's line at w */
            acc -= slope * dw;
            if (j != i && j + 1 != i)                     /* the two touching w cancel */
                acc += at_w * log(fabs((w - x0) / (w - x1)));
        }
        re[i] = -acc / M_PI;
    }
}

int orc_sigma2(const orc_model *m, double T, double U, const double *V, int n_w, double *w_out,
               double *im_out, double *re_out, double *Z_out, int nthreads)
{
    geom g;
    if (!(T > 0.0) || n_w < 16 || geom_build(m, &g)) return -1;
    set_threads(nthreads);
    int N = g.N, L = g.L, np = g.np;
    double W0 = orc_sigma_wmax(m), dw = 2.0 * W0 / (n_w - 1);
    if (!(W0 > 0.0)) { geom_free(&g); return -1; }
    double *f = (double *)malloc(sizeof(double) * np);
    for (int j = 0; j < np; ++j) f[j] = fermi(g.xi[j], T);
    for (int i = 0; i < n_w; ++i) if (w_out) w_out[i] = -W0 + dw * i;
#pragma omp parallel for schedule(dynamic)
    for (int a = 0; a < N; ++a) {
        double kx, ky;
        patch_point(m, a, &kx, &ky);
        double *h = (double *)calloc(n_w, sizeof(double));
        for (int j1 = 0; j1 < np; ++j1) {
            double k1x = grid_k(j1 % L, L), k1y = grid_k(j1 / L, L);
            for (int j3 = 0; j3 < np; ++j3) {
                double k3x = grid_k(j3 % L, L), k3y = grid_k(j3 / L, L);
                double x2 = disp(m, kx + k1x - k3x, ky + k1y - k3y);
                double f2 = fermi(x2, T);
                double F = f[j1] * (1.0 - f2) * (1.0 - f[j3]) + (1.0 - f[j1]) * f2 * f[j3];
                double W = U * U;
                if (V) {
                    int b = g.patch[j1], c = g.patch[j3];
                    double v = V[VIX(N, a, b, c)], vx = V[VIX(N, b, a, c)];
                    W = v * v + 0.5 * (v - vx) * (v - vx);
                }
                double E = x2 + g.xi[j3] - g.xi[j1];
                double x = (E + W0) / dw;
                int i = (int)floor(x);
                double fr = x - i;
                h[i] += (1.0 - fr) * W * F;
                h[i + 1] += fr * W * F;
            }
        }
        double *im = im_out + (size_t)a * n_w;
        for (int i = 0; i < n_w; ++i) im[i] = -M_PI * h[i] / ((double)np * np * dw);
        double *re = (double *)malloc(sizeof(double) * n_w);
        orc_kramers_kronig(n_w, -W0, dw, im, re);
        if (re_out) memcpy(re_out + (size_t)a * n_w, re, sizeof(double) * n_w);
        double sx = 0, sy = 0, sxx = 0, sxy = 0;
        int cnt = 0;
        for (int i = 0; i < n_w; ++i) {
            double w = -W0 + dw * i;
            if (fabs(w) < 2.0 * T || fabs(w) > 4.0 * T) continue;
            sx += w; sy += re[i]; sxx += w * w; sxy += w * re[i]; ++cnt;
        }
        double slope = (cnt * sxy - sx * sy) / (cnt * sxx - sx * sx);
        if (Z_out) Z_out[a] = cnt >= 8 ? 1.0 / (1.0 - slope) : NAN;
        free(re); free(h);
    }
    free(f);
    geom_free(&g);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Katanin factor and A_g of the interaction flow (App. A, Steps 2 and 3) from Z tabulated */
/* on n >= 3 nodes g_0 < ... < g_{n-1} (Z_g from the self-energy at scale g, so that      */
/* s_g = 1 - 1/Z_g is the slope of Re(g Sigma_g) at the Fermi level, Eq. definition_Z):   */
/*   K_g = 1 + g^2 d_w Re(d Sigma_g/dg) = 1 - s_g + g ds_g/dg   (Eq. K_definition, with     */
/*         d_w Re Sigma_g = s_g / g),                                                      */
/*   A_g = -(2/g)(1 - Z_g K_g)                                  (Eq. A_g_simple),          */
/* which equals 2 (dZ_g/dg)/Z_g = 2 s_g'/(1 - s_g), the form used at g = 0.  ds/dg is the  */
/* derivative of the parabola through three neighbouring nodes (one-sided at the ends).    */
/* z_tab, k_tab, a_tab: [n][N]; a_tab may be NULL.                                          */
/* ------------------------------------------------------------------------------------ */
int orc_katanin(int n, const double *g, int N, const double *z_tab, double *k_tab,
                double *a_tab)
{
    if (n < 3 || N < 1 || !g || !z_tab || !k_tab) return -1;
    for (int i = 1; i < n; ++i) if (!(g[i] > g[i - 1])) return -1;
    for (int i = 0; i < n; ++i) {
        /* three nodes i0, i0+1, i0+2 around i, and the derivative weights at g_i */
        int i0 = i == 0 ? 0 : (i == n - 1 ? n - 3 : i - 1);
        double x0 = g[i0], x1 = g[i0 + 1], x2 = g[i0 + 2], x = g[i];
        /* d/dx of the Lagrange basis polynomials at x */
        double w0 = ((x - x1) + (x - x2)) / ((x0 - x1) * (x0 - x2));
        double w1 = ((x - x0) + (x - x2)) / ((x1 - x0) * (x1 - x2));
        double w2 = ((x - x0) + (x - x1)) / ((x2 - x0) * (x2 - x1));
        for (int a = 0; a < N; ++a) {
            double s0 = 1.0 - 1.0 / z_tab[(size_t)i0 * N + a];
            double s1 = 1.0 - 1.0 / z_tab[(size_t)(i0 + 1) * N + a];
            double s2 = 1.0 - 1.0 / z_tab[(size_t)(i0 + 2) * N + a];
            double z = z_tab[(size_t)i * N + a], s = 1.0 - 1.0 / z;
            double ds = w0 * s0 + w1 * s1 + w2 * s2;
            double K = 1.0 - s + x * ds;
            k_tab[(size_t)i * N + a] = K;
            if (a_tab)
                a_tab[(size_t)i * N + a] = x > 0.0 ? -(2.0 / x) * (1.0 - z * K)
                                                   : 2.0 * ds / (1.0 - s);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Quasi-particle weights along the flow: a table Z_a(s_i) in the flow parameter (ln T, or  */
/* g for the interaction flow), linear in s between nodes, clamped outside.               */
/* ------------------------------------------------------------------------------------ */
static void table_at(const orc_flowcfg *f, const double *tab, int N, double s, double *Z)
{
    if (f->n_z <= 0 || !tab) { for (int a = 0; a < N; ++a) Z[a] = 1.0; return; }
    int n = f->n_z;
    if (n == 1 || s <= f->z_lnT[0]) { memcpy(Z, tab, sizeof(double) * N); return; }
    if (s >= f->z_lnT[n - 1]) { memcpy(Z, tab + (size_t)(n - 1) * N, sizeof(double) * N); return; }
    int i = 0;
    while (i + 1 < n - 1 && f->z_lnT[i + 1] <= s) ++i;
    double w = (s - f->z_lnT[i]) / (f->z_lnT[i + 1] - f->z_lnT[i]);
    for (int a = 0; a < N; ++a)
        Z[a] = (1.0 - w) * tab[(size_t)i * N + a] + w * tab[(size_t)(i + 1) * N + a];
}

static void z_at(const orc_flowcfg *f, int N, double s, double *Z) { table_at(f, f->z_tab, N, s, Z); }

/* ------------------------------------------------------------------------------------ */
/* Integrators in s = ln T (temperature flow) or s = g (interaction flow).              */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    const geom *g;
    const orc_model *m;
    const orc_flowcfg *f;
    double *Z;
    long n_rhs;
    double *K;           /* Katanin factors at the current s (k_tab set) */
} flowctx;

static void eval_f(flowctx *cx, double s, const double *V, double *k)
{
    z_at(cx->f, cx->g->N, s, cx->Z);
    if (cx->f->k_tab) table_at(cx->f, cx->f->k_tab, cx->g->N, s, cx->K);
    wkind wk = {cx->f->gflow != 0, cx->f->gflow ? cx->f->T0 : exp(s), cx->f->gflow ? s : 0.0,
                cx->f->k_tab ? cx->K : NULL};
    if (cx->f->rhs_binned)
        rhs_binned_geom(cx->g, cx->m->channels, wk, cx->f->n_z > 0 ? cx->Z : NULL, V, k);
    else
        rhs_geom(cx->g, cx->m->channels, wk, cx->f->n_z > 0 ? cx->Z : NULL, V, k);
    cx->n_rhs++;
}

static double max_abs(const double *V, size_t n, int *finite)
{
    double m = 0.0;
    *finite = 1;
    for (size_t i = 0; i < n; ++i) {
        if (!isfinite(V[i])) { *finite = 0; return INFINITY; }
        if (fabs(V[i]) > m) m = fabs(V[i]);
    }
    return m;
}

/* Dormand & Prince (1980), RK5(4)7M: nodes, coupling, 5th-order weights (= last coupling
 * row, first-same-as-last) and the 5th-minus-4th-order error weights. */
static const double DP_C[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
static const double DP_A[7][6] = {
    {0},
    {1.0 / 5},
    {3.0 / 40, 9.0 / 40},
    {44.0 / 45, -56.0 / 15, 32.0 / 9},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656},
    {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
static const double DP_E[7] = {71.0 / 57600, 0.0, -71.0 / 16695, 71.0 / 1920,
                               -17253.0 / 339200, 22.0 / 525, -1.0 / 40};

int orc_dopri_tableau(double *c, double *a, double *e)
{
    memcpy(c, DP_C, sizeof(DP_C));
    memcpy(a, DP_A, sizeof(DP_A));
    memcpy(e, DP_E, sizeof(DP_E));
    return 0;
}

/* One Dormand-Prince attempt from (s, V) with step h, k[0] = f(s, V) given.  Fills k[1..6],
 * Vn = the 5th-order solution (also the last stage's argument), returns the scaled error
 * norm max_i |E_i| / (atol + rtol max(|V_i|, |Vn_i|)), or INFINITY if anything is
 * non-finite. */
static double dopri_attempt(flowctx *cx, double s, double h, const double *V, double **k,
                            double *Vn, double *tmp, size_t n)
{
    const orc_flowcfg *f = cx->f;
    for (int st = 1; st < 7; ++st) {
        double *arg = (st == 6) ? Vn : tmp;
        for (size_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int l = 0; l < st; ++l) acc += DP_A[st][l] * k[l][i];
            arg[i] = V[i] + h * acc;
        }
        eval_f(cx, s + DP_C[st] * h, arg, k[st]);
    }
    double err = 0.0;
    for (size_t i = 0; i < n; ++i) {
        double e = 0.0;
        for (int l = 0; l < 7; ++l) e += DP_E[l] * k[l][i];
        e = fabs(h * e);
        double sc = f->atol + f->rtol * fmax(fabs(V[i]), fabs(Vn[i]));
        double r = e / sc;
        if (!isfinite(r) || !isfinite(Vn[i])) return INFINITY;
        if (r > err) err = r;
    }
    return err;
}

static double step_factor(double err)
{
    if (err == 0.0) return 5.0;
    double fac = 0.9 * pow(err, -0.2);
    return fmin(5.0, fmax(0.2, fac));
}

/* Stop rule (Sec. 3.2: the flow is followed until the coupling grows beyond a threshold):
 * the largest |V| above the threshold vth (or a non-finite value) ends the flow.  The
 * temperature flow uses an absolute threshold v_max; the interaction flow the paper's own
 * criterion, relative to the bare coupling, vth = v_rel |U|: since g^2 V_g depends on g^2 U
 * only (without Z), the crossing U* = g*^2 U is then a function of T alone.
 * The crossing max|V| = vth is located on 1/max|V| as a function of x = ln T (temperature
 * flow) or x = g^2 (interaction flow): near an instability the one-loop flow grows like a
 * simple pole in that variable (for one patch 1/v = 1/U - [c(T) - c(T0)], resp.
 * 1/v = 1/U - g^2 c, exactly), so 1/max|V| is smooth and nearly linear.  Its curvature over
 * a long last step still shifts a straight-line crossing (by ~5e-4 in T_c for the N = 128
 * workloads at rtol 1e-6), so the crossing is the root of the parabola through the last
 * three accepted points (x_prev2, x_prev, x_new), inside the last step; with only two points,
 * or no root inside the step, the straight line through the last two. */
static double crossing_x(double x0, double m0, double x1, double m1, double x2, double m2,
                         double vth)
{
    if (!(m1 > 0.0) || m2 == m1) return x2;
    double y1 = 1.0 / m1, y2 = 1.0 / m2, ys = 1.0 / vth;
    double lin = x1 + (ys - y1) * (x2 - x1) / (y2 - y1);
    if (!(m0 > 0.0) || x0 == x1) return lin;
    /* Newton form: y(x) = y1 + (x - x1) d1 + (x - x1)(x - x2) d2 */
    double d0 = (y1 - 1.0 / m0) / (x1 - x0);
    double d1 = (y2 - y1) / (x2 - x1);
    double d2 = (d1 - d0) / (x2 - x0);
    if (d2 == 0.0) return lin;
    /* in t = x - x1: d2 t^2 + (d1 - d2 (x2 - x1)) t + (y1 - ys) = 0 */
    double A = d2, B = d1 - d2 * (x2 - x1), C = y1 - ys;
    double disc = B * B - 4.0 * A * C;
    if (!(disc >= 0.0)) return lin;
    double q = -0.5 * (B + copysign(sqrt(disc), B));
    double lo = fmin(0.0, x2 - x1), hi = fmax(0.0, x2 - x1);
    double best = lin, dist = INFINITY;
    double r[2] = {q != 0.0 ? q / A : NAN, q != 0.0 ? C / q : NAN};
    for (int i = 0; i < 2; ++i) {
        if (!(r[i] >= lo && r[i] <= hi)) continue;
        double x = x1 + r[i];
        if (fabs(x - lin) < dist) { dist = fabs(x - lin); best = x; }
    }
    return best;
}

/* (s_pp, m_pp): the accepted point before (s_prev, m_prev); m_pp = 0 when there is none. */
static int stop_test(const orc_flowcfg *f, double vth, double s_pp, double m_pp, double s_prev,
                     double m_prev, double s_new, double m_new, int finite, double *sc)
{
    if (!finite) { *sc = s_new; return ORC_NONFINITE; }
    if (m_new > vth) {
        if (f->gflow)
            *sc = sqrt(crossing_x(s_pp * s_pp, m_pp, s_prev * s_prev, m_prev, s_new * s_new,
                                  m_new, vth));
        else
            *sc = crossing_x(s_pp, m_pp, s_prev, m_prev, s_new, m_new, vth);
        return ORC_DIVERGED;
    }
    return ORC_RUNNING;
}

/* A Katanin table needs the interaction flow and a Z table's nodes. */
static int katanin_ok(const orc_flowcfg *f) { return !f->k_tab || (f->gflow && f->n_z > 0); }

/*
 * Full flow from V = U: temperature flow from T0 down to T_end, or interaction flow at
 * T = T0 from g = 0 up to g_end.  trace (optional) receives (s, max|V|) after every
 * accepted step, starting with the initial point; *n_trace is its length (capped at
 * max_trace).
 */
int orc_flow(const orc_model *m, const orc_flowcfg *f, double U, double *V_out,
             orc_result *res, double *trace, int max_trace, int *n_trace, int nthreads)
{
    geom g;
    if (f->gflow ? !(f->T0 > 0.0 && f->g_end > 0.0)
                 : (!(f->T0 > f->T_end) || !(f->T_end > 0.0)))
        return -1;
    if (!katanin_ok(f) || geom_build(m, &g)) return -1;
    set_threads(nthreads);
    size_t n = (size_t)g.N * g.N * g.N;
    double *V = (double *)malloc(sizeof(double) * n);
    double *Vn = (double *)malloc(sizeof(double) * n);
    double *tmp = (double *)malloc(sizeof(double) * n);
    double *kb = (double *)malloc(sizeof(double) * n * 7);
    double *k[7];
    for (int i = 0; i < 7; ++i) k[i] = kb + (size_t)i * n;
    double *Z = (double *)malloc(sizeof(double) * g.N);
    double *Kz = (double *)malloc(sizeof(double) * g.N);
    flowctx cx = {&g, m, f, Z, 0, Kz};
    for (size_t i = 0; i < n; ++i) V[i] = U;

    double s0 = f->gflow ? 0.0 : log(f->T0), s_end = f->gflow ? f->g_end : log(f->T_end);
    double s = s0, dir = s_end > s0 ? 1.0 : -1.0;   /* direction of the flow parameter */
    double vth = f->gflow ? (f->v_rel > 0.0 ? f->v_rel : 100.0) * fabs(U) : f->v_max;
    int finite, status = ORC_RUNNING, nacc = 0, nrej = 0, ntr = 0;
    double mV = max_abs(V, n, &finite), lnTc = NAN;
    double sp = s, mp = 0.0;      /* the accepted point before (s, mV); none yet */
    if (trace && ntr < max_trace) { trace[2 * ntr] = s; trace[2 * ntr + 1] = mV; ++ntr; }
    if (!finite) { status = ORC_NONFINITE; lnTc = s; }
    else if (mV > vth) { status = ORC_DIVERGED; lnTc = s; }

    if (status == ORC_RUNNING && f->integrator == 0) {
        double h = (s_end - s0) / f->n_steps;
        for (int st = 0; st < f->n_steps && status == ORC_RUNNING; ++st) {
            double sn = s0 + st * h;
            eval_f(&cx, sn, V, k[0]);
            for (size_t i = 0; i < n; ++i) tmp[i] = V[i] + 0.5 * h * k[0][i];
            eval_f(&cx, sn + 0.5 * h, tmp, k[1]);
            for (size_t i = 0; i < n; ++i) tmp[i] = V[i] + 0.5 * h * k[1][i];
            eval_f(&cx, sn + 0.5 * h, tmp, k[2]);
            for (size_t i = 0; i < n; ++i) tmp[i] = V[i] + h * k[2][i];
            eval_f(&cx, sn + h, tmp, k[3]);
            for (size_t i = 0; i < n; ++i)
                V[i] += h / 6.0 * (k[0][i] + 2.0 * k[1][i] + 2.0 * k[2][i] + k[3][i]);
            double s_new = (st + 1 == f->n_steps) ? s_end : s0 + (st + 1) * h;
            double m_new = max_abs(V, n, &finite);
            ++nacc;
            status = stop_test(f, vth, sp, mp, s, mV, s_new, m_new, finite, &lnTc);
            sp = s; mp = mV;
            s = s_new; mV = m_new;
            if (trace && ntr < max_trace) { trace[2 * ntr] = s; trace[2 * ntr + 1] = mV; ++ntr; }
        }
        if (status == ORC_RUNNING) status = ORC_REACHED_TEND;
    } else if (status == ORC_RUNNING) {
        double span = fabs(s_end - s0);
        double h = f->h0 != 0.0 ? f->h0 : (s_end - s0) / 200.0;
        double hmin = f->h_min > 0.0 ? f->h_min : 1e-8 * span;
        eval_f(&cx, s, V, k[0]);
        while (status == ORC_RUNNING) {
            if (dir * (s - s_end) >= 0.0) { status = ORC_REACHED_TEND; break; }
            int last = (dir * (s + h - s_end) >= 0.0);
            double ht = last ? (s_end - s) : h;
            double err = dopri_attempt(&cx, s, ht, V, k, Vn, tmp, n);
            if (f->progress) {
                fprintf(stderr, "oracle flow: s %.6f h %.3e err %.3g max|V| %.4g\n", s, ht, err,
                        mV);
                fflush(stderr);
            }
            if (err <= 1.0) {
                double s_new = last ? s_end : s + ht;
                double m_new = max_abs(Vn, n, &finite);
                memcpy(V, Vn, sizeof(double) * n);
                memcpy(k[0], k[6], sizeof(double) * n);
                ++nacc;
                status = stop_test(f, vth, sp, mp, s, mV, s_new, m_new, finite, &lnTc);
                sp = s; mp = mV;
                s = s_new; mV = m_new;
                if (trace && ntr < max_trace) { trace[2 * ntr] = s; trace[2 * ntr + 1] = mV; ++ntr; }
                h = ht * step_factor(err);
            } else {
                ++nrej;
                h = isfinite(err) ? ht * step_factor(err) : 0.5 * ht;
            }
            if (status == ORC_RUNNING && fabs(h) < hmin) status = ORC_STEPFAIL;
        }
    }
    if (res) {
        int stopped = status == ORC_DIVERGED || status == ORC_NONFINITE;
        res->status = status;
        res->T_c = (stopped && !f->gflow) ? exp(lnTc) : NAN;
        res->T_final = f->gflow ? f->T0 : exp(s);
        res->g_c = (stopped && f->gflow) ? lnTc : NAN;
        res->U_star = (stopped && f->gflow) ? lnTc * lnTc * U : NAN;
        res->g_final = f->gflow ? s : NAN;
        res->max_abs_V = mV;
        res->n_accepted = nacc;
        res->n_rejected = nrej;
        res->n_rhs = (int)cx.n_rhs;
    }
    if (V_out) memcpy(V_out, V, sizeof(double) * n);
    if (n_trace) *n_trace = ntr;
    free(V); free(Vn); free(tmp); free(kb); free(Z); free(Kz);
    geom_free(&g);
    return 0;
}

/*
 * Flows on one step schedule: nf flows from V = U[i], all from the same start (T0, or g = 0
 * at T = T0), Dormand-Prince only.  Every attempt is made by every running flow with the
 * same step; it is accepted only if each flow's error norm is <= 1, and the next step follows
 * from the largest norm of the running flows (the smallest step any of them proposes).  Each
 * flow keeps its own stop rule and crossing.  Sharing one schedule makes every stage
 * temperature common to the flows, which is what lets their bubble sums be shared.  atol <= 0
 * selects 1e-9 max(1, |U_i|) per flow.  V_out: [nf][N^3] or NULL; res: [nf].
 */
int orc_flow_sync(const orc_model *m, const orc_flowcfg *f, int nf, const double *U,
                  double *V_out, orc_result *res, int nthreads)
{
    geom g;
    if (nf < 1 || f->integrator != 1) return -1;
    if (f->gflow ? !(f->T0 > 0.0 && f->g_end > 0.0) : (!(f->T0 > f->T_end) || !(f->T_end > 0.0)))
        return -1;
    if (!katanin_ok(f) || geom_build(m, &g)) return -1;
    set_threads(nthreads);
    size_t n = (size_t)g.N * g.N * g.N;
    double *V = (double *)malloc(sizeof(double) * n * nf);
    double *Vn = (double *)malloc(sizeof(double) * n * nf);
    double *tmp = (double *)malloc(sizeof(double) * n);
    double *kb = (double *)malloc(sizeof(double) * n * 7 * nf);
    double *Z = (double *)malloc(sizeof(double) * g.N);
    double *err = (double *)malloc(sizeof(double) * nf);
    double *mV = (double *)malloc(sizeof(double) * nf);
    double *lnTc = (double *)malloc(sizeof(double) * nf);
    double *sl = (double *)malloc(sizeof(double) * nf);    /* each flow's last accepted s */
    double *spp = (double *)malloc(sizeof(double) * nf);   /* and the accepted point before */
    double *mpp = (double *)calloc(nf, sizeof(double));
    int *status = (int *)malloc(sizeof(int) * nf);
    int *nacc = (int *)calloc(nf, sizeof(int));
    int *nrej = (int *)calloc(nf, sizeof(int));
    long *nrhs = (long *)calloc(nf, sizeof(long));
    orc_flowcfg fi = *f;
    double *Kz = (double *)malloc(sizeof(double) * g.N);
    flowctx cx = {&g, m, &fi, Z, 0, Kz};
    double s0 = f->gflow ? 0.0 : log(f->T0), s_end = f->gflow ? f->g_end : log(f->T_end);
    double s = s0, dir = s_end > s0 ? 1.0 : -1.0;
    double h = f->h0 != 0.0 ? f->h0 : (s_end - s0) / 200.0;
    double hmin = f->h_min > 0.0 ? f->h_min : 1e-8 * fabs(s_end - s0);
    for (int i = 0; i < nf; ++i) {
        double *Vi = V + (size_t)i * n, *k0 = kb + (size_t)i * 7 * n;
        for (size_t e = 0; e < n; ++e) Vi[e] = U[i];
        double vth = f->gflow ? (f->v_rel > 0.0 ? f->v_rel : 100.0) * fabs(U[i]) : f->v_max;
        int finite;
        mV[i] = max_abs(Vi, n, &finite);
        lnTc[i] = NAN;
        sl[i] = s;
        spp[i] = s;
        status[i] = ORC_RUNNING;
        if (!finite) { status[i] = ORC_NONFINITE; lnTc[i] = s; }
        else if (mV[i] > vth) { status[i] = ORC_DIVERGED; lnTc[i] = s; }
        if (status[i] == ORC_RUNNING) { cx.n_rhs = 0; eval_f(&cx, s, Vi, k0); nrhs[i] += cx.n_rhs; }
    }
    for (;;) {
        int any = 0;
        for (int i = 0; i < nf; ++i) any |= status[i] == ORC_RUNNING;
        if (!any) break;
        if (dir * (s - s_end) >= 0.0) {
            for (int i = 0; i < nf; ++i) if (status[i] == ORC_RUNNING) status[i] = ORC_REACHED_TEND;
            break;
        }
        int last = (dir * (s + h - s_end) >= 0.0);
        double ht = last ? (s_end - s) : h;
        double eg = 0.0;
        for (int i = 0; i < nf; ++i) {
            if (status[i] != ORC_RUNNING) continue;
            double *k[7];
            for (int l = 0; l < 7; ++l) k[l] = kb + ((size_t)i * 7 + l) * n;
            fi.atol = f->atol > 0.0 ? f->atol : 1e-9 * fmax(1.0, fabs(U[i]));
            cx.n_rhs = 0;
            err[i] = dopri_attempt(&cx, s, ht, V + (size_t)i * n, k, Vn + (size_t)i * n, tmp, n);
            nrhs[i] += cx.n_rhs;
            if (!(err[i] <= eg)) eg = err[i];          /* a non-finite norm is the largest */
        }
        if (eg <= 1.0) {
            double s_new = last ? s_end : s + ht;
            for (int i = 0; i < nf; ++i) {
                if (status[i] != ORC_RUNNING) continue;
                double *Vi = V + (size_t)i * n, *k0 = kb + (size_t)i * 7 * n;
                int finite;
                double m_new = max_abs(Vn + (size_t)i * n, n, &finite);
                memcpy(Vi, Vn + (size_t)i * n, sizeof(double) * n);
                memcpy(k0, k0 + 6 * n, sizeof(double) * n);
                ++nacc[i];
                double vth = f->gflow ? (f->v_rel > 0.0 ? f->v_rel : 100.0) * fabs(U[i]) : f->v_max;
                status[i] = stop_test(f, vth, spp[i], mpp[i], s, mV[i], s_new, m_new, finite,
                                      &lnTc[i]);
                spp[i] = s; mpp[i] = mV[i];
                mV[i] = m_new;
                sl[i] = s_new;
            }
            s = s_new;
            h = ht * step_factor(eg);
        } else {
            for (int i = 0; i < nf; ++i) if (status[i] == ORC_RUNNING) ++nrej[i];
            h = isfinite(eg) ? ht * step_factor(eg) : 0.5 * ht;
        }
        if (fabs(h) < hmin)
            for (int i = 0; i < nf; ++i) if (status[i] == ORC_RUNNING) status[i] = ORC_STEPFAIL;
    }
    for (int i = 0; i < nf; ++i) {
        if (res) {
            orc_result *r = res + i;
            int stopped = status[i] == ORC_DIVERGED || status[i] == ORC_NONFINITE;
            r->status = status[i];
            r->T_c = (stopped && !f->gflow) ? exp(lnTc[i]) : NAN;
            r->T_final = f->gflow ? f->T0 : exp(sl[i]);
            r->g_c = (stopped && f->gflow) ? lnTc[i] : NAN;
            r->U_star = (stopped && f->gflow) ? lnTc[i] * lnTc[i] * U[i] : NAN;
            r->g_final = f->gflow ? sl[i] : NAN;
            r->max_abs_V = mV[i];
            r->n_accepted = nacc[i];
            r->n_rejected = nrej[i];
            r->n_rhs = (int)nrhs[i];
        }
        if (V_out) memcpy(V_out + (size_t)i * n, V + (size_t)i * n, sizeof(double) * n);
    }
    free(V); free(Vn); free(tmp); free(kb); free(Z); free(Kz); free(err); free(mV); free(lnTc); free(sl);
    free(spp); free(mpp); free(status); free(nacc); free(nrej); free(nrhs);
    geom_free(&g);
    return 0;
}

/*
 * One step from (s, V) with step *h, for step-by-step comparison; s = ln T, or g for the
 * interaction flow (at T = f->T0).  RK4: always accepted, *h unchanged.  Dormand-Prince: k1
 * evaluated here (no carry-over between calls); on acceptance V and s advance; *h becomes
 * the proposed next step either way.
 */
int orc_step(const orc_model *m, const orc_flowcfg *f, double *lnT, double *h, double *V,
             int *accepted, double *err_out, int nthreads)
{
    geom g;
    if (!katanin_ok(f) || geom_build(m, &g)) return -1;
    set_threads(nthreads);
    size_t n = (size_t)g.N * g.N * g.N;
    double *Vn = (double *)malloc(sizeof(double) * n);
    double *tmp = (double *)malloc(sizeof(double) * n);
    double *kb = (double *)malloc(sizeof(double) * n * 7);
    double *k[7];
    for (int i = 0; i < 7; ++i) k[i] = kb + (size_t)i * n;
    double *Z = (double *)malloc(sizeof(double) * g.N);
    double *Kz = (double *)malloc(sizeof(double) * g.N);
    flowctx cx = {&g, m, f, Z, 0, Kz};
    double s = *lnT, hh = *h;
    eval_f(&cx, s, V, k[0]);
    if (f->integrator == 0) {
        for (size_t i = 0; i < n; ++i) tmp[i] = V[i] + 0.5 * hh * k[0][i];
        eval_f(&cx, s + 0.5 * hh, tmp, k[1]);
        for (size_t i = 0; i < n; ++i) tmp[i] = V[i] + 0.5 * hh * k[1][i];
        eval_f(&cx, s + 0.5 * hh, tmp, k[2]);
        for (size_t i = 0; i < n; ++i) tmp[i] = V[i] + hh * k[2][i];
        eval_f(&cx, s + hh, tmp, k[3]);
        for (size_t i = 0; i < n; ++i)
            V[i] += hh / 6.0 * (k[0][i] + 2.0 * k[1][i] + 2.0 * k[2][i] + k[3][i]);
        *lnT = s + hh;
        *accepted = 1;
        if (err_out) *err_out = 0.0;
    } else {
        double err = dopri_attempt(&cx, s, hh, V, k, Vn, tmp, n);
        if (err_out) *err_out = err;
        if (err <= 1.0) {
            memcpy(V, Vn, sizeof(double) * n);
            *lnT = s + hh;
            *accepted = 1;
            *h = hh * step_factor(err);
        } else {
            *accepted = 0;
            *h = isfinite(err) ? hh * step_factor(err) : 0.5 * hh;
        }
    }
    free(Vn); free(tmp); free(kb); free(Z); free(Kz);
    geom_free(&g);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
