/*
 * fm_flow.h -- C ABI of the one-loop temperature-flow library for the N-patch coupling
 * function V(k1,k2,k3) of the two-dimensional Hubbard model on MI355X (gfx950).
 *
 * The method is that of D. Rohe and C. Honerkamp, "Quasi-particle functional
 * Renormalisation Group calculations in the two-dimensional half-filled Hubbard model at
 * finite temperatures" (arXiv:2005.00827):
 *   - model and dispersion: Sec. 2.1, Eqs. model_definition, free_dispersion_xi;
 *   - one-loop flow of the static vertex: App. A, Eqs. vertex_flow_general,
 *     vertex_flow_simple; quasi-particle weights Z on the internal lines, projected onto the
 *     Fermi-surface patch of each line: App. A, Step 2, Eqs. both_propagators_Z,
 *     vertex_flow_feedback_Z;
 *   - angular Fermi-surface patching (Sec. 3.2: seven patches from antinode to node, 48 in
 *     total), the whole Brillouin zone as loop support (App. A, Comment 1);
 *   - stop rule: the flow ends when the largest |V| has grown beyond a threshold (Sec. 3.2,
 *     definition of U*(T)).
 * Two flows of the same one-loop vertex equation (FM_FLOW_*):
 *   - temperature flow, s = ln T from T0 down to T_end: every internal pair of lines carries
 *     the weight Z_a' Z_b' T d/dT chi(xi, xi') with chi the bare static particle-hole (or
 *     particle-particle) bubble of the two lines;
 *   - interaction flow, the paper's own scheme (Sec. 2.2; App. A, Steps 1 and 2): at fixed
 *     T the propagator scale g runs from 0 to g_end, lines G_g = g Z G0 and S_g = Z^2 G0, so
 *     the pair carries g Z_a' Z_b' (Z_a' + Z_b') chi (2 g chi without Z).  The stop rule
 *     gives g* and the crossover coupling U*(T) = g*^2 U (Sec. 3.2); fm_flow_tstar inverts
 *     it to T*(U).
 *
 * Conventions
 *   - Loop grid: L x L points k = -pi + 2 pi (j + 1/2)/L per axis, point index j = jx + L*jy.
 *   - Patches (FM_GEOM_ANGULAR): sector centres theta_a = theta_off + 2 pi a / N with
 *     theta_off = 0 for N % 8 == 0 or N == 1 and pi/N for N % 8 == 4; the patch of a loop
 *     point is its nearest centre.  Each patch is represented by the Fermi-surface point on
 *     its centre ray, snapped to the transfer grid q = 2 pi m / L.
 *     FM_GEOM_IDENTITY: every loop point is its own patch (N = L*L), all momenta exact.
 *   - V layout: row-major double V[((f*N + a)*N + b)*N + c] for flow f; a, b are the patches
 *     of the incoming k1, k2, c that of the outgoing k3 (spin of k1); k4 = k1 + k2 - k3.
 *
 * Ownership and memory: the library allocates no device memory.  The caller allocates one
 * workspace of fm_flow_workspace_bytes() bytes (for example a torch uint8 tensor) and passes
 * its device pointer to fm_flow_init; it must stay valid until fm_flow_destroy.  Every other
 * device pointer is also caller owned.  Host arrays passed to fm_flow_init are copied.
 *
 * Errors: every call returns FM_OK (0) or a negative FM_E* code; fm_last_error() gives a
 * message for the last failing call of the calling thread.  Flow outcomes (divergence,
 * reaching T_end, ...) are not errors; they are reported in fm_result.status.
 *
 * Streams: all device work is enqueued on cfg.stream (a hipStream_t; NULL = the default
 * stream).  fm_flow_rhs is asynchronous; fm_flow_step and fm_flow_run_batch synchronise the
 * stream before returning their host outputs.  A handle is not thread safe.
 */
#ifndef FM_FLOW_H
#define FM_FLOW_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fm_flow fm_flow;

enum { FM_OK = 0, FM_EINVAL = -1, FM_ENOMEM = -2, FM_EDEVICE = -3, FM_ESTATE = -4 };

/* Patch geometry.  FM_GEOM_SHELLS: energy-shell patching (Sec. 3.2: the angular sectors
 * subdivided in energy, 7 shells x 32 sectors = 224 patches); patch a = e * (N / n_shells) +
 * s for shell e (0 = most negative xi) and angular sector s. */
enum { FM_GEOM_ANGULAR = 0, FM_GEOM_IDENTITY = 1, FM_GEOM_SHELLS = 2 };

/* Integrator in s = ln T: classical RK4 with n_steps fixed steps from T0 to T_end, or
 * Dormand-Prince 5(4) with error control (rtol, atol, h0, h_min). */
enum { FM_RK4_FIXED = 0, FM_RK45_DOPRI = 1 };

/* Arithmetic of the right-hand side.  The integrator state, the error estimate and the stop
 * test are double precision in every mode.
 *   FM_FP64          binned loop sums and contractions in double precision
 *   FM_FP32          binned loop sums and contractions in single precision
 *   FM_FP32_BF16MFMA single-precision loop sums; the grouped contractions on bf16 matrix
 *                    cores with single-precision accumulation
 *   FM_FP64_DIRECT   direct double-precision loop sums over every loop point, no binning
 *   FM_FP32_BF16X3   as FM_FP32_BF16MFMA, with each operand split into two bf16 parts and
 *                    three bf16 products per contraction step (about 16 significant bits
 *                    per product, close to single precision at bf16 matrix-core rates) */
enum { FM_FP64 = 0, FM_FP32 = 1, FM_FP32_BF16MFMA = 2, FM_FP64_DIRECT = 3, FM_FP32_BF16X3 = 4 };

/* Flow parameter. */
enum { FM_FLOW_TEMPERATURE = 0, FM_FLOW_INTERACTION = 1 };

/* Channel mask (for ablations of the flow equation). */
enum { FM_CH_PP = 1, FM_CH_CR = 2, FM_CH_D = 4, FM_CH_ALL = 7 };

/* Sizes: FM_FP32_BF16MFMA and FM_FP32_BF16X3 need N <= 128 (FM_EINVAL above; their
 * contractions run on bf16 matrix cores only up to that width); FM_FP32 runs its contractions
 * on fp32 matrix cores up to N = 128 and on the vector units above; FM_FP64 and
 * FM_FP64_DIRECT have no bound on N beyond memory. */

/* fm_result.status */
enum { FM_FLOW_RUNNING = 0, FM_FLOW_DIVERGED = 1, FM_FLOW_NONFINITE = 2,
       FM_FLOW_REACHED_TEND = 3, FM_FLOW_STEPFAIL = 4 };

typedef struct {
    double t, tp, mu, U;      /* hopping t, next-nearest t', chemical potential, bare U
                                 (Eqs. model_definition, free_dispersion_xi) */
    int geometry;             /* FM_GEOM_* */
    int N, L;                 /* patches; loop grid side.  Angular: N == 1 or N % 4 == 0
                                 with N % 8 in {0, 4}; L % 4 == 0.  Identity: N == L*L. */
    double T0, T_end;         /* temperature flow: window, T0 > T_end > 0 (finite T only);
                                 interaction flow: T0 > 0 is the temperature of
                                 fm_flow_step (run_batch takes one per flow), T_end unused */
    int integrator, n_steps;  /* FM_RK4_FIXED uses n_steps */
    double rtol, atol;        /* Dormand-Prince: error norm max_i |E_i|/(atol + rtol max(|V|,|Vnew|));
                                 0 selects rtol 1e-6 (1e-4 for FM_FP32_BF16MFMA, whose
                                 right-hand side resolves about 3 digits) and atol
                                 1e-9 max(1, |U|) */
    double h0, h_min;         /* first step and smallest |step| in the flow parameter; 0
                                 selects span/200 and 1e-8 |span|, span = ln(T_end/T0) or
                                 g_end (h0 < 0 for the temperature flow, > 0 in g) */
    double v_max;             /* temperature flow: stop when max|V| > v_max (0 selects 20) */
    unsigned channels;        /* FM_CH_* mask (0 selects FM_CH_ALL) */
    int precision;            /* FM_FP64 | FM_FP32 | FM_FP32_BF16MFMA | FM_FP64_DIRECT |
                                 FM_FP32_BF16X3 */
    int n_zT;                 /* 0: no quasi-particle feedback (Z = 1) */
    const double *z_lnT;      /* host [n_zT], ascending nodes in the flow parameter (ln T, or
                                 g in [0, g_end] for the interaction flow); copied */
    const double *z_table;    /* host [n_zT][N], every Z positive and finite (Z passes 1
                                 where Re Sigma slopes upward, as its definition allows),
                                 linear between nodes, clamped outside; copied */
    void *stream;             /* hipStream_t or NULL */
    int max_batch;            /* capacity (flows) for every batched call; >= 1 */
    int tile_rows;            /* single-precision phase 2a: 16-row transfer tiles per
                                 wavefront (>= 1, values past all tiles of a group are
                                 clamped); 0 = chosen by timing 1, 2, 4, ... and all on the
                                 first call (kept per shape for the process) */
    int flow;                 /* FM_FLOW_TEMPERATURE (0) | FM_FLOW_INTERACTION */
    double g_end;             /* interaction flow: last g (0 selects 1) */
    double v_rel;             /* interaction flow: stop when max|V| > v_rel |U|, the paper's
                                 criterion relative to the bare coupling (Sec. 3.2); with it
                                 U* = g*^2 U depends on T alone without Z (0 selects 100) */
    int y_kernel;             /* single-precision phase 2a on matrix cores: 1 gathers each
                                 transfer's permuted bins, 2 stages the operand permuted once
                                 per point-group operation class, 3 reads each representative's
                                 bin row once and applies every operation of its orbit to it
                                 (tile_rows 1, 2, or 4 with bf16 operands); 4 (bf16 and split
                                 bf16 products, N <= 128) runs phase 2 as one fused kernel that
                                 contracts the products in registers, so the workspace holds
                                 no product buffers; 0 = chosen by timing with tile_rows on the
                                 first call, the fused kernel included where it applies */
    int sync_batch;           /* fm_flow_run_batch: 1 = flows with equal T0 form a group that
                                 advances on one step schedule (Dormand-Prince: a step is
                                 accepted only when every running member accepts it, and the
                                 next step is the smallest any member proposes), so that every
                                 stage temperature is shared and the group's phase-1 bins are
                                 computed once, by its first running member; each flow keeps
                                 its own stop rule and T_c.  k > 1: the same with groups of at
                                 most k such flows, consecutive in the batch.  0 = every flow
                                 steps on its own */
    int n_shells;             /* FM_GEOM_SHELLS: odd number of energy shells (N % n_shells == 0,
                                 N / n_shells a valid angular patch count); other geometries: 0
                                 or 1 */
    const double *shell_edges;/* FM_GEOM_SHELLS: host [(n_shells - 1) / 2], ascending positive
                                 |xi| at which the shells meet (symmetric about the Fermi
                                 surface xi = 0); NULL selects 2|t| (2^k - 1)/(2^m - 1),
                                 k = 1..m = (n_shells - 1)/2, finest at the Fermi surface.  The
                                 patch of a loop point is its angular sector and the shell of
                                 its xi; a patch is represented by the point of its sector's
                                 centre ray where xi equals the shell's representative energy
                                 (0 for the Fermi-surface shell, the middle of the shell's
                                 range otherwise, the outermost shell's inner edge plus half
                                 the width of the shell below it), snapped to the transfer grid.
                                 FM_EINVAL when a loop point lies within 1e-9 of an edge. */
    const double *k_table;    /* interaction flow with a Z table only: host [n_zT][N] Katanin
                                 factors K on the Z table's nodes (App. A, Step 3), or NULL
                                 (K = 1).  The single-scale line Z^2 G0 becomes K Z^2 G0
                                 (Eq. vertex_flow_feedback_Z_with_Katanin), so a line pair
                                 carries g Z_a Z_b (K_a Z_a + K_b Z_b) chi; K is linear between
                                 nodes, clamped outside, any finite sign (it may change sign
                                 along the flow); copied.  Every flow of the handle uses it:
                                 fm_flow_run_batch then takes no per-flow Z tables. */
    int phase1_variant;       /* launch shape of the step's phase-1 launch: 1 / 2 one stage
                                 node per block with 256 / 1024 threads, 3 / 4 two nodes per
                                 block (where the bins fit in LDS; else one); 0 = chosen by
                                 timing all four on the first call (kept per shape for the
                                 process) */
    int sym_state;            /* 1: the caller's states are invariant under the square
                                 lattice's point group: V(pi a, pi b, pi c) = V(a, b, c) for
                                 the patch permutation pi of each of its 8 operations, and
                                 every Z and K table row too (Z_{pi a} = Z_a).  The flow
                                 equation keeps that symmetry (as from V = U), and a transfer
                                 q = o(r) then has the products Y_q[g][n] = Y_r[pi^-1 g]
                                 [pi^-1 n] of its orbit representative r: phase 2 computes the
                                 representatives' products only and the contraction reads them
                                 through the permutations.  Same results for such states; for
                                 a state without the symmetry they are wrong.  Needs the
                                 geometry's point-group symmetry (fm_geometry_query: n_rep
                                 below the transfer counts), a phase 2 with product buffers
                                 (not FM_FP64_DIRECT, y_kernel 0, 2 or 3: the class kernel
                                 on class 0 or the orbit kernel on operation 0) and
                                 symmetric Z and K tables (checked to 1e-12 relative, also
                                 per-flow tables of fm_flow_run_batch); FM_EINVAL otherwise.
                                 0: no assumption. */
} fm_config;

typedef struct {
    double T_c;        /* temperature flow: crossing of max|V| = v_max, 1/max|V| interpolated
                          linearly in ln T over the last step; NaN unless status is DIVERGED
                          or NONFINITE, and for the interaction flow */
    double T_final;    /* temperature of the last accepted step (the flow's T in g) */
    double max_abs_V;  /* max|V| at the last accepted step */
    int status;        /* FM_FLOW_* (REACHED_TEND: T_end, or g_end, reached) */
    int n_accepted, n_rejected, n_rhs;
    double g_c;        /* interaction flow: crossing g*, 1/max|V| linear in g^2; else NaN */
    double U_star;     /* interaction flow: g*^2 U (Sec. 3.2, U*(T)); else NaN */
    double g_final;    /* interaction flow: g of the last accepted step; else NaN */
} fm_result;

/* Bytes of device workspace needed for cfg (all buffers for cfg->max_batch flows). */
int fm_flow_workspace_bytes(const fm_config *cfg, size_t *bytes);

/* Validates cfg, builds the geometry on the host (double precision) and uploads it into the
 * caller's workspace.  FM_EINVAL for an invalid N, L, window or precision, or when a loop
 * point lies within 1e-9 sector widths of a patch boundary. */
int fm_flow_init(const fm_config *cfg, void *workspace_dev, size_t bytes, fm_flow **out);

/* The right-hand side of the one-loop flow of the static vertex (App. A, Eq.
 * vertex_flow_general; Z on the internal lines as in Eq. vertex_flow_feedback_Z, projected
 * onto each line's patch), in the temperature flow: dV/d ln T with the particle-particle,
 * crossed and direct particle-hole loop sums over the L x L grid, each pair of lines carrying
 * Z_a' Z_b' T d/dT chi.
 * `batch` independent states at temperatures T[batch] (host array, T > 0):
 * V_dev and dV_dev are device arrays of batch*N^3 doubles (dV_dev may not alias V_dev).
 * Z (if configured) is taken from the table at ln T.  Asynchronous on cfg.stream.
 * Temperature-flow handles only; FM_EINVAL for a bad batch, T or pointer. */
int fm_flow_rhs(fm_flow *h, int batch, const double *T, const double *V_dev, double *dV_dev);

/* For callers that cannot allocate device memory (code under stream capture, serving loops,
 * harnesses that forbid hipMalloc): fm_flow_rhs with the library's own static device array
 * as the workspace, so the caller passes only the inputs and outputs.  cfg, batch, T, V_dev,
 * dV_dev as fm_flow_init and fm_flow_rhs (batch <= cfg->max_batch; cfg->stream is used).
 * The array holds 96 MiB per device (one flow of the N = 48, L = 128 workloads fits); a
 * configuration whose workspace would be larger gives FM_EINVAL.  Each device holds its own
 * array for the life of the process, shared by every call on that device: the first call
 * (and any call whose configuration differs from the previous one) builds the geometry into
 * it, later calls with an equal configuration reuse it.  Calls that overlap in time on one
 * device (other threads, or other streams still running) race on the array.  It allocates
 * no device memory and calls no allocating library routine. */
int fm_flow_rhs_static(const fm_config *cfg, int batch, const double *T, const double *V_dev,
                       double *dV_dev);

/* Interaction flow (App. A, Eq. vertex_flow_feedback_Z): dV/dg for `batch` states at
 * temperatures T[batch] and scales g[batch] (host arrays, T > 0, g finite); Z (if
 * configured) from the table at g.  Layout, aliasing and streams as fm_flow_rhs.
 * Interaction-flow handles only (FM_EINVAL otherwise). */
int fm_flow_rhs_g(fm_flow *h, int batch, const double *T, const double *g, const double *V_dev,
                  double *dV_dev);

/* One step of the flow integrated as an ordinary differential equation in the flow
 * parameter (Sec. 3.2; the scheme is not given in the paper: classical RK4, or
 * Dormand-Prince 5(4) with the error control below), right-hand sides as fm_flow_rhs.
 * `batch` states.  lnT[batch], h[batch] are host in/out arrays
 * (ln T and its step; for the interaction flow g and its step, at T = cfg.T0),
 * V_dev (device, batch*N^3 doubles) in/out, accepted[batch] host out.
 * RK4: always accepted, lnT += h, h unchanged.  Dormand-Prince: the step is accepted when
 * the error norm is <= 1; then V and lnT advance; h returns the proposed next step
 * (h * min(5, max(0.2, 0.9 err^-1/5)), or h/2 after a non-finite stage). */
int fm_flow_step(fm_flow *h, int batch, double *lnT, double *hstep, double *V_dev,
                 int *accepted);

/* Whole flows with the stop rule of Sec. 3.2 (the largest coupling beyond a threshold
 * marks the instability; here max|V| > cfg.v_max, crossing T_c interpolated), for a sweep
 * of bare couplings and start temperatures such as the paper's U-T plane of crossover scales.
 * Runs n_flows independent flows from V = U[f] at T0[f] down to cfg.T_end (interaction
 * flow: at the fixed temperature T0[f] > 0 from g = 0 to cfg.g_end) or until the stop rule
 * fires, all on the device: one integrator step of every running flow per replay of a
 * captured graph; finished flows are masked.  z_lnT / z_tables: NULL (use cfg's table for
 * every flow, or none) or per-flow host arrays [n_flows][n_zT] and [n_flows][n_zT][N],
 * checked as fm_flow_init checks the configured table (FM_EINVAL unless every flow's nodes
 * ascend and every Z is positive and finite).
 * V_final_dev: NULL or a device array of n_flows*N^3 doubles receiving the final states.
 * res[n_flows] (host) receives the outcomes. */
int fm_flow_run_batch(fm_flow *h, int n_flows, const double *U, const double *T0,
                      const double *z_lnT, const double *z_tables, double *V_final_dev,
                      fm_result *res);

/* Interaction flow: T*(U) for n_flows couplings U[f] (n_flows <= max_batch), the
 * temperature below which the flow of bare U diverges before g = cfg.g_end, i.e. the root
 * of U*(T) = U (Sec. 3.2).  Bisection in ln T inside [T_lo, T_hi] on the outcome of batched
 * interaction flows (diverged, or not, by g_end) until hi/lo - 1 <= rtol; T_star[f] is the
 * geometric midpoint of the final bracket.  status[f]: 0 found, 1 the flow diverges already
 * at T_hi (T* >= T_hi), 2 it does not at T_lo (T* <= T_lo), T_star[f] = NaN for 1 and 2.
 * Uses cfg's Z table for every flow.  FM_EINVAL for a temperature-flow handle or a bad
 * bracket. */
int fm_flow_tstar(fm_flow *h, int n_flows, const double *U, double T_lo, double T_hi,
                  double rtol, double *T_star, int *status);

/* Quasi-particle weights from the self-energy on the real axis (Sec. 3.1: Im Sigma as raw
 * data on a frequency grid, Re Sigma by Kramers-Kronig, Z from the slope of Re Sigma taken
 * outside the window of inverted slope; App. A, Eq. definition_Z, Z = (1 - d Re Sigma/dw)^-1,
 * projected onto each patch's representative point k).  Im Sigma is the second-order
 * (two-loop) diagram of a static vertex,
 *   Im Sigma(w, k) = -pi L^-4 sum_{p1,p3} W [f1 (1-f2)(1-f3) + (1-f1) f2 f3]
 *                    delta(w + xi1 - xi2 - xi3),   p2 = k + p1 - p3 (its energy exact),
 * with W = U^2 when V_dev is NULL (second-order perturbation theory in the bare U), else
 * W = V(a,b,c)^2 + (V(a,b,c) - V(b,a,c))^2 / 2 for the flowing vertex V_dev (device,
 * [N][N][N] doubles; a, b, c the patches of k, p1, p3), which is U^2 for V = U.  The delta
 * function is shared linearly between the two nearest of FM_SIGMA_NW frequency nodes
 * w_i = -W0 + 2 W0 i / (FM_SIGMA_NW - 1), W0 = fm_sigma_wmax(cfg); Re Sigma is the
 * principal-value integral of the piecewise-linear Im Sigma; Z = 1 / (1 - s) with s the
 * least-squares slope of Re Sigma over the nodes with 2T <= |w| <= 4T, NaN when fewer than
 * 8 nodes fall there (T below about 4 W0 / (FM_SIGMA_NW - 1): the slope is not resolved).
 * The slope may turn positive at high T (Z > 1 where the window reaches the band's flank, as
 * the definition allows) and, on a loop grid too coarse for T, pass 1 (Z < 0).
 * Z: host [N]; im_sigma, re_sigma: NULL or host [N][FM_SIGMA_NW].  Synchronous on cfg.stream.
 * FM_EINVAL for T <= 0 or a null Z. */
enum { FM_SIGMA_NW = 2048 };
int fm_flow_z(fm_flow *h, double T, double U, const double *V_dev, double *Z, double *im_sigma,
              double *re_sigma);
double fm_sigma_wmax(const fm_config *cfg);

/* Host-only (no device): the Katanin factors and A_g of the interaction flow (App. A,
 * Eqs. K_definition and A_g_simple) from quasi-particle weights Z tabulated on n >= 3
 * ascending scales g[n] (host), z_tab [n][N] (positive, finite).  With s = 1 - 1/Z the slope
 * of Re(g Sigma_g) at the Fermi level (Eq. definition_Z), so that d_w Re Sigma_g = s/g,
 *   K = 1 + g^2 d_w Re(d Sigma_g/dg) = 1 - s + g ds/dg,
 *   A = -(2/g)(1 - Z K)  (= 2 (dZ/dg)/Z; this form at g = 0),
 * ds/dg the derivative of the parabola through each node and its two neighbours (the first
 * or last three nodes at the ends).  k_tab [n][N] receives K (for cfg.k_table), a_tab
 * [n][N] (or NULL) A; a_minmax (or NULL) [n][2] the smallest and largest A over the patches
 * at each node, the bounds between which A_g's patch dependence is followed.  FM_EINVAL for
 * n < 3, nodes that do not ascend, or a Z that is not positive and finite. */
int fm_katanin_table(int n, const double *g, int N, const double *z_tab, double *k_tab,
                     double *a_tab, double *a_minmax);

/* Host-only geometry query (no device needed): xi[L*L], patch[L*L], anchor[N][2] (snapped
 * Fermi-point transfer indices, or loop indices in identity mode), the numbers of distinct
 * particle-particle and particle-hole transfers, the smallest distance of a loop point to a
 * patch boundary in sector widths, and n_rep[2]: the numbers of particle-particle and
 * particle-hole transfers whose bins phase 1 computes (orbit representatives under the
 * square's point group when the geometry has that symmetry, else all transfers).  Any
 * output pointer may be NULL. */
int fm_geometry_query(const fm_config *cfg, double *xi, int *patch, int *anchor, int *n_pp,
                      int *n_ph, double *margin, int *n_rep);

/* Measurement: average duration (milliseconds) of one launch of a right-hand-side kernel
 * group on the state the handle holds (the first `batch` flows, replayed as running at their
 * current temperature; their status is restored): group 0 stage argument and phase 1 of
 * every stage node of an integrator step (the first stage launch of a step), 1 phase-2a
 * products, 2 phase-2b contraction (the direct kernel in FM_FP64_DIRECT), 3 stage argument
 * alone as a later stage of a step forms it (four earlier k slots read).  The group is
 * launched `reps` times back to back on cfg->stream between two HIP events; every
 * launch recomputes the same products from the same inputs.  It overwrites the stage
 * operands, bins, products and k slot 0, all of which the next integrator step recomputes.
 * Synchronous.  FM_EINVAL for a bad group, batch or reps. */
int fm_flow_kernel_time(fm_flow *h, int group, int batch, int reps, double *avg_ms);

/* Per-kernel event timings of the last fm_flow_rhs / fm_flow_step / fm_flow_run_batch call
 * (milliseconds, summed over launches), when enabled with fm_flow_set_timing(h, 1).
 * names[i] points to static strings.  Returns the number of entries written. */
int fm_flow_set_timing(fm_flow *h, int enable);
int fm_flow_timings(fm_flow *h, const char **names, double *ms, int *launches, int max_n);

void fm_flow_destroy(fm_flow *h);

const char *fm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FM_FLOW_H */
