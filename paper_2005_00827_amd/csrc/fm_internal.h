// Internal declarations shared by the host driver and the gfx950 kernels of libfmflow.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fm_flow.h"

namespace fm {

// ------------------------------------------------------------------------------------
// Host geometry (double precision), see geometry.cpp.
// ------------------------------------------------------------------------------------
struct HostGeometry {
    int N = 0, L = 0, np = 0, identity = 0, pp_shift = 0;
    int nsec = 0;                    // angular sectors (N / n_shells; N for identity patches)
    std::vector<double> xi;          // [np] dispersion at each loop point
    std::vector<int> patch;          // [np] patch of each loop point
    std::vector<int> anchor;         // [N][2] transfer-grid index of each patch's Fermi point
    std::vector<double> kpt;         // [N][2] each patch's representative point (not snapped)
    std::vector<int> q_pp, q_ph;     // distinct transfers, flat index mx + L*my
    std::vector<int> map_pp;         // [a*N+b] -> index into q_pp of k_a + k_b
    std::vector<int> map_cr;         // [b*N+c] -> index into q_ph of k_c - k_b
    std::vector<int> map_d;          // [a*N+c] -> index into q_ph of k_a - k_c
    double margin = 0.5;             // smallest distance to a sector boundary (sectors)

    // Point-group reduction.  The eight operations o = 4*swap + 2*flip_x + flip_y act on
    // loop indices, transfer indices and (through perm) patch labels.  Bins of transfer
    // q = o(r) are those of its representative r with both patch labels mapped by o^-1.
    bool sym = false;                // the geometry is invariant under all eight
    std::vector<int> pinv;           // [8][N] patch permutation of o^-1
    bool inv_ok = false;             // the geometry is invariant under k -> -k alone
    std::vector<int> inv_perm;       // [N] patch permutation of k -> -k
    std::vector<int> rep_pp, rep_ph; // representative transfers (flat index)
    std::vector<int> qrep_pp, qg_pp; // [nP] representative index and operation
    std::vector<int> qrep_ph, qg_ph; // [nD]
    std::vector<int> perm;           // [8][N] patch permutation of o (pinv is its inverse)
    // Transfers are ordered by (operation, representative); cls_*[o] .. cls_*[o+1] are the
    // transfers obtained with operation o.
    std::vector<int> cls_pp, cls_ph; // [9]
    // Orbit kernel: representatives in 16-row tiles per channel kind (pp tiles first), the
    // transfer of each (tile, operation, row) and each tile's operation set; patches in
    // groups of 8, orbit by orbit (-1 pads).
    std::vector<int> orb_rows;       // [16 (nt0 + nt1)] representative or -1
    std::vector<int> orb_q;          // [(nt0 + nt1) * 8 * 16] transfer or -1
    std::vector<int> orb_mask;       // [nt0 + nt1] bit o: some row has a transfer by o
    int orb_nt[2] = {0, 0};
    std::vector<int> porder;         // [8 nG]
    // Output pairs grouped by transfer (CSR): pp pairs (a,b), crossed (b,c), direct (a,c),
    // each packed as x*N + y.
    std::vector<int> pp_off, pp_pairs, cr_off, cr_pairs, d_off, d_pairs;
    // Phase-2b work items: (transfer, first pair) with at most 8 pairs each, per channel
    std::vector<int> item_q, item_p0;
    std::vector<int> item_rec;       // [items][16]: transfer, pair count, channel, first pair, 8 pairs
    int n_items[3] = {0, 0, 0};
    // Fused phase 2: rows (transfer, up to kFusedPairs of its output pairs) per channel kind,
    // ordered by (operation, representative) like the transfers, each operation class padded
    // to whole blocks of kFusedRows rows (padding rows: transfer -1, no pairs); per block its
    // operation and first row.
    std::vector<int> fz_row;         // [rows] transfer or -1
    std::vector<int> fz_pair;        // [rows][kFusedPairs] packed pair or -1
    std::vector<int> fz_blk;         // [blocks][2] operation, first row
    int fz_nblk[3] = {0, 0, 0};      // blocks of the pp, crossed and direct kinds, in order
    // Phase 2b of symmetric states on the matrix cores: per channel kind and representative
    // r, records of 4 + kSymPairs ints: r, pair count, kind, 0, then (pair * 8 + o) of the
    // transfers q = o(r) of r's orbit (-1 pads)
    std::vector<int> sym_rec;
    int n_sym_items[3] = {0, 0, 0};
};

// Fused phase 2: output pairs per row and rows per block (16-row tiles, one per wavefront).
constexpr int kFusedPairs = 4;
constexpr int kFusedRows = 128;
// Matrix-core phase 2b of symmetric states: output pairs per work item (4 wavefronts of
// 16-row tiles) of one representative's orbit.
constexpr int kSymPairs = 64;

bool build_geometry(const fm_config& cfg, HostGeometry& g, std::string& err);

// The message fm_last_error() returns on the calling thread.
void set_last_error(const std::string& msg);

// ------------------------------------------------------------------------------------
// Device-side per-flow integrator state (double precision throughout).
// ------------------------------------------------------------------------------------
// s is ln T for the temperature flow and -g for the interaction flow, so that both run
// towards smaller s; dV/ds = -dV/dg in the latter.
struct FlowState {
    double lnT;      // accepted s (ln T, or -g)
    double h;        // proposed next step
    double ht;       // step being attempted (h, or clamped to reach ln T_end)
    double lnT_end;  // -inf for free stepping
    double m;        // max|V| at lnT
    double lnTc;     // crossing of the stop threshold
    double err;      // error norm of the last attempt
    double hmin;     // smallest allowed |h|
    double s0;       // ln T0 (fixed-step grid origin)
    double atol;     // absolute error tolerance of this flow
    double Tfix;     // interaction flow: the flow's temperature
    double vmax;     // stop threshold on max|V| (v_max, or v_rel |U| in the interaction flow)
    double sp, mp;   // the accepted point before (lnT, m): s and max|V| (mp = 0: none yet)
    int status;      // FM_FLOW_*
    int accepted;    // outcome of the last attempt
    int n_acc, n_rej, n_rhs;
    int gflow;       // 1: interaction flow
    int bshare;      // 0: phase 1 bins this flow's own temperatures; else 1 + the flow whose
                     // bins it reads (flows on one step schedule share every stage temperature)
};

// Geometry as the kernels see it.
struct DevGeom {
    int N, L, np, nP, nD, NN;
    int nRp, nRd;          // representative transfers (pp, ph)
    const int* rep_pp;     // [nRp]
    const int* rep_ph;     // [nRd]
    const int* qrep_pp;    // [nP]
    const int* qg_pp;      // [nP]
    const int* qrep_ph;    // [nD]
    const int* qg_ph;      // [nD]
    const int* pinv;       // [8][N]
    const int* perm;       // [8][N], inverse of pinv
    int cls[2][9];         // transfer classes by operation: particle-particle, particle-hole
    const int* orb_rows;   // orbit kernel tables (see HostGeometry)
    const int* orb_q;
    const int* orb_mask;
    int orb_nt[2];
    const int* porder;
    int nG;                // patch groups of 8
    const int* pI;         // [N] patch permutation of k -> -k
    int inv_ok;            // pI is valid (k -> -k maps patches and dispersion onto themselves)
    int inv_rot;           // pI[a] = (a + N/2) mod N
    int gflow;             // interaction flow: bins of chi instead of T d/dT chi
    int lds_max;           // LDS bytes one work group may allocate on the device
    int sym;               // states invariant under the point group: products of
                           // representatives only, read through the permutations
    const int* pp_off; const int* pp_pairs;
    const int* cr_off; const int* cr_pairs;
    const int* d_off;  const int* d_pairs;
    const int* item_q; const int* item_p0;
    const int* item_rec;   // [items][16] (one 64-byte record per phase-2b work item)
    int n_items[3];
    const int* fz_row;     // fused phase 2 tables (see HostGeometry)
    const int* fz_pair;
    const int* fz_blk;
    int fz_nblk[3];
    const int* sym_rec;    // matrix-core phase 2b of symmetric states (see HostGeometry)
    int n_sym_items[3];
    const double* xi;      // [np]
    const int* patch;      // [np]
    const int2* xp;        // [np] (xi as float bits, patch): single-precision phase 1
    const int* q_pp;       // [nP]
    const int* q_ph;       // [nD]
    const int* map_pp;     // [NN]
    const int* map_cr;     // [NN]
    const int* map_d;      // [NN]
};

// LDS bytes of one phase-1 bin matrix held by a work group: N rows of stride N + 1 (R values).
inline size_t bins_lds_bytes(int N, size_t rs) { return static_cast<size_t>(N) * (N + 1) * rs; }

// Per-flow Z tables, and the Katanin factors on the same nodes (interaction flow).
struct DevZ {
    int n;                 // nodes (0: Z = 1)
    const double* lnT;     // [B][n]
    const double* tab;     // [B][n][N]
    const double* ktab;    // [B][n][N] K, or nullptr (K = 1)
};

// Integrator constants for one stage.
struct StageCoef {
    double c;              // node
    double a[7];           // coupling to previous stages
    int ns;                // number of previous stages used
};

// Stage nodes whose phase-1 bins one stage launch computes: every distinct node of an
// integrator step (bins depend on the stage temperature only, not on V), one bin set each.
struct BinPlan {
    int n;                 // sets (0: the launch forms the stage argument only)
    double c[6];           // node of each set
};

// Values of padding after each bin buffer: phase 2a reads a row up to 4 KE <= 128 values.
constexpr size_t kBinPad = 256;

// Device buffers carved out of the caller's workspace.
struct Buffers {
    // geometry
    double* xi; int* patch; int2* xp; int* q_pp; int* q_ph; int* map_pp; int* map_cr; int* map_d;
    // per flow
    FlowState* fs;
    double* z_lnT; double* z_tab;      // [B][nz], [B][nz][N]
    double* k_tab;                     // [B][nz][N] Katanin factors, or nullptr
    double* T_stage;                   // [B]
    double* Z_stage;                   // [B][2][N]: Z, then W = K Z (W = Z without K)
    double* zw_stage;                  // [B][2]: line-pair factor Z_a Z_b (al + be (W_a + W_b))
    int* rep_pp; int* rep_ph; int* qrep_pp; int* qg_pp; int* qrep_ph; int* qg_ph; int* pinv;
    int* perm;
    int* orb_rows; int* orb_q; int* orb_mask; int* porder;
    int* pI;
    int* pp_off; int* pp_pairs; int* cr_off; int* cr_pairs; int* d_off; int* d_pairs;
    int* item_q; int* item_p0; int* item_rec; int* sym_rec;
    int* fz_row; int* fz_pair; int* fz_blk;
    void* bins;                        // [S][B][nRp + nRd][NN] real, representative transfers
    void* binsT;                       // [S][B][nRd][NN] real, particle-hole bins transposed
    int nbset;                         // S: bin sets (stage nodes of one step)
    size_t bins_bytes, binsT_bytes;    // with kBinPad values of zeroed padding each
    void* y1; void* y2; void* y3; void* y4;  // [B][n][NN] real (bf16 when y_bf16)
    int y_bf16;                        // bf16 operands: the products Y are stored as bf16
    int y_split;                       // split-bf16 operands (f32 products)
    void* v0; void* va; void* vc;      // operands [B][N^3] real
    void* k;                           // [7][B][3][N^3] real: per stage, flow and channel (parts in phase-2b order)
    void* ksum;                        // [7][B][N^3] real: a slot's three parts summed, V order
    double* V; double* Vnew;           // [B][N^3] state, candidate
    double* part;                      // [B][nblk][2] reduction partials
    double* wtab;                      // direct mode: [B][nP+nD][np]
    double* U;                         // [B] bare couplings of run_batch
    double* kpt;                       // [N][2] patch representative points (self-energy)
    double* sig_f;                     // [L^2] Fermi factors of the self-energy's temperature
    double* sig_hist; double* sig_im; double* sig_re;   // [N][kSigmaW]
    double* sig_Z;                     // [N]
    int* grp_members;                  // [B] flows of run_batch's step-sharing groups, by group
    int* grp_off;                      // [B + 1] group g: members grp_off[g] .. grp_off[g+1]
    int nblk;                          // reduction blocks per flow
    int bstride;                       // flows per buffer (max_batch)
    int ph1var;                        // phase-1 launch shape: 0 by rule, 1..4 fixed (threads
                                       // 256 or 1024, one or two stage nodes per block)
};

// Dormand-Prince error weights (5th minus embedded 4th order).
struct ErrWeights {
    double e[7];
};

// Launchers (kernels.hip).  `dbl` selects the double-precision instantiation, nf is the
// number of flows launched; buffers are strided by b.bstride flows.
// Stage argument and operand layouts; with bins, phase 1 of the stage in the same launch.
// bp.n > 0: phase 1 of every node of bp in the same launch, into bin sets 0 .. bp.n-1.
void launch_stage(hipStream_t s, bool dbl, const DevGeom& g, const DevZ& z, const Buffers& b,
                  int nf, const StageCoef& sc, const BinPlan& bp, int write_new,
                  const double* Vbase);
// Largest useful tiles per wavefront of the operation-class kernel: all tiles of the
// largest class in the 4 waves of one block.
int y_max_tpw(const DevGeom& g);
// The buffers with bin set `set` in place of set 0 (phase 2a reads the bins of its stage).
Buffers with_bin_set(const Buffers& b, const DevGeom& g, bool dbl, int set);
// mma: 0 VALU, 1 f32 matrix cores, 2 bf16 matrix cores, 3 split-bf16 matrix cores (single
// precision only, N <= 128);
// tpw: row tiles per wavefront on matrix cores (1, 2, 4; 0 = by size);
// yvar: matrix-core kernel, 1 per-row gather of permuted bins, 2 operation classes (the
// permutation applied to the staged operand), 3 orbits (each representative's bin row read
// once, every operation applied to it in the block)
void launch_y(hipStream_t s, bool dbl, const DevGeom& g, const Buffers& b, int nf, unsigned ch,
              int mma, int tpw, int yvar);
// Largest useful tiles per wavefront of the per-row kernel.
int y_rows_max_tpw(const DevGeom& g);
// Largest useful tiles per wavefront of the orbit kernel (1, 2, or 4 with bf16 operands).
int y_orb_max_tpw(const DevGeom& g, int mma);
void launch_contract(hipStream_t s, bool dbl, const DevGeom& g, const Buffers& b, int nf,
                     unsigned ch, int slot);
// Fused phase 2 (FM_FP32_BF16MFMA, FM_FP32_BF16X3 with N <= 128): products and contraction
// in one launch into k slot `slot`, with the bins of b's set.
void launch_fused(hipStream_t s, const DevGeom& g, const Buffers& b, int nf, unsigned ch,
                  int slot, int mma);
void launch_wtable(hipStream_t s, const DevGeom& g, const Buffers& b, int nf);
void launch_direct(hipStream_t s, const DevGeom& g, const Buffers& b, int nf, unsigned ch,
                   int slot);
void launch_k_to_f64(hipStream_t s, bool dbl, const Buffers& b, int nf, int N, int slot,
                     double* out);
void launch_fill_u(hipStream_t s, const Buffers& b, int nf, size_t N3, const double* U);
void launch_rk4_update(hipStream_t s, bool dbl, const Buffers& b, int nf, int N, double* V);
void launch_dopri_err(hipStream_t s, bool dbl, const Buffers& b, int nf, int N,
                      const double* V, double rtol, const ErrWeights& ew);
// Accept/reject and the stop test against each flow's own threshold (FlowState::vmax).
void launch_finish(hipStream_t s, const Buffers& b, int nf, int rk45, int fixed_steps);
// The same for groups of flows on one step schedule (members[off[g] .. off[g+1]) of group g):
// a step is accepted when every running member accepts it, and the group's next step is the
// smallest any member proposes; the first running member bins for the group (its bins are
// recomputed every step unless `rebind` is 0, as for the interaction flow's fixed bins).
void launch_finish_sync(hipStream_t s, const Buffers& b, int ngroups, int max_members, int rk45,
                        int fixed_steps, int rebind);
void launch_commit(hipStream_t s, bool dbl, const Buffers& b, int nf, size_t N3, double* V);
void launch_copy(hipStream_t s, const double* from, double* to, size_t n);

// Quasi-particle weight provider (sigma.hip): frequency nodes of the real-axis self-energy.
constexpr int kSigmaW = 2048;
struct SigmaArgs {
    int N, L;
    double t, tp, mu, T, U;
    double w0, dw;            // nodes -w0 + dw i, i < kSigmaW
    const double* xi;         // [L^2]
    const int* patch;         // [L^2]
    const double* kpt;        // [N][2] representative points
    double* f;                // [L^2] Fermi factors at T (filled by the launch)
};
// Im Sigma, Re Sigma [N][kSigmaW] and Z [N] at temperature s.T; V = null: bare U^2 weights.
void launch_sigma(hipStream_t st, const SigmaArgs& s, const double* V, double* hist, double* im,
                  double* re, double* Z);

}  // namespace fm
