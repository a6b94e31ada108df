// Host side of libfmflow: the C ABI of include/fm_flow.h, workspace layout and the integrator
// driver.  Every step of the flow runs in the kernels of kernels.hip; this file only carves
// the caller's workspace, uploads the geometry and sequences launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "fm_internal.h"

using namespace fm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(FM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Classical RK4 and Dormand & Prince (1980) RK5(4)7M in s = ln T.
const double kRK4C[4] = {0.0, 0.5, 0.5, 1.0};
const double kRK4A[4][3] = {{0, 0, 0}, {0.5, 0, 0}, {0, 0.5, 0}, {0, 0, 1.0}};

const double kDPC[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
const double kDPA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
const double kDPE[7] = {71.0 / 57600, 0.0, -71.0 / 16695, 71.0 / 1920, -17253.0 / 339200,
                        22.0 / 525, -1.0 / 40};

StageCoef rk4_stage(int s) {
    StageCoef c{};
    c.c = kRK4C[s];
    c.ns = s;
    for (int l = 0; l < s; ++l) c.a[l] = kRK4A[s][l];
    return c;
}

StageCoef dp_stage(int s) {
    StageCoef c{};
    c.c = kDPC[s];
    c.ns = s;
    for (int l = 0; l < s; ++l) c.a[l] = kDPA[s][l];
    return c;
}

// Bins of one integrator step: phase 1 depends on the stage temperature only, so the first
// stage launch of a step bins every distinct node of the step (Dormand-Prince: 1/5, 3/10,
// 4/5, 8/9, 1 for stages 2-7, whose last two share c = 1; RK4: 0, 1/2, 1), and each stage's
// phase 2a reads the set of its node.
struct StepPlan {
    BinPlan bp{};
    int set[7] = {0, 0, 0, 0, 0, 0, 0};
    int first = 0;           // the stage whose launch computes the bins
};

StepPlan step_plan(bool rk45) {
    StepPlan p;
    p.first = rk45 ? 1 : 0;
    const int last = rk45 ? 7 : 4;
    for (int s = p.first; s < last; ++s) {
        const double c = rk45 ? kDPC[s] : kRK4C[s];
        int k = 0;
        while (k < p.bp.n && p.bp.c[k] != c) ++k;
        if (k == p.bp.n) p.bp.c[p.bp.n++] = c;
        p.set[s] = k;
    }
    return p;
}

// One node (the stage temperature of a lone right-hand side or a step's first stage).
const BinPlan kOneNode{1, {0.0}};
const BinPlan kNoBins{0, {0.0}};

struct Layout {
    size_t off = 0;
    char* base = nullptr;
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~static_cast<size_t>(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// Phase 2 as one fused kernel is possible for bf16 or split-bf16 products at N <= 128;
// y_kernel 4 asks for it alone (and the workspace then holds no product buffers), y_kernel 0
// lets the tuner choose between it and the two-kernel path by timing.
bool fusable(const fm_config& c) {
    return (c.precision == FM_FP32_BF16MFMA || c.precision == FM_FP32_BF16X3) && c.N <= 128 &&
           !c.sym_state;
}

// Rows of a [n][N] table that are invariant under the point group's patch permutations
// (perm: [8][N]), to 1e-12 relative.
bool rows_symmetric(const std::vector<int>& perm, const double* tab, int n, int N) {
    for (int i = 0; i < n; ++i) {
        const double* t = tab + static_cast<size_t>(i) * N;
        for (int o = 1; o < 8; ++o)
            for (int a = 0; a < N; ++a) {
                const double x = t[a], y = t[perm[static_cast<size_t>(o) * N + a]];
                if (!(std::fabs(x - y) <= 1e-12 * std::max(1.0, std::fabs(x)))) return false;
            }
    }
    return true;
}
bool fused_phase2(const fm_config& c) { return fusable(c) && c.y_kernel == 4; }

// sym_state: the geometry is invariant under the point group, and the representatives' own
// transfers (operation 0) lead each kind's transfer list in representative order (transfer r
// holds representative r's products); the configured Z and K tables are invariant too.
bool sym_ok(const fm_config& c, const HostGeometry& hg, std::string& why) {
    if (!c.sym_state) return true;
    bool lead = hg.sym;
    for (int k = 0; k < 2 && lead; ++k) {
        const std::vector<int>& qr = k == 0 ? hg.qrep_pp : hg.qrep_ph;
        const std::vector<int>& qg = k == 0 ? hg.qg_pp : hg.qg_ph;
        const size_t nr = k == 0 ? hg.rep_pp.size() : hg.rep_ph.size();
        for (size_t r = 0; r < nr && lead; ++r) lead = qr[r] == static_cast<int>(r) && qg[r] == 0;
    }
    if (!lead) { why = "sym_state needs a geometry invariant under the point group"; return false; }
    if (c.n_zT > 0 && (!rows_symmetric(hg.perm, c.z_table, c.n_zT, c.N) ||
                       (c.k_table && !rows_symmetric(hg.perm, c.k_table, c.n_zT, c.N)))) {
        why = "sym_state needs Z and K tables invariant under the point group";
        return false;
    }
    return true;
}

int resolve(const fm_config* in, fm_config& c, std::string& why) {
    if (!in) { why = "null config"; return FM_EINVAL; }
    c = *in;
    if (c.flow != FM_FLOW_TEMPERATURE && c.flow != FM_FLOW_INTERACTION) { why = "bad flow"; return FM_EINVAL; }
    if (c.flow == FM_FLOW_INTERACTION) {
        if (!(c.T0 > 0.0) || !std::isfinite(c.T0)) { why = "interaction flow needs T0 > 0"; return FM_EINVAL; }
        if (c.g_end == 0.0) c.g_end = 1.0;
        if (!(c.g_end > 0.0) || !std::isfinite(c.g_end)) { why = "g_end must be positive"; return FM_EINVAL; }
    } else if (!(c.T0 > c.T_end) || !(c.T_end > 0.0)) {
        why = "need T0 > T_end > 0";
        return FM_EINVAL;
    }
    if (c.integrator != FM_RK4_FIXED && c.integrator != FM_RK45_DOPRI) { why = "bad integrator"; return FM_EINVAL; }
    if (c.integrator == FM_RK4_FIXED && c.n_steps < 1) { why = "RK4 needs n_steps >= 1"; return FM_EINVAL; }
    if (c.precision < FM_FP64 || c.precision > FM_FP32_BF16X3) { why = "bad precision"; return FM_EINVAL; }
    if (c.max_batch < 1) { why = "max_batch must be >= 1"; return FM_EINVAL; }
    if (c.n_zT < 0 || (c.n_zT > 0 && (!c.z_lnT || !c.z_table))) { why = "bad Z table"; return FM_EINVAL; }
    if (c.k_table && (c.flow != FM_FLOW_INTERACTION || c.n_zT < 1)) {
        why = "a Katanin table needs the interaction flow and a Z table's nodes";
        return FM_EINVAL;
    }
    if (c.k_table)
        for (size_t i = 0; i < static_cast<size_t>(c.n_zT) * c.N; ++i)
            if (!std::isfinite(c.k_table[i])) { why = "Katanin factors must be finite"; return FM_EINVAL; }
    for (int i = 1; i < c.n_zT; ++i)
        if (!(c.z_lnT[i] > c.z_lnT[i - 1])) { why = "Z nodes must ascend"; return FM_EINVAL; }
    // the relative tolerance must not ask for more than the right-hand side resolves:
    // bf16 operands carry about 3 significant digits, so their default is 1e-4
    if (c.rtol <= 0.0) c.rtol = c.precision == FM_FP32_BF16MFMA ? 1e-4 : 1e-6;
    if (c.v_max <= 0.0) c.v_max = 20.0;
    if (c.v_rel <= 0.0) c.v_rel = 100.0;
    if (c.channels == 0) c.channels = FM_CH_ALL;
    if (c.channels & ~7u) { why = "bad channel mask"; return FM_EINVAL; }
    if (c.tile_rows < 0) { why = "tile_rows must be >= 0"; return FM_EINVAL; }
    // the bf16 matrix-core products stage a whole operand row (N values) per lane group;
    // there is no bf16 path beyond that width (FP32 runs phase 2a on the vector units there)
    if ((c.precision == FM_FP32_BF16MFMA || c.precision == FM_FP32_BF16X3) && c.N > 128) {
        why = "bf16 and split-bf16 precisions support N <= 128";
        return FM_EINVAL;
    }
    if (c.y_kernel < 0 || c.y_kernel > 4) { why = "y_kernel must be 0 .. 4"; return FM_EINVAL; }
    if (c.phase1_variant < 0 || c.phase1_variant > 4) { why = "phase1_variant must be 0 .. 4"; return FM_EINVAL; }
    if (c.y_kernel == 4 && !fused_phase2(c)) {
        why = "y_kernel 4 (fused phase 2) needs bf16 or split-bf16 products and N <= 128";
        return FM_EINVAL;
    }
    if (c.sync_batch < 0) { why = "sync_batch must be >= 0"; return FM_EINVAL; }
    if (c.sym_state != 0 && c.sym_state != 1) { why = "sym_state must be 0 or 1"; return FM_EINVAL; }
    if (c.sym_state && (c.precision == FM_FP64_DIRECT || c.y_kernel == 1 || c.y_kernel == 4)) {
        why = "sym_state needs product buffers from the class or orbit kernel (not FM_FP64_DIRECT, y_kernel 0, 2 or 3)";
        return FM_EINVAL;
    }
    return FM_OK;
}

}  // namespace

struct fm_flow {
    fm_config cfg{};
    HostGeometry hg;
    DevGeom g{};
    DevZ z{};
    Buffers b{};
    hipStream_t stream = nullptr;      // caller's stream (may be null)
    hipStream_t own = nullptr;         // capture stream for graphs when the caller's is null
    bool dbl = false, direct = false, fused = false;
    size_t N3 = 0;
    std::vector<double> zlnT, ztab;    // configured table (host copy)
    std::vector<double> ktab;          // configured Katanin factors on the same nodes, or empty
    std::vector<FlowState> hfs;
    // phase-2a kernel variant and row tiles per wavefront (cfg.y_kernel, cfg.tile_rows, or
    // tuned for tuned_nf flows)
    int tpw = 0, yvar = 1, tuned_nf = -1;
    int ph1_nf = -1;                   // flows the phase-1 launch shape was timed for
    // graphs of one integrator step, keyed by the number of flows captured and the
    // step-sharing groups (count, largest)
    hipGraphExec_t step_exec = nullptr;
    int step_nf = -1, step_ng = -1, step_gmax = -1;
    // run_batch's step-sharing groups (0: every flow steps on its own)
    int ngroups = 0, gmax = 0;
    // timings
    bool timing = false;
    std::vector<hipEvent_t> ev;
    std::vector<std::pair<int, int>> ev_use;  // (kernel id, event index of start; end = start + 1)
    int ev_last = -1;                  // event ending the last timed group, if nothing followed
    size_t ev_next = 0;                // next free event
    std::vector<int> ev_end;           // end event of each entry of ev_use
    double t_ms[16] = {0};
    int t_n[16] = {0};
};

namespace {

enum { T_STAGE, T_Y, T_CONTRACT, T_WTABLE, T_DIRECT, T_UPDATE, T_FINISH, T_STAGE_ONLY, T_COUNT };
const char* kTimerNames[T_COUNT] = {"stage_bins", "y", "contract", "wtable", "direct",
                                    "update", "finish", "stage"};

int carve(fm_flow& h, const fm_config& c, const HostGeometry& hg, char* base, size_t* bytes) {
    const int B = c.max_batch, N = c.N, np = hg.np;
    const size_t NN = static_cast<size_t>(N) * N, N3 = NN * N;
    const int nP = static_cast<int>(hg.q_pp.size()), nD = static_cast<int>(hg.q_ph.size());
    const bool dbl = c.precision == FM_FP64 || c.precision == FM_FP64_DIRECT;
    const bool direct = c.precision == FM_FP64_DIRECT;
    const size_t rs = dbl ? 8 : 4;
    const int nz = std::max(c.n_zT, 1);
    Layout L;
    L.base = base;
    Buffers& b = h.b;
    b.xi = L.take<double>(np);
    b.patch = L.take<int>(np);
    b.xp = L.take<int2>(np);
    b.q_pp = L.take<int>(nP);
    b.q_ph = L.take<int>(nD);
    b.map_pp = L.take<int>(NN);
    b.map_cr = L.take<int>(NN);
    b.map_d = L.take<int>(NN);
    const int nRp = static_cast<int>(hg.rep_pp.size()), nRd = static_cast<int>(hg.rep_ph.size());
    b.rep_pp = L.take<int>(nRp);
    b.rep_ph = L.take<int>(nRd);
    b.qrep_pp = L.take<int>(nP);
    b.qg_pp = L.take<int>(nP);
    b.qrep_ph = L.take<int>(nD);
    b.qg_ph = L.take<int>(nD);
    b.pinv = L.take<int>(8 * static_cast<size_t>(N));
    b.perm = L.take<int>(8 * static_cast<size_t>(N));
    b.orb_rows = L.take<int>(hg.orb_rows.size());
    b.orb_q = L.take<int>(hg.orb_q.size());
    b.orb_mask = L.take<int>(hg.orb_mask.size());
    b.porder = L.take<int>(hg.porder.size());
    b.pI = L.take<int>(N);
    b.pp_off = L.take<int>(nP + 1);
    b.pp_pairs = L.take<int>(NN);
    b.cr_off = L.take<int>(nD + 1);
    b.cr_pairs = L.take<int>(NN);
    b.d_off = L.take<int>(nD + 1);
    b.d_pairs = L.take<int>(NN);
    b.item_q = L.take<int>(hg.item_q.size());
    b.item_p0 = L.take<int>(hg.item_p0.size());
    b.item_rec = L.take<int>(hg.item_rec.size());
    b.sym_rec = L.take<int>(hg.sym_rec.size());
    b.fz_row = L.take<int>(hg.fz_row.size());
    b.fz_pair = L.take<int>(hg.fz_pair.size());
    b.fz_blk = L.take<int>(hg.fz_blk.size());
    b.fs = L.take<FlowState>(B);
    b.z_lnT = L.take<double>(static_cast<size_t>(B) * nz);
    b.z_tab = L.take<double>(static_cast<size_t>(B) * nz * N);
    b.k_tab = c.k_table ? L.take<double>(static_cast<size_t>(B) * nz * N) : nullptr;
    b.T_stage = L.take<double>(B);
    b.Z_stage = L.take<double>(static_cast<size_t>(B) * 2 * N);
    b.zw_stage = L.take<double>(2 * static_cast<size_t>(B));
    b.U = L.take<double>(B);
    b.kpt = L.take<double>(2 * static_cast<size_t>(N));
    b.sig_f = L.take<double>(np);
    b.sig_hist = L.take<double>(static_cast<size_t>(N) * kSigmaW);
    b.sig_im = L.take<double>(static_cast<size_t>(N) * kSigmaW);
    b.sig_re = L.take<double>(static_cast<size_t>(N) * kSigmaW);
    b.sig_Z = L.take<double>(N);
    b.grp_members = L.take<int>(B);
    b.grp_off = L.take<int>(static_cast<size_t>(B) + 1);
    // integrator reduction blocks per flow: one per 8 x 8 x 16 element tile, at most 512
    {
        const size_t nx = (static_cast<size_t>(N) + 7) / 8, nz = (static_cast<size_t>(N) + 15) / 16;
        b.nblk = static_cast<int>(std::min<size_t>(nx * nx * nz, 512));
    }
    b.part = L.take<double>(static_cast<size_t>(B) * b.nblk * 2);
    b.bstride = B;
    if (!direct) {
        // the interaction flow bins once per flow (T is fixed): one set
        const size_t S = c.flow == FM_FLOW_INTERACTION
                             ? 1 : static_cast<size_t>(step_plan(c.integrator == FM_RK45_DOPRI).bp.n);
        b.nbset = static_cast<int>(S);
        // padding: phase-2a row reads run up to kBinPad values past a row's end
        b.bins = L.take<char>((S * B * (nRp + nRd) * NN + kBinPad) * rs);
        b.binsT = L.take<char>((S * B * nRd * NN + kBinPad) * rs);
        b.bins_bytes = (S * B * (nRp + nRd) * NN + kBinPad) * rs;
        b.binsT_bytes = (S * B * nRd * NN + kBinPad) * rs;
        // the products of bf16 operands are stored as bf16 (the same 8-bit significand); the
        // fused phase 2 keeps them in registers and needs no buffers for them
        b.y_bf16 = c.precision == FM_FP32_BF16MFMA ? 1 : 0;
        b.y_split = c.precision == FM_FP32_BF16X3 ? 1 : 0;
        const size_t ys = b.y_bf16 ? 2 : rs;
        const bool fz = fused_phase2(c);
        b.y1 = fz ? nullptr : L.take<char>(static_cast<size_t>(B) * nP * NN * ys);
        b.y2 = fz ? nullptr : L.take<char>(static_cast<size_t>(B) * nD * NN * ys);
        b.y3 = fz ? nullptr : L.take<char>(static_cast<size_t>(B) * nD * NN * ys);
        b.y4 = fz ? nullptr : L.take<char>(static_cast<size_t>(B) * nD * NN * ys);
        b.wtab = nullptr;
    } else {
        b.bins = b.binsT = b.y1 = b.y2 = b.y3 = b.y4 = nullptr;
        b.y_bf16 = 0;
        b.y_split = 0;
        b.bins_bytes = b.binsT_bytes = 0;
        b.nbset = 0;
        b.wtab = L.take<double>(static_cast<size_t>(B) * (nP + nD) * np);
    }
    b.v0 = L.take<char>(static_cast<size_t>(B) * N3 * rs);
    b.va = L.take<char>(static_cast<size_t>(B) * N3 * rs);
    b.vc = L.take<char>(static_cast<size_t>(B) * N3 * rs);
    b.k = L.take<char>(7 * 3 * static_cast<size_t>(B) * N3 * rs);
    b.ksum = L.take<char>(7 * static_cast<size_t>(B) * N3 * rs);
    b.V = L.take<double>(static_cast<size_t>(B) * N3);
    b.Vnew = L.take<double>(static_cast<size_t>(B) * N3);
    *bytes = L.off + 256;
    return FM_OK;
}

// Phase-2a product mode of a precision: 0 vector units (double), 1 f32 matrix cores, 2 bf16,
// 3 split bf16.
int mma_mode(int precision) {
    switch (precision) {
        case FM_FP32: return 1;
        case FM_FP32_BF16MFMA: return 2;
        case FM_FP32_BF16X3: return 3;
        default: return 0;
    }
}

// Timed launch group: records events around `fn` when timing is on.  Back-to-back groups
// share one event (the end of one is the start of the next), so an interval holds one
// event record and matches a profiler's duration of serialized kernels.  Untimed work
// between groups must call untimed() first.
template <typename F>
void timed(fm_flow* h, int id, F&& fn) {
    if (!h->timing) { fn(); return; }
    auto ev_at = [&](size_t i) -> bool {
        while (h->ev.size() <= i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return false;
            h->ev.push_back(e);
        }
        return true;
    };
    int start = h->ev_last;
    if (start < 0) {
        start = static_cast<int>(h->ev_next);
        if (!ev_at(start)) { fn(); return; }
        (void)hipEventRecord(h->ev[start], h->stream);
        ++h->ev_next;
    }
    const int end = static_cast<int>(h->ev_next);
    if (!ev_at(end)) { fn(); h->ev_last = -1; return; }
    fn();
    (void)hipEventRecord(h->ev[end], h->stream);
    ++h->ev_next;
    h->ev_use.emplace_back(id, start);
    h->ev_end.push_back(end);
    h->ev_last = end;
}
void untimed(fm_flow* h) { h->ev_last = -1; }

void collect_timings(fm_flow* h) {
    if (!h->timing || h->ev_use.empty()) { h->ev_last = -1; h->ev_next = 0; return; }
    (void)hipStreamSynchronize(h->stream);
    for (size_t k = 0; k < h->ev_use.size(); ++k) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->ev[h->ev_use[k].second], h->ev[h->ev_end[k]]) == hipSuccess) {
            h->t_ms[h->ev_use[k].first] += ms;
            h->t_n[h->ev_use[k].first] += 1;
        }
    }
    h->ev_use.clear();
    h->ev_end.clear();
    h->ev_last = -1;
    h->ev_next = 0;
}

// One right-hand-side evaluation of the current stage operands into k slot `slot`, with the
// stage's bins in set `set`.
void rhs_launch(fm_flow* h, int nf, int slot, int set) {
    const unsigned ch = h->cfg.channels;
    if (h->direct) {
        timed(h, T_WTABLE, [&] { launch_wtable(h->stream, h->g, h->b, nf); });
        timed(h, T_DIRECT, [&] { launch_direct(h->stream, h->g, h->b, nf, ch, slot); });
        return;
    }
    const int mma = mma_mode(h->cfg.precision);
    const Buffers bs = with_bin_set(h->b, h->g, h->dbl, set);
    if (h->fused) {
        timed(h, T_Y, [&] { launch_fused(h->stream, h->g, bs, nf, ch, slot, mma); });
        return;
    }
    timed(h, T_Y, [&] { launch_y(h->stream, h->dbl, h->g, bs, nf, ch, mma, h->tpw, h->yvar); });
    timed(h, T_CONTRACT, [&] { launch_contract(h->stream, h->dbl, h->g, h->b, nf, ch, slot); });
}

void stage_launch(fm_flow* h, int nf, const StageCoef& sc, const BinPlan& bp, int write_new,
                  const double* Vbase) {
    const BinPlan& p = h->direct ? kNoBins : bp;
    timed(h, p.n > 0 ? T_STAGE : T_STAGE_ONLY, [&] {
        launch_stage(h->stream, h->dbl, h->g, h->z, h->b, nf, sc, p, write_new, Vbase);
    });
}

// Phase-2a choice: the kernel variant (cfg.y_kernel, or all three) and row tiles per
// wavefront (cfg.tile_rows, or 1, 2, 4, ... up to all of a group's or a class's tiles in one
// block: few blocks, each staging its B chunk once, against many blocks with more
// parallelism); the fastest candidate, timed with events on the operands of a stage at the
// flows' current state.  The per-row kernel gathers permuted bins; the operation-class
// kernel reads plain bin rows and stages a permuted operand once per class, which pays where
// the gathers dominate (large N, bf16) and costs where blocks are few; the orbit kernel
// reads each representative's bin row once and stages the operand once per operation,
// which cuts the bins' re-reads where they dominate the traffic.
// Every later stage recomputes these products, so the timing runs change no result.
// Choices are kept for the process, per shape, settings and number of flows.
using TuneKey = std::tuple<int, int, int, int, int, double, double, double, int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune;

// Phase-1 launch shape (cfg.phase1_variant, or timed): the step's first stage launch, which
// bins every node of the step, with 256- or 1024-thread blocks and one or two nodes per
// block; the fastest of the applicable shapes on the flows' current state.  Kept for the
// process per shape, settings, flows and step-sharing groups.
using Tune1Key = std::tuple<int, int, int, int, int, double, double, double, int, int, int>;
std::map<Tune1Key, int> g_tune1;

int tune_phase1(fm_flow* h, int nf, const double* Vbase) {
    const fm_config& c = h->cfg;
    if (h->direct || !h->b.bins || h->g.gflow) return FM_OK;
    if (c.phase1_variant != 0) { h->b.ph1var = c.phase1_variant; return FM_OK; }
    if (h->ph1_nf == nf) return FM_OK;
    const Tune1Key key{c.N, c.L, c.precision, nf, c.geometry, c.t, c.tp, c.mu, c.sync_batch,
                       c.integrator, c.n_shells};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune1.find(key);
        if (it != g_tune1.end()) {
            h->b.ph1var = it->second;
            h->ph1_nf = nf;
            return FM_OK;
        }
    }
    const BinPlan bp = step_plan(c.integrator == FM_RK45_DOPRI).bp;
    const size_t rs = h->dbl ? sizeof(double) : sizeof(float);
    const bool two = bp.n > 1 && 2 * bins_lds_bytes(h->g.N, rs) <= static_cast<size_t>(h->g.lds_max);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    StageCoef sc{};
    int best = 0;
    float best_ms = std::numeric_limits<float>::infinity();
    for (int v = 1; v <= (two ? 4 : 2); ++v) {
        Buffers bb = h->b;
        bb.ph1var = v;
        launch_stage(h->stream, h->dbl, h->g, h->z, bb, nf, sc, bp, 0, Vbase);
        (void)hipEventRecord(e0, h->stream);
        for (int r = 0; r < 3; ++r) launch_stage(h->stream, h->dbl, h->g, h->z, bb, nf, sc, bp, 0, Vbase);
        (void)hipEventRecord(e1, h->stream);
        float ms = 0.f;
        const bool ok = hipGetLastError() == hipSuccess;   // a shape that cannot launch is skipped
        if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
            ok && ms < best_ms) {
            best_ms = ms;
            best = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(hipGetLastError());
    h->b.ph1var = best;
    h->ph1_nf = nf;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune1[key] = best;
    return FM_OK;
}

int ensure_tuned(fm_flow* h, int nf, const double* Vbase) {
    if (int rc = tune_phase1(h, nf, Vbase)) return rc;
    const fm_config& c = h->cfg;
    const int mma = mma_mode(c.precision);
    if (h->dbl || h->direct || fused_phase2(c) || mma == 0 || c.N > 128) return FM_OK;
    std::vector<std::pair<int, int>> cand;    // (variant, tiles per wavefront)
    for (int var = 1; var <= 3; ++var) {
        if (c.y_kernel != 0 && var != c.y_kernel) continue;
        // representatives' products: the operation-class kernel on class 0, or the orbit
        // kernel on operation 0
        if (c.sym_state && var == 1) continue;
        if (c.tile_rows > 0) { cand.emplace_back(var, c.tile_rows); continue; }
        const int maxt = var == 3 ? y_orb_max_tpw(h->g, mma)
                         : var == 2 ? y_max_tpw(h->g) : y_rows_max_tpw(h->g);
        for (int t = 1; t < maxt; t *= 2) cand.emplace_back(var, t);
        cand.emplace_back(var, maxt);
    }
    if (cand.size() == 1) { h->yvar = cand[0].first; h->tpw = cand[0].second; return FM_OK; }
    if (h->tuned_nf == nf) return FM_OK;
    const TuneKey key{c.N, c.L, c.precision, nf, c.geometry, c.t, c.tp, c.mu, c.y_kernel,
                      c.tile_rows, c.n_shells, c.sym_state};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            h->yvar = it->second.first;
            h->tpw = it->second.second;
            h->fused = h->yvar == 4;
            h->tuned_nf = nf;
            return FM_OK;
        }
    }
    StageCoef sc{};
    launch_stage(h->stream, h->dbl, h->g, h->z, h->b, nf, sc, kOneNode, 0, Vbase);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    std::pair<int, int> best = cand[0];
    float best_ms = std::numeric_limits<float>::infinity();
    for (const auto& cv : cand) {
        launch_y(h->stream, false, h->g, h->b, nf, c.channels, mma, cv.second, cv.first);
        (void)hipEventRecord(e0, h->stream);
        for (int r = 0; r < 5; ++r)
            launch_y(h->stream, false, h->g, h->b, nf, c.channels, mma, cv.second, cv.first);
        (void)hipEventRecord(e1, h->stream);
        float ms = 0.f;
        if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
            ms < best_ms) {
            best_ms = ms;
            best = cv;
        }
    }
    // the fused phase 2 against the best phase 2a plus phase 2b
    if (fusable(c) && c.y_kernel == 0) {
        auto time5 = [&](auto&& launch) {
            launch();
            (void)hipEventRecord(e0, h->stream);
            for (int r = 0; r < 5; ++r) launch();
            (void)hipEventRecord(e1, h->stream);
            float ms = std::numeric_limits<float>::infinity();
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                ms = std::numeric_limits<float>::infinity();
            return ms;
        };
        const float c_ms = time5([&] { launch_contract(h->stream, false, h->g, h->b, nf, c.channels, 0); });
        const float f_ms = time5([&] { launch_fused(h->stream, h->g, h->b, nf, c.channels, 0, mma); });
        if (f_ms < best_ms + c_ms) best = {4, 0};
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPCHK(hipGetLastError());
    h->yvar = best.first;
    h->tpw = best.second;
    h->fused = best.first == 4;
    h->tuned_nf = nf;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    return FM_OK;
}

// One integrator step of every running flow (no host interaction).  V is the state array.
void step_launch(fm_flow* h, int nf, double* V, int fixed_steps) {
    const bool rk45 = h->cfg.integrator == FM_RK45_DOPRI;
    StepPlan plan = step_plan(rk45);
    if (h->g.gflow) {          // bins of the flow's fixed T, computed when the flow starts
        plan.bp = kNoBins;
        for (int& s : plan.set) s = 0;
    }
    if (!rk45) {
        for (int s = 0; s < 4; ++s) {
            stage_launch(h, nf, rk4_stage(s), s == plan.first ? plan.bp : kNoBins, 0, V);
            rhs_launch(h, nf, s, plan.set[s]);
        }
        timed(h, T_UPDATE, [&] { launch_rk4_update(h->stream, h->dbl, h->b, nf, h->g.N, V); });
        timed(h, T_FINISH, [&] {
            if (h->ngroups > 0)
                launch_finish_sync(h->stream, h->b, h->ngroups, h->gmax, 0, fixed_steps, !h->g.gflow);
            else
                launch_finish(h->stream, h->b, nf, 0, fixed_steps);
        });
        return;
    }
    for (int s = 1; s < 7; ++s) {
        stage_launch(h, nf, dp_stage(s), s == plan.first ? plan.bp : kNoBins, s == 6, V);
        rhs_launch(h, nf, s, plan.set[s]);
    }
    ErrWeights ew;
    std::memcpy(ew.e, kDPE, sizeof ew.e);
    timed(h, T_UPDATE, [&] { launch_dopri_err(h->stream, h->dbl, h->b, nf, h->g.N, V, h->cfg.rtol, ew); });
    timed(h, T_FINISH, [&] {
        if (h->ngroups > 0)
            launch_finish_sync(h->stream, h->b, h->ngroups, h->gmax, 1, 0, !h->g.gflow);
        else
            launch_finish(h->stream, h->b, nf, 1, 0);
        launch_commit(h->stream, h->dbl, h->b, nf, h->N3, V);
    });
}

int upload_z(fm_flow* h, int nf, const double* zl, const double* zt) {
    const int nz = h->cfg.n_zT;
    if (nz == 0) return FM_OK;
    const int N = h->cfg.N;
    const bool kat = !h->ktab.empty();   // the configured K table, for every flow
    std::vector<double> l(static_cast<size_t>(nf) * nz), t(static_cast<size_t>(nf) * nz * N);
    std::vector<double> k(kat ? t.size() : 0);
    for (int f = 0; f < nf; ++f) {
        const double* sl = zl ? zl + static_cast<size_t>(f) * nz : h->zlnT.data();
        const double* st = zt ? zt + static_cast<size_t>(f) * nz * N : h->ztab.data();
        for (int i = 0; i < nz; ++i) {
            // interaction flow: nodes in s = -g, negated, in reversed (ascending) order
            const int src = h->g.gflow ? nz - 1 - i : i;
            l[static_cast<size_t>(f) * nz + i] = h->g.gflow ? -sl[src] : sl[src];
            std::memcpy(&t[(static_cast<size_t>(f) * nz + i) * N], st + static_cast<size_t>(src) * N,
                        sizeof(double) * N);
            if (kat)
                std::memcpy(&k[(static_cast<size_t>(f) * nz + i) * N],
                            h->ktab.data() + static_cast<size_t>(src) * N, sizeof(double) * N);
        }
    }
    HIPCHK(hipMemcpyAsync(h->b.z_lnT, l.data(), l.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->b.z_tab, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
    if (kat)
        HIPCHK(hipMemcpyAsync(h->b.k_tab, k.data(), k.size() * sizeof(double), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return FM_OK;
}

}  // namespace

void fm::set_last_error(const std::string& msg) { g_err = msg; }

extern "C" {

const char* fm_last_error(void) { return g_err.c_str(); }

int fm_geometry_query(const fm_config* cfg, double* xi, int* patch, int* anchor, int* n_pp,
                      int* n_ph, double* margin, int* n_rep) {
    if (!cfg) return fail(FM_EINVAL, "null config");
    HostGeometry g;
    std::string why;
    if (!build_geometry(*cfg, g, why)) return fail(FM_EINVAL, why);
    if (xi) std::memcpy(xi, g.xi.data(), sizeof(double) * g.np);
    if (patch) std::memcpy(patch, g.patch.data(), sizeof(int) * g.np);
    if (anchor) std::memcpy(anchor, g.anchor.data(), sizeof(int) * 2 * g.N);
    if (n_pp) *n_pp = static_cast<int>(g.q_pp.size());
    if (n_ph) *n_ph = static_cast<int>(g.q_ph.size());
    if (margin) *margin = g.margin;
    if (n_rep) {
        n_rep[0] = static_cast<int>(g.rep_pp.size());
        n_rep[1] = static_cast<int>(g.rep_ph.size());
    }
    return FM_OK;
}

int fm_flow_workspace_bytes(const fm_config* in, size_t* bytes) {
    fm_config c;
    std::string why;
    int rc = resolve(in, c, why);
    if (rc) return fail(rc, why);
    if (!bytes) return fail(FM_EINVAL, "null bytes");
    HostGeometry g;
    if (!build_geometry(c, g, why)) return fail(FM_EINVAL, why);
    if (!sym_ok(c, g, why)) return fail(FM_EINVAL, why);
    fm_flow tmp;
    return carve(tmp, c, g, nullptr, bytes);
}

int fm_flow_init(const fm_config* in, void* ws, size_t bytes, fm_flow** out) {
    if (!out) return fail(FM_EINVAL, "null handle pointer");
    *out = nullptr;
    fm_config c;
    std::string why;
    int rc = resolve(in, c, why);
    if (rc) return fail(rc, why);
    fm_flow* h = new fm_flow;
    h->cfg = c;
    if (!build_geometry(c, h->hg, why)) { delete h; return fail(FM_EINVAL, why); }
    if (!sym_ok(c, h->hg, why)) { delete h; return fail(FM_EINVAL, why); }
    size_t need = 0;
    carve(*h, c, h->hg, nullptr, &need);
    if (!ws || bytes < need) {
        delete h;
        return fail(FM_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
    }
    // align the base to 256 bytes
    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) & ~static_cast<uintptr_t>(255));
    carve(*h, c, h->hg, base, &need);
    h->stream = static_cast<hipStream_t>(c.stream);
    h->dbl = c.precision == FM_FP64 || c.precision == FM_FP64_DIRECT;
    h->direct = c.precision == FM_FP64_DIRECT;
    h->fused = fused_phase2(c);
    const HostGeometry& hg = h->hg;
    const int N = c.N;
    h->N3 = static_cast<size_t>(N) * N * N;
    DevGeom& g = h->g;
    g.N = N; g.L = c.L; g.np = hg.np;
    g.nP = static_cast<int>(hg.q_pp.size());
    g.nD = static_cast<int>(hg.q_ph.size());
    g.NN = N * N;
    g.xi = h->b.xi; g.patch = h->b.patch; g.xp = h->b.xp; g.q_pp = h->b.q_pp; g.q_ph = h->b.q_ph;
    g.map_pp = h->b.map_pp; g.map_cr = h->b.map_cr; g.map_d = h->b.map_d;
    g.nRp = static_cast<int>(hg.rep_pp.size());
    g.nRd = static_cast<int>(hg.rep_ph.size());
    g.rep_pp = h->b.rep_pp; g.rep_ph = h->b.rep_ph;
    g.qrep_pp = h->b.qrep_pp; g.qg_pp = h->b.qg_pp;
    g.qrep_ph = h->b.qrep_ph; g.qg_ph = h->b.qg_ph;
    g.pinv = h->b.pinv;
    g.perm = h->b.perm;
    g.orb_rows = h->b.orb_rows; g.orb_q = h->b.orb_q; g.orb_mask = h->b.orb_mask;
    g.orb_nt[0] = hg.orb_nt[0];
    g.orb_nt[1] = hg.orb_nt[1];
    g.porder = h->b.porder;
    g.nG = static_cast<int>(hg.porder.size() / 8);
    for (int o = 0; o < 9; ++o) {
        g.cls[0][o] = hg.cls_pp[o];
        g.cls[1][o] = hg.cls_ph[o];
    }
    g.pI = h->b.pI;
    g.inv_ok = hg.inv_ok ? 1 : 0;
    g.gflow = c.flow == FM_FLOW_INTERACTION ? 1 : 0;
    g.sym = c.sym_state;
    {
        int dev = 0, lds = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        if (e != hipSuccess) {
            delete h;
            return fail(FM_EDEVICE, std::string("device query: ") + hipGetErrorString(e));
        }
        g.lds_max = lds;
    }
    g.inv_rot = 0;
    if (hg.inv_ok && N % 2 == 0) {
        g.inv_rot = 1;
        for (int a = 0; a < N; ++a)
            if (hg.inv_perm[a] != (a + N / 2) % N) g.inv_rot = 0;
    }
    g.pp_off = h->b.pp_off; g.pp_pairs = h->b.pp_pairs;
    g.cr_off = h->b.cr_off; g.cr_pairs = h->b.cr_pairs;
    g.d_off = h->b.d_off; g.d_pairs = h->b.d_pairs;
    g.item_q = h->b.item_q; g.item_p0 = h->b.item_p0; g.item_rec = h->b.item_rec;
    for (int k = 0; k < 3; ++k) g.n_items[k] = hg.n_items[k];
    g.sym_rec = h->b.sym_rec;
    for (int k = 0; k < 3; ++k) g.n_sym_items[k] = hg.n_sym_items[k];
    g.fz_row = h->b.fz_row; g.fz_pair = h->b.fz_pair; g.fz_blk = h->b.fz_blk;
    for (int k = 0; k < 3; ++k) g.fz_nblk[k] = hg.fz_nblk[k];
    auto up = [&](void* dst, const void* src, size_t n) {
        return hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, h->stream);
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up(h->b.xi, hg.xi.data(), sizeof(double) * hg.np);
    if (e == hipSuccess) e = up(h->b.patch, hg.patch.data(), sizeof(int) * hg.np);
    std::vector<int2> xp(hg.np);
    for (int j = 0; j < hg.np; ++j) {
        const float x = static_cast<float>(hg.xi[j]);
        std::memcpy(&xp[j].x, &x, sizeof x);
        xp[j].y = hg.patch[j];
    }
    if (e == hipSuccess) e = up(h->b.xp, xp.data(), sizeof(int2) * hg.np);
    if (e == hipSuccess) e = up(h->b.q_pp, hg.q_pp.data(), sizeof(int) * g.nP);
    if (e == hipSuccess) e = up(h->b.q_ph, hg.q_ph.data(), sizeof(int) * g.nD);
    if (e == hipSuccess) e = up(h->b.map_pp, hg.map_pp.data(), sizeof(int) * g.NN);
    if (e == hipSuccess) e = up(h->b.map_cr, hg.map_cr.data(), sizeof(int) * g.NN);
    if (e == hipSuccess) e = up(h->b.map_d, hg.map_d.data(), sizeof(int) * g.NN);
    auto upv = [&](int* dst, const std::vector<int>& v) {
        return v.empty() ? hipSuccess : up(dst, v.data(), sizeof(int) * v.size());
    };
    if (e == hipSuccess) e = upv(h->b.rep_pp, hg.rep_pp);
    if (e == hipSuccess) e = upv(h->b.rep_ph, hg.rep_ph);
    if (e == hipSuccess) e = upv(h->b.qrep_pp, hg.qrep_pp);
    if (e == hipSuccess) e = upv(h->b.qg_pp, hg.qg_pp);
    if (e == hipSuccess) e = upv(h->b.qrep_ph, hg.qrep_ph);
    if (e == hipSuccess) e = upv(h->b.qg_ph, hg.qg_ph);
    if (e == hipSuccess) e = upv(h->b.pinv, hg.pinv);
    if (e == hipSuccess) e = upv(h->b.perm, hg.perm);
    if (e == hipSuccess) e = upv(h->b.orb_rows, hg.orb_rows);
    if (e == hipSuccess) e = upv(h->b.orb_q, hg.orb_q);
    if (e == hipSuccess) e = upv(h->b.orb_mask, hg.orb_mask);
    if (e == hipSuccess) e = upv(h->b.porder, hg.porder);
    if (e == hipSuccess) e = upv(h->b.pI, hg.inv_perm);
    if (e == hipSuccess) e = upv(h->b.pp_off, hg.pp_off);
    if (e == hipSuccess) e = upv(h->b.pp_pairs, hg.pp_pairs);
    if (e == hipSuccess) e = upv(h->b.cr_off, hg.cr_off);
    if (e == hipSuccess) e = upv(h->b.cr_pairs, hg.cr_pairs);
    if (e == hipSuccess) e = upv(h->b.d_off, hg.d_off);
    if (e == hipSuccess) e = upv(h->b.d_pairs, hg.d_pairs);
    if (e == hipSuccess) e = upv(h->b.item_q, hg.item_q);
    if (e == hipSuccess) e = upv(h->b.item_p0, hg.item_p0);
    if (e == hipSuccess) e = upv(h->b.item_rec, hg.item_rec);
    if (e == hipSuccess) e = upv(h->b.sym_rec, hg.sym_rec);
    if (e == hipSuccess) e = upv(h->b.fz_row, hg.fz_row);
    if (e == hipSuccess) e = upv(h->b.fz_pair, hg.fz_pair);
    if (e == hipSuccess) e = upv(h->b.fz_blk, hg.fz_blk);
    if (e == hipSuccess) e = up(h->b.kpt, hg.kpt.data(), sizeof(double) * hg.kpt.size());
    // bins start zeroed (with their padding): phase 2a may read past a row's end, and only
    // finite values may meet the zero operand there
    if (e == hipSuccess && h->b.bins) e = hipMemsetAsync(h->b.bins, 0, h->b.bins_bytes, h->stream);
    if (e == hipSuccess && h->b.binsT) e = hipMemsetAsync(h->b.binsT, 0, h->b.binsT_bytes, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        delete h;
        return fail(FM_EDEVICE, std::string("geometry upload: ") + hipGetErrorString(e));
    }
    if (c.n_zT > 0) {
        h->zlnT.assign(c.z_lnT, c.z_lnT + c.n_zT);
        h->ztab.assign(c.z_table, c.z_table + static_cast<size_t>(c.n_zT) * N);
        if (c.k_table) h->ktab.assign(c.k_table, c.k_table + static_cast<size_t>(c.n_zT) * N);
        for (double z : h->ztab)
            if (!(z > 0.0 && std::isfinite(z))) {
                delete h;
                return fail(FM_EINVAL, "Z must be positive and finite");
            }

        rc = upload_z(h, c.max_batch, nullptr, nullptr);
        if (rc) { delete h; return rc; }
    }
    h->z.n = c.n_zT;
    h->z.lnT = h->b.z_lnT;
    h->z.tab = h->b.z_tab;
    h->z.ktab = c.k_table ? h->b.k_tab : nullptr;
    h->hfs.resize(c.max_batch);
    *out = h;
    return FM_OK;
}

void fm_flow_destroy(fm_flow* h) {
    if (!h) return;
    if (h->step_exec) (void)hipGraphExecDestroy(h->step_exec);
    for (auto e : h->ev) (void)hipEventDestroy(e);
    if (h->own) (void)hipStreamDestroy(h->own);
    delete h;
}

int fm_flow_set_timing(fm_flow* h, int enable) {
    if (!h) return fail(FM_EINVAL, "null handle");
    h->timing = enable != 0;
    h->ev_use.clear();
    h->ev_end.clear();
    h->ev_last = -1;
    h->ev_next = 0;
    std::fill(std::begin(h->t_ms), std::end(h->t_ms), 0.0);
    std::fill(std::begin(h->t_n), std::end(h->t_n), 0);
    return FM_OK;
}

int fm_flow_timings(fm_flow* h, const char** names, double* ms, int* launches, int max_n) {
    if (!h) return fail(FM_EINVAL, "null handle");
    collect_timings(h);
    int n = 0;
    for (int i = 0; i < T_COUNT && n < max_n; ++i) {
        if (!h->t_n[i]) continue;
        if (names) names[n] = kTimerNames[i];
        if (ms) ms[n] = h->t_ms[i];
        if (launches) launches[n] = h->t_n[i];
        ++n;
    }
    return n;
}

int fm_flow_kernel_time(fm_flow* h, int group, int batch, int reps, double* avg_ms) {
    if (!h) return fail(FM_EINVAL, "null handle");
    if (batch < 1 || batch > h->cfg.max_batch) return fail(FM_EINVAL, "batch outside [1, max_batch]");
    if (reps < 1 || !avg_ms) return fail(FM_EINVAL, "need reps >= 1 and an output");
    if (group < 0 || group > 3 || (h->direct && group == 1))
        return fail(FM_EINVAL, "group: 0 stage and phase 1, 1 phase 2a, 2 phase 2b, 3 stage alone");
    if (h->fused && group == 2)
        return fail(FM_EINVAL, "phase 2 is one fused launch here: time group 1");
    // flows replayed as running at their current temperature; their status is restored
    std::vector<FlowState> saved(batch);
    HIPCHK(hipMemcpyAsync(saved.data(), h->b.fs, sizeof(FlowState) * batch, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    std::vector<FlowState> run = saved;
    for (auto& f : run) { f.status = FM_FLOW_RUNNING; f.ht = 0.0; }
    HIPCHK(hipMemcpyAsync(h->b.fs, run.data(), sizeof(FlowState) * batch, hipMemcpyHostToDevice, h->stream));
    const StageCoef sc{};
    // the stage alone as in the middle of a step: four earlier k slots read
    StageCoef mid{};
    mid.ns = 4;
    for (int l = 0; l < 4; ++l) mid.a[l] = 0.25;
    const BinPlan step_bins = h->direct ? kNoBins
                              : h->g.gflow ? kOneNode
                                           : step_plan(h->cfg.integrator == FM_RK45_DOPRI).bp;
    auto once = [&] {
        const int mma = mma_mode(h->cfg.precision);
        if (group == 0)
            launch_stage(h->stream, h->dbl, h->g, h->z, h->b, batch, sc, step_bins, 0, h->b.V);
        else if (group == 3)
            launch_stage(h->stream, h->dbl, h->g, h->z, h->b, batch, mid, kNoBins, 0, h->b.V);
        else if (group == 1 && h->fused)
            launch_fused(h->stream, h->g, h->b, batch, h->cfg.channels, 0, mma);
        else if (group == 1)
            launch_y(h->stream, h->dbl, h->g, h->b, batch, h->cfg.channels, mma, h->tpw, h->yvar);
        else if (h->direct)
            launch_direct(h->stream, h->g, h->b, batch, h->cfg.channels, 0);
        else
            launch_contract(h->stream, h->dbl, h->g, h->b, batch, h->cfg.channels, 0);
    };
    // inputs of the later groups: one stage and phase 1 first
    launch_stage(h->stream, h->dbl, h->g, h->z, h->b, batch, sc, h->direct ? kNoBins : kOneNode, 0,
                 h->b.V);
    if (h->direct) launch_wtable(h->stream, h->g, h->b, batch);
    once();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    (void)hipEventRecord(e0, h->stream);
    for (int r = 0; r < reps; ++r) once();
    (void)hipEventRecord(e1, h->stream);
    hipError_t e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(FM_EDEVICE, std::string("kernel timing: ") + hipGetErrorString(e));
    HIPCHK(hipMemcpyAsync(h->b.fs, saved.data(), sizeof(FlowState) * batch, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    HIPCHK(hipGetLastError());
    *avg_ms = ms / reps;
    return FM_OK;
}

int fm_flow_rhs(fm_flow* h, int batch, const double* T, const double* V_dev, double* dV_dev) {
    if (!h) return fail(FM_EINVAL, "null handle");
    if (batch < 1 || batch > h->cfg.max_batch) return fail(FM_EINVAL, "batch outside [1, max_batch]");
    if (!T || !V_dev || !dV_dev) return fail(FM_EINVAL, "null argument");
    if (V_dev == dV_dev) return fail(FM_EINVAL, "dV_dev must not alias V_dev");
    if (h->g.gflow) return fail(FM_EINVAL, "interaction-flow handle: use fm_flow_rhs_g");
    for (int f = 0; f < batch; ++f) {
        if (!(T[f] > 0.0) || !std::isfinite(T[f])) return fail(FM_EINVAL, "T must be positive and finite");
        FlowState s{};
        s.lnT = std::log(T[f]);
        s.status = FM_FLOW_RUNNING;
        h->hfs[f] = s;
    }
    HIPCHK(hipMemcpyAsync(h->b.fs, h->hfs.data(), sizeof(FlowState) * batch, hipMemcpyHostToDevice, h->stream));
    if (int rc = ensure_tuned(h, batch, V_dev)) return rc;
    untimed(h);
    StageCoef sc{};
    stage_launch(h, batch, sc, kOneNode, 0, V_dev);
    rhs_launch(h, batch, 0, 0);
    launch_k_to_f64(h->stream, h->dbl, h->b, batch, h->g.N, 0, dV_dev);
    HIPCHK(hipGetLastError());
    return FM_OK;
}

int fm_flow_step(fm_flow* h, int batch, double* lnT, double* hstep, double* V_dev, int* accepted) {
    if (!h) return fail(FM_EINVAL, "null handle");
    if (batch < 1 || batch > h->cfg.max_batch) return fail(FM_EINVAL, "batch outside [1, max_batch]");
    if (!lnT || !hstep || !V_dev || !accepted) return fail(FM_EINVAL, "null argument");
    const bool rk45 = h->cfg.integrator == FM_RK45_DOPRI;
    const bool gf = h->g.gflow != 0;   // lnT holds g, and s = -g internally
    for (int f = 0; f < batch; ++f) {
        if (!std::isfinite(lnT[f]) || !std::isfinite(hstep[f]) || hstep[f] == 0.0)
            return fail(FM_EINVAL, "lnT and h must be finite, h nonzero");
        FlowState s{};
        s.lnT = gf ? -lnT[f] : lnT[f];
        s.h = s.ht = gf ? -hstep[f] : hstep[f];
        s.gflow = gf ? 1 : 0;
        s.Tfix = gf ? h->cfg.T0 : 0.0;
        s.vmax = std::numeric_limits<double>::infinity();   // no stop test in a lone step
        s.lnT_end = -std::numeric_limits<double>::infinity();
        s.hmin = 0.0;
        s.atol = h->cfg.atol > 0.0 ? h->cfg.atol : 1e-9 * std::max(1.0, std::fabs(h->cfg.U));
        s.status = FM_FLOW_RUNNING;
        h->hfs[f] = s;
    }
    HIPCHK(hipMemcpyAsync(h->b.fs, h->hfs.data(), sizeof(FlowState) * batch, hipMemcpyHostToDevice, h->stream));
    if (int rc = ensure_tuned(h, batch, V_dev)) return rc;
    untimed(h);
    h->ngroups = h->gmax = 0;      // a lone step: every state on its own step
    if (rk45) {
        stage_launch(h, batch, dp_stage(0), kOneNode, 0, V_dev);
        rhs_launch(h, batch, 0, 0);
    } else if (gf) {        // the interaction flow's bins, at its fixed temperature
        stage_launch(h, batch, rk4_stage(0), kOneNode, 0, V_dev);
    }
    step_launch(h, batch, V_dev, 0);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h->hfs.data(), h->b.fs, sizeof(FlowState) * batch, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int f = 0; f < batch; ++f) {
        const FlowState& s = h->hfs[f];
        accepted[f] = s.accepted;
        if (s.accepted) lnT[f] = gf ? -s.lnT : s.lnT;
        if (rk45) hstep[f] = gf ? -s.h : s.h;
    }
    return FM_OK;
}

int fm_flow_rhs_g(fm_flow* h, int batch, const double* T, const double* g, const double* V_dev,
                  double* dV_dev) {
    if (!h) return fail(FM_EINVAL, "null handle");
    if (batch < 1 || batch > h->cfg.max_batch) return fail(FM_EINVAL, "batch outside [1, max_batch]");
    if (!T || !g || !V_dev || !dV_dev) return fail(FM_EINVAL, "null argument");
    if (V_dev == dV_dev) return fail(FM_EINVAL, "dV_dev must not alias V_dev");
    if (!h->g.gflow) return fail(FM_EINVAL, "temperature-flow handle: use fm_flow_rhs");
    for (int f = 0; f < batch; ++f) {
        if (!(T[f] > 0.0) || !std::isfinite(T[f])) return fail(FM_EINVAL, "T must be positive and finite");
        if (!std::isfinite(g[f])) return fail(FM_EINVAL, "g must be finite");
        FlowState s{};
        s.lnT = -g[f];
        s.Tfix = T[f];
        s.gflow = 1;
        s.status = FM_FLOW_RUNNING;
        h->hfs[f] = s;
    }
    HIPCHK(hipMemcpyAsync(h->b.fs, h->hfs.data(), sizeof(FlowState) * batch, hipMemcpyHostToDevice, h->stream));
    if (int rc = ensure_tuned(h, batch, V_dev)) return rc;
    untimed(h);
    StageCoef sc{};
    stage_launch(h, batch, sc, kOneNode, 0, V_dev);
    rhs_launch(h, batch, 0, 0);
    launch_k_to_f64(h->stream, h->dbl, h->b, batch, h->g.N, 0, dV_dev);   // -dV/ds = dV/dg
    HIPCHK(hipGetLastError());
    return FM_OK;
}

int fm_flow_run_batch(fm_flow* h, int n, const double* U, const double* T0, const double* z_lnT,
                      const double* z_tables, double* V_final_dev, fm_result* res) {
    if (!h) return fail(FM_EINVAL, "null handle");
    if (n < 1 || n > h->cfg.max_batch) return fail(FM_EINVAL, "n_flows outside [1, max_batch]");
    if (!U || !T0 || !res) return fail(FM_EINVAL, "null argument");
    if ((z_lnT == nullptr) != (z_tables == nullptr)) return fail(FM_EINVAL, "give both Z arrays or neither");
    if (z_tables && h->cfg.n_zT == 0) return fail(FM_EINVAL, "per-flow Z tables need cfg.n_zT > 0");
    if (z_tables && !h->ktab.empty())
        return fail(FM_EINVAL, "per-flow Z tables cannot be combined with a configured Katanin table");
    if (z_tables) {   // each flow's table as fm_flow_init checks the configured one
        const int nz = h->cfg.n_zT, N = h->cfg.N;
        for (int f = 0; f < n; ++f) {
            const double* l = z_lnT + static_cast<size_t>(f) * nz;
            const double* t = z_tables + static_cast<size_t>(f) * nz * N;
            for (int i = 1; i < nz; ++i)
                if (!(l[i] > l[i - 1])) return fail(FM_EINVAL, "per-flow Z nodes must ascend");
            for (size_t i = 0; i < static_cast<size_t>(nz) * N; ++i)
                if (!(t[i] > 0.0 && std::isfinite(t[i])))
                    return fail(FM_EINVAL, "per-flow Z must be positive and finite");
            if (h->g.sym && !rows_symmetric(h->hg.perm, t, nz, N))
                return fail(FM_EINVAL, "sym_state needs per-flow Z tables invariant under the point group");
        }
    }
    const fm_config& c = h->cfg;
    const bool rk45 = c.integrator == FM_RK45_DOPRI;
    const bool gf = h->g.gflow != 0;
    // temperature flow: s = ln T from ln T0 down to ln T_end; interaction flow: s = -g from 0
    // down to -g_end at the fixed T0[f]
    const double lnTe = gf ? -c.g_end : std::log(c.T_end);
    for (int f = 0; f < n; ++f) {
        if (gf ? !(T0[f] > 0.0 && std::isfinite(T0[f])) : !(T0[f] > c.T_end))
            return fail(FM_EINVAL, gf ? "need T0[f] > 0" : "need T0[f] > T_end");
        if (!std::isfinite(U[f])) return fail(FM_EINVAL, "need a finite U");
        FlowState s{};
        s.s0 = s.lnT = gf ? 0.0 : std::log(T0[f]);
        s.lnT_end = lnTe;
        s.gflow = gf ? 1 : 0;
        s.Tfix = gf ? T0[f] : 0.0;
        const double span = lnTe - s.s0;
        if (rk45) {
            s.h = c.h0 != 0.0 ? (gf ? -c.h0 : c.h0) : span / 200.0;
            s.ht = (s.lnT + s.h <= lnTe) ? lnTe - s.lnT : s.h;
            s.hmin = c.h_min > 0.0 ? c.h_min : 1e-8 * std::fabs(span);
        } else {
            s.h = s.ht = span / c.n_steps;
        }
        s.atol = c.atol > 0.0 ? c.atol : 1e-9 * std::max(1.0, std::fabs(U[f]));
        s.m = std::fabs(U[f]);
        s.status = FM_FLOW_RUNNING;
        // the paper's threshold is relative to the bare coupling (Sec. 3.2); the temperature
        // flow uses an absolute one
        s.vmax = gf ? c.v_rel * std::fabs(U[f]) : c.v_max;
        if (s.m > s.vmax) { s.status = FM_FLOW_DIVERGED; s.lnTc = s.lnT; }
        s.n_rhs = (rk45 && s.status == FM_FLOW_RUNNING) ? 1 : 0;
        h->hfs[f] = s;
    }
    // step-sharing groups: flows with equal T0, in order of first appearance, at most
    // cfg.sync_batch of them per group (1 = no limit); the first running member bins for
    // the group
    h->ngroups = h->gmax = 0;
    if (c.sync_batch) {
        const int cap = c.sync_batch == 1 ? n : c.sync_batch;
        std::vector<int> members, off{0};
        std::vector<char> done(n, 0);
        for (int f = 0; f < n; ++f) {
            if (done[f]) continue;
            int lead = -1;
            for (int k = f; k < n && static_cast<int>(members.size()) - off.back() < cap; ++k) {
                if (done[k] || T0[k] != T0[f]) continue;
                done[k] = 1;
                members.push_back(k);
                if (lead < 0 && h->hfs[k].status == FM_FLOW_RUNNING) lead = k;
            }
            for (size_t i = off.back(); i < members.size(); ++i)
                h->hfs[members[i]].bshare = lead >= 0 ? lead + 1 : 0;
            h->gmax = std::max(h->gmax, static_cast<int>(members.size()) - off.back());
            off.push_back(static_cast<int>(members.size()));
        }
        h->ngroups = static_cast<int>(off.size()) - 1;
        HIPCHK(hipMemcpyAsync(h->b.grp_members, members.data(), sizeof(int) * members.size(),
                              hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->b.grp_off, off.data(), sizeof(int) * off.size(),
                              hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    if (z_tables) {
        int rc = upload_z(h, n, z_lnT, z_tables);
        if (rc) return rc;
    } else if (c.n_zT > 0) {
        int rc = upload_z(h, n, nullptr, nullptr);
        if (rc) return rc;
    }
    HIPCHK(hipMemcpyAsync(h->b.fs, h->hfs.data(), sizeof(FlowState) * n, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->b.U, U, sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
    launch_fill_u(h->stream, h->b, n, h->N3, h->b.U);
    if (int rc = ensure_tuned(h, n, h->b.V)) return rc;
    untimed(h);
    if (rk45) {
        stage_launch(h, n, dp_stage(0), kOneNode, 0, h->b.V);
        rhs_launch(h, n, 0, 0);
    } else if (gf) {        // the interaction flow's bins, at its fixed temperature
        stage_launch(h, n, rk4_stage(0), kOneNode, 0, h->b.V);
    }
    HIPCHK(hipGetLastError());
    // fixed steps: flow f advances on its own grid ln T0_f + k (ln T_end - ln T0_f)/n_steps
    const int fixed = rk45 ? 0 : c.n_steps;
    const int max_steps = rk45 ? 1000000 : c.n_steps;
    const int check_every = rk45 ? 4 : 8;
    int done_steps = 0;
    bool use_graph = !h->timing;
    hipStream_t cap = h->stream;
    if (use_graph && cap == nullptr) {
        if (!h->own) HIPCHK(hipStreamCreateWithFlags(&h->own, hipStreamNonBlocking));
        cap = h->own;
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    hipStream_t saved = h->stream;
    if (use_graph && (h->step_nf != n || h->step_ng != h->ngroups || h->step_gmax != h->gmax)) {
        if (h->step_exec) { (void)hipGraphExecDestroy(h->step_exec); h->step_exec = nullptr; }
        h->stream = cap;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            step_launch(h, n, h->b.V, fixed);
            e = hipStreamEndCapture(cap, &graph);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&h->step_exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        h->stream = saved;
        if (e != hipSuccess) {
            // eager steps on the caller's stream, and every readback on the same stream
            (void)hipGetLastError();
            h->step_exec = nullptr;
            use_graph = false;
            cap = h->stream;
        } else {
            h->step_nf = n;
            h->step_ng = h->ngroups;
            h->step_gmax = h->gmax;
        }
    }
    while (done_steps < max_steps) {
        const int k = std::min(check_every, max_steps - done_steps);
        for (int i = 0; i < k; ++i) {
            if (use_graph) {
                HIPCHK(hipGraphLaunch(h->step_exec, cap));
            } else {
                step_launch(h, n, h->b.V, fixed);
            }
        }
        done_steps += k;
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(h->hfs.data(), h->b.fs, sizeof(FlowState) * n, hipMemcpyDeviceToHost, cap));
        HIPCHK(hipStreamSynchronize(cap));
        collect_timings(h);
        bool any = false;
        for (int f = 0; f < n; ++f) any |= h->hfs[f].status == FM_FLOW_RUNNING;
        if (!any) break;
    }
    if (z_tables) {   // later rhs/step calls use the configured table again
        int rc = upload_z(h, n, nullptr, nullptr);
        if (rc) return rc;
    }
    if (V_final_dev) {
        launch_copy(cap, h->b.V, V_final_dev, static_cast<size_t>(n) * h->N3);
        HIPCHK(hipStreamSynchronize(cap));
    }
    for (int f = 0; f < n; ++f) {
        const FlowState& s = h->hfs[f];
        fm_result& r = res[f];
        r.status = s.status == FM_FLOW_RUNNING ? FM_FLOW_STEPFAIL : s.status;
        const bool stopped = s.status == FM_FLOW_DIVERGED || s.status == FM_FLOW_NONFINITE;
        const double nan = std::numeric_limits<double>::quiet_NaN();
        r.T_c = (stopped && !gf) ? std::exp(s.lnTc) : nan;
        r.T_final = gf ? s.Tfix : std::exp(s.lnT);
        r.g_c = (stopped && gf) ? 0.0 - s.lnTc : nan;
        r.U_star = (stopped && gf) ? s.lnTc * s.lnTc * U[f] : nan;
        r.g_final = gf ? 0.0 - s.lnT : nan;
        r.max_abs_V = s.m;
        r.n_accepted = s.n_acc;
        r.n_rejected = s.n_rej;
        r.n_rhs = s.n_rhs;
    }
    return FM_OK;
}

int fm_flow_z(fm_flow* h, double T, double U, const double* V_dev, double* Z, double* im_sigma,
              double* re_sigma) {
    if (!h) return fail(FM_EINVAL, "null handle");
    if (!(T > 0.0) || !std::isfinite(T) || !std::isfinite(U)) return fail(FM_EINVAL, "need T > 0, finite U");
    if (!Z) return fail(FM_EINVAL, "null Z");
    const fm_config& c = h->cfg;
    SigmaArgs s{};
    s.N = c.N;
    s.L = c.L;
    s.t = c.t; s.tp = c.tp; s.mu = c.mu; s.T = T; s.U = U;
    s.w0 = fm_sigma_wmax(&c);
    s.dw = 2.0 * s.w0 / (kSigmaW - 1);
    if (!(s.w0 > 0.0) || !std::isfinite(s.w0)) return fail(FM_EINVAL, "the band has no width (t, t', mu)");
    s.xi = h->b.xi;
    s.patch = h->b.patch;
    s.kpt = h->b.kpt;
    s.f = h->b.sig_f;
    launch_sigma(h->stream, s, V_dev, h->b.sig_hist, h->b.sig_im, h->b.sig_re, h->b.sig_Z);
    HIPCHK(hipGetLastError());
    const size_t nw = static_cast<size_t>(c.N) * kSigmaW;
    HIPCHK(hipMemcpyAsync(Z, h->b.sig_Z, sizeof(double) * c.N, hipMemcpyDeviceToHost, h->stream));
    if (im_sigma)
        HIPCHK(hipMemcpyAsync(im_sigma, h->b.sig_im, sizeof(double) * nw, hipMemcpyDeviceToHost, h->stream));
    if (re_sigma)
        HIPCHK(hipMemcpyAsync(re_sigma, h->b.sig_re, sizeof(double) * nw, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return FM_OK;
}

double fm_sigma_wmax(const fm_config* cfg) {
    if (!cfg) return 0.0;
    return 3.0001 * (4.0 * std::fabs(cfg->t) + 4.0 * std::fabs(cfg->tp) + std::fabs(cfg->mu));
}

int fm_katanin_table(int n, const double* g, int N, const double* z_tab, double* k_tab,
                     double* a_tab, double* a_minmax) {
    if (n < 3 || N < 1 || !g || !z_tab || !k_tab) return fail(FM_EINVAL, "need n >= 3 nodes, N >= 1 and the tables");
    for (int i = 1; i < n; ++i)
        if (!(g[i] > g[i - 1])) return fail(FM_EINVAL, "Katanin table: nodes must ascend");
    for (size_t i = 0; i < static_cast<size_t>(n) * N; ++i)
        if (!(z_tab[i] > 0.0 && std::isfinite(z_tab[i]))) return fail(FM_EINVAL, "Katanin table: Z must be positive and finite");
    for (int i = 0; i < n; ++i) {
        // the three nodes whose parabola gives ds/dg at g_i
        const int c = std::min(std::max(i, 1), n - 2);
        const double xm = g[c - 1], x0 = g[c], xp = g[c + 1], x = g[i];
        // derivative of the Lagrange basis polynomials of (xm, x0, xp) at x
        const double dm = (2.0 * x - x0 - xp) / ((xm - x0) * (xm - xp));
        const double d0 = (2.0 * x - xm - xp) / ((x0 - xm) * (x0 - xp));
        const double dp = (2.0 * x - xm - x0) / ((xp - xm) * (xp - x0));
        double amin = std::numeric_limits<double>::infinity(), amax = -amin;
        for (int a = 0; a < N; ++a) {
            auto s_at = [&](int j) { return 1.0 - 1.0 / z_tab[static_cast<size_t>(j) * N + a]; };
            const double ds = dm * s_at(c - 1) + d0 * s_at(c) + dp * s_at(c + 1);
            const double z = z_tab[static_cast<size_t>(i) * N + a], s = s_at(i);
            const double K = 1.0 - s + x * ds;
            const double A = x > 0.0 ? -2.0 / x * (1.0 - z * K) : 2.0 * ds / (1.0 - s);
            k_tab[static_cast<size_t>(i) * N + a] = K;
            if (a_tab) a_tab[static_cast<size_t>(i) * N + a] = A;
            amin = std::min(amin, A);
            amax = std::max(amax, A);
        }
        if (a_minmax) {
            a_minmax[2 * i] = amin;
            a_minmax[2 * i + 1] = amax;
        }
    }
    return FM_OK;
}

int fm_flow_tstar(fm_flow* h, int n, const double* U, double T_lo, double T_hi, double rtol,
                  double* T_star, int* status) {
    if (!h) return fail(FM_EINVAL, "null handle");
    if (!h->g.gflow) return fail(FM_EINVAL, "T*(U) needs an interaction-flow handle");
    if (n < 1 || n > h->cfg.max_batch) return fail(FM_EINVAL, "n_flows outside [1, max_batch]");
    if (!U || !T_star || !status) return fail(FM_EINVAL, "null argument");
    if (!(T_lo > 0.0) || !(T_hi > T_lo) || !std::isfinite(T_hi) || !(rtol > 0.0))
        return fail(FM_EINVAL, "need 0 < T_lo < T_hi and rtol > 0");
    const double nan = std::numeric_limits<double>::quiet_NaN();
    std::vector<double> lo(n, std::log(T_lo)), hi(n, std::log(T_hi));
    std::vector<double> Ua, Ta;
    std::vector<int> idx;
    std::vector<fm_result> r(n);
    auto diverged = [](const fm_result& x) {
        return x.status == FM_FLOW_DIVERGED || x.status == FM_FLOW_NONFINITE;
    };
    // the bracket: below T* the flow diverges before g_end, above it does not
    std::vector<double> Tv(n, T_hi);
    if (int rc = fm_flow_run_batch(h, n, U, Tv.data(), nullptr, nullptr, nullptr, r.data())) return rc;
    for (int f = 0; f < n; ++f) status[f] = diverged(r[f]) ? 1 : 0;
    std::fill(Tv.begin(), Tv.end(), T_lo);
    if (int rc = fm_flow_run_batch(h, n, U, Tv.data(), nullptr, nullptr, nullptr, r.data())) return rc;
    for (int f = 0; f < n; ++f)
        if (status[f] == 0 && !diverged(r[f])) status[f] = 2;
    const double width = std::log1p(rtol);
    for (;;) {
        idx.clear(); Ua.clear(); Ta.clear();
        for (int f = 0; f < n; ++f)
            if (status[f] == 0 && hi[f] - lo[f] > width) {
                idx.push_back(f);
                Ua.push_back(U[f]);
                Ta.push_back(std::exp(0.5 * (lo[f] + hi[f])));
            }
        if (idx.empty()) break;
        const int m = static_cast<int>(idx.size());
        if (int rc = fm_flow_run_batch(h, m, Ua.data(), Ta.data(), nullptr, nullptr, nullptr, r.data()))
            return rc;
        for (int i = 0; i < m; ++i) {
            const int f = idx[i];
            (diverged(r[i]) ? lo[f] : hi[f]) = std::log(Ta[i]);
        }
    }
    for (int f = 0; f < n; ++f) T_star[f] = status[f] == 0 ? std::exp(0.5 * (lo[f] + hi[f])) : nan;
    return FM_OK;
}

}  // extern "C"
