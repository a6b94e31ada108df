// fm_flow_rhs_static: the right-hand side of fm_flow_rhs for callers that cannot allocate
// device memory.  The handle's whole workspace (geometry tables, bins, stage operands,
// products and k slots) is carved out of one file-scope device array instead of a caller
// allocation; nothing here calls hipMalloc, hipFree or an allocating library routine.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fm_internal.h"

namespace {

// Largest workspace a static handle may use: one flow of the N = 48, L = 128 workloads in
// single or double precision (at most 80 MiB) fits.
constexpr size_t kScratchBytes = size_t(96) << 20;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

int fail(int code, const std::string& msg) {
    fm::set_last_error(msg);
    return code;
}

// One static handle per device, with the configuration it was built for (host arrays copied,
// so that a later call with equal values reuses the handle).
struct Slot {
    bool have_ptr = false;
    void* ptr = nullptr;          // device address of `scratch` on this device
    fm_flow* h = nullptr;
    fm_config cfg{};
    std::vector<double> zl, zt;
};

std::mutex g_mu;
std::vector<Slot> g_slots;

bool same_config(const Slot& s, const fm_config& c) {
    if (!s.h) return false;
    const fm_config& a = s.cfg;
    const bool same = a.t == c.t && a.tp == c.tp && a.mu == c.mu && a.U == c.U &&
                      a.geometry == c.geometry && a.N == c.N && a.L == c.L && a.T0 == c.T0 &&
                      a.T_end == c.T_end && a.integrator == c.integrator &&
                      a.n_steps == c.n_steps && a.rtol == c.rtol && a.atol == c.atol &&
                      a.h0 == c.h0 && a.h_min == c.h_min && a.v_max == c.v_max &&
                      a.channels == c.channels && a.precision == c.precision &&
                      a.n_zT == c.n_zT && a.stream == c.stream && a.max_batch == c.max_batch &&
                      a.tile_rows == c.tile_rows && a.flow == c.flow && a.g_end == c.g_end &&
                      a.v_rel == c.v_rel && a.y_kernel == c.y_kernel &&
                      a.sync_batch == c.sync_batch && a.n_shells == c.n_shells &&
                      a.shell_edges == nullptr && c.shell_edges == nullptr &&
                      a.k_table == nullptr && c.k_table == nullptr &&
                      a.phase1_variant == c.phase1_variant && a.sym_state == c.sym_state;
    if (!same) return false;
    if (c.n_zT <= 0) return true;
    const size_t nz = static_cast<size_t>(c.n_zT), nt = nz * static_cast<size_t>(c.N);
    return s.zl.size() == nz && s.zt.size() == nt &&
           std::memcmp(s.zl.data(), c.z_lnT, nz * sizeof(double)) == 0 &&
           std::memcmp(s.zt.data(), c.z_table, nt * sizeof(double)) == 0;
}

}  // namespace

extern "C" int fm_flow_rhs_static(const fm_config* cfg, int batch, const double* T,
                                  const double* V_dev, double* dV_dev) {
    if (!cfg) return fail(FM_EINVAL, "null config");
    if (cfg->n_zT > 0 && (!cfg->z_lnT || !cfg->z_table)) return fail(FM_EINVAL, "bad Z table");
    if (batch < 1 || batch > cfg->max_batch) return fail(FM_EINVAL, "batch outside [1, max_batch]");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(FM_EDEVICE, "hipGetDevice failed");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_slots.size() <= static_cast<size_t>(dev)) g_slots.resize(dev + 1);
    Slot& s = g_slots[dev];
    if (!s.have_ptr) {
        // the array's address on this device (each device holds its own copy); host code
        // uses only this pointer, never the array's name
        hipError_t e = hipGetSymbolAddress(&s.ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !s.ptr)
            return fail(FM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                        hipGetErrorString(e));
        s.have_ptr = true;
    }
    if (!same_config(s, *cfg)) {
        size_t need = 0;
        if (int rc = fm_flow_workspace_bytes(cfg, &need)) return rc;
        if (need > kScratchBytes)
            return fail(FM_EINVAL, "fm_flow_rhs_static: the configuration needs " +
                                       std::to_string(need) + " bytes of workspace, more than the " +
                                       std::to_string(kScratchBytes) + " of the static array");
        if (s.h) {
            // the previous handle's work may still read the array: finish it first
            (void)hipStreamSynchronize(static_cast<hipStream_t>(s.cfg.stream));
            fm_flow_destroy(s.h);
            s.h = nullptr;
        }
        fm_flow* h = nullptr;
        if (int rc = fm_flow_init(cfg, s.ptr, kScratchBytes, &h)) return rc;
        s.h = h;
        s.cfg = *cfg;
        const size_t nz = cfg->n_zT > 0 ? static_cast<size_t>(cfg->n_zT) : 0;
        s.zl.assign(cfg->z_lnT, cfg->z_lnT + nz);
        s.zt.assign(cfg->z_table, cfg->z_table + nz * static_cast<size_t>(cfg->N));
    }
    return fm_flow_rhs(s.h, batch, T, V_dev, dV_dev);
}
