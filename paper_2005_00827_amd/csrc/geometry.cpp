// Host-side geometry of the loop grid and Fermi-surface patches, in double precision.
//
// Loop grid: half-shifted, k = -pi + 2 pi (j + 1/2)/L per axis, so it contains neither Gamma
// nor the zone boundary and, for even L, maps onto itself under k -> k + (pi, pi).  The loops
// run over the whole Brillouin zone (App. A, Comment 1: the interaction-flow propagators do
// not shrink around the Fermi surface).
//
// Patches: N angular sectors around Gamma with centres theta_off + 2 pi a / N; with N % 8 == 0
// they include the antinodal and nodal directions (Sec. 3.2 counts seven patches from
// antinode to node, 48 in total).  Each patch is represented by the Fermi-surface point on
// its centre ray (App. A, Step 2: quantities are projected onto the patch's Fermi point),
// snapped to the transfer grid 2 pi m / L so that all transfer bookkeeping is integer.
//
// Dispersion: Sec. 2.1, Eq. free_dispersion_xi.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>

#include "fm_internal.h"

namespace fm {
namespace {

struct Disp {
    double t, tp, mu;
    double operator()(double kx, double ky) const {
        double cx = std::cos(kx), cy = std::cos(ky);
        return -2.0 * t * (cx + cy) - 4.0 * tp * cx * cy - mu;
    }
};

inline int wrap(long v, int L) {
    long r = v % L;
    return static_cast<int>(r < 0 ? r + L : r);
}

double sector_offset(int N) {
    if (N == 1 || N % 8 == 0) return 0.0;
    if (N % 8 == 4) return M_PI / N;
    return std::nan("");
}

// Radius of the first point along the ray (cos th, sin th) inside the zone where xi equals
// `level` (0: the Fermi surface): scan 4096 equal steps from Gamma to the zone edge for the
// first sign change of xi - level and bisect it; without a sign change take the scanned
// radius of smallest |xi - level|.
double fermi_radius(const Disp& disp, double th, double level = 0.0) {
    const int n_scan = 4096;
    const double c = std::cos(th), s = std::sin(th);
    const double r_edge = M_PI / std::max(std::fabs(c), std::fabs(s));
    auto xi = [&](double kx, double ky) { return disp(kx, ky) - level; };
    double f_prev = xi(0.0, 0.0);
    if (f_prev == 0.0) return 0.0;
    double r_prev = 0.0, r_min = 0.0, f_min = std::fabs(f_prev);
    for (int i = 1; i <= n_scan; ++i) {
        const double r = r_edge * i / n_scan;
        const double f = xi(r * c, r * s);
        const bool crossed = (f_prev < 0.0) ? (f >= 0.0) : (f <= 0.0);
        if (crossed) {
            const bool neg_side = f_prev < 0.0;
            double lo = r_prev, hi = r;
            for (int it = 0; it < 200; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (!(mid > lo && mid < hi)) break;
                const double fm = xi(mid * c, mid * s);
                if ((fm < 0.0) == neg_side && fm != 0.0) lo = mid; else hi = mid;
            }
            return hi;
        }
        if (std::fabs(f) < f_min) { f_min = std::fabs(f); r_min = r; }
        r_prev = r;
        f_prev = f;
    }
    return r_min;
}

// Point-group operation o on a loop index (half-shifted grid: k -> -k is j -> L-1-j).
inline void op_point(int o, int L, int jx, int jy, int& ox, int& oy) {
    int x = (o & 4) ? jy : jx, y = (o & 4) ? jx : jy;
    if (o & 2) x = L - 1 - x;
    if (o & 1) y = L - 1 - y;
    ox = x; oy = y;
}

// The same operation on a transfer index (unshifted grid: q -> -q is m -> -m mod L).
inline int op_transfer(int o, int L, int m) {
    const int mx = m % L, my = m / L;
    int x = (o & 4) ? my : mx, y = (o & 4) ? mx : my;
    if (o & 2) x = (L - x) % L;
    if (o & 1) y = (L - y) % L;
    return x + L * y;
}

// Fills the permutation of patches that no loop point lies in (energy shells of a sector the
// band does not reach): within their shell, by the permutation of their sector learned from a
// patch of the same sector that has points.  False if that is impossible or the result is not
// a permutation mapping empty patches onto empty ones.
bool fill_empty(const HostGeometry& g, const std::vector<char>& used, int* p) {
    const int N = g.N, ns = g.nsec;
    for (int a = 0; a < N; ++a) {
        if (p[a] >= 0) continue;
        int s = -1;
        for (int b = a % ns; b < N && s < 0; b += ns)
            if (p[b] >= 0) s = p[b] % ns;
        if (s < 0) return false;
        p[a] = (a / ns) * ns + s;
    }
    std::vector<char> seen(N, 0);
    for (int a = 0; a < N; ++a) {
        if (seen[p[a]] || used[a] != used[p[a]]) return false;
        seen[p[a]] = 1;
    }
    return true;
}

void build_symmetry(HostGeometry& g) {
    const int N = g.N, L = g.L;
    std::vector<int> perm(8 * static_cast<size_t>(N), -1);
    std::vector<char> used(N, 0);
    for (int j = 0; j < g.np; ++j) used[g.patch[j]] = 1;
    bool ok = true;
    for (int o = 0; o < 8 && ok; ++o) {
        for (int jy = 0; jy < L && ok; ++jy)
            for (int jx = 0; jx < L && ok; ++jx) {
                int ox, oy;
                op_point(o, L, jx, jy, ox, oy);
                const int j = jx + L * jy, oj = ox + L * oy;
                const double d = std::fabs(g.xi[oj] - g.xi[j]);
                if (d > 1e-12 * std::max(1.0, std::fabs(g.xi[j]))) { ok = false; break; }
                int& p = perm[o * static_cast<size_t>(N) + g.patch[j]];
                if (p < 0) p = g.patch[oj];
                else if (p != g.patch[oj]) ok = false;
            }
        if (ok) ok = fill_empty(g, used, &perm[o * static_cast<size_t>(N)]);
    }
    g.sym = ok;
    // inversion k -> -k alone (operation 3), used to pair the particle-hole loop points of
    // phase 1: needs xi(-k) = xi(k) and a patch permutation P with patch(-k) = P(patch(k))
    {
        std::vector<int> p(N, -1);
        bool iok = true;
        for (int jy = 0; jy < L && iok; ++jy)
            for (int jx = 0; jx < L && iok; ++jx) {
                int ox, oy;
                op_point(3, L, jx, jy, ox, oy);
                const int j = jx + L * jy, oj = ox + L * oy;
                if (std::fabs(g.xi[oj] - g.xi[j]) > 1e-12 * std::max(1.0, std::fabs(g.xi[j]))) iok = false;
                else if (p[g.patch[j]] < 0) p[g.patch[j]] = g.patch[oj];
                else if (p[g.patch[j]] != g.patch[oj]) iok = false;
            }
        if (iok) iok = fill_empty(g, used, p.data());
        g.inv_ok = iok;
        g.inv_perm.resize(N);
        for (int a = 0; a < N; ++a) g.inv_perm[a] = iok ? p[a] : a;
    }
    g.pinv.assign(8 * static_cast<size_t>(N), 0);
    for (int o = 0; o < 8; ++o)
        for (int a = 0; a < N; ++a) {
            if (ok) g.pinv[o * static_cast<size_t>(N) + perm[o * static_cast<size_t>(N) + a]] = a;
            else g.pinv[o * static_cast<size_t>(N) + a] = a;
        }
    auto reduce = [&](const std::vector<int>& q, std::vector<int>& reps, std::vector<int>& qrep,
                      std::vector<int>& qg) {
        std::map<int, int> idx;
        for (size_t i = 0; i < q.size(); ++i) idx.emplace(q[i], static_cast<int>(i));
        qrep.assign(q.size(), -1);
        qg.assign(q.size(), 0);
        reps.clear();
        for (size_t i = 0; i < q.size(); ++i) {
            if (qrep[i] >= 0) continue;
            const int r = static_cast<int>(reps.size());
            reps.push_back(q[i]);
            qrep[i] = r;
            qg[i] = 0;
            if (!ok) continue;
            for (int o = 1; o < 8; ++o) {
                auto it = idx.find(op_transfer(o, L, q[i]));
                if (it != idx.end() && qrep[it->second] < 0) {
                    qrep[it->second] = r;
                    qg[it->second] = o;
                }
            }
        }
    };
    reduce(g.q_pp, g.rep_pp, g.qrep_pp, g.qg_pp);
    reduce(g.q_ph, g.rep_ph, g.qrep_ph, g.qg_ph);
    g.perm.assign(8 * static_cast<size_t>(N), 0);
    for (int o = 0; o < 8; ++o)
        for (int a = 0; a < N; ++a)
            g.perm[o * static_cast<size_t>(N) + a] = ok ? perm[o * static_cast<size_t>(N) + a] : a;
    // Transfers ordered by (operation, representative): the rows of a phase-2a tile then
    // share one point-group operation, whose patch permutation the kernel applies to the
    // operand it stages once instead of to every bin it reads.  The transfer index is only
    // a label; the maps are renumbered with it.
    auto order = [](std::vector<int>& q, std::vector<int>& qrep, std::vector<int>& qg,
                    std::vector<std::vector<int>*> maps, std::vector<int>& cls) {
        const size_t n = q.size();
        std::vector<int> idx(n);
        for (size_t i = 0; i < n; ++i) idx[i] = static_cast<int>(i);
        std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
            return qg[x] != qg[y] ? qg[x] < qg[y] : qrep[x] < qrep[y];
        });
        std::vector<int> pos(n), q2(n), r2(n), g2(n);
        for (size_t i = 0; i < n; ++i) {
            pos[idx[i]] = static_cast<int>(i);
            q2[i] = q[idx[i]];
            r2[i] = qrep[idx[i]];
            g2[i] = qg[idx[i]];
        }
        q.swap(q2);
        qrep.swap(r2);
        qg.swap(g2);
        for (auto* m : maps)
            for (int& v : *m) v = pos[v];
        cls.assign(9, 0);
        for (size_t i = 0; i < n; ++i) cls[qg[i] + 1]++;
        for (int o = 0; o < 8; ++o) cls[o + 1] += cls[o];
    };
    order(g.q_pp, g.qrep_pp, g.qg_pp, {&g.map_pp}, g.cls_pp);
    order(g.q_ph, g.qrep_ph, g.qg_ph, {&g.map_cr, &g.map_d}, g.cls_ph);
}

// Tables of the orbit phase-2a kernel, which reads each representative's bins once and
// produces every transfer of the representative's orbit from them.
//   Row tiles: per channel kind, the representatives in 16-row tiles, grouped by the set of
//   operations that yield their transfers (a tile holds one set; rows past a set's end are
//   -1), with the transfer index of each (tile, operation, row), -1 where none.
//   Patch groups: patches listed orbit by orbit, orbits by decreasing size, in groups of 8
//   (-1 padding).  Orbit sizes divide 8, so no orbit straddles two groups; the slabs of the
//   operand that a group's blocks read are those of its orbits.
void build_orbit_tables(HostGeometry& g) {
    const int N = g.N;
    g.orb_rows.clear();
    g.orb_q.clear();
    g.orb_mask.clear();
    for (int cc = 0; cc < 2; ++cc) {
        const std::vector<int>& qrep = cc == 0 ? g.qrep_pp : g.qrep_ph;
        const std::vector<int>& qg = cc == 0 ? g.qg_pp : g.qg_ph;
        const int nR = static_cast<int>(cc == 0 ? g.rep_pp.size() : g.rep_ph.size());
        std::vector<int> mask(nR, 0), qof(8 * static_cast<size_t>(nR), -1);
        for (size_t q = 0; q < qrep.size(); ++q) {
            mask[qrep[q]] |= 1 << qg[q];
            qof[static_cast<size_t>(qg[q]) * nR + qrep[q]] = static_cast<int>(q);
        }
        std::vector<int> idx(nR);
        for (int r = 0; r < nR; ++r) idx[r] = r;
        std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return mask[x] > mask[y]; });
        std::vector<int> rows;
        for (int i = 0; i < nR; ++i) {
            if (i > 0 && mask[idx[i]] != mask[idx[i - 1]])
                while (rows.size() % 16) rows.push_back(-1);
            rows.push_back(idx[i]);
        }
        while (rows.size() % 16) rows.push_back(-1);
        const int nt = static_cast<int>(rows.size() / 16);
        g.orb_nt[cc] = nt;
        for (int t = 0; t < nt; ++t) {
            int m = 0;
            for (int j = 0; j < 16; ++j)
                if (rows[16 * t + j] >= 0) m |= mask[rows[16 * t + j]];
            g.orb_mask.push_back(m);
            for (int o = 0; o < 8; ++o)
                for (int j = 0; j < 16; ++j) {
                    const int r = rows[16 * t + j];
                    g.orb_q.push_back(r < 0 ? -1 : qof[static_cast<size_t>(o) * nR + r]);
                }
        }
        g.orb_rows.insert(g.orb_rows.end(), rows.begin(), rows.end());
    }
    std::vector<int> seen(N, 0);
    std::vector<std::vector<int>> orbits;
    for (int a = 0; a < N; ++a) {
        if (seen[a]) continue;
        std::vector<int> orb;
        for (int o = 0; o < 8; ++o) {
            const int b = g.perm[o * static_cast<size_t>(N) + a];
            if (!seen[b]) { seen[b] = 1; orb.push_back(b); }
        }
        std::sort(orb.begin(), orb.end());
        orbits.push_back(orb);
    }
    std::stable_sort(orbits.begin(), orbits.end(),
                     [](const std::vector<int>& x, const std::vector<int>& y) { return x.size() > y.size(); });
    g.porder.clear();
    for (const auto& orb : orbits) g.porder.insert(g.porder.end(), orb.begin(), orb.end());
    while (g.porder.size() % 8) g.porder.push_back(-1);
}

void csr(const std::vector<int>& map, int nq, std::vector<int>& off, std::vector<int>& pairs) {
    off.assign(nq + 1, 0);
    for (int v : map) off[v + 1]++;
    for (int i = 0; i < nq; ++i) off[i + 1] += off[i];
    pairs.assign(map.size(), 0);
    std::vector<int> fill(off.begin(), off.end() - 1);
    for (size_t xy = 0; xy < map.size(); ++xy) pairs[fill[map[xy]]++] = static_cast<int>(xy);
}

void build_pairs(HostGeometry& g) {
    csr(g.map_pp, static_cast<int>(g.q_pp.size()), g.pp_off, g.pp_pairs);
    csr(g.map_cr, static_cast<int>(g.q_ph.size()), g.cr_off, g.cr_pairs);
    csr(g.map_d, static_cast<int>(g.q_ph.size()), g.d_off, g.d_pairs);
    const int chunk = 8;   // pairs per phase-2b work item (the kernel's kChunk)
    g.item_q.clear();
    g.item_p0.clear();
    g.item_rec.clear();
    const std::vector<int>* offs[3] = {&g.pp_off, &g.cr_off, &g.d_off};
    const std::vector<int>* prs[3] = {&g.pp_pairs, &g.cr_pairs, &g.d_pairs};
    for (int k = 0; k < 3; ++k) {
        const std::vector<int>& off = *offs[k];
        const std::vector<int>& pr = *prs[k];
        int n = 0;
        for (size_t q = 0; q + 1 < off.size(); ++q)
            for (int p = off[q]; p < off[q + 1]; p += chunk) {
                g.item_q.push_back(static_cast<int>(q));
                g.item_p0.push_back(p);
                // record: transfer, pair count, 2 spare, then the pairs (padded with the last)
                const int cnt = std::min(chunk, off[q + 1] - p);
                int rec[16] = {static_cast<int>(q), cnt, k, p};
                for (int i = 0; i < chunk; ++i) rec[4 + i] = pr[p + std::min(i, cnt - 1)];
                g.item_rec.insert(g.item_rec.end(), rec, rec + 16);
                ++n;
            }
        g.n_items[k] = n;
    }
    // fused phase 2: each transfer's pairs in rows of at most kFusedPairs, rows of one
    // operation class in whole blocks
    g.fz_row.clear();
    g.fz_pair.clear();
    g.fz_blk.clear();
    for (int k = 0; k < 3; ++k) {
        const std::vector<int>& off = *offs[k];
        const std::vector<int>& pr = *prs[k];
        const std::vector<int>& cls = k == 0 ? g.cls_pp : g.cls_ph;
        int nb = 0;
        for (int o = 0; o < 8; ++o) {
            const size_t r0 = g.fz_row.size();
            for (int q = cls[o]; q < cls[o + 1]; ++q)
                for (int p = off[q]; p < off[q + 1]; p += kFusedPairs) {
                    g.fz_row.push_back(q);
                    for (int i = 0; i < kFusedPairs; ++i)
                        g.fz_pair.push_back(p + i < off[q + 1] ? pr[p + i] : -1);
                }
            if (g.fz_row.size() == r0) continue;
            while ((g.fz_row.size() - r0) % kFusedRows) {
                g.fz_row.push_back(-1);
                for (int i = 0; i < kFusedPairs; ++i) g.fz_pair.push_back(-1);
            }
            for (size_t r = r0; r < g.fz_row.size(); r += kFusedRows) {
                g.fz_blk.push_back(o);
                g.fz_blk.push_back(static_cast<int>(r));
                ++nb;
            }
        }
        g.fz_nblk[k] = nb;
    }
    // symmetric states: per channel kind and representative r, the output pairs of every
    // transfer q = o(r) of r's orbit, each with its o, in items of at most kSymPairs
    g.sym_rec.clear();
    for (int k = 0; k < 3; ++k) {
        const std::vector<int>& off = *offs[k];
        const std::vector<int>& pr = *prs[k];
        const std::vector<int>& qrep = k == 0 ? g.qrep_pp : g.qrep_ph;
        const std::vector<int>& qg = k == 0 ? g.qg_pp : g.qg_ph;
        const int nr = static_cast<int>(k == 0 ? g.rep_pp.size() : g.rep_ph.size());
        std::vector<std::vector<int>> ent(nr);
        for (size_t q = 0; q + 1 < off.size(); ++q)
            for (int p = off[q]; p < off[q + 1]; ++p) ent[qrep[q]].push_back(pr[p] * 8 + qg[q]);
        int n = 0;
        for (int r = 0; r < nr; ++r)
            for (size_t e0 = 0; e0 < ent[r].size(); e0 += kSymPairs) {
                const int cnt = static_cast<int>(std::min<size_t>(kSymPairs, ent[r].size() - e0));
                const int head[4] = {r, cnt, k, 0};
                g.sym_rec.insert(g.sym_rec.end(), head, head + 4);
                for (int i = 0; i < kSymPairs; ++i)
                    g.sym_rec.push_back(i < cnt ? ent[r][e0 + i] : -1);
                ++n;
            }
        g.n_sym_items[k] = n;
    }
}

}  // namespace

bool build_geometry(const fm_config& cfg, HostGeometry& g, std::string& err) {
    const int N = cfg.N, L = cfg.L;
    char buf[256];
    if (L < 2 || (L % 2) != 0) { err = "L must be even and >= 2"; return false; }
    if (L > 2048) { err = "L must be <= 2048"; return false; }
    // energy shells: ns shells, m = (ns - 1)/2 edges E_1 < ... < E_m on each side of xi = 0
    const bool shells = cfg.geometry == FM_GEOM_SHELLS;
    const int ns = shells ? cfg.n_shells : 1;
    std::vector<double> edge;
    if (cfg.geometry == FM_GEOM_IDENTITY) {
        if (N != L * L) { err = "identity geometry needs N == L*L"; return false; }
    } else if (cfg.geometry == FM_GEOM_ANGULAR || shells) {
        if (shells && (ns < 1 || ns % 2 == 0 || N % ns != 0)) {
            err = "shell geometry needs an odd n_shells dividing N";
            return false;
        }
        const int Na = N / ns;
        if (Na < 1 || std::isnan(sector_offset(Na))) {
            err = "angular geometry needs N == 1 or N % 8 in {0, 4} (per shell)";
            return false;
        }
        if (L % 4 != 0) { err = "angular geometry needs L % 4 == 0"; return false; }
        const int m = (ns - 1) / 2;
        for (int k = 1; k <= m; ++k)
            edge.push_back(cfg.shell_edges ? cfg.shell_edges[k - 1]
                                           : 2.0 * std::fabs(cfg.t) * (std::ldexp(1.0, k) - 1.0) /
                                                 (std::ldexp(1.0, m) - 1.0));
        for (int k = 0; k < m; ++k)
            if (!(edge[k] > (k ? edge[k - 1] : 0.0)) || !std::isfinite(edge[k])) {
                err = "shell edges must be positive and ascending";
                return false;
            }
    } else {
        err = "unknown geometry";
        return false;
    }
    const Disp xi{cfg.t, cfg.tp, cfg.mu};
    g = HostGeometry{};
    g.N = N; g.L = L; g.np = L * L;
    g.identity = cfg.geometry == FM_GEOM_IDENTITY;
    const int Nsec = g.identity ? N : N / ns;
    g.nsec = Nsec;
    // shell of an energy: m - k below the Fermi surface, m + k above, k = edges below |x|
    const int m = (ns - 1) / 2;
    auto shell_of = [&](double x) {
        int k = 0;
        while (k < m && std::fabs(x) > edge[k]) ++k;
        return x < 0.0 ? m - k : m + k;
    };
    double emargin = INFINITY;   // smallest distance of a loop point's |xi| to an edge
    g.xi.resize(g.np);
    g.patch.resize(g.np);
    g.anchor.resize(2 * N);
    std::vector<double> kg(L);
    for (int j = 0; j < L; ++j) kg[j] = -M_PI + 2.0 * M_PI * (j + 0.5) / L;
    const double off = g.identity ? 0.0 : sector_offset(Nsec);
    g.margin = 0.5;
    for (int jy = 0; jy < L; ++jy) {
        for (int jx = 0; jx < L; ++jx) {
            const int j = jx + L * jy;
            g.xi[j] = xi(kg[jx], kg[jy]);
            if (g.identity) { g.patch[j] = j; continue; }
            const double u = (std::atan2(kg[jy], kg[jx]) - off) * Nsec / (2.0 * M_PI);
            const double r = std::round(u);   // nearest centre (ties cannot pass the margin test)
            g.margin = std::min(g.margin, 0.5 - std::fabs(u - r));
            g.patch[j] = shell_of(g.xi[j]) * Nsec + wrap(static_cast<long>(r), Nsec);
            for (double e : edge) emargin = std::min(emargin, std::fabs(std::fabs(g.xi[j]) - e));
        }
    }
    if (!g.identity && g.margin < 1e-9) {
        std::snprintf(buf, sizeof buf, "a loop point lies %.3g sectors from a patch boundary",
                      g.margin);
        err = buf;
        return false;
    }
    if (emargin < 1e-9) {
        std::snprintf(buf, sizeof buf, "a loop point lies %.3g from a shell edge", emargin);
        err = buf;
        return false;
    }
    g.kpt.resize(2 * static_cast<size_t>(N));
    if (g.identity) {
        for (int a = 0; a < N; ++a) {
            g.anchor[2 * a] = a % L; g.anchor[2 * a + 1] = a / L;
            g.kpt[2 * a] = kg[a % L]; g.kpt[2 * a + 1] = kg[a / L];
        }
        g.pp_shift = 1;   // k_a + k_b of two half-shifted points has index ja + jb + 1
    } else {
        for (int a = 0; a < N; ++a) {
            // representative energy of the patch's shell: 0 on the Fermi surface, the middle
            // of an inner shell, the outermost shell's edge plus half the width below it
            const int e = a / Nsec, k = std::abs(e - m);
            double level = 0.0;
            if (k > 0) {
                const double lo = edge[k - 1], below = k > 1 ? edge[k - 2] : 0.0;
                level = k < m ? 0.5 * (lo + edge[k]) : lo + 0.5 * (lo - below);
                if (e < m) level = -level;
            }
            const double th = off + 2.0 * M_PI * (a % Nsec) / Nsec;
            const double r = fermi_radius(xi, th, level);
            const double kx = r * std::cos(th), ky = r * std::sin(th);
            g.kpt[2 * a] = kx;
            g.kpt[2 * a + 1] = ky;
            g.anchor[2 * a] = wrap(std::lround(kx * L / (2.0 * M_PI)), L);
            g.anchor[2 * a + 1] = wrap(std::lround(ky * L / (2.0 * M_PI)), L);
        }
        g.pp_shift = 0;
    }
    // distinct transfers, first-occurrence order
    std::map<int, int> ipp, iph;
    auto intern = [](std::map<int, int>& m, std::vector<int>& list, int key) {
        auto it = m.find(key);
        if (it != m.end()) return it->second;
        const int id = static_cast<int>(list.size());
        m.emplace(key, id);
        list.push_back(key);
        return id;
    };
    auto flat = [L](int mx, int my) { return wrap(mx, L) + L * wrap(my, L); };
    g.map_pp.resize(static_cast<size_t>(N) * N);
    g.map_cr.resize(static_cast<size_t>(N) * N);
    g.map_d.resize(static_cast<size_t>(N) * N);
    for (int x = 0; x < N; ++x) {
        for (int y = 0; y < N; ++y) {
            const int* ax = &g.anchor[2 * x];
            const int* ay = &g.anchor[2 * y];
            g.map_pp[x * N + y] = intern(ipp, g.q_pp, flat(ax[0] + ay[0] + g.pp_shift,
                                                           ax[1] + ay[1] + g.pp_shift));
            // k_x - k_y: map_d uses (a, c) = (x, y); map_cr uses (b, c) with k_c - k_b
            g.map_d[x * N + y] = intern(iph, g.q_ph, flat(ax[0] - ay[0], ax[1] - ay[1]));
        }
    }
    for (int b = 0; b < N; ++b)
        for (int c = 0; c < N; ++c) {
            const int* ab = &g.anchor[2 * b];
            const int* ac = &g.anchor[2 * c];
            g.map_cr[b * N + c] = intern(iph, g.q_ph, flat(ac[0] - ab[0], ac[1] - ab[1]));
        }
    build_symmetry(g);
    build_orbit_tables(g);
    build_pairs(g);
    return true;
}

}  // namespace fm
