// gfx950 kernels of the one-loop temperature-flow right-hand side and its integrator.
//
// Right-hand side (App. A, Eq. vertex_flow_general with Z on internal lines as in
// Eq. vertex_flow_feedback_Z, written out per channel for the spin-rotation-invariant
// coupling function, temperature flow s = ln T):
//
//   dV/ds(a,b,c) = - sum_{a'b'} Bpp_{k1+k2}(a',b') Z_a' Z_b' V(a,b,a') V(a',b',c)
//                  + sum_{a'b'} Bph_{k3-k2}(a',b') Z_a' Z_b' V(a,a',b') V(b',b,c)
//                  + sum_{a'b'} Bph_{k1-k3}(a',b') Z_a' Z_b' [ -2 V(a,a',c) V(b',b,a')
//                                     + V(a',a,c) V(b',b,a') + V(a,a',c) V(b,b',a') ]
//
// with the bins B_q(a',b') = (1/L^2) sum over loop points j whose line pair (j, j') falls in
// patches (a', b') of T d/dT chi(xi_j, xi_j'), j' = q - j (particle-particle) or j + q
// (particle-hole).  The bins are an exact regrouping of the loop sum.
//
// Stage and phase 1 (k_stage_bins, one launch): the stage argument and its operand layouts,
//   and in the same grid the bubble-weight derivatives, evaluated on the fly for every loop
//   point j and every representative transfer q (one per orbit of the lattice point group),
//   summed into per-transfer bin matrices held in LDS.
// Phase 2a (k_y_mfma_rows / k_y_mfma_cls on matrix cores, k_y on vector units): per-transfer
//   grouped products
//   Y_q = B_q x V-slab, four kinds.
// Phase 2b (k_contract): the remaining contraction over one patch index per channel,
//   written straight into the stage's k slot, one part per channel.
// Integrator (k_rk4_update, k_dopri_err, k_finish, k_commit): double precision.
// Z weights: a line pair (a', b') carries Z_a' Z_b' (al + be (W_a' + W_b')) per flow, with
// (al, be) = (1, 0) for the temperature flow and (0, g) for the interaction flow, where W = Z,
// or W = K Z with the Katanin factors K on the single-scale line (App. A, Step 3: dG/dg =
// K Z^2 G0 replaces S = Z^2 G0, Eq. vertex_flow_feedback_Z_with_Katanin).  The stage writes Z
// and W per flow, [flow][2][N].
// Direct path (k_wtable, k_direct): the same sums over every loop point, no bins.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "fm_internal.h"

namespace fm {
namespace {

constexpr int kThreads = 256;
constexpr int kStepThreads = 1024;   // integrator kernels: one 8 x 8 x 16 tile per block round

__device__ inline int wrapi(int v, int L) {
    int r = v % L;
    return r < 0 ? r + L : r;
}

// Partner of loop point j (jx + L jy) for transfer m (mx + L my).
__device__ inline int partner_pp(int m, int j, int L) {
    const int jy = j / L, jx = j - jy * L;
    const int my = m / L, mx = m - my * L;
    return wrapi(mx - jx - 1, L) + L * wrapi(my - jy - 1, L);
}
__device__ inline int partner_ph(int m, int j, int L) {
    const int jy = j / L, jx = j - jy * L;
    const int my = m / L, mx = m - my * L;
    return wrapi(jx + mx, L) + L * wrapi(jy + my, L);
}

// phi(u) = u sech^2 u, from exp(-2|u|) only (no overflow).
__device__ inline double phi_d(double u) {
    const double e = exp(-2.0 * fabs(u));
    const double d = 1.0 + e;
    return 4.0 * u * e / (d * d);
}

// Divided difference phi[a,b] given pa = phi(a), pb = phi(b).  Away from a == b it is the
// plain quotient; within |a-b| < cut it is the Taylor series about the midpoint m,
//   phi[a,b] = phi'(m) + phi'''(m) d^2/24 + phi^(5)(m) d^4/1920 + O(d^6),  d = a - b,
// with, for s = sech^2 m, tau = tanh m,
//   phi'     = s (1 - 2 m tau)
//   phi'''   = s (-6 (1 - 3 tau^2) + 8 m tau (2 - 3 tau^2))
//   phi^(5)  = s (40 (2 - 15 tau^2 + 15 tau^4) - 16 m tau (17 - 60 tau^2 + 45 tau^4)).
template <typename R> struct WeightCut;
template <> struct WeightCut<float> { static constexpr float v = 0.1f; };
template <> struct WeightCut<double> { static constexpr double v = 0.01; };

__device__ inline float quot(float x, float y) { return x * __builtin_amdgcn_rcpf(y); }
__device__ inline double quot(double x, double y) { return x / y; }

template <typename R>
__device__ inline R phi_dd(R a, R pa, R b, R pb) {
    const R d = a - b;
    if (fabs(d) >= WeightCut<R>::v) return quot(pa - pb, d);
    const R m = R(0.5) * (a + b);
    const R e = exp(R(-2) * fabs(m));
    const R rden = quot(R(1), R(1) + e);
    const R s = R(4) * e * rden * rden;
    const R tau = copysign((R(1) - e) * rden, m);
    const R t2 = tau * tau;
    const R mt = m * tau;
    const R d2 = d * d;
    const R p1 = R(1) - R(2) * mt;
    const R p3 = R(-6) * (R(1) - R(3) * t2) + R(8) * mt * (R(2) - R(3) * t2);
    const R p5 = R(40) * (R(2) - R(15) * t2 + R(15) * t2 * t2) -
                 R(16) * mt * (R(17) - R(60) * t2 + R(45) * t2 * t2);
    return s * (p1 + d2 * (p3 * (R(1) / R(24)) + d2 * p5 * (R(1) / R(1920))));
}

__device__ inline double z_interp(const DevZ& z, int f, int N, int a, double lnT) {
    if (z.n <= 0) return 1.0;
    const double* x = z.lnT + static_cast<size_t>(f) * z.n;
    const double* t = z.tab + static_cast<size_t>(f) * z.n * N;
    if (z.n == 1 || lnT <= x[0]) return t[a];
    if (lnT >= x[z.n - 1]) return t[static_cast<size_t>(z.n - 1) * N + a];
    int i = 0;
    while (i + 1 < z.n - 1 && x[i + 1] <= lnT) ++i;
    const double w = (lnT - x[i]) / (x[i + 1] - x[i]);
    return (1.0 - w) * t[static_cast<size_t>(i) * N + a] + w * t[static_cast<size_t>(i + 1) * N + a];
}

// Katanin factor K of patch a (the K table shares the Z table's nodes); 1 without one.
__device__ inline double k_interp(const DevZ& z, int f, int N, int a, double lnT) {
    if (!z.ktab) return 1.0;
    const DevZ zk{z.n, z.lnT, z.ktab, nullptr};
    return z_interp(zk, f, N, a, lnT);
}

__device__ inline bool running(const FlowState* fs, int f) { return fs[f].status == FM_FLOW_RUNNING; }

// The flow whose phase-1 bins flow f reads: its own, or, for flows that share one step
// schedule (and so every stage temperature), the group's first running flow.
__device__ inline int bin_flow(const FlowState* fs, int f) {
    const int b = fs[f].bshare;
    return b ? b - 1 : f;
}

// k slots [slot][flow][pp, crossed, direct][N^3] (R).  Each channel part is stored in the
// order phase 2b writes it: a phase-2b lane owns the free index n of an output pair's row,
//   pp part       V(x,y,z) at (x N + y) N + z   (n = z)
//   crossed part  V(x,y,z) at (y N + z) N + x   (n = x)
//   direct part   V(x,y,z) at (x N + z) N + y   (n = y)
// so each of its stores is contiguous over the wave.  The first kernel after phase 2b that
// needs a slot (the next stage argument, or the step's update or error norm for the last slot)
// tiles the cube, brings the crossed and direct parts to V order through LDS (tile_parts, each
// read along its own contiguous index), and writes the slot's sum (pp + crossed) + direct,
// rounded to R as each addition is, to ksum[slot][flow][N^3] in V order; later readers in the
// same step read that sum.
__host__ __device__ inline size_t kpos(int ch, int N, int x, int y, int z) {
    const size_t n = static_cast<size_t>(N);
    return ch == 0 ? (x * n + y) * n + z : (ch == 1 ? (y * n + z) * n + x : (x * n + z) * n + y);
}

// k of stage l, flow f, element (x, y, z): the three parts summed in that order.
template <typename R>
__device__ inline R kval_at(const R* K, int l, int B, int f, size_t N3, int N, int x, int y,
                            int z) {
    const R* p = K + (static_cast<size_t>(l) * B + f) * 3 * N3;
    R v = p[kpos(0, N, x, y, z)];
    v += p[N3 + kpos(1, N, x, y, z)];
    v += p[2 * N3 + kpos(2, N, x, y, z)];
    return v;
}

// Element tiles of w (x) x w (y) x 16 (z), w = 2^TL, with padded LDS strides; tile t of a
// flow starts at (x0, y0, z0), z fastest over t.
constexpr int kTZ = 16, kTSY = kTZ + 1;

__host__ __device__ inline int stage_tiles(int N, int tl) {
    const int w = 1 << tl, nx = (N + w - 1) / w;
    return nx * nx * ((N + kTZ - 1) / kTZ);
}
__host__ __device__ constexpr int stage_tile_lds(int tl) {  // elements of one LDS tile
    return (1 << tl) * ((1 << tl) * kTSY + 1);
}
__device__ inline void tile_origin(int t, int N, int tl, int& x0, int& y0, int& z0) {
    const int nx = (N + (1 << tl) - 1) >> tl, nz = (N + kTZ - 1) / kTZ;
    const int txy = t / nz;
    x0 = (txy / nx) << tl;
    y0 = (txy % nx) << tl;
    z0 = (t - txy * nz) * kTZ;
}

// The crossed and direct parts of one k slot (Kp: the slot's flow base) at one tile's
// elements, read along x and along y respectively, left in LDS (exactly, as double) at the
// element's tile position; the caller synchronises before use.
template <int TL, typename R>
__device__ inline void tile_parts(const R* Kp, size_t N3, int N, int x0, int y0, int z0,
                                  double* p1, double* p2) {
    constexpr int w = 1 << TL, m = w - 1, tsx = w * kTSY + 1, tile_n = kTZ * w * w;
    for (int e = threadIdx.x; e < tile_n; e += blockDim.x) {
        const int u = e & m, v = (e >> TL) & m, lz = e >> (2 * TL);
        const int zz = z0 + lz;
        // crossed: (lx, ly) = (u, v); direct: (lx, ly) = (v, u)
        const bool ok1 = x0 + u < N && y0 + v < N && zz < N;
        const bool ok2 = x0 + v < N && y0 + u < N && zz < N;
        const R k1 = Kp[N3 + (ok1 ? kpos(1, N, x0 + u, y0 + v, zz) : 0)];
        const R k2 = Kp[2 * N3 + (ok2 ? kpos(2, N, x0 + v, y0 + u, zz) : 0)];
        if (ok1) p1[u * tsx + v * kTSY + lz] = static_cast<double>(k1);
        if (ok2) p2[v * tsx + u * kTSY + lz] = static_cast<double>(k2);
    }
}

// Sum of the three parts of a slot at one element, in the order and precision kval_at uses.
template <typename R>
__device__ inline R part_sum(R pp, double cr, double d) {
    R v = pp;
    v += static_cast<R>(cr);
    v += static_cast<R>(d);
    return v;
}

// The stage argument is formed in element tiles, w = 8 or 16 (chosen per launch).  The newest
// slot's crossed and direct parts go to LDS first (tile_parts); then each element's loads
// (the newest slot's pp part, the earlier slots' sums, V) are summed as the slots' order
// gives, V_s = V + h sum_l a_l k_l, the newest slot's sum is written to ksum, V_s and v0 are
// written along z, and V_s in operand precision takes the element's crossed-part slot (read
// only by the same thread), from which va is written along y and vc along x, w consecutive
// elements per run.  LDS: two double tiles.
template <int NS, int TL, int BT, bool PRE, typename R>
__device__ inline void stage_elems(const DevGeom& g, const StageCoef& sc, double ht, int f,
                                   int write_new, const double* Vf, const R* K, R* KS,
                                   double* Vnew, R* v0, R* va, R* vc, int B, double* tile,
                                   int blk, int nblk) {
    const int N = g.N, NN = g.NN;
    const size_t N3 = static_cast<size_t>(NN) * N;
    constexpr int tl = TL, w = 1 << tl, m = w - 1, tsx = w * kTSY + 1, tile_n = kTZ * w * w;
    constexpr int NL = NS > 0 ? NS : 1;
    // with PRE (and at most 96 bytes of them per thread) this thread's element loads are
    // issued before the LDS parts and held in registers across the barrier: one memory round
    // trip per tile instead of two
    constexpr int EPT = tile_n / BT;
    constexpr bool kPre = PRE && EPT * NS * sizeof(R) <= 96;
    double* p1 = tile;
    double* p2 = tile + stage_tile_lds(TL);
    const int ntile = stage_tiles(N, tl);
    R* v0f = v0 + f * N3;
    R* vaf = va + f * N3;
    R* vcf = vc + f * N3;
    const size_t ks = static_cast<size_t>(B) * N3;               // ksum slot stride
    const R* Kn = K + ((static_cast<size_t>(NL - 1) * B + f) * 3) * N3;   // newest slot, flow f
    const R* KSf = KS + static_cast<size_t>(f) * N3;
    R* KSn = KS + (static_cast<size_t>(NL - 1) * B + f) * N3;
    for (int t = blk; t < ntile; t += nblk) {          // uniform over the block
        int x0, y0, z0;
        tile_origin(t, N, tl, x0, y0, z0);
        R kp[kPre ? EPT : 1][NL];
        double vp[kPre ? EPT : 1];
        if constexpr (kPre) {
#pragma unroll
            for (int r = 0; r < EPT; ++r) {
                const int e = threadIdx.x + r * BT;
                const int lz = e & (kTZ - 1), ly = (e >> 4) & m, lx = e >> (4 + tl);
                const int x = x0 + lx, y = y0 + ly, zz = z0 + lz;
                const size_t i =
                    x < N && y < N && zz < N ? (static_cast<size_t>(x) * N + y) * N + zz : 0;
#pragma unroll
                for (int l = 0; l + 1 < NS; ++l) kp[r][l] = KSf[l * ks + i];
                if constexpr (NS > 0) kp[r][NS - 1] = Kn[i];
                vp[r] = Vf[i];
            }
        }
        if constexpr (NS > 0) {
            tile_parts<TL>(Kn, N3, N, x0, y0, z0, p1, p2);
            __syncthreads();
        }
        // unrolled only with the preload (else one element's loads at a time)
#pragma unroll (kPre ? EPT : 1)
        for (int r = 0; r < EPT; ++r) {
            const int e = threadIdx.x + r * BT;
            const int lz = e & (kTZ - 1), ly = (e >> 4) & m, lx = e >> (4 + tl);
            const int x = x0 + lx, y = y0 + ly, zz = z0 + lz;
            if (x >= N || y >= N || zz >= N) continue;
            const size_t i = (static_cast<size_t>(x) * N + y) * N + zz;
            const int j = lx * tsx + ly * kTSY + lz;
            R kv[NL];
            double vb;
            if constexpr (kPre) {
#pragma unroll
                for (int l = 0; l < NS; ++l) kv[l] = kp[r][l];
                vb = vp[r];
            } else {
#pragma unroll
                for (int l = 0; l + 1 < NS; ++l) kv[l] = KSf[l * ks + i];
                if constexpr (NS > 0) kv[NS - 1] = Kn[i];
                vb = Vf[i];
            }
            double acc = 0.0;
            if constexpr (NS > 0) {
                kv[NS - 1] = part_sum(kv[NS - 1], p1[j], p2[j]);
                KSn[i] = kv[NS - 1];
            }
#pragma unroll
            for (int l = 0; l < NS; ++l) acc += sc.a[l] * static_cast<double>(kv[l]);
            const double v = vb + ht * acc;
            if (write_new) Vnew[f * N3 + i] = v;
            const R rv = static_cast<R>(v);
            v0f[i] = rv;
            p1[j] = static_cast<double>(rv);
        }
        __syncthreads();
        // va[z][x][y]: runs along y
        for (int e = threadIdx.x; e < tile_n; e += BT) {
            const int ly = e & m, lx = (e >> tl) & m, lz = e >> (2 * tl);
            const int x = x0 + lx, y = y0 + ly, zz = z0 + lz;
            if (x < N && y < N && zz < N)
                vaf[static_cast<size_t>(zz) * NN + x * N + y] =
                    static_cast<R>(p1[lx * tsx + ly * kTSY + lz]);
        }
        // vc[z][y][x]: runs along x
        for (int e = threadIdx.x; e < tile_n; e += BT) {
            const int lx = e & m, ly = (e >> tl) & m, lz = e >> (2 * tl);
            const int x = x0 + lx, y = y0 + ly, zz = z0 + lz;
            if (x < N && y < N && zz < N)
                vcf[static_cast<size_t>(zz) * NN + y * N + x] =
                    static_cast<R>(p1[lx * tsx + ly * kTSY + lz]);
        }
        __syncthreads();                                // the tiles are rewritten next round
    }
}

// The tile width as a compile-time constant (a run-time width costs 17% at 16 wide).
template <int NS, int BT, bool PRE, typename R>
__device__ inline void stage_ns(const DevGeom& g, const StageCoef& sc, double ht, int f,
                                int write_new, const double* Vf, const R* K, R* KS,
                                double* Vnew, R* v0, R* va, R* vc, int B, double* tile, int tl,
                                int blk, int nblk) {
    if (tl == 4)
        stage_elems<NS, 4, BT, PRE>(g, sc, ht, f, write_new, Vf, K, KS, Vnew, v0, va, vc, B, tile,
                                    blk, nblk);
    else
        stage_elems<NS, 3, BT, PRE>(g, sc, ht, f, write_new, Vf, K, KS, Vnew, v0, va, vc, B, tile,
                                    blk, nblk);
}

template <typename R, int BT, bool PRE>
__device__ inline void stage_part(const DevGeom& g, const DevZ& z, const FlowState& st, int f,
                                  const StageCoef& sc, int write_new, const double* Vbase,
                                  const R* K, R* KS, double* Vnew, R* v0, R* va, R* vc,
                                  double* T_stage, double* Z_stage, double* zw, int B,
                                  double* tile, int tl, int blk, int nblk) {
    const int N = g.N;
    const size_t N3 = static_cast<size_t>(g.NN) * N;
    const double ht = st.ht;
    const double lnTs = st.lnT + sc.c * ht;
    if (blk == 0) {
        if (threadIdx.x == 0) {
            T_stage[f] = st.gflow ? st.Tfix : exp(lnTs);
            zw[2 * f] = st.gflow ? 0.0 : 1.0;
            zw[2 * f + 1] = st.gflow ? lnTs : 0.0;
        }
        for (int a = threadIdx.x; a < N; a += blockDim.x) {
            const double za = z_interp(z, f, N, a, lnTs);
            Z_stage[static_cast<size_t>(f) * 2 * N + a] = za;
            Z_stage[static_cast<size_t>(f) * 2 * N + N + a] = z.ktab ? za * k_interp(z, f, N, a, lnTs) : za;
        }
    }
    const double* Vf = Vbase + f * N3;
    switch (sc.ns) {                                   // uniform: earlier stages of this stage
    case 0:
        stage_ns<0, BT, PRE>(g, sc, ht, f, write_new, Vf, K, KS, Vnew, v0, va, vc, B, tile, tl, blk,
                             nblk);
        break;
    case 1:
        stage_ns<1, BT, PRE>(g, sc, ht, f, write_new, Vf, K, KS, Vnew, v0, va, vc, B, tile, tl, blk,
                             nblk);
        break;
    case 2:
        stage_ns<2, BT, PRE>(g, sc, ht, f, write_new, Vf, K, KS, Vnew, v0, va, vc, B, tile, tl, blk,
                             nblk);
        break;
    case 3:
        stage_ns<3, BT, PRE>(g, sc, ht, f, write_new, Vf, K, KS, Vnew, v0, va, vc, B, tile, tl, blk,
                             nblk);
        break;
    case 4:
        stage_ns<4, BT, PRE>(g, sc, ht, f, write_new, Vf, K, KS, Vnew, v0, va, vc, B, tile, tl, blk,
                             nblk);
        break;
    case 5:
        stage_ns<5, BT, PRE>(g, sc, ht, f, write_new, Vf, K, KS, Vnew, v0, va, vc, B, tile, tl, blk,
                             nblk);
        break;
    default:
        stage_ns<6, BT, PRE>(g, sc, ht, f, write_new, Vf, K, KS, Vnew, v0, va, vc, B, tile, tl, blk,
                             nblk);
        break;
    }
}


// Point quantities at the stage temperature, a = xi / 2T (single precision: xi rounded to
// float times 1/2T rounded to float):
//   single precision (a, phi(a), phi'(a), phi3(a)), double precision (a, phi(a)),
// where phi(u) = u sech^2 u, phi' = s (1 - 2 a tau) and the third derivative
//   phi3 = s (-6 (1 - 3 tau^2) + 8 a tau (2 - 3 tau^2)),  s = sech^2 a, tau = tanh a,
// with s and tau from e = exp(-2|a|) <= 1 (no overflow): s = 4e/(1+e)^2, |tau| = (1-e)/(1+e).

__device__ inline float4 point_q(float xi, float inv2T) {
    const float a = xi * inv2T;
    const float e = __expf(-2.0f * fabsf(a));
    const float rd = __builtin_amdgcn_rcpf(1.0f + e);
    const float sh = 4.0f * e * rd * rd;
    const float tau = copysignf((1.0f - e) * rd, a);
    const float t2 = tau * tau, at = a * tau;
    return make_float4(a, a * sh, sh * (1.0f - 2.0f * at),
                       sh * (-6.0f * (1.0f - 3.0f * t2) + 8.0f * at * (2.0f - 3.0f * t2)));
}
__device__ inline double2 point_q(double xi, double twoT) {
    const double a = xi / twoT;
    return make_double2(a, phi_d(a));
}

// Single-precision weight phi[a,b] without branches: away from a == b the quotient;
// within |a - b| < 0.05 the trapezoid value with its end correction,
//   phi[a,b] = (phi'(a) + phi'(b))/2 - (a-b)^2 (phi3(a) + phi3(b))/24 + O((a-b)^4).
__device__ inline float phi_dd_pt(float4 u, float4 v) {
    const float d = u.x - v.x;
    const float qt = (u.y - v.y) * __builtin_amdgcn_rcpf(d);
    const float sr = 0.5f * (u.z + v.z) - (d * d) * (u.w + v.w) * (1.0f / 24.0f);
    return fabsf(d) >= 0.05f ? qt : sr;
}
__device__ inline double phi_dd_pt(double2 u, double2 v) { return phi_dd<double>(u.x, u.y, v.x, v.y); }
// Particle-particle partner: chi_pp(x, y) = chi_ph(x, -y); a and phi are odd in a, phi'
// and phi3 even.
__device__ inline float4 flip(float4 v) { return make_float4(-v.x, -v.y, v.z, v.w); }
__device__ inline double2 flip(double2 v) { return make_double2(-v.x, -v.y); }

// Single-precision weight of one loop-point pair for phase 1, straight from xi: a quarter of
// phi_dd_pt(point_q(.), point_q(.)) (the factor 4 goes into the bins' scale).  With
// e = exp(-2|x|), p = 1 + e and sech^2 x = 4e/p^2, the quotient away from the diagonal is
//   phi[a,b] = (a s_a - b s_b)/(a - b) = 4 (a e_a p_b^2 - b e_b p_a^2) / ((a - b) p_a^2 p_b^2)
// (p in [1, 2]: one reciprocal instead of three).  Arguments: tp = 1/2T, tq = 1/2T, or -1/2T
// for particle-particle (b = -xv/2T), and ce = -log2(e)/T, so that e_a = exp2(ce |xu|).
// phi', phi3 and the trapezoid are evaluated for the lanes with |a - b| < 0.05 only (a branch
// the wave skips when none has), with tanh entering only as |a| tanh|a| and tanh^2.
__device__ inline float pair_weight_q(float xu, float xv, float tp, float tq, float ce) {
    const float a = xu * tp, b = xv * tq;
    const float ea = __builtin_amdgcn_exp2f(ce * fabsf(xu));
    const float eb = __builtin_amdgcn_exp2f(ce * fabsf(xv));
    const float pa = 1.0f + ea, pb = 1.0f + eb;
    const float pa2 = pa * pa, pb2 = pb * pb;
    const float d = a - b;
    const float num = (a * ea) * pb2 - (b * eb) * pa2;
    float w = num * __builtin_amdgcn_rcpf(d * pa2 * pb2);
    const bool near = fabsf(d) < 0.05f;
    if (near) {
        const float ra = __builtin_amdgcn_rcpf(pa), rb = __builtin_amdgcn_rcpf(pb);
        const float sa = ea * ra * ra, sb = eb * rb * rb;       // sech^2 / 4
        const float ta = (1.0f - ea) * ra, tb = (1.0f - eb) * rb;   // tanh|a|, tanh|b|
        const float xa = fabsf(a) * ta, xb = fabsf(b) * tb, qa = ta * ta, qb = tb * tb;
        const float d1 = sa * (1.0f - 2.0f * xa) + sb * (1.0f - 2.0f * xb);
        const float d3 = sa * (-6.0f * (1.0f - 3.0f * qa) + 8.0f * xa * (2.0f - 3.0f * qa)) +
                         sb * (-6.0f * (1.0f - 3.0f * qb) + 8.0f * xb * (2.0f - 3.0f * qb));
        w = 0.5f * d1 - (d * d) * d3 * (1.0f / 24.0f);
    }
    return w;
}
__device__ inline double pair_weight(double xu, double xv, double twoT, bool pp) {
    const double2 u = point_q(xu, twoT), v = point_q(xv, twoT);
    return phi_dd_pt(u, pp ? flip(v) : v);
}

// Interaction-flow weight of one loop-point pair: the divided difference
// tanh[a,b] = (tanh a - tanh b)/(a - b), a = xi/2T (b negated for particle-particle), so
// that chi = tanh[a,b] / 4T.  With e = exp(-2|x|), tanh|x| = (1 - e)/(1 + e) and, for a and
// b of one sign, tanh a - tanh b = sgn(a) 2 (e_b/(1 + e_b) - e_a/(1 + e_a)) without
// cancellation.
// Near the diagonal (|a - b| < 0.05) the trapezoid value with its end correction,
//   tanh[a,b] = (s_a + s_b)/2 - (a-b)^2 (s_a (6 t_a^2 - 2) + s_b (6 t_b^2 - 2))/24 + O((a-b)^4),
// with s = sech^2, t = tanh (the third derivative of tanh is sech^2 (6 tanh^2 - 2)), for the
// lanes that need it only.
__device__ inline float pair_chi(float xu, float xv, float inv2T, bool pp) {
    const float a = xu * inv2T;
    const float b0 = xv * inv2T;
    const float b = pp ? -b0 : b0;
    const float ea = __expf(-2.0f * fabsf(a)), eb = __expf(-2.0f * fabsf(b));
    const float ra = __builtin_amdgcn_rcpf(1.0f + ea), rb = __builtin_amdgcn_rcpf(1.0f + eb);
    const float ta = copysignf((1.0f - ea) * ra, a), tb = copysignf((1.0f - eb) * rb, b);
    const bool same = (a >= 0.0f) == (b >= 0.0f);
    const float diff = same ? (a >= 0.0f ? 2.0f : -2.0f) * (eb * rb - ea * ra) : ta - tb;
    const float d = a - b;
    float w = diff * __builtin_amdgcn_rcpf(d);
    const bool near = fabsf(d) < 0.05f;
    if (near) {
        const float sa = 4.0f * ea * ra * ra, sb = 4.0f * eb * rb * rb;
        const float c3 = sa * (6.0f * ta * ta - 2.0f) + sb * (6.0f * tb * tb - 2.0f);
        w = 0.5f * (sa + sb) - (d * d) * c3 * (1.0f / 24.0f);
    }
    return w;
}
// Double precision: the quotient away from the diagonal; within |a - b| < 0.01 the series
// about the midpoint m, tanh[a,b] = s (1 + (6 t^2 - 2) d^2/24 + (16 - 120 t^2 + 120 t^4) d^4/1920)
// + O(d^6), s = sech^2 m, t = tanh m, d = a - b.
__device__ inline double tanh_abs(double x, double& e) {
    e = exp(-2.0 * fabs(x));
    return (1.0 - e) / (1.0 + e);
}
__device__ inline double pair_chi(double xu, double xv, double twoT, bool pp) {
    const double a = xu / twoT;
    const double b = pp ? -(xv / twoT) : xv / twoT;
    const double d = a - b;
    if (fabs(d) >= 0.01) {
        double ea, eb;
        const double ta = copysign(tanh_abs(a, ea), a), tb = copysign(tanh_abs(b, eb), b);
        const bool same = (a >= 0.0) == (b >= 0.0);
        const double diff = same ? (a >= 0.0 ? 2.0 : -2.0) * (eb / (1.0 + eb) - ea / (1.0 + ea))
                                 : ta - tb;
        return diff / d;
    }
    const double m = 0.5 * (a + b);
    double e;
    const double t = copysign(tanh_abs(m, e), m);
    const double s = 4.0 * e / ((1.0 + e) * (1.0 + e));
    const double t2 = t * t, d2 = d * d;
    return s * (1.0 + (6.0 * t2 - 2.0) * d2 * (1.0 / 24.0) +
                (16.0 - 120.0 * t2 + 120.0 * t2 * t2) * d2 * d2 * (1.0 / 1920.0));
}

// ------------------------------------------------------------------------------------
// Phase 1: bins of the representative transfers.  One 1024-thread block per
// (representative, flow) accumulates the N x N bin matrix in LDS and stores it scaled by
// -1/(4 T L^2) (plus its transpose for particle-hole representatives, which the crossed
// channel reads).  Point quantities are evaluated on the fly from xi.
//
// Lane layout: the 16 lanes of a DPP row take 16 consecutive loop points, so every load
// (own xi, partner xi, both patches) is a contiguous segment.  Consecutive points mostly
// share their patch pair, so a segmented scan over the row (DPP shifts 1, 2, 4, 8) sums
// each run of equal keys and only the last lane of a run issues the atomic.  The four
// rows of a wave work in bands a quarter of the grid apart, so their keys rarely collide.
//   kMode 0: bins in LDS; kMode 1 (bin matrix above 128 KB): the block accumulates its own
//   representative's bins in global memory with atomics, after clearing them.
// ------------------------------------------------------------------------------------
// Block size of stage and phase 1: 1024 threads for few (flow, representative) pairs, so
// one flow's bins spread over many waves, and wherever the LDS bins allow few blocks per
// CU; otherwise 256, so several blocks share a CU and one block's fill and drain overlap
// another's work.
// 16-point units per row whose loads are in flight together
template <typename R> struct BinBatch;
template <> struct BinBatch<float> { static constexpr int v = 8; };
template <> struct BinBatch<double> { static constexpr int v = 4; };

// xi and patch of loop point j: single precision reads the packed (float xi, patch) table.
// The byte offset is formed in 32 bits (L <= 2048: under 32 MiB), so a load is the table's
// base plus one 32-bit offset.
__device__ inline void xi_patch(const DevGeom& g, int j, float& x, int& p) {
    const unsigned off = static_cast<unsigned>(j) * 8u;
    const int2 v = *reinterpret_cast<const int2*>(reinterpret_cast<const char*>(g.xp) + off);
    x = __int_as_float(v.x);
    p = v.y;
}
__device__ inline void xi_patch(const DevGeom& g, int j, double& x, int& p) {
    x = g.xi[j];
    p = g.patch[j];
}

template <int kCtrl>
__device__ inline float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xf, 0xf, false));
}
template <int kCtrl>
__device__ inline double dpp_f(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), kCtrl, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), kCtrl, 0xf, 0xf, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}
template <int kCtrl>
__device__ inline int dpp_i(int v) { return __builtin_amdgcn_update_dpp(0, v, kCtrl, 0xf, 0xf, false); }

// One step of the segmented inclusive scan within a 16-lane row (Hillis-Steele): lane s adds
// the partial sum of lane s - D when that lane lies in its own run, i.e. s - D >= st, st the
// first lane of the run.
template <int D, typename R>
__device__ inline void seg_step(R& v, int st, int s) {
    const R vp = dpp_f<0x110 | D>(v);   // row_shr:D
    if (s - D >= st) v += vp;
}
// First lane of each lane's run of equal keys within its 16-lane row: the inclusive prefix
// maximum of the run heads' lane numbers (row_shr reads 0 past the row's start).
__device__ inline int run_start(int key, int s) {
    const int kprev = dpp_i<0x111>(key);   // row_shr:1
    int st = (s == 0 || kprev != key) ? s : 0;
    st = max(st, dpp_i<0x111>(st));
    st = max(st, dpp_i<0x112>(st));
    st = max(st, dpp_i<0x114>(st));
    st = max(st, dpp_i<0x118>(st));
    return st;
}

// Pairing (exact, halves the weight evaluations): the particle-particle partner map
// j -> q - j and the particle-hole map j -> -(j + q) are involutions s of the loop grid, per
// axis j -> (c - 1 - j) mod L (c = q, resp. -q), whose pairs carry equal weights.  The pair
// of s(j) has key (pi(j'), pi(j)) (particle-particle) or (P pi(j'), P pi(j)) (particle-hole,
// P the patch permutation of k -> -k), so each unordered pair {j, s(j)} is evaluated once
// and added under both keys.  Rows pair up as jy <-> (c - 1 - jy) mod L: one row of each
// pair is visited in full; in a row that s fixes (two when c - 1 is even) the columns pair
// up the same way and one column of each pair is visited; the at most four points that s
// fixes are their own pair and are added once, at the end.  Without the inversion symmetry
// the particle-hole sum visits every point once.  With the bins in LDS a pair is added under
// its first key only, and the second key's share is taken when the block stores its bins:
// the map of keys k = (a, b) -> k' = (b, a) (particle-particle) or (P b, P a) (particle-hole)
// is an involution, so bin k is the LDS sum at k plus that at k'; a point that s fixes has
// k' = k and adds half its weight.
struct Half {
    int h1, h2, nfix, c;   // [0, h1) and [c + 1, c + 1 + h2) are one side; fixed c/2, c/2 + L/2
};
__device__ inline Half half_of(int cc, int L) {
    const int c = (cc + 2 * L - 1) % L;
    return Half{(c + 1) / 2, (L - c - 1) / 2, c % 2 == 0 ? 2 : 0, c};
}
__device__ inline int half_map(const Half& h, int i) { return i < h.h1 ? i : h.c + 1 + (i - h.h1); }
__device__ inline int half_fix(const Half& h, int i, int L) { return h.c / 2 + i * (L / 2); }

// Patch permutation of k -> -k: a rotation by half a turn for angular patches, else the table.
__device__ inline int inv_patch(const DevGeom& g, int a) {
    if (g.inv_rot) {
        const int b = a + g.N / 2;
        return b >= g.N ? b - g.N : b;
    }
    return g.pI[a];
}

// kG = 1: interaction-flow bins, chi = tanh[a,b]/4T, stored scaled by +1/(4 T L^2).
// NODES > 1 (bins in LDS): the block bins one representative at nn <= NODES stage
// temperatures T[0..nn) at once, one LDS bin matrix each: the loads, indices, keys and run
// starts of a pair serve every node, only the weights, scans and atomics are per node.
// bins / binsT point to the first node's set; consecutive nodes' sets are set_bins /
// set_binsT values apart.
template <typename R, int kMode, int BT, int kG, int NODES>
__device__ inline void bins_part(const DevGeom& g, int f, int r, const double (&T)[NODES],
                                 int nn, R* bins, R* binsT, size_t set_bins, size_t set_binsT,
                                 R* lb) {
    static_assert(kMode == 0 || NODES == 1, "several nodes per block need the LDS bins");
    static_assert(NODES <= 2, "a block's last node group holds NODES or one node");
    const int N = g.N, NN = g.NN, L = g.L, np = g.np;
    // LDS bin rows have stride N + 1, so the column walks of the store fall on distinct banks
    const int S = kMode == 0 ? N + 1 : N, NS = kMode == 0 ? N * (N + 1) : NN;
    const int nR = g.nRp + g.nRd;
    const bool pp = r < g.nRp;
    const int m = pp ? g.rep_pp[r] : g.rep_ph[r - g.nRp];
    const int mx = m % L, my = m / L;
    R* out = bins + (static_cast<size_t>(f) * nR + r) * NN;
    R scale[NODES], tp[NODES];
    float tq[NODES], ce[NODES];                        // single-precision weight: +-1/2T, -log2(e)/T
    constexpr double kWq = (!kG && sizeof(R) == 4) ? 4.0 : 1.0;   // that weight is a quarter
#pragma unroll
    for (int j = 0; j < NODES; ++j) {
        const double Tj = T[j];
        scale[j] = static_cast<R>(kWq * (kG ? 1.0 : -1.0) / (4.0 * Tj * np));
        tp[j] = static_cast<R>(sizeof(R) == 4 ? 1.0 / (2.0 * Tj) : 2.0 * Tj);   // 1/2T or 2T
        tq[j] = static_cast<float>((pp ? -1.0 : 1.0) / (2.0 * Tj));
        ce[j] = static_cast<float>(-1.4426950408889634 / Tj);
    }
    constexpr int kBinBatch = BinBatch<R>::v;
    const bool half = (pp || g.inv_ok) && L % 2 == 0;
    const Half hy = half_of(pp ? my : L - my, L), hx = half_of(pp ? mx : L - mx, L);
    const int nrow = half ? hy.h1 + hy.h2 : L;            // rows visited in full
    const int ncol = hx.h1 + hx.h2;                        // columns visited in a fixed row
    const int npt = nrow * L + (half ? hy.nfix * ncol : 0);
    const float invL = 1.0f / static_cast<float>(L);
    R* acc = kMode == 0 ? lb : out;                   // node j: acc + j NS
    for (int i = threadIdx.x; i < nn * NS; i += blockDim.x) acc[i] = R(0);
    if (kMode == 1) __threadfence();
    __syncthreads();                                   // every thread of the block
    // BT/16 rows of 16 lanes per block; row rr works on band rr of BT/16 contiguous bands of
    // units, the 4 rows of a wave a quarter of the bands apart
    constexpr int kBands = BT / 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int s = lane & 15;
    const int band = (lane >> 4) * (BT / 64) + wv;
    // Weights of one batch (kBinBatch points per lane), the segmented scan of equal keys
    // within each 16-lane row, and one atomic per run of equal keys (global bins: two under
    // the pairing).
    auto weight = [&](R xa, R xb, int j) -> R {
        if constexpr (kG) return pair_chi(xa, xb, tp[j], pp);
        else if constexpr (sizeof(R) == 4) return pair_weight_q(xa, xb, tp[j], tq[j], ce[j]);
        else return pair_weight(xa, xb, tp[j], pp);
    };
    auto add_batch = [&](const R (&xu)[kBinBatch], const R (&xv)[kBinBatch],
                         const int (&pa)[kBinBatch], const int (&pq)[kBinBatch],
                         const bool (&ok)[kBinBatch]) {
#pragma unroll
        for (int i = 0; i < kBinBatch; ++i) {
            // keys < N (N + 1) (24-bit products)
            const int key = static_cast<int>(__umul24(pa[i], S)) + pq[i];
            const int knext = dpp_i<0x101>(key);   // row_shl:1
            const int st = run_start(key, s);
            const bool end = s == 15 || knext != key;
#pragma unroll
            for (int j = 0; j < NODES; ++j) {
                if (j >= nn) break;                    // uniform over the block
                const R w = weight(xu[i], xv[i], j);
                R x = ok[i] ? (kMode == 0 ? w : w * scale[j]) : R(0);
                seg_step<1>(x, st, s);
                seg_step<2>(x, st, s);
                seg_step<4>(x, st, s);
                seg_step<8>(x, st, s);
                if (end) {
                    R* aj = acc + j * NS;
                    atomicAdd(&aj[key], x);
                    if constexpr (kMode == 1) {        // the second key (bijective in the first)
                        if (half) {
                            const int key2 = pp ? static_cast<int>(__umul24(pq[i], N)) + pa[i]
                                                : static_cast<int>(__umul24(inv_patch(g, pq[i]), N)) +
                                                      inv_patch(g, pa[i]);
                            atomicAdd(&aj[key2], x);
                        }
                    }
                }
            }
        }
    };
    auto partner = [&](int jx, int jy, int& px, int& py) {
        px = pp ? mx - jx - 1 : jx + mx;
        py = pp ? my - jy - 1 : jy + my;
        px += px < 0 ? L : (px >= L ? -L : 0);
        py += py < 0 ? L : (py >= L ? -L : 0);
    };
    // the rows the pairing fixes (at most two): one column of each column pair, few points,
    // one atomic per key
    auto fixed_rows = [&]() {
        for (int t = threadIdx.x; t < hy.nfix * ncol; t += BT) {
            const int fr = t >= ncol ? 1 : 0;
            const int jx = half_map(hx, t - fr * ncol), jy = half_fix(hy, fr, L);
            int px, py;
            partner(jx, jy, px, py);
            R xa, xb;
            int qa, qb;
            xi_patch(g, jy * L + jx, xa, qa);
            xi_patch(g, py * L + px, xb, qb);
            const int k1 = qa * S + qb, k2 = pp ? qb * N + qa : inv_patch(g, qb) * N + inv_patch(g, qa);
#pragma unroll
            for (int j = 0; j < NODES; ++j) {
                if (j >= nn) break;                    // uniform over the block
                const R w = weight(xa, xb, j);
                const R x = kMode == 0 ? w : w * scale[j];
                atomicAdd(&acc[j * NS + k1], x);
                if constexpr (kMode == 1) atomicAdd(&acc[k2], x);
            }
        }
    };
    if constexpr (kMode == 0) {
        // Column walks (bins in LDS): a lane takes one grid column -- consecutive lanes take
        // consecutive columns, so the loads of a row are contiguous over the wave -- and one
        // segment of the visited rows, and walks down it keeping each node's sum over the
        // current run of equal keys in a register.  The sum goes to LDS when the key changes
        // (along a column only where the point or its partner crosses a patch boundary) and
        // at the segment's end: no scan across lanes, one atomic per run.
        const int nseg = BT > L ? BT / L : 1;
        const int seglen = (nrow + nseg - 1) / nseg;
        bool walked = false;
        if constexpr (sizeof(R) == 4) if (L % 64 == 0) {
            // L a multiple of 64 (single precision): a wave's 64 lanes take 64 consecutive
            // columns of one segment, so the row of each step, its partner row and both rows'
            // offsets are the same for every lane and are formed on the scalar unit; the
            // table is read by raw buffer loads (lane offset in a vector register, row offset
            // in a scalar one, range np entries), so per point a lane forms only its key, the
            // weights and the run update.  The run starts at key 0 with a zero sum, so its
            // first flush adds nothing.
            // resource word 3: raw buffer with a 32-bit data format (gfx9 encoding)
            const __amdgpu_buffer_rsrc_t xr = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<int2*>(g.xp), 0, np * 8, 0x00020000);
            // the walk for KN nodes (all of a block's nodes, or one for the last group)
            auto walk64 = [&](auto kn) {
                constexpr int KN = decltype(kn)::value;
                const int wave0 = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) & ~63);
                for (int it0 = wave0; it0 < L * nseg; it0 += BT) {
                    const int sg = it0 / L;
                    const int jx = it0 - sg * L + lane;
                    const int r0 = sg * seglen, r1 = min(r0 + seglen, nrow);
                    int px = pp ? mx - jx - 1 : jx + mx;
                    px += px < 0 ? L : (px >= L ? -L : 0);
                    const unsigned ou = static_cast<unsigned>(jx) * 8u, ov = static_cast<unsigned>(px) * 8u;
                    int prev = 0;
                    R run[KN];
    #pragma unroll
                    for (int j = 0; j < KN; ++j) run[j] = R(0);
                    // The segment in pieces over which the row and the partner row each advance
                    // by one per step (a piece ends at the pairing's jump from visited row h1 to
                    // grid row c + 1 and where the partner row wraps), so a step's two row
                    // offsets are the previous ones plus constants.  Full batches of a piece add
                    // every point; the last, partial one repeats the piece's last row in its
                    // unused slots and stops at the piece's end.
                    const int L8 = L * 8;
                    // one batch: kTail = false, kBinBatch rows; true, cnt < kBinBatch rows
                    auto batch = [&](auto tail, int& su, int& sv, int dv, int su1, int sv1, int cnt) {
                        constexpr bool kTail = decltype(tail)::value;
                        R xu[kBinBatch], xv[kBinBatch];
                        int ka[kBinBatch];
    #pragma unroll
                        for (int i = 0; i < kBinBatch; ++i) {
                            const int oy = kTail ? min(su, su1) : su;
                            const int oq = kTail ? (pp ? max(sv, sv1) : min(sv, sv1)) : sv;
                            const auto u = __builtin_amdgcn_raw_buffer_load_b64(xr, ou, oy, 0);
                            const auto v = __builtin_amdgcn_raw_buffer_load_b64(xr, ov, oq, 0);
                            xu[i] = __int_as_float(static_cast<int>(u[0]));
                            xv[i] = __int_as_float(static_cast<int>(v[0]));
                            ka[i] = static_cast<int>(__umul24(u[1], S)) + static_cast<int>(v[1]);
                            su += L8;
                            sv += dv;
                        }
    #pragma unroll
                        for (int i = 0; i < kBinBatch; ++i) {
                            if (kTail && i >= cnt) break;       // uniform over the wave
                            const int key = ka[i];
                            const bool chg = key != prev;
                            if (chg) {
    #pragma unroll
                                for (int j = 0; j < KN; ++j) {
                                    atomicAdd(&acc[j * NS + prev], run[j]);
                                }
                            }
    #pragma unroll
                            for (int j = 0; j < KN; ++j) {
                                const R w = weight(xu[i], xv[i], j);
                                run[j] = (chg ? R(0) : run[j]) + w;
                            }
                            prev = key;
                        }
                    };
                    for (int rr = r0; rr < r1;) {                // uniform over the wave
                        const int jy0 = half ? half_map(hy, rr) : rr;
                        int py0 = pp ? my - jy0 - 1 : jy0 + my;
                        py0 += py0 < 0 ? L : (py0 >= L ? -L : 0);
                        int len = r1 - rr;
                        if (half && rr < hy.h1) len = min(len, hy.h1 - rr);
                        len = min(len, pp ? py0 + 1 : L - py0);
                        const int dv = pp ? -L8 : L8;
                        int su = jy0 * L8, sv = py0 * L8;
                        const int su1 = su + (len - 1) * L8, sv1 = sv + (len - 1) * dv;
                        int t0 = 0;
                        for (; t0 + kBinBatch <= len; t0 += kBinBatch)
                            batch(std::false_type{}, su, sv, dv, su1, sv1, kBinBatch);
                        if (t0 < len) batch(std::true_type{}, su, sv, dv, su1, sv1, len - t0);
                        rr += len;
                    }
    #pragma unroll
                    for (int j = 0; j < KN; ++j) {
                        atomicAdd(&acc[j * NS + prev], run[j]);
                    }
                }
            };
            if constexpr (NODES == 1) walk64(std::integral_constant<int, 1>{});
            else if (nn == NODES) walk64(std::integral_constant<int, NODES>{});
            else walk64(std::integral_constant<int, 1>{});   // nn == 1 (NODES <= 2)
            walked = true;
        }
        if (!walked)
        for (int it = threadIdx.x; it < L * nseg; it += BT) {
            const int jx = it % L, sg = it / L;
            const int r0 = sg * seglen, r1 = min(r0 + seglen, nrow);
            int px = pp ? mx - jx - 1 : jx + mx;
            px += px < 0 ? L : (px >= L ? -L : 0);
            int prev = -1;                             // key of the current run (none yet)
            R run[NODES];
#pragma unroll
            for (int j = 0; j < NODES; ++j) run[j] = R(0);
            for (int rb = r0; rb < r1; rb += kBinBatch) {   // uniform over the wave
                R xu[kBinBatch], xv[kBinBatch];
                int ka[kBinBatch];
#pragma unroll
                for (int i = 0; i < kBinBatch; ++i) {
                    const int rr = min(rb + i, r1 - 1);
                    const int jy = half ? half_map(hy, rr) : rr;
                    int py = pp ? my - jy - 1 : jy + my;
                    py += py < 0 ? L : (py >= L ? -L : 0);
                    int qa, qb;
                    xi_patch(g, static_cast<int>(__umul24(jy, L)) + jx, xu[i], qa);
                    xi_patch(g, static_cast<int>(__umul24(py, L)) + px, xv[i], qb);
                    ka[i] = static_cast<int>(__umul24(qa, S)) + qb;
                }
#pragma unroll
                for (int i = 0; i < kBinBatch; ++i) {
                    const bool ok = rb + i < r1;
                    const int key = ok ? ka[i] : prev;
                    const bool chg = key != prev;
                    if (chg && prev >= 0) {
#pragma unroll
                        for (int j = 0; j < NODES; ++j) {
                            if (j >= nn) break;        // uniform over the block
                            atomicAdd(&acc[j * NS + prev], run[j]);
                        }
                    }
#pragma unroll
                    for (int j = 0; j < NODES; ++j) {
                        if (j >= nn) break;            // uniform over the block
                        const R w = weight(xu[i], xv[i], j);
                        run[j] = (chg ? R(0) : run[j]) + (ok ? w : R(0));
                    }
                    prev = key;
                }
            }
            if (prev >= 0) {
#pragma unroll
                for (int j = 0; j < NODES; ++j) {
                    if (j >= nn) break;                // uniform over the block
                    atomicAdd(&acc[j * NS + prev], run[j]);
                }
            }
        }
        if (half) fixed_rows();
    } else if (L % 16 == 0) {
        // The visited rows in full: a 16-point unit never crosses a grid row, so the row is
        // found once per unit and the column is the lane's offset.  The loop is specialised
        // per kind: a particle-particle partner coordinate m - j - 1 can only fall below 0,
        // a particle-hole one j + m only reach L.
        const int upr = L >> 4;                                   // units per row
        const float invu = 1.0f / static_cast<float>(upr);
        const int nmain = nrow * upr;
        const int per_band = (nmain + kBands - 1) / kBands;
        const int u_begin = band * per_band;
        const int u_end = min(u_begin + per_band, nmain);
        auto main_rows = [&](auto kind) {
            constexpr bool kPP = decltype(kind)::value;
            auto wrap = [&](int v) {
                if constexpr (kPP) return v + (v < 0 ? L : 0);
                else return v - (v >= L ? L : 0);
            };
            if (upr >= kBinBatch) {
                // A batch of consecutive units crosses at most one row end: unit u0 + i is
                // column block cb0 + i of row rr0, or of row rr0 + 1 past the end; the two
                // rows' offsets are formed once per batch (24-bit products).  Units past the
                // band's end read the last row (valid addresses, never added).
                int rr0 = u_begin / upr, cb0 = u_begin - rr0 * upr;
                for (int u0 = u_begin; u0 < u_begin + per_band; u0 += kBinBatch) {   // same trip count for all rows
                    const int ra = min(rr0, nrow - 1), rb = min(rr0 + 1, nrow - 1);
                    const int jya = half ? half_map(hy, ra) : ra;
                    const int jyb = half ? half_map(hy, rb) : rb;
                    const int pya = wrap(kPP ? my - jya - 1 : jya + my);
                    const int pyb = wrap(kPP ? my - jyb - 1 : jyb + my);
                    const int oa = static_cast<int>(__umul24(jya, L)), ob = static_cast<int>(__umul24(jyb, L));
                    const int qa = static_cast<int>(__umul24(pya, L)), qb = static_cast<int>(__umul24(pyb, L));
                    R xu[kBinBatch], xv[kBinBatch];
                    int pa[kBinBatch], pq[kBinBatch];
                    bool ok[kBinBatch];
#pragma unroll
                    for (int i = 0; i < kBinBatch; ++i) {
                        const int c = cb0 + i;
                        const bool nx = c >= upr;
                        const int jx = ((nx ? c - upr : c) << 4) + s;
                        const int px = wrap(kPP ? mx - jx - 1 : jx + mx);
                        xi_patch(g, (nx ? ob : oa) + jx, xu[i], pa[i]);
                        xi_patch(g, (nx ? qb : qa) + px, xv[i], pq[i]);
                        ok[i] = u0 + i < u_end;
                    }
                    add_batch(xu, xv, pa, pq, ok);
                    cb0 += kBinBatch;
                    if (cb0 >= upr) {
                        cb0 -= upr;
                        ++rr0;
                    }
                }
                return;
            }
            for (int u0 = u_begin; u0 < u_begin + per_band; u0 += kBinBatch) {   // same trip count for all rows
                R xu[kBinBatch], xv[kBinBatch];
                int pa[kBinBatch], pq[kBinBatch];
                bool ok[kBinBatch];
#pragma unroll
                for (int i = 0; i < kBinBatch; ++i) {
                    const int u = min(u0 + i, nmain - 1);
                    const int rr = static_cast<int>((u + 0.5f) * invu);   // u / upr (exact, L <= 2048)
                    const int jx = ((u - rr * upr) << 4) + s;
                    const int jy = half ? half_map(hy, rr) : rr;
                    int px = kPP ? mx - jx - 1 : jx + mx;
                    int py = kPP ? my - jy - 1 : jy + my;
                    if constexpr (kPP) {
                        px += px < 0 ? L : 0;
                        py += py < 0 ? L : 0;
                    } else {
                        px -= px >= L ? L : 0;
                        py -= py >= L ? L : 0;
                    }
                    xi_patch(g, jy * L + jx, xu[i], pa[i]);
                    xi_patch(g, py * L + px, xv[i], pq[i]);
                    ok[i] = u0 + i < u_end;
                }
                add_batch(xu, xv, pa, pq, ok);
            }
        };
        if (pp) main_rows(std::true_type{});
        else main_rows(std::false_type{});
        if (half) fixed_rows();
    } else {
        // any L: visited rows and fixed rows as one numbered list of points
        const int nunits = (npt + 15) / 16;
        const int per_band = (nunits + kBands - 1) / kBands;
        const int u_begin = band * per_band;
        const int u_end = min(u_begin + per_band, nunits);
        for (int u0 = u_begin; u0 < u_begin + per_band; u0 += kBinBatch) {   // same trip count for all rows
            R xu[kBinBatch], xv[kBinBatch];
            int pa[kBinBatch], pq[kBinBatch];
            bool ok[kBinBatch];
#pragma unroll
            for (int i = 0; i < kBinBatch; ++i) {
                const int p = min((u0 + i) * 16 + s, npt - 1);
                // p < nrow L: row rr of the visited rows; else column of a row fixed by s
                const int rr = static_cast<int>((p + 0.5f) * invL);       // p / L (L <= 2048)
                const int q2 = p - nrow * L, fr = q2 >= ncol ? 1 : 0;
                const bool mainpart = q2 < 0;
                const int jx = mainpart ? p - rr * L : half_map(hx, q2 - fr * ncol);
                const int jy = mainpart ? (half ? half_map(hy, rr) : rr) : half_fix(hy, fr, L);
                int px, py;
                partner(jx, jy, px, py);
                xi_patch(g, jy * L + jx, xu[i], pa[i]);
                xi_patch(g, py * L + px, xv[i], pq[i]);
                ok[i] = u0 + i < u_end && (u0 + i) * 16 + s < npt;
            }
            add_batch(xu, xv, pa, pq, ok);
        }
    }
    // points fixed by s: their own pair, added once (in LDS half of it, at a key that is its
    // own second key)
    if (half && static_cast<int>(threadIdx.x) < hy.nfix * hx.nfix) {
        const int jy = half_fix(hy, threadIdx.x >> 1, L), jx = half_fix(hx, threadIdx.x & 1, L);
        int px = pp ? mx - jx - 1 : jx + mx;
        int py = pp ? my - jy - 1 : jy + my;
        px += px < 0 ? L : (px >= L ? -L : 0);
        py += py < 0 ? L : (py >= L ? -L : 0);
        R xa, xb;
        int qa, qb;
        xi_patch(g, jy * L + jx, xa, qa);
        xi_patch(g, py * L + px, xb, qb);
#pragma unroll
        for (int j = 0; j < NODES; ++j) {
            if (j >= nn) break;                        // uniform over the block
            const R w = weight(xa, xb, j);
            atomicAdd(&acc[j * NS + qa * S + qb], kMode == 0 ? R(0.5) * w : w * scale[j]);
        }
    }
    if (kMode == 1) __threadfence();
    __syncthreads();                                   // every thread of the block
    R* outT = pp ? nullptr : binsT + (static_cast<size_t>(f) * g.nRd + (r - g.nRp)) * NN;
#pragma unroll
    for (int j = 0; j < NODES; ++j) {
        if (j >= nn) break;                            // uniform over the block
        R* oj = out + j * set_bins;
        R* oTj = outT ? outT + j * set_binsT : nullptr;
        if constexpr (kMode == 0) {
            // bin (a, b) = L(a, b) + L(k'(a, b)) under the pairing, with k'(a, b) = (b, a) or
            // (P b, P a), and the particle-hole transpose T(a, b) = bin (b, a); every LDS
            // read walks a row or a column (stride N + 1), every store a row
            const R* lj = lb + j * NS;
            // (a, b) of element i, advanced by blockDim.x elements per round without a division
            const int bd = blockDim.x, da = bd / N, db = bd - da * N;
            int a = static_cast<int>(threadIdx.x) / N, b = static_cast<int>(threadIdx.x) - a * N;
            for (int i = threadIdx.x; i < NN; i += bd) {
                const int pa = pp ? a : inv_patch(g, a), pb = pp ? b : inv_patch(g, b);
                oj[i] = (lj[a * S + b] + (half ? lj[pb * S + pa] : R(0))) * scale[j];
                if (oTj) oTj[i] = (lj[b * S + a] + (half ? lj[pa * S + pb] : R(0))) * scale[j];
                a += da;
                b += db;
                if (b >= N) {
                    b -= N;
                    ++a;
                }
            }
        } else if (oTj) {
            for (int i = threadIdx.x; i < NN; i += blockDim.x) {
                const int bb = i / N, aa = i - bb * N;
                oTj[i] = oj[aa * N + bb];
            }
        }
    }
}

// One launch per stage: blocks [0, nRb ceil(bp.n / NODES)) bin the representatives (phase
// 1, which needs only T) at every node of the plan, NODES consecutive nodes per block -- the
// first stage of an integrator step bins all the step's distinct nodes at once, the later
// stages none -- and the remaining blocks form the stage argument and its operand layouts.
// Grid (nRb ceil(bp.n / NODES) + stage blocks, flows).
template <typename R, int kMode, int BT, int kG, int NODES>
__global__ void __launch_bounds__(BT, 4) k_stage_bins(DevGeom g, DevZ z, const FlowState* fs,
                                                            StageCoef sc, BinPlan bp,
                                                            int write_new, const double* Vbase,
                                                            const R* K, R* KS, double* Vnew,
                                                            R* v0, R* va, R* vc, double* T_stage,
                                                            double* Z_stage, double* zw,
                                                            R* bins, R* binsT, int nRb, int B,
                                                            int tl) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int f = blockIdx.y;
    if (!running(fs, f)) return;                      // uniform over the block
    const FlowState st = fs[f];
    const int nbin = nRb * ((bp.n + NODES - 1) / NODES);
    if (static_cast<int>(blockIdx.x) < nbin) {
        if (bin_flow(fs, f) != f) return;             // another flow bins this temperature
        const int grp = static_cast<int>(blockIdx.x) / nRb;
        const int r = static_cast<int>(blockIdx.x) - grp * nRb;
        const int set0 = grp * NODES;
        const int nn = min(NODES, bp.n - set0);
        double T[NODES];
#pragma unroll
        for (int j = 0; j < NODES; ++j)
            T[j] = kG ? st.Tfix : exp(st.lnT + bp.c[min(set0 + j, bp.n - 1)] * st.ht);
        const size_t NN = static_cast<size_t>(g.NN);
        const size_t sb = static_cast<size_t>(B) * nRb * NN, sbT = static_cast<size_t>(B) * g.nRd * NN;
        bins_part<R, kMode, BT, kG, NODES>(g, f, r, T, nn, bins + set0 * sb, binsT + set0 * sbT,
                                           sb, sbT, reinterpret_cast<R*>(smem_raw));
    } else {
        stage_part<R, BT, false>(g, z, st, f, sc, write_new, Vbase, K, KS, Vnew, v0, va, vc,
                                 T_stage, Z_stage, zw, B, reinterpret_cast<double*>(smem_raw),
                                 tl, blockIdx.x - nbin, gridDim.x - nbin);
    }
}

// The stage argument alone (the later stages of a step): 1024-thread blocks, one element tile
// per block round, each element's loads (newest slot's pp part, earlier slots' sums, V) held
// across the tile's barrier.  Grid (tiles, flows).
template <typename R>
__global__ void __launch_bounds__(1024) k_stage(DevGeom g, DevZ z, const FlowState* fs,
                                                StageCoef sc, int write_new, const double* Vbase,
                                                const R* K, R* KS, double* Vnew, R* v0, R* va,
                                                R* vc,
                                                double* T_stage, double* Z_stage, double* zw,
                                                int B, int tl) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int f = blockIdx.y;
    if (!running(fs, f)) return;                      // uniform over the block
    const FlowState st = fs[f];
    stage_part<R, 1024, true>(g, z, st, f, sc, write_new, Vbase, K, KS, Vnew, v0, va, vc,
                              T_stage, Z_stage, zw, B, reinterpret_cast<double*>(smem_raw), tl,
                              blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------------------------------
// Phase 2a: grouped products.  For group g (one patch index) and kind k:
//   C[q][n] = sum_kk A[q][kk] Bm[kk][n],  Bm[kk][n] = Vsrc[g][kk][n],
//   A[q][kk] = Z_g Z_kk B_q(row, col) with B_q(x, y) = Brep_r(pinv_o x, pinv_o y), q = o(r),
// stored as Y[q][g][n]:
//   kind 0 (pp):      (row, col) = (g, kk), Vsrc = v0 -> Y1[q][a'][c]
//   kind 1 (crossed): (row, col) = (kk, g), Vsrc = vc -> Y2[q][b'][a]
//   kind 2 (direct):  (row, col) = (g, kk), Vsrc = va -> Y3[q][a'][b]
//   kind 3 (direct):  (row, col) = (g, kk), Vsrc = vc -> Y4[q][a'][b]
// 64 x 64 output tile, K in steps of 16, 4 x 4 per thread.
// ------------------------------------------------------------------------------------
template <typename R>
struct YArgs {
    const R* Vs[4];
    R* Y[4];
    int on[4];
};

template <typename R>
__global__ void __launch_bounds__(kThreads) k_y(DevGeom g, const FlowState* fs,
                                                const double* Z_stage, const double* zw,
                                                const R* bins, const R* binsT, YArgs<R> args) {
    constexpr int TM = 64, TN = 64, TK = 16;
    __shared__ R As[TK][TM + 4];
    __shared__ R Bs[TK][TN + 4];
    const int kind = blockIdx.z % 4;
    const int f = blockIdx.z / 4;
    if (!running(fs, f) || !args.on[kind]) return;
    const int N = g.N, NN = g.NN;
    const bool ppk = kind == 0;
    // transfers of the kind (the per-flow stride of Y); symmetric states compute the
    // representatives' own transfers (the first nR) only
    const int Mq = ppk ? g.nP : g.nD;
    const int M = g.sym ? (ppk ? g.nRp : g.nRd) : Mq;
    const int ntn = (N + TN - 1) / TN;
    const int tm = blockIdx.x / ntn, tn = blockIdx.x - tm * ntn;
    if (tm * TM >= M) return;
    const int grp = blockIdx.y;
    const size_t N3 = static_cast<size_t>(NN) * N;
    const int nR = g.nRp + g.nRd;
    // kind 1 reads the transposed particle-hole bins, so every kind reads a contiguous row
    const int fb = bin_flow(fs, f);
    const R* Bf = kind == 1 ? binsT + static_cast<size_t>(fb) * g.nRd * NN
                            : bins + static_cast<size_t>(fb) * nR * NN + (ppk ? 0 : static_cast<size_t>(g.nRp) * NN);
    const int* qrep = ppk ? g.qrep_pp : g.qrep_ph;
    const int* qg = ppk ? g.qg_pp : g.qg_ph;
    const R* Vg = args.Vs[kind] + f * N3 + static_cast<size_t>(grp) * NN;
    const double* Zf = Z_stage + static_cast<size_t>(f) * 2 * N;
    const double* Wf = Zf + N;
    const R zg = static_cast<R>(Zf[grp]), wg = static_cast<R>(Wf[grp]);
    const R al = static_cast<R>(zw[2 * f]), be = static_cast<R>(zw[2 * f + 1]);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    __shared__ int pis[8 * 256];
    for (int i = threadIdx.x; i < 8 * N && i < 8 * 256; i += blockDim.x) pis[i] = g.pinv[i];
    __syncthreads();
    R acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) acc[i][jj] = R(0);
    // A-tile loads: thread t always loads column kk = t % TK of rows t / TK + 16 i, so the
    // row metadata (representative bins, permutation, permuted group index) is fixed.
    const int kk_t = threadIdx.x % TK;
    const R* rowp[4];
    const int* pir[4];
    int gxr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int q = tm * TM + threadIdx.x / TK + 16 * i;
        if (q < M) {
            pir[i] = (N <= 256 ? pis : g.pinv) + qg[q] * N;
            gxr[i] = pir[i][grp];
            rowp[i] = Bf + static_cast<size_t>(qrep[q]) * NN;
        } else {
            pir[i] = nullptr; gxr[i] = 0; rowp[i] = nullptr;
        }
    }
    for (int k0 = 0; k0 < N; k0 += TK) {
        const int k = k0 + kk_t;
        const R zkk = k < N ? static_cast<R>(Zf[k]) : R(0);
        const R wkk = k < N ? static_cast<R>(Wf[k]) : R(0);
        const R zk = k < N ? zg * zkk * (al + be * (wg + wkk)) : R(0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr = threadIdx.x / TK + 16 * i;
            R v = R(0);
            if (rowp[i] && k < N) {
                v = rowp[i][gxr[i] * N + pir[i][k]] * zk;
            }
            As[kk_t][rr] = v;
        }
        for (int e = threadIdx.x; e < TK * TN; e += blockDim.x) {
            const int kk = e / TN, c = e - kk * TN;
            const int k = k0 + kk, n = tn * TN + c;
            Bs[kk][c] = (k < N && n < N) ? Vg[static_cast<size_t>(k) * N + n] : R(0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            R a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) b[jj] = Bs[kk][tx * 4 + jj];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) acc[i][jj] += a[i] * b[jj];
        }
        __syncthreads();
    }
    R* Y = args.Y[kind] + static_cast<size_t>(f) * Mq * NN;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int q = tm * TM + ty * 4 + i;
        if (q >= M) continue;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int n = tn * TN + tx * 4 + jj;
            if (n < N) Y[static_cast<size_t>(q) * NN + grp * N + n] = acc[i][jj];
        }
    }
}

// Phase 2a on matrix cores (single-precision storage, N <= 128).  Same products as k_y.
// One wave computes, for one group g, a column chunk of NT 16-wide tiles and a run of
// 16-row tiles of transfers of one operation class:
//   B'[k'][n] = Z_g Z_k (al + be (W_g + W_k)) Vsrc[g][k][n], k = perm_o k', is staged in
//     LDS once per block (for the direct channel two such operands, va and vc, share one A);
//   A[q][k'] = Brep_r(pinv_o g, k') is read straight from a representative's bin row into
//     the MFMA register layout.
// kM = 0: v_mfma_f32_16x16x4_f32, lane holds k = 4 e + lane / 16 (e < KE);
// kM = 1: v_mfma_f32_16x16x32_bf16, k = 32 (e / 8) + 8 (lane / 16) + e % 8, operands rounded
//         to bf16;
// kM = 2: the same layout with each operand split x = hi + lo (both bf16, lo = bf16(x - hi)):
//         A B = hi hi + hi lo + lo hi in three bf16 MFMAs (lo lo, of relative size 2^-16
//         squared, dropped), about 16 significant bits per product, f32 accumulation.
// A row and B column = lane % 16; D row = 4 (lane / 16) + r, column = lane % 16.
// k >= N (and n >= N) are zero in both operands.
typedef float fm_f4 __attribute__((ext_vector_type(4)));
typedef __bf16 fm_bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 fm_bf4 __attribute__((ext_vector_type(4)));

// Storage of the products Y: bf16 operands (kM = 1) leave about 3 significant digits in a
// product, so Y is stored rounded to bf16 (half the bytes phase 2a writes and phase 2b
// reads); the f32 and split-bf16 modes keep f32.
template <int kM> struct YStore { using T = float; };
template <> struct YStore<1> { using T = __bf16; };

template <int kM>
__device__ inline int mfma_k(int e, int lane) {
    return kM > 0 ? 32 * (e >> 3) + 8 * (lane >> 4) + (e & 7) : 4 * e + (lane >> 4);
}

// LDS row stride of a B chunk of W = 16 NT columns: a fragment read touches rows k..k+3
// (16 consecutive columns each); a stride of 16 mod 32 words spreads them over the banks.
template <int NT>
constexpr int b_stride() { return (16 * NT) % 32 == 16 ? 16 * NT : 16 * NT + 16; }

// A operand of one row tile as the matrix cores take it: kM > 0 packed bf16 (kM = 2 with the
// low parts), kM = 0 the f32 values.
template <int kM, int KE>
struct AFrag {
    fm_bf8 h[KE / 8];
    fm_bf8 l[kM == 2 ? KE / 8 : 1];
};
template <int KE>
struct AFrag<0, KE> {
    float a[KE];
};

template <int kM, int KE>
__device__ inline AFrag<kM, KE> make_afrag(const float (&a)[KE]) {
    AFrag<kM, KE> r;
    if constexpr (kM > 0) {
#pragma unroll
        for (int s = 0; s < KE / 8; ++s)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                r.h[s][e] = static_cast<__bf16>(a[8 * s + e]);
                if constexpr (kM == 2) r.l[s][e] = static_cast<__bf16>(a[8 * s + e] - static_cast<float>(r.h[s][e]));
            }
    } else {
#pragma unroll
        for (int e = 0; e < KE; ++e) r.a[e] = a[e];
    }
    return r;
}

// One 16-row tile on the matrix cores: c0 += A B0 (and c1 += A B1 for the direct channel).
// kM = 0: B fragments read from LDS as [k][n] floats (stride b_stride).  kM > 0: B staged as
// bf16, transposed [n][k] with row stride 4 KE + 8, so a lane's 8 consecutive k of one column
// are a single 16-byte read; kM = 2 keeps a second plane with the low parts right after the
// first.  Both zero beyond N.
template <int kM, int KE, int NT, bool kTwo>
__device__ inline void mfma_tile_f(const AFrag<kM, KE>& A, const void* Bs0v, const void* Bs1v,
                                   fm_f4 (&c0)[NT], fm_f4 (&c1)[NT], int lane) {
    const int col = lane & 15;
    if constexpr (kM > 0) {
        constexpr int KBS = 4 * KE + 8;
        constexpr int PL = 16 * NT * KBS;              // elements per plane
        const __bf16* Bh0 = static_cast<const __bf16*>(Bs0v);
        const __bf16* Bh1 = static_cast<const __bf16*>(Bs1v);
#pragma unroll
        for (int s = 0; s < KE / 8; ++s) {
            const fm_bf8 ah = A.h[s];
            const int kb = 32 * s + 8 * (lane >> 4);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int o = (16 * t + col) * KBS + kb;
                const fm_bf8 bh = *reinterpret_cast<const fm_bf8*>(Bh0 + o);
                if constexpr (kM == 2) {
                    const fm_bf8 bl = *reinterpret_cast<const fm_bf8*>(Bh0 + PL + o);
                    c0[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.l[s], bh, c0[t], 0, 0, 0);
                    c0[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c0[t], 0, 0, 0);
                }
                c0[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c0[t], 0, 0, 0);
                if constexpr (kTwo) {
                    const fm_bf8 wh = *reinterpret_cast<const fm_bf8*>(Bh1 + o);
                    if constexpr (kM == 2) {
                        const fm_bf8 wl = *reinterpret_cast<const fm_bf8*>(Bh1 + PL + o);
                        c1[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.l[s], wh, c1[t], 0, 0, 0);
                        c1[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, wl, c1[t], 0, 0, 0);
                    }
                    c1[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, wh, c1[t], 0, 0, 0);
                }
            }
        }
    } else {
        constexpr int S = b_stride<NT>();
        const float* Bs0 = static_cast<const float*>(Bs0v);
        const float* Bs1 = static_cast<const float*>(Bs1v);
#pragma unroll
        for (int e = 0; e < KE; ++e) {
            const int k = 4 * e + (lane >> 4);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                c0[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.a[e], Bs0[k * S + 16 * t + col], c0[t], 0, 0, 0);
                if constexpr (kTwo)
                    c1[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.a[e], Bs1[k * S + 16 * t + col], c1[t], 0, 0, 0);
            }
        }
    }
}

// The same from the f32 values of the lane's k-values.
template <int kM, int KE, int NT, bool kTwo>
__device__ inline void mfma_tile(const float (&a)[KE], const void* Bs0v, const void* Bs1v,
                                 fm_f4 (&c0)[NT], fm_f4 (&c1)[NT], int lane) {
    mfma_tile_f<kM, KE, NT, kTwo>(make_afrag<kM, KE>(a), Bs0v, Bs1v, c0, c1, lane);
}

// A operand of one row tile: lane row q = 16 tile + lane % 16 (rep r, operation o), k-values
// of the lane: A[q][k] = Z_g Z_k (al + be (W_g + W_k)) Brep_r(pinv_o g, pinv_o k), zero for
// k >= N; zs holds Z in [0, N) and W = K Z in [N, 2N).
template <int kM, int KE>
__device__ inline void gather_rows(float (&a)[KE], const float* Bf, int NN, int N, int grp,
                                int rep, int op, const int* pis, const float* zs, float zg,
                                float al, float be, int lane) {
    const int* pi = pis + op * N;
    const float* row = Bf + static_cast<size_t>(rep) * NN + pi[grp] * N;
    // all permutation entries, then all loads in flight together, then the Z factors
    int col[KE];
#pragma unroll
    for (int e = 0; e < KE; ++e) col[e] = pi[min(mfma_k<kM>(e, lane), N - 1)];
#pragma unroll
    for (int e = 0; e < KE; ++e) a[e] = row[col[e]];
    const float wg = zs[N + grp];
#pragma unroll
    for (int e = 0; e < KE; ++e) {
        const int k = mfma_k<kM>(e, lane);
        const float zk = zs[min(k, N - 1)], wk = zs[N + min(k, N - 1)];
        a[e] = k < N ? a[e] * (zg * zk * (al + be * (wg + wk))) : 0.f;
    }
}

// Representative and operation of the lane's row in row tile `tile` (clamped to the last
// transfer, so tiles past the end read valid entries).
__device__ inline void tile_rep(const int* qrep, const int* qg, int M, int tile, int col,
                                int& rep, int& op) {
    const int q = min(tile * 16 + col, M - 1);
    rep = qrep[q];
    op = qg[q];
}

// Row tiles [t_begin, t_end) of one wavefront: the A gather of tile t+1 and the table
// entries of tile t+2 are in flight while tile t runs on the matrix cores and is stored.
template <int kM, int KE, int NT, bool kTwo>
__device__ inline void y_tiles_rows(const float* Bf, const int* qrep, const int* qg, int NN, int N,
                               int M, int grp, int n0, int t_begin, int t_end, const int* pis,
                               const float* zs, float al, float be, const void* Bs0,
                               const void* Bs1, typename YStore<kM>::T* Y0,
                               typename YStore<kM>::T* Y1, int lane, int r0, int o0,
                               int r1, int o1) {
    using YT = typename YStore<kM>::T;
    const int col = lane & 15;
    const float zg = zs[grp];
    float a0[KE], a1[KE];
    gather_rows<kM, KE>(a0, Bf, NN, N, grp, r0, o0, pis, zs, zg, al, be, lane);
    for (int tile = t_begin; tile < t_end; ++tile) {
        // B fragments are re-read from LDS every tile instead of being kept in registers
        asm volatile("" ::: "memory");
        int r2, o2;
        tile_rep(qrep, qg, M, tile + 2, col, r2, o2);
        if (tile + 1 < t_end) gather_rows<kM, KE>(a1, Bf, NN, N, grp, r1, o1, pis, zs, zg, al, be, lane);
        fm_f4 c0[NT], c1[NT];
#pragma unroll
        for (int u = 0; u < NT; ++u) c0[u] = c1[u] = fm_f4{0.f, 0.f, 0.f, 0.f};
        mfma_tile<kM, KE, NT, kTwo>(a0, Bs0, Bs1, c0, c1, lane);
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int n = n0 + 16 * u + col;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int qq = tile * 16 + 4 * (lane >> 4) + r;
                if (qq < M && n < N) {
                    const size_t o = static_cast<size_t>(qq) * NN + grp * N + n;
                    Y0[o] = static_cast<YT>(c0[u][r]);
                    if constexpr (kTwo) Y1[o] = static_cast<YT>(c1[u][r]);
                }
            }
        }
#pragma unroll
        for (int e = 0; e < KE; ++e) a0[e] = a1[e];
        r1 = r2;
        o1 = o2;
    }
}

// Per-row variant (any transfer order).  1D grid.  A work group is (row-tile run x, group g,
// channel, flow), numbered
// w = ((flow * 3 + channel) * N + g) * bx + x; its nchunk column chunks read the same A rows.
// Workgroups are dealt to the 8 XCDs round-robin, so the chunks of one work group get
// block ids 8 apart (same XCD, launched together) and its A rows come from one L2:
//   id = (w / 8) * 8 nchunk + chunk * 8 + w % 8.
// The block stages its B chunk(s) in LDS once and reuses them for all 4 tpw row tiles;
// every wave gathers its tiles' A operands straight into MFMA layout.
template <int kM, int KE, int NT>
__global__ void __launch_bounds__(kThreads) k_y_mfma_rows(DevGeom g, const FlowState* fs,
                                                     const double* Z_stage, const double* zw,
                                                     const float* bins, const float* binsT,
                                                     YArgs<float> args, int nchunk, int tpw,
                                                     int bx, int nwork) {
    constexpr int S = b_stride<NT>(), KP = 4 * KE, W = 16 * NT, KBS = KP + 8;
    constexpr int kBytes = kM == 0 ? KP * S * 4 : W * KBS * 2 * kM;   // one B chunk (kM planes)
    __shared__ int pis[8 * 128];                      // patch permutations (N <= 128)
    __shared__ float zs[256];                         // Z and W = K Z of the stage
    __shared__ __align__(16) unsigned char Braw[2 * kBytes];   // B chunks
    const int id = blockIdx.x;
    const int rem = id % (8 * nchunk);
    const int work = (id / (8 * nchunk)) * 8 + rem % 8;
    const int chunk = rem / 8;
    if (work >= nwork) return;                        // padding of the last 8 work groups
    const int N = g.N, NN = g.NN;
    const int xr = work % bx;
    const int grp = (work / bx) % N;
    const int ch = (work / (bx * N)) % 3;
    const int f = work / (bx * N * 3);
    const int M = ch == 0 ? g.nP : g.nD;
    const int n0 = chunk * W;
    const int ntiles = (M + 15) / 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int t_begin = (xr * 4 + wv) * tpw;
    const int t_end = min(t_begin + tpw, ntiles);
    const bool two = ch == 2;
    const int* qrep = ch == 0 ? g.qrep_pp : g.qrep_ph;
    const int* qg = ch == 0 ? g.qg_pp : g.qg_ph;
    // the first two tiles' transfer tables need no LDS: loaded with the flow's status and in
    // flight across the barrier
    int r0, o0, r1, o1;
    tile_rep(qrep, qg, M, t_begin, lane & 15, r0, o0);
    tile_rep(qrep, qg, M, t_begin + 1, lane & 15, r1, o1);
    if (!running(fs, f) || !args.on[ch]) return;      // uniform over the block
    const int nR = g.nRp + g.nRd;
    const int fb = bin_flow(fs, f);
    const float* Bf = ch == 1 ? binsT + static_cast<size_t>(fb) * g.nRd * NN
                              : bins + static_cast<size_t>(fb) * nR * NN + (ch == 0 ? 0 : static_cast<size_t>(g.nRp) * NN);
    // The permutation table, Z and the B chunk: every load in flight before any LDS store
    // (one round trip instead of one per element).
    int pv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) pv[v] = g.pinv[min(static_cast<int>(threadIdx.x) + v * kThreads, 8 * N - 1)];
    const double* Zf = Z_stage + static_cast<size_t>(f) * 2 * N;
    const float zv = static_cast<float>(Zf[min(static_cast<int>(threadIdx.x), N - 1)]);
    const float kzv = static_cast<float>(Zf[N + min(static_cast<int>(threadIdx.x), N - 1)]);
    const size_t N3 = static_cast<size_t>(NN) * N;
    const size_t slab = f * N3 + static_cast<size_t>(grp) * NN;
    const float* V0 = args.Vs[two ? 2 : ch] + slab;
    const float* V1 = args.Vs[3] + slab;
    // B chunk: every element's load in flight before any is stored
    constexpr int kPer = KP * W / kThreads;
    static_assert(KP * W % kThreads == 0, "staging covers the chunk in whole rounds");
    float sv0[kPer], sv1[kPer];
    auto stage_index = [&](int j) {
        const int e = threadIdx.x + j * kThreads;
        const int k = e / W, n = e - k * W;            // W is a compile-time constant
        return static_cast<size_t>(min(k, N - 1)) * N + min(n0 + n, N - 1);
    };
    // the second operand only for the direct channel; elsewhere the same loads repeat the
    // first one's addresses (cache hits, no branch between the loads)
    const float* V1s = two ? V1 : V0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        sv0[j] = V0[stage_index(j)];
        sv1[j] = V1s[stage_index(j)];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)          // the permutation table (8 N <= 1024 entries)
        if (static_cast<int>(threadIdx.x) + v * kThreads < 8 * N) pis[threadIdx.x + v * kThreads] = pv[v];
    if (threadIdx.x < N) {
        zs[threadIdx.x] = zv;
        zs[N + threadIdx.x] = kzv;
    }
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        const int e = threadIdx.x + j * kThreads;
        const int k = e / W, n = e - k * W;
        const bool ok = k < N && n0 + n < N;
        const float x0 = ok ? sv0[j] : 0.f;
        const float x1 = (two && ok) ? sv1[j] : 0.f;
        if constexpr (kM > 0) {
            __bf16* Bh = reinterpret_cast<__bf16*>(Braw);
            const __bf16 h0 = static_cast<__bf16>(x0), h1 = static_cast<__bf16>(x1);
            Bh[n * KBS + k] = h0;
            if (two) Bh[kBytes / 2 + n * KBS + k] = h1;
            if constexpr (kM == 2) {                   // low parts: the second plane
                Bh[W * KBS + n * KBS + k] = static_cast<__bf16>(x0 - static_cast<float>(h0));
                if (two) Bh[kBytes / 2 + W * KBS + n * KBS + k] = static_cast<__bf16>(x1 - static_cast<float>(h1));
            }
        } else {
            float* Bf32 = reinterpret_cast<float*>(Braw);
            Bf32[k * S + n] = x0;
            if (two) Bf32[KP * S + k * S + n] = x1;
        }
    }
    __syncthreads();                                   // every thread of the block
    if (t_begin >= t_end) return;
    using YT = typename YStore<kM>::T;
    const size_t yoff = static_cast<size_t>(f) * M * NN;
    const void* B0 = Braw;
    const void* B1 = Braw + kBytes;
    const float al = static_cast<float>(zw[2 * f]), be = static_cast<float>(zw[2 * f + 1]);
    if (two)
        y_tiles_rows<kM, KE, NT, true>(Bf, qrep, qg, NN, N, M, grp, n0, t_begin, t_end, pis, zs,
                                     al, be, B0, B1, reinterpret_cast<YT*>(args.Y[2]) + yoff,
                                     reinterpret_cast<YT*>(args.Y[3]) + yoff, lane, r0, o0, r1,
                                     o1);
    else
        y_tiles_rows<kM, KE, NT, false>(Bf, qrep, qg, NN, N, M, grp, n0, t_begin, t_end, pis, zs,
                                      al, be, B0, B1, reinterpret_cast<YT*>(args.Y[ch]) + yoff,
                                      nullptr, lane, r0, o0, r1, o1);
}

// Row tiles of one operation class.  Transfers are ordered by (operation o, representative),
// so a 16-row tile shares o and its A rows are plain rows of representatives' bins:
//   A[q][k'] = Brep_r(pinv_o g, k')   (k' = pinv_o k; the permutation moves to B, below).
// Rows past the class end are clamped to its last transfer (valid reads; never stored).
// A lane's k-values: kM = 0, k' = 4 e + lane / 16 (the four lane groups of a row read 16
// contiguous bytes); kM > 0, eight consecutive k' per 32-wide step, two 16-byte loads
// (N % 4 == 0; else one value at a time).  Every address is the lane's base plus a
// constant.  k' in [N, 4 KE) reads past the row's end, into the next row or the zeroed
// padding that follows the bin buffers (finite values either way); the staged B is zero
// there.
template <int kM, int KE>
__device__ inline void gather_a(float (&a)[KE], const float* row, int N, int lane) {
    if constexpr (kM == 0) {
        const float* r = row + (lane >> 4);
#pragma unroll
        for (int e = 0; e < KE; ++e) a[e] = r[4 * e];
    } else {
        const float* r = row + 8 * (lane >> 4);
        if ((N & 3) == 0) {
#pragma unroll
            for (int s = 0; s < KE / 8; ++s) {
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    const float4 v = *reinterpret_cast<const float4*>(r + 32 * s + 4 * hh);
                    a[8 * s + 4 * hh] = v.x;
                    a[8 * s + 4 * hh + 1] = v.y;
                    a[8 * s + 4 * hh + 2] = v.z;
                    a[8 * s + 4 * hh + 3] = v.w;
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < KE; ++e) a[e] = r[32 * (e >> 3) + (e & 7)];
        }
    }
}

// Row tiles [t_begin, t_end) of one wavefront within class [q0, q1): the A rows of tile t+1
// are loaded while tile t runs on the matrix cores and is stored, and the representative
// of tile t+2 is in flight.
template <int kM, int KE, int NT, bool kTwo>
__device__ inline void y_tiles(const float* Bf, const int* qrep, int NN, int N, int q0,
                               int q1, int prow, int grp, int n0, int t_begin, int t_end,
                               const void* Bs0, const void* Bs1, typename YStore<kM>::T* Y0,
                               typename YStore<kM>::T* Y1, int lane, int r0, int r1) {
    using YT = typename YStore<kM>::T;
    const int col = lane & 15;
    const size_t roff = static_cast<size_t>(prow) * N;
    float a0[KE], a1[KE];
    gather_a<kM, KE>(a0, Bf + static_cast<size_t>(r0) * NN + roff, N, lane);
#pragma unroll 1
    for (int tile = t_begin; tile < t_end; ++tile) {
        // B fragments are re-read from LDS every tile instead of being kept in registers
        asm volatile("" ::: "memory");
        const int r2 = qrep[min(q0 + 16 * (tile + 2) + col, q1 - 1)];
        if (tile + 1 < t_end) gather_a<kM, KE>(a1, Bf + static_cast<size_t>(r1) * NN + roff, N, lane);
        fm_f4 c0[NT], c1[NT];
#pragma unroll
        for (int u = 0; u < NT; ++u) c0[u] = c1[u] = fm_f4{0.f, 0.f, 0.f, 0.f};
        mfma_tile<kM, KE, NT, kTwo>(a0, Bs0, Bs1, c0, c1, lane);
#pragma unroll
        for (int u = 0; u < NT; ++u) {
            const int n = n0 + 16 * u + col;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int qq = q0 + tile * 16 + 4 * (lane >> 4) + r;
                if (qq < q1 && n < N) {
                    const size_t o = static_cast<size_t>(qq) * NN + grp * N + n;
                    Y0[o] = static_cast<YT>(c0[u][r]);
                    if constexpr (kTwo) Y1[o] = static_cast<YT>(c1[u][r]);
                }
            }
        }
#pragma unroll
        for (int e = 0; e < KE; ++e) a0[e] = a1[e];
        r1 = r2;
    }
}

// Row-tile runs of the operation classes for one launch: run count of class o per channel
// kind (0 particle-particle, 1 particle-hole) and in total, for `tpw` tiles per wavefront.
struct YRuns {
    int nr[2][8];
    int tot[2];
};

// 1D grid.  A work group is (class run x, group g, channel, flow), numbered
// w = ((flow * 3 + channel) * N + g) * bx + x; its nchunk column chunks read the same A rows.
// Workgroups are dealt to the 8 XCDs round-robin, so the chunks of one work group get
// block ids 8 apart (same XCD, launched together) and its A rows come from one L2:
//   id = (w / 8) * 8 nchunk + chunk * 8 + w % 8.
// Run x of channel kind c is run r of class o; the block stages its B chunk once, for that
// operation:
//   B'[k'][n] = Z_g Z_k (al + be (W_g + W_k)) Vsrc[g][k][n],  k = perm_o k',
// so that sum_k' A[q][k'] B'[k'][n] is the product of the gathered, permuted and Z-weighted
// bins with the slab.  The 4 waves take tpw consecutive row tiles each.
template <int kM, int KE, int NT>
__global__ void __launch_bounds__(kThreads) k_y_mfma_cls(DevGeom g, const FlowState* fs,
                                                     const double* Z_stage, const double* zw,
                                                     const float* bins, const float* binsT,
                                                     YArgs<float> args, YRuns runs, int nchunk,
                                                     int tpw, int bx, int nwork) {
    constexpr int S = b_stride<NT>(), KP = 4 * KE, W = 16 * NT, KBS = KP + 8;
    constexpr int kBytes = kM == 0 ? KP * S * 4 : W * KBS * 2 * kM;   // one B chunk (kM planes)
    __shared__ __align__(16) unsigned char Braw[2 * kBytes];   // B chunks
    __shared__ int kperm[4 * KE];                     // perm_o k' (k' < N)
    __shared__ float kfac[4 * KE];                    // Z_g Z_k (al + be (W_g + W_k)), k = perm_o k' 
    const int id = blockIdx.x;
    const int rem = id % (8 * nchunk);
    const int work = (id / (8 * nchunk)) * 8 + rem % 8;
    const int chunk = rem / 8;
    if (work >= nwork) return;                        // padding of the last 8 work groups
    const int N = g.N, NN = g.NN;
    int x = work % bx;
    const int grp = (work / bx) % N;
    const int ch = (work / (bx * N)) % 3;
    const int f = work / (bx * N * 3);
    if (!running(fs, f) || !args.on[ch]) return;      // uniform over the block
    const int cc = ch == 0 ? 0 : 1;
    int o = 0;
    for (; o < 8; ++o) {
        if (x < runs.nr[cc][o]) break;
        x -= runs.nr[cc][o];
    }
    if (o == 8) return;                               // past this kind's runs (uniform)
    const int q0 = g.cls[cc][o], q1 = g.cls[cc][o + 1];
    const int M = ch == 0 ? g.nP : g.nD;
    const int n0 = chunk * W;
    const int ntiles = (q1 - q0 + 15) / 16;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int t_begin = (x * 4 + wv) * tpw;
    const int t_end = min(t_begin + tpw, ntiles);
    const bool two = ch == 2;
    const int* qrep = ch == 0 ? g.qrep_pp : g.qrep_ph;
    // the first two tiles' representatives: in flight across the barrier
    const int col = lane & 15;
    const int r0 = qrep[min(q0 + 16 * t_begin + col, q1 - 1)];
    const int r1 = qrep[min(q0 + 16 * (t_begin + 1) + col, q1 - 1)];
    const int prow = g.pinv[o * N + grp];
    const size_t N3 = static_cast<size_t>(NN) * N;
    const size_t slab = f * N3 + static_cast<size_t>(grp) * NN;
    const float* V0 = args.Vs[two ? 2 : ch] + slab;
    const float* V1 = args.Vs[3] + slab;
    if (threadIdx.x < KP) {                           // per-k' permutation and factor
        const double* Zf = Z_stage + static_cast<size_t>(f) * 2 * N;
        const float zg = static_cast<float>(Zf[grp]), wg = static_cast<float>(Zf[N + grp]);
        const float al = static_cast<float>(zw[2 * f]), be = static_cast<float>(zw[2 * f + 1]);
        const int kp = g.perm[o * N + min(static_cast<int>(threadIdx.x), N - 1)];
        const float zk = static_cast<float>(Zf[kp]), wk = static_cast<float>(Zf[N + kp]);
        kperm[threadIdx.x] = kp;
        kfac[threadIdx.x] = zg * zk * (al + be * (wg + wk));
    }
    __syncthreads();                                   // every thread of the block
    for (int e = threadIdx.x; e < KP * W; e += kThreads) {
        const int k = e / W, n = e - k * W;            // W is a compile-time constant
        const bool ok = k < N && n0 + n < N;
        const int kp = kperm[k];
        const float fac = kfac[k];
        const size_t ia = static_cast<size_t>(kp) * N + min(n0 + n, N - 1);
        const float x0 = ok ? fac * V0[ia] : 0.f;
        const float x1 = (two && ok) ? fac * V1[ia] : 0.f;
        if constexpr (kM > 0) {
            __bf16* Bh = reinterpret_cast<__bf16*>(Braw);
            const __bf16 h0 = static_cast<__bf16>(x0), h1 = static_cast<__bf16>(x1);
            Bh[n * KBS + k] = h0;
            if (two) Bh[kBytes / 2 + n * KBS + k] = h1;
            if constexpr (kM == 2) {                   // low parts: the second plane
                Bh[W * KBS + n * KBS + k] = static_cast<__bf16>(x0 - static_cast<float>(h0));
                if (two) Bh[kBytes / 2 + W * KBS + n * KBS + k] = static_cast<__bf16>(x1 - static_cast<float>(h1));
            }
        } else {
            float* Bf32 = reinterpret_cast<float*>(Braw);
            Bf32[k * S + n] = x0;
            if (two) Bf32[KP * S + k * S + n] = x1;
        }
    }
    __syncthreads();                                   // every thread of the block
    if (t_begin >= t_end) return;
    const int nR = g.nRp + g.nRd;
    const int fb = bin_flow(fs, f);
    const float* Bf = ch == 1 ? binsT + static_cast<size_t>(fb) * g.nRd * NN
                              : bins + static_cast<size_t>(fb) * nR * NN + (ch == 0 ? 0 : static_cast<size_t>(g.nRp) * NN);
    using YT = typename YStore<kM>::T;
    const size_t yoff = static_cast<size_t>(f) * M * NN;
    const void* B0 = Braw;
    const void* B1 = Braw + kBytes;
    if (two)
        y_tiles<kM, KE, NT, true>(Bf, qrep, NN, N, q0, q1, prow, grp, n0, t_begin, t_end, B0,
                                  B1, reinterpret_cast<YT*>(args.Y[2]) + yoff,
                                  reinterpret_cast<YT*>(args.Y[3]) + yoff, lane, r0, r1);
    else
        y_tiles<kM, KE, NT, false>(Bf, qrep, NN, N, q0, q1, prow, grp, n0, t_begin, t_end, B0,
                                   B1, reinterpret_cast<YT*>(args.Y[ch]) + yoff, nullptr, lane,
                                   r0, r1);
}

// B operand of one wavefront's tiles in registers: the fragments of every k-step and column
// tile, read from the staged chunk once and used by all of the wave's row tiles.
template <int kM, int KE, int NT>
struct BFrag {
    fm_bf8 h[KE / 8][NT];
    fm_bf8 l[kM == 2 ? KE / 8 : 1][NT];
};
template <int KE, int NT>
struct BFrag<0, KE, NT> {
    float b[KE][NT];
};

template <int kM, int KE, int NT>
__device__ inline void load_bfrag(BFrag<kM, KE, NT>& B, const void* Bsv, int lane) {
    const int col = lane & 15;
    if constexpr (kM > 0) {
        constexpr int KBS = 4 * KE + 8;
        constexpr int PL = 16 * NT * KBS;
        const __bf16* Bh = static_cast<const __bf16*>(Bsv);
#pragma unroll
        for (int s = 0; s < KE / 8; ++s)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int o = (16 * t + col) * KBS + 32 * s + 8 * (lane >> 4);
                B.h[s][t] = *reinterpret_cast<const fm_bf8*>(Bh + o);
                if constexpr (kM == 2) B.l[s][t] = *reinterpret_cast<const fm_bf8*>(Bh + PL + o);
            }
    } else {
        constexpr int S = b_stride<NT>();
        const float* Bs = static_cast<const float*>(Bsv);
#pragma unroll
        for (int e = 0; e < KE; ++e)
#pragma unroll
            for (int t = 0; t < NT; ++t) B.b[e][t] = Bs[(4 * e + (lane >> 4)) * S + 16 * t + col];
    }
}

// c += A B with both operands in registers (the fragment layouts of mfma_tile_f): lane holds
// rows 4 (lane / 16) .. + 3 of column lane % 16 of each 16 x 16 tile c[t].
template <int kM, int KE, int NT>
__device__ inline void mfma_ab(const AFrag<kM, KE>& A, const BFrag<kM, KE, NT>& B, fm_f4 (&c)[NT]) {
    if constexpr (kM > 0) {
#pragma unroll
        for (int s = 0; s < KE / 8; ++s)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if constexpr (kM == 2) {
                    c[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.l[s], B.h[s][t], c[t], 0, 0, 0);
                    c[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.h[s], B.l[s][t], c[t], 0, 0, 0);
                }
                c[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.h[s], B.h[s][t], c[t], 0, 0, 0);
            }
    } else {
#pragma unroll
        for (int e = 0; e < KE; ++e)
#pragma unroll
            for (int t = 0; t < NT; ++t)
                c[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(A.a[e], B.b[e][t], c[t], 0, 0, 0);
    }
}

// c += (A B)^T with both operands in registers (the fragment layouts of mfma_tile_f).  The A
// and B fragments of these shapes have the same lane layout (lane % 16 the row of A or the
// column of B, lane / 16 the k group), so passing B first gives the transposed tile: lane
// holds rows 4 (lane / 16) .. + 3 of column lane % 16 of c[t] = (A B)^T, i.e. four
// consecutive n of row tile row lane % 16.
template <int kM, int KE, int NT>
__device__ inline void mfma_abt(const AFrag<kM, KE>& A, const BFrag<kM, KE, NT>& B, fm_f4 (&c)[NT]) {
    if constexpr (kM > 0) {
#pragma unroll
        for (int s = 0; s < KE / 8; ++s)
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                if constexpr (kM == 2) {
                    c[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(B.h[s][t], A.l[s], c[t], 0, 0, 0);
                    c[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(B.l[s][t], A.h[s], c[t], 0, 0, 0);
                }
                c[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(B.h[s][t], A.h[s], c[t], 0, 0, 0);
            }
    } else {
#pragma unroll
        for (int e = 0; e < KE; ++e)
#pragma unroll
            for (int t = 0; t < NT; ++t)
                c[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(B.b[e][t], A.a[e], c[t], 0, 0, 0);
    }
}

// Loads a thread keeps in flight while staging: the largest divisor of its count up to 16.
constexpr int stage_group(int per) {
    int gsz = per < 16 ? per : 16;
    while (per % gsz) --gsz;
    return gsz;
}

// Stages B'_o[k'][n] = fac(k) Vsrc[k][n0 + n], k = perm_o k' (fac from the stage's Z), for
// one or two operand slabs into the block's chunk(s).  Loads are issued in groups before
// any of them is used, so a thread has a group in flight instead of one.
template <int kM, int KE, int NT, bool kTwo, int BT = kThreads>
__device__ inline void stage_orbit_b(unsigned char* Braw, const float* V0, const float* V1,
                                     const int* pm, const float* zs, float zg, float wg,
                                     float al, float be, int N, int n0) {
    constexpr int S = b_stride<NT>(), KP = 4 * KE, W = 16 * NT, KBS = KP + 8;
    constexpr int kBytes = kM == 0 ? KP * S * 4 : W * KBS * 2 * kM;
    constexpr int kPer = KP * W / BT > 0 ? KP * W / BT : 1;
    static_assert(kM > 0 || KP * W % BT == 0, "staging covers the chunk in whole rounds");
    constexpr int kGrp = stage_group(kPer);
    if constexpr (kM > 0) {
        // bf16 planes [n][k']: a task is 8 consecutive k' of one column n, loaded together
        // (each load coalesced over the wave's columns) and stored as one 16-byte row
        // segment per plane
        constexpr int kTasks = KP / 8 * W;
        constexpr int kTPT = (kTasks + BT - 1) / BT;
        constexpr int R = kTPT < 2 ? kTPT : 2;          // tasks whose loads are in flight
        __bf16* Bh = reinterpret_cast<__bf16*>(Braw);
#pragma unroll 1
        for (int j0 = 0; j0 < kTPT; j0 += R) {
            float x0[R][8], x1[R][8];
            int kq[R][8];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int task = min(static_cast<int>(threadIdx.x) + (j0 + j) * BT, kTasks - 1);
                const int n = task % W, kb = 8 * (task / W);
                const int nc = min(n0 + n, N - 1);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int kp = pm[min(kb + i, N - 1)];
                    kq[j][i] = kp;
                    x0[j][i] = V0[static_cast<size_t>(kp) * N + nc];
                    if constexpr (kTwo) x1[j][i] = V1[static_cast<size_t>(kp) * N + nc];
                }
            }
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int task = static_cast<int>(threadIdx.x) + (j0 + j) * BT;
                if (task >= kTasks) continue;
                const int n = task % W, kb = 8 * (task / W);
                const bool nok = n0 + n < N;
                fm_bf8 h0, h1, l0, l1;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int kp = kq[j][i];
                    const float fac = (nok && kb + i < N) ? zg * zs[kp] * (al + be * (wg + zs[N + kp])) : 0.f;
                    const float y0 = fac * x0[j][i];
                    h0[i] = static_cast<__bf16>(y0);
                    if constexpr (kM == 2) l0[i] = static_cast<__bf16>(y0 - static_cast<float>(h0[i]));
                    if constexpr (kTwo) {
                        const float y1 = fac * x1[j][i];
                        h1[i] = static_cast<__bf16>(y1);
                        if constexpr (kM == 2) l1[i] = static_cast<__bf16>(y1 - static_cast<float>(h1[i]));
                    }
                }
                const int o = n * KBS + kb;
                *reinterpret_cast<fm_bf8*>(Bh + o) = h0;
                if constexpr (kM == 2) *reinterpret_cast<fm_bf8*>(Bh + W * KBS + o) = l0;
                if constexpr (kTwo) {
                    *reinterpret_cast<fm_bf8*>(Bh + kBytes / 2 + o) = h1;
                    if constexpr (kM == 2) *reinterpret_cast<fm_bf8*>(Bh + kBytes / 2 + W * KBS + o) = l1;
                }
            }
        }
        return;
    }
#pragma unroll 1
    for (int j0 = 0; j0 < kPer; j0 += kGrp) {
        float v0[kGrp], v1[kGrp];
        int kq[kGrp];
#pragma unroll
        for (int j = 0; j < kGrp; ++j) {
            const int e = threadIdx.x + (j0 + j) * BT;
            const int k = e / W, n = e - k * W;
            const int kp = pm[min(k, N - 1)];
            kq[j] = kp;
            const size_t ia = static_cast<size_t>(kp) * N + min(n0 + n, N - 1);
            v0[j] = V0[ia];
            if constexpr (kTwo) v1[j] = V1[ia];
        }
#pragma unroll
        for (int j = 0; j < kGrp; ++j) {
            const int e = threadIdx.x + (j0 + j) * BT;
            const int k = e / W, n = e - k * W;
            const bool ok = k < N && n0 + n < N;
            const float zk = zs[kq[j]], wk = zs[N + kq[j]];
            const float fac = ok ? zg * zk * (al + be * (wg + wk)) : 0.f;
            const float x0 = fac * v0[j];
            const float x1 = kTwo ? fac * v1[j] : 0.f;
            if constexpr (kM > 0) {
                __bf16* Bh = reinterpret_cast<__bf16*>(Braw);
                const __bf16 h0 = static_cast<__bf16>(x0), h1 = static_cast<__bf16>(x1);
                Bh[n * KBS + k] = h0;
                if constexpr (kTwo) Bh[kBytes / 2 + n * KBS + k] = h1;
                if constexpr (kM == 2) {               // low parts: the second plane
                    Bh[W * KBS + n * KBS + k] = static_cast<__bf16>(x0 - static_cast<float>(h0));
                    if constexpr (kTwo) Bh[kBytes / 2 + W * KBS + n * KBS + k] = static_cast<__bf16>(x1 - static_cast<float>(h1));
                }
            } else {
                float* Bf32 = reinterpret_cast<float*>(Braw);
                Bf32[k * S + n] = x0;
                if constexpr (kTwo) Bf32[KP * S + k * S + n] = x1;
            }
        }
    }
}

// Orbit kernel.  Transfer q = o(r) of representative r needs row pinv_o(g) of r's bins for
// slab g; for fixed bin row p that is slab g = perm_o(p).  A block takes one bin row p, a run
// of representative tiles (4 waves x TPW tiles of 16 representatives) and one column chunk;
// it loads its A rows once, keeps them in registers, and for each operation o that yields
// transfers of its tiles stages
//   B'_o[k'][n] = Z_g Z_k (al + be (W_g + W_k)) Vsrc[g][k][n],  g = perm_o p,  k = perm_o k',
// and stores the tile product into the rows of the transfers o(r) at slab g.  Every (q, g)
// is produced once (q by its own (o, r), g by p = pinv_o g), and every bin row is read by
// one block per column chunk instead of once per transfer of its orbit.  A wave reads B'_o
// from LDS into registers once and applies it to all its tiles.
// Grid: a work group is (patch group G of 8 bin rows, channel, flow), numbered
// gw = (flow * 3 + channel) * nG + G; its 8 bx nchunk blocks (member i, run x, chunk) read
// the operand slabs of G's orbits only and go to one XCD, launched together:
//   id = (gw / 8) * 8 gsize + m * 8 + gw % 8,  m = (i * bx + x) * nchunk + chunk.
template <int kM, int KE, int NT, int TPW, bool kTwo>
__device__ inline void y_orbit_block(const DevGeom& g, const float* Bf, const float* Vs0,
                                     const float* Vs1, typename YStore<kM>::T* Y0,
                                     typename YStore<kM>::T* Y1, int p, int tb,
                                     int nt, int toff, int n0, float al, float be,
                                     const double* Zf, unsigned char* Braw, int* pms,
                                     float* zs, int* qs, int* msk) {
    constexpr int S = b_stride<NT>(), KP = 4 * KE, W = 16 * NT, KBS = KP + 8;
    constexpr int kBytes = kM == 0 ? KP * S * 4 : W * KBS * 2 * kM;   // one B chunk (kM planes)
    const int N = g.N, NN = g.NN;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int col = lane & 15;
    const int tn = min(tb + 4 * TPW, nt);
    const int tw0 = tb + wv * TPW;
    // Loads in dependency order, each group in flight together: the representatives of the
    // wave's tiles, the block's tables (permutations, transfers, operation sets, Z), then the
    // A rows (row p of each representative's bins), which need the representatives.
    int rr[TPW];
#pragma unroll
    for (int j = 0; j < TPW; ++j) rr[j] = g.orb_rows[16 * (toff + min(tw0 + j, nt - 1)) + col];
    int pv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) pv[v] = g.perm[min(static_cast<int>(threadIdx.x) + v * kThreads, 8 * N - 1)];
    constexpr int kQ = 4 * TPW * 128 / kThreads;
    const int nq = (tn - tb) * 128;
    const int* qsrc = g.orb_q + static_cast<size_t>(toff + tb) * 128;
    int qv[kQ];
#pragma unroll
    for (int v = 0; v < kQ; ++v) qv[v] = qsrc[min(static_cast<int>(threadIdx.x) + v * kThreads, nq - 1)];
    const int mv = g.orb_mask[toff + tb + min(static_cast<int>(threadIdx.x), tn - tb - 1)];
    const float zv = static_cast<float>(Zf[min(static_cast<int>(threadIdx.x), N - 1)]);
    const float kzv = static_cast<float>(Zf[N + min(static_cast<int>(threadIdx.x), N - 1)]);
    float a[TPW][KE];
#pragma unroll
    for (int j = 0; j < TPW; ++j)
        gather_a<kM, KE>(a[j], Bf + static_cast<size_t>(max(rr[j], 0)) * NN + static_cast<size_t>(p) * N, N, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v)
        if (static_cast<int>(threadIdx.x) + v * kThreads < 8 * N) pms[threadIdx.x + v * kThreads] = pv[v];
#pragma unroll
    for (int v = 0; v < kQ; ++v)
        if (static_cast<int>(threadIdx.x) + v * kThreads < nq) qs[threadIdx.x + v * kThreads] = qv[v];
    if (static_cast<int>(threadIdx.x) < tn - tb) msk[threadIdx.x] = mv;
    if (static_cast<int>(threadIdx.x) < N) {
        zs[threadIdx.x] = zv;
        zs[N + threadIdx.x] = kzv;
    }
    AFrag<kM, KE> A[TPW];
#pragma unroll
    for (int j = 0; j < TPW; ++j) A[j] = make_afrag<kM, KE>(a[j]);
    __syncthreads();                                   // tables; every thread of the block
    int bmask = 0;                                     // operations used by the block's tiles
    for (int t = 0; t < tn - tb; ++t) bmask |= msk[t];
    if (g.sym) bmask &= 1;                             // symmetric states: representatives only
#pragma unroll 1
    for (int o = 0; o < 8; ++o) {
        if (!((bmask >> o) & 1)) continue;             // uniform over the block
        const int grp = pms[o * N + p];
        stage_orbit_b<kM, KE, NT, kTwo>(Braw, Vs0 + static_cast<size_t>(grp) * NN,
                                        Vs1 + static_cast<size_t>(grp) * NN, pms + o * N,
                                        zs, zs[grp], zs[N + grp], al, be, N, n0);
        __syncthreads();                               // B'_o staged; every thread
#pragma unroll
        for (int w = 0; w < (kTwo ? 2 : 1); ++w) {
            BFrag<kM, KE, NT> B;
            load_bfrag<kM, KE, NT>(B, Braw + w * kBytes, lane);
            typename YStore<kM>::T* Yw = w ? Y1 : Y0;
#pragma unroll
            for (int j = 0; j < TPW; ++j) {
                const int tl = tw0 + j - tb;           // tile within the block (wave-uniform)
                if (tw0 + j >= nt || !((msk[tl] >> o) & 1)) continue;
                fm_f4 c[NT];
#pragma unroll
                for (int u = 0; u < NT; ++u) c[u] = fm_f4{0.f, 0.f, 0.f, 0.f};
                if constexpr (kM == 0) {
                    // f32 operands: the untransposed tile (fewer registers live here), one
                    // value per store
                    mfma_ab<kM, KE, NT>(A[j], B, c);
                    const int* qt = qs + (tl * 8 + o) * 16 + 4 * (lane >> 4);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int q = qt[r];
                        if (q < 0) continue;
                        auto* yrow = Yw + static_cast<size_t>(q) * NN + static_cast<size_t>(grp) * N;
#pragma unroll
                        for (int u = 0; u < NT; ++u) {
                            const int n = n0 + 16 * u + col;
                            if (n < N) yrow[n] = c[u][r];
                        }
                    }
                    continue;
                }
                const int q = qs[(tl * 8 + o) * 16 + col];
                mfma_abt<kM, KE, NT>(A[j], B, c);
                // four consecutive n of transfer q per lane: one 16-byte store when N % 4 == 0
                // (rows then start 16-byte aligned and a group of four lies wholly below N or
                // at or above it), else one value at a time
                if (q >= 0) {
                    auto* yrow = Yw + static_cast<size_t>(q) * NN + static_cast<size_t>(grp) * N;
#pragma unroll
                    for (int u = 0; u < NT; ++u) {
                        const int n = n0 + 16 * u + 4 * (lane >> 4);
                        if ((N & 3) == 0) {
                            if (n < N) {
                                if constexpr (kM == 1)   // bf16 products: one 8-byte store
                                    *reinterpret_cast<fm_bf4*>(yrow + n) = __builtin_convertvector(c[u], fm_bf4);
                                else
                                    *reinterpret_cast<fm_f4*>(yrow + n) = c[u];
                            }
                        } else {
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                if (n + r < N) yrow[n + r] = static_cast<typename YStore<kM>::T>(c[u][r]);
                        }
                    }
                }
            }
        }
        __syncthreads();                               // B'_o consumed before the next stage
    }
}

template <int kM, int KE, int NT, int TPW>
__global__ void __launch_bounds__(kThreads) k_y_mfma_orb(DevGeom g, const FlowState* fs,
                                                     const double* Z_stage, const double* zw,
                                                     const float* bins, const float* binsT,
                                                     YArgs<float> args, int nchunk, int bx,
                                                     int ngw) {
    constexpr int S = b_stride<NT>(), KP = 4 * KE, W = 16 * NT, KBS = KP + 8;
    constexpr int kBytes = kM == 0 ? KP * S * 4 : W * KBS * 2 * kM;   // one B chunk (kM planes)
    __shared__ __align__(16) unsigned char Braw[2 * kBytes];   // B chunks (two for direct)
    __shared__ int pms[8 * 128];                      // perm_o (N <= 128)
    __shared__ float zs[256];                         // Z and W = K Z of the stage
    __shared__ int qs[4 * TPW * 8 * 16];              // transfers of the block's (tile, o, row)
    __shared__ int msk[4 * TPW];                      // operation sets of the block's tiles
    const int gsize = 8 * bx * nchunk;
    const int id = blockIdx.x;
    const int gw = (id / (8 * gsize)) * 8 + id % 8;
    if (gw >= ngw) return;                            // padding of the last 8 work groups
    const int m = (id % (8 * gsize)) / 8;
    const int chunk = m % nchunk;
    const int x = (m / nchunk) % bx;
    const int i = m / (nchunk * bx);
    const int G = gw % g.nG;
    const int ch = (gw / g.nG) % 3;
    const int f = gw / (g.nG * 3);
    const int p = g.porder[8 * G + i];                // loaded with the flow's status
    if (!running(fs, f) || !args.on[ch]) return;      // uniform over the block
    if (p < 0) return;                                // padding of the last patch group
    const int cc = ch == 0 ? 0 : 1;
    const int nt = g.orb_nt[cc];
    const int tb = x * 4 * TPW;
    if (tb >= nt) return;                             // past this kind's tiles
    const int N = g.N, NN = g.NN;
    const int M = ch == 0 ? g.nP : g.nD;
    const int nR = g.nRp + g.nRd;
    const int fb = bin_flow(fs, f);
    const float* Bf = ch == 1 ? binsT + static_cast<size_t>(fb) * g.nRd * NN
                              : bins + static_cast<size_t>(fb) * nR * NN + (ch == 0 ? 0 : static_cast<size_t>(g.nRp) * NN);
    const float al = static_cast<float>(zw[2 * f]), be = static_cast<float>(zw[2 * f + 1]);
    const size_t N3 = static_cast<size_t>(NN) * N;
    const size_t yoff = static_cast<size_t>(f) * M * NN;
    const int toff = cc == 0 ? 0 : g.orb_nt[0];
    using YT = typename YStore<kM>::T;
    if (ch == 2)
        y_orbit_block<kM, KE, NT, TPW, true>(g, Bf, args.Vs[2] + f * N3, args.Vs[3] + f * N3,
                                             reinterpret_cast<YT*>(args.Y[2]) + yoff,
                                             reinterpret_cast<YT*>(args.Y[3]) + yoff, p, tb, nt,
                                             toff, chunk * 16 * NT, al, be,
                                             Z_stage + static_cast<size_t>(f) * 2 * N, Braw, pms, zs, qs,
                                             msk);
    else
        y_orbit_block<kM, KE, NT, TPW, false>(g, Bf, args.Vs[ch] + f * N3, args.Vs[ch] + f * N3,
                                              reinterpret_cast<YT*>(args.Y[ch]) + yoff,
                                              reinterpret_cast<YT*>(args.Y[ch]) + yoff, p, tb, nt,
                                              toff, chunk * 16 * NT, al, be,
                                              Z_stage + static_cast<size_t>(f) * 2 * N, Braw, pms, zs,
                                              qs, msk);
}

// Orbit kernel for point-group-invariant states with bf16 products: only operation 0 yields
// products (the representatives' own), so B'_0 of a (flow, channel, bin row p, column chunk)
// serves every representative tile.  A 1024-thread block takes one (channel, p) of one flow,
// or of two flows that read the same bins (flows of a step-sharing group sit at the same
// stage temperatures).  Its 16 waves take the tiles, wave w tiles w, w + 16 and w + 32 (then
// w + 48, ...: at N = 128 the 34 tiles of a class are one run, staged once per chunk and
// flow); the tiles' A rows (row p of the 16 representatives' bins) are loaded once and kept
// in registers for every chunk, every flow of the block and the direct channel's second
// product.  For each column chunk and flow all threads stage that
// flow's B'_0, into one of two LDS buffers while the other one's products are formed.
// Products and stores are the orbit kernel's for operation 0.
// Grid: one block per unit u = (flow * 3 + channel) N + p.  The running flows that share a
// flow's bins are taken in pairs in index order; the block of a pair's second flow returns.
constexpr int kSymThreads = 1024;

template <int kM, int KE, int NT>
__device__ inline void mfma_bt(const AFrag<kM, KE>& A, const __bf16* Bh, fm_f4 (&c)[NT], int lane);

// One flow's operands and outputs in a symmetric phase-2a block.
struct SymFlow {
    const float* V0;     // operand slab base (the direct channel's first)
    const float* V1;     // the direct channel's second operand (else = V0)
    __bf16* Y0;          // products of the representatives
    __bf16* Y1;          // the direct channel's second products (else = Y0)
    const double* Z;     // the flow's Z at the stage nodes, 2N values
    float al, be;        // stage weights of the two Z factors
};

template <int KE, int NT, bool kTwo>
__device__ inline void y_orb_sym_block(const DevGeom& g, const float* Bf, SymFlow F0,
                                       SymFlow F1, int nfl, int p, int nt, int toff,
                                       int nchunk, unsigned char* Braw, int* pm0, float* zs) {
    constexpr int kM = 1, KBS = 4 * KE + 8, W = 16 * NT;
    constexpr int kBytes = W * KBS * 2;
    constexpr int kWaves = kSymThreads / 64;
    constexpr int kTiles = 3;                          // tiles per wave in a run of tiles
    const int N = g.N, NN = g.NN;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int col = lane & 15;
    if (static_cast<int>(threadIdx.x) < N) {
        pm0[threadIdx.x] = g.perm[threadIdx.x];
        zs[threadIdx.x] = static_cast<float>(F0.Z[threadIdx.x]);
        zs[N + threadIdx.x] = static_cast<float>(F0.Z[N + threadIdx.x]);
        if (nfl > 1) {
            zs[256 + threadIdx.x] = static_cast<float>(F1.Z[threadIdx.x]);
            zs[256 + N + threadIdx.x] = static_cast<float>(F1.Z[N + threadIdx.x]);
        }
    }
    __syncthreads();                                   // tables; every thread of the block
    const int grp = pm0[p];
    auto arow = [&](int t) {                           // row p of the bins of tile t's row col
        const int rr = g.orb_rows[16 * (toff + min(t, nt - 1)) + col];
        return Bf + static_cast<size_t>(max(rr, 0)) * NN + static_cast<size_t>(p) * N;
    };
    // steps i = ((tile run) nchunk + chunk) nfl + flow; step i's B'_0 sits in buffer i & 1 and
    // step i + 1's is staged into the other one while step i is multiplied, so one barrier
    // per step separates a buffer's staging from its use and its use from its next staging
    const int nsteps = (nt + kTiles * kWaves - 1) / (kTiles * kWaves) * nchunk * nfl;
    auto stage = [&](int i) {
        const int fl = i % nfl, n0 = (i / nfl) % nchunk * W;
        const float* V0 = fl ? F1.V0 : F0.V0;
        const float* V1 = fl ? F1.V1 : F0.V1;
        const float al = fl ? F1.al : F0.al, be = fl ? F1.be : F0.be;
        const float* zf = zs + (fl ? 256 : 0);
        stage_orbit_b<kM, KE, NT, kTwo, kSymThreads>(Braw + (i & 1) * 2 * kBytes,
                                                     V0 + static_cast<size_t>(grp) * NN,
                                                     V1 + static_cast<size_t>(grp) * NN, pm0, zf,
                                                     zf[grp], zf[N + grp], al, be, N, n0);
    };
    AFrag<kM, KE> A[kTiles];
    if (nsteps > 0) stage(0);
    for (int i = 0; i < nsteps; ++i) {                 // uniform over the block
        const int fl = i % nfl, chunk = (i / nfl) % nchunk;
        const int t0 = i / (nfl * nchunk) * kTiles * kWaves + wv;
        const int n0 = chunk * W;
        if (chunk == 0 && fl == 0) {                   // the tiles' A rows, for every chunk and flow
#pragma unroll
            for (int j = 0; j < kTiles; ++j) {
                if (t0 + j * kWaves >= nt) break;      // uniform over the wave
                float a[KE];
                gather_a<kM, KE>(a, arow(t0 + j * kWaves), N, lane);
                A[j] = make_afrag<kM, KE>(a);
            }
        }
        __syncthreads();                               // step i staged; step i - 1's buffer free
        if (i + 1 < nsteps) stage(i + 1);
        __bf16* Y0 = fl ? F1.Y0 : F0.Y0;
        __bf16* Y1 = fl ? F1.Y1 : F0.Y1;
        const unsigned char* Bi = Braw + (i & 1) * 2 * kBytes;
#pragma unroll
        for (int w = 0; w < (kTwo ? 2 : 1); ++w) {
            const __bf16* Bw = reinterpret_cast<const __bf16*>(Bi + w * kBytes);
            __bf16* Yw = w ? Y1 : Y0;
#pragma unroll
            for (int j = 0; j < kTiles; ++j) {
                const int t = t0 + j * kWaves;
                if (t >= nt) continue;
                if (!(g.orb_mask[toff + t] & 1)) continue;
                const int q = g.orb_q[static_cast<size_t>(toff + t) * 128 + col];   // operation 0
                fm_f4 c[NT];
#pragma unroll
                for (int u = 0; u < NT; ++u) c[u] = fm_f4{0.f, 0.f, 0.f, 0.f};
                mfma_bt<kM, KE, NT>(A[j], Bw, c, lane);
                if (q >= 0) {
                    __bf16* yrow = Yw + static_cast<size_t>(q) * NN + static_cast<size_t>(grp) * N;
#pragma unroll
                    for (int u = 0; u < NT; ++u) {
                        const int n = n0 + 16 * u + 4 * (lane >> 4);
                        if ((N & 3) == 0) {
                            if (n < N) *reinterpret_cast<fm_bf4*>(yrow + n) = __builtin_convertvector(c[u], fm_bf4);
                        } else {
#pragma unroll
                            for (int r = 0; r < 4; ++r)
                                if (n + r < N) yrow[n + r] = static_cast<__bf16>(c[u][r]);
                        }
                    }
                }
            }
        }
    }
}

template <int KE, int NT>
__global__ void __launch_bounds__(kSymThreads) k_y_orb_sym(DevGeom g, const FlowState* fs,
                                                           const double* Z_stage, const double* zw,
                                                           const float* bins, const float* binsT,
                                                           YArgs<float> args, int nchunk, int nu) {
    constexpr int KBS = 4 * KE + 8, kBytes = 16 * NT * KBS * 2;
    __shared__ __align__(16) unsigned char Braw[2 * 2 * kBytes];   // two buffers of two planes
    __shared__ int pm0[128];
    __shared__ float zs[512];
    const int u = blockIdx.x;
    if (u >= nu) return;
    const int N = g.N, NN = g.NN;
    const int p = u % N, ch = (u / N) % 3, f = u / (3 * N);
    if (!running(fs, f) || !args.on[ch]) return;      // uniform over the block
    const int fb = bin_flow(fs, f);
    // the running flows reading the same bins, in index order, are taken two at a time:
    // this block serves f and the next such flow when f's rank among them is even
    const int nf = nu / (3 * N);
    int rank = 0, f2 = -1;
    for (int k = 0; k < nf; ++k) {                     // uniform over the block
        if (k == f || !running(fs, k) || bin_flow(fs, k) != fb) continue;
        if (k < f) ++rank;
        else if (f2 < 0) f2 = k;
    }
    if (rank & 1) return;                              // the pair's first flow's block serves f
    const int nfl = f2 >= 0 ? 2 : 1;
    const int cc = ch == 0 ? 0 : 1;
    const int nt = g.orb_nt[cc], toff = cc == 0 ? 0 : g.orb_nt[0];
    const int M = ch == 0 ? g.nP : g.nD;
    const int nR = g.nRp + g.nRd;
    const float* Bf = ch == 1 ? binsT + static_cast<size_t>(fb) * g.nRd * NN
                              : bins + static_cast<size_t>(fb) * nR * NN + (ch == 0 ? 0 : static_cast<size_t>(g.nRp) * NN);
    const size_t N3 = static_cast<size_t>(NN) * N;
    auto flow = [&](int h) {
        SymFlow F;
        const size_t yoff = static_cast<size_t>(h) * M * NN;
        F.V0 = args.Vs[ch] + h * N3;
        F.V1 = args.Vs[ch == 2 ? 3 : ch] + h * N3;
        F.Y0 = reinterpret_cast<__bf16*>(args.Y[ch]) + yoff;
        F.Y1 = reinterpret_cast<__bf16*>(args.Y[ch == 2 ? 3 : ch]) + yoff;
        F.Z = Z_stage + static_cast<size_t>(h) * 2 * N;
        F.al = static_cast<float>(zw[2 * h]);
        F.be = static_cast<float>(zw[2 * h + 1]);
        return F;
    };
    const SymFlow F0 = flow(f), F1 = flow(nfl > 1 ? f2 : f);
    if (ch == 2)
        y_orb_sym_block<KE, NT, true>(g, Bf, F0, F1, nfl, p, nt, toff, nchunk, Braw, pm0, zs);
    else
        y_orb_sym_block<KE, NT, false>(g, Bf, F0, F1, nfl, p, nt, toff, nchunk, Braw, pm0, zs);
}

// ------------------------------------------------------------------------------------
// Phase 2b: per transfer q, a small product over the output pairs that use q.
//   kind 0 (pp, pairs (a,b)):     k(a,b,n) -= sum_x V(a,b,x)            Y1[q][x][n]
//   kind 1 (crossed, pairs (b,c)):k(n,b,c) += sum_x V(x,b,c)            Y2[q][x][n]
//   kind 2 (direct, pairs (a,c)): k(a,n,c) += sum_x (V(x,a,c) - 2V(a,x,c)) Y3[q][x][n]
//                                                 + V(a,x,c)             Y4[q][x][n]
// The pairs' vectors are staged in LDS (kChunk at a time, read from the operand layout in
// which they are contiguous); every thread then owns independent (pair, n) outputs, reading
// Y rows coalesced over n.  Every output element receives exactly one contribution per
// channel, stored in that channel's part of the k slot (no atomics).
// ------------------------------------------------------------------------------------
constexpr int kChunk = 8;      // output pairs per work item

template <typename R> struct YGroup;              // rows of Y held in registers per lane
template <> struct YGroup<float> { static constexpr int v = 48; };
template <> struct YGroup<double> { static constexpr int v = 24; };
// the direct channel holds two Y columns, so half as many rows each

// CW consecutive columns of a Y row at p (CW = 2 or 4: one bf16 or f32 vector load, p
// CW-aligned), widened to R.
template <typename R, typename YT, int CW>
__device__ inline void load_cols(const YT* p, R* out) {
    if constexpr (CW == 1) {
        out[0] = static_cast<R>(p[0]);
    } else {
        typedef YT ytn __attribute__((ext_vector_type(CW)));
        const ytn v = *reinterpret_cast<const ytn*>(p);
#pragma unroll
        for (int c = 0; c < CW; ++c) out[c] = static_cast<R>(v[c]);
    }
}

// One wave per work item (kind, q, first pair, count <= kChunk), with KC = 4 accumulators per
// column for items of at most four pairs and KC = kChunk otherwise.  Each lane owns CW
// consecutive free indices n (CW = 2 for single precision and even N > 64: one wider load per
// Y row, and each pair value read from LDS serves two columns; at N = 128 with bf16 products
// 2.63 -> 1.90 ms for 16 flows): its columns of Y (a group of
// rows at a time) are loaded into registers while the item's pair vectors are gathered into
// LDS (zero-padded to KC, laid out [x][pair] so one x is a 128-bit broadcast read), so
// every group costs one memory round trip.
// pm (symmetric states, item transfer q = o(r), o != 0): perm_o.  Y_q[x][n] = Y_r[pinv_o x]
// [pinv_o n], so the item reads representative r's rows x' in order with the pair vectors
// taken at x = perm_o x', and the lane holding Y_r column n' writes output column perm_o n'.
// XH = 2 (N a multiple of 128, CW = 4): the two half-waves take alternate rows x with the
// same 32 x 4 columns and their sums are added at the end, so one broadcast LDS read of a
// row's pair values feeds 4 columns per lane (LDS bytes per multiply-add halved; with 2
// columns per lane the broadcast reads bound the kernel together with the multiply-adds).
template <typename R, typename YT, int KIND, int CW, int KC, int XH = 1>
__device__ __attribute__((always_inline)) inline void contract_item(
    const DevGeom& g, const R* V, const R* VA, const R* VC, const YT* Ya, const YT* Yb,
    const int* pairs, int cnt, R* vu, R* vw, R* Kf, const int* pm) {
    constexpr int G = (KIND == 2 ? YGroup<R>::v / 2 : YGroup<R>::v) / CW;   // rows per lane
    constexpr int GR = G * XH;                                              // rows per group
    const int N = g.N, NN = g.NN;
    const int lc = XH == 2 ? static_cast<int>(threadIdx.x & 31) : static_cast<int>(threadIdx.x);
    const int h = XH == 2 ? static_cast<int>(threadIdx.x >> 5) : 0;
    // the item's output pairs, read once with the first loads (the stores at the end would
    // otherwise each wait for their pair's load)
    int pr[KC];
#pragma unroll
    for (int i = 0; i < KC; ++i) pr[i] = pairs[min(i, cnt - 1)];
    for (int n0 = 0; n0 < N; n0 += 64 / XH * CW) {
        const int n = min(n0 + CW * lc, N - CW);
        R acc[KC][CW];
#pragma unroll
        for (int i = 0; i < KC; ++i)
#pragma unroll
            for (int c = 0; c < CW; ++c) acc[i][c] = R(0);
        for (int xg = 0; xg < N; xg += GR) {
            R ya[G][CW], yb[KIND == 2 ? G : 1][CW];
#pragma unroll
            for (int j = 0; j < G; ++j) {
                const int x = min(xg + XH * j + h, N - 1);
                load_cols<R, YT, CW>(Ya + static_cast<size_t>(x) * N + n, ya[j]);
                if (KIND == 2) load_cols<R, YT, CW>(Yb + static_cast<size_t>(x) * N + n, yb[j]);
            }
            if (n0 == 0 && xg == 0) {
                // gather the pair vectors while the first Y rows are in flight (KC * 128
                // values per round, kVec per lane, loaded to registers before any store; one
                // round for N <= 128)
                constexpr int kVec = KC * 128 / 64;
                for (int e0 = 0; e0 < KC * N; e0 += 64 * kVec) {
                R av[kVec], bv[kVec];
#pragma unroll
                for (int v = 0; v < kVec; ++v) {
                    const int e = min(e0 + static_cast<int>(threadIdx.x) + 64 * v, KC * N - 1);
                    const int i = e / N, xr = e - i * N;
                    const int x = pm ? pm[xr] : xr;
                    const int xy = pairs[min(i, cnt - 1)];
                    const int u = xy / N, w = xy - u * N;
                    // contiguous in x: V(u,w,x) = v0[u][w][x], V(x,u,w) = vc[w][u][x],
                    // V(u,x,w) = va[w][u][x]
                    const size_t ia = KIND == 0 ? static_cast<size_t>(xy) * N + x
                                                : static_cast<size_t>(w) * NN + u * N + x;
                    av[v] = KIND == 0 ? V[ia] : VC[ia];
                    bv[v] = KIND == 2 ? VA[ia] : R(0);
                }
#pragma unroll
                for (int v = 0; v < kVec; ++v) {
                    const int e = e0 + threadIdx.x + 64 * v;
                    const int ec = min(e, KC * N - 1);
                    const int i = ec / N, x = ec - i * N;
                    const bool ok = e < KC * N;
                    const bool live = i < cnt;          // padding pairs contribute zero
                    const R a = live ? av[v] : R(0), b = live ? bv[v] : R(0);
                    if (ok) {
                        if (KIND == 2) {
                            vu[x * KC + i] = a - R(2) * b;
                            vw[x * KC + i] = b;
                        } else {
                            vu[x * KC + i] = a;
                        }
                    }
                }
                }
                __syncthreads();
            }
            // rows past N repeat row N-1 (clamped loads) and are weighted by zero; a group
            // wholly below N needs no weights
            if (xg + GR <= N) {
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    const R* u = vu + (xg + XH * j + h) * KC;
#pragma unroll
                    for (int i = 0; i < KC; ++i)
#pragma unroll
                        for (int c = 0; c < CW; ++c) acc[i][c] += u[i] * ya[j][c];
                    if (KIND == 2) {
                        const R* w = vw + (xg + XH * j + h) * KC;
#pragma unroll
                        for (int i = 0; i < KC; ++i)
#pragma unroll
                            for (int c = 0; c < CW; ++c) acc[i][c] += w[i] * yb[j][c];
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < G; ++j) {
                    const int x = min(xg + XH * j + h, N - 1);
                    const R mask = xg + XH * j + h < N ? R(1) : R(0);
                    const R* u = vu + x * KC;
#pragma unroll
                    for (int i = 0; i < KC; ++i)
#pragma unroll
                        for (int c = 0; c < CW; ++c) acc[i][c] += u[i] * (mask * ya[j][c]);
                    if (KIND == 2) {
                        const R* w = vw + x * KC;
#pragma unroll
                        for (int i = 0; i < KC; ++i)
#pragma unroll
                            for (int c = 0; c < CW; ++c) acc[i][c] += w[i] * (mask * yb[j][c]);
                    }
                }
            }
        }
        if constexpr (XH == 2) {
            // the two halves' sums over alternate rows
#pragma unroll
            for (int i = 0; i < KC; ++i)
#pragma unroll
                for (int c = 0; c < CW; ++c) acc[i][c] += __shfl_xor(acc[i][c], 32);
            if (h) continue;
        }
        if (n0 + CW * lc >= N) continue;
        int col[CW];
#pragma unroll
        for (int c = 0; c < CW; ++c) col[c] = pm ? pm[n + c] : n + c;
#pragma unroll
        for (int i = 0; i < KC; ++i) {   // every part at (pair) N + n: contiguous in n
            if (i >= cnt) break;
#pragma unroll
            for (int c = 0; c < CW; ++c)
                Kf[static_cast<size_t>(pr[i]) * N + col[c]] = KIND == 0 ? -acc[i][c] : acc[i][c];
        }
    }
}

template <typename R, typename YT>
__global__ void __launch_bounds__(64) k_contract(DevGeom g, const FlowState* fs,
                                                 const R* v0, const R* va, const R* vc,
                                                 const YT* y1, const YT* y2, const YT* y3,
                                                 const YT* y4, R* K, unsigned ch, int slot,
                                                 int B) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int f = blockIdx.y;
    if (!running(fs, f)) return;
    const int it = blockIdx.x;
    const int kind = it < g.n_items[0] ? 0 : (it < g.n_items[0] + g.n_items[1] ? 1 : 2);
    // one record per item (uniform address: scalar loads): transfer, count, pairs
    const int* rec = g.item_rec + static_cast<size_t>(it) * 16;
    const int q = rec[0];
    const int cnt = rec[1];
    const int* pairs = rec + 4;
    const int nq = kind == 0 ? g.nP : g.nD;
    const int N = g.N, NN = g.NN;
    const size_t N3 = static_cast<size_t>(NN) * N;
    // k slot part of this channel: [slot][flow][channel][N^3]
    R* Kf = K + ((static_cast<size_t>(slot) * B + f) * 3 + kind) * N3;
    const unsigned bit = kind == 0 ? FM_CH_PP : (kind == 1 ? FM_CH_CR : FM_CH_D);
    if (!(ch & bit)) {   // a channel that is switched off contributes zero
        for (int e = threadIdx.x; e < cnt * N; e += blockDim.x) {
            const int i = e / N, n = e - i * N;
            Kf[static_cast<size_t>(pairs[i]) * N + n] = R(0);
        }
        return;
    }
    const R* V = v0 + f * N3;
    const R* VA = va + f * N3;
    const R* VC = vc + f * N3;
    // symmetric states: the products of the transfer's representative, through perm_o
    int qy = q;
    const int* pm = nullptr;
    if (g.sym) {
        qy = (kind == 0 ? g.qrep_pp : g.qrep_ph)[q];
        const int o = (kind == 0 ? g.qg_pp : g.qg_ph)[q];
        if (o != 0) pm = g.perm + o * N;
    }
    const YT* Ya = (kind == 0 ? y1 : (kind == 1 ? y2 : y3)) + (static_cast<size_t>(f) * nq + qy) * NN;
    const YT* Yb = y4 + (static_cast<size_t>(f) * nq + qy) * NN;
    R* vu = reinterpret_cast<R*>(smem_raw);            // [N][kChunk]
    R* vw = vu + kChunk * N;                            // [N][kChunk] (direct only)
    // two columns per lane where one per lane would take more than one pass over the row
    // (N > 64; at N = 48 two per lane leave 40 of 64 lanes idle: 11.6 -> 13.5 us measured)
    // items of at most four pairs (most transfers have four) carry four accumulators per
    // column instead of eight, half of them padding
    if (sizeof(R) == 4 && N % 128 == 0) {
        if (cnt <= 4) {
            if (kind == 0) contract_item<R, YT, 0, 4, 4, 2>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
            else if (kind == 1) contract_item<R, YT, 1, 4, 4, 2>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
            else contract_item<R, YT, 2, 4, 4, 2>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
            return;
        }
        if (kind == 0) contract_item<R, YT, 0, 4, kChunk, 2>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
        else if (kind == 1) contract_item<R, YT, 1, 4, kChunk, 2>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
        else contract_item<R, YT, 2, 4, kChunk, 2>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
        return;
    }
    if (sizeof(R) == 4 && (N & 1) == 0 && N > 64) {
        if (cnt <= 4) {
            if (kind == 0) contract_item<R, YT, 0, 2, 4>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
            else if (kind == 1) contract_item<R, YT, 1, 2, 4>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
            else contract_item<R, YT, 2, 2, 4>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
            return;
        }
        if (kind == 0) contract_item<R, YT, 0, 2, kChunk>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
        else if (kind == 1) contract_item<R, YT, 1, 2, kChunk>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
        else contract_item<R, YT, 2, 2, kChunk>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
        return;
    }
    if (cnt <= 4) {
        if (kind == 0) contract_item<R, YT, 0, 1, 4>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
        else if (kind == 1) contract_item<R, YT, 1, 1, 4>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
        else contract_item<R, YT, 2, 1, 4>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
        return;
    }
    if (kind == 0) contract_item<R, YT, 0, 1, kChunk>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
    else if (kind == 1) contract_item<R, YT, 1, 1, kChunk>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
    else contract_item<R, YT, 2, 1, kChunk>(g, V, VA, VC, Ya, Yb, pairs, cnt, vu, vw, Kf, pm);
}

// ------------------------------------------------------------------------------------
// Phase 2b of symmetric states on the matrix cores (bf16 products, N <= 128, N % 16 == 0).
// One 4-wavefront block per (channel kind, representative r, at most kSymPairs output pairs
// of the transfers q = o(r) of r's orbit) and flow.  Every such transfer's products are r's,
// Y_q[x][n] = Y_r[pinv_o x][pinv_o n], so for a pair of transfer o(r)
//   out(pair, perm_o n') = sum_x' L(pair, perm_o x') Y_r[x'][n']
// (L the pair's vector of its channel, as in k_contract): one product of the pairs' vectors,
// gathered at perm_o x' and split into bf16 high and low parts (two products: the vectors
// keep f32 accuracy), with Y_r as stored (bf16), which the block stages once in LDS in the
// B operand layout [n'][x'] and shares between its four 16-pair tiles.  The direct channel
// adds a second product, (V(x,a,c) - 2 V(a,x,c)) Y3 + V(a,x,c) Y4.  A lane ends with four
// consecutive n' of its tile row (the staged operand goes first) and writes them to columns
// perm_o n'.
// ------------------------------------------------------------------------------------
constexpr int kMmaKE = 32;                        // k values per lane: x' < 128
constexpr int kMmaKBS = 4 * kMmaKE + 8;           // staged row stride (bf16 values)

// YT = __bf16: bf16 products as stored, all of an item's products staged at once.  YT = float
// (split-bf16 products): each product staged as high and low bf16 planes, one product per
// pass, three products per k-step (the low-by-low term dropped, as in phase 2a's split mode).
// TWO: the launch of the direct channel's items (two products); the pp and crossed items'
// launch holds no second operand (fewer registers, more blocks per CU).
template <typename YT, bool TWO>
__global__ void __launch_bounds__(256) k_contract_mma(DevGeom g, const FlowState* fs,
                                                      const float* v0, const float* va,
                                                      const float* vc, const YT* y1,
                                                      const YT* y2, const YT* y3,
                                                      const YT* y4, float* K, unsigned ch,
                                                      int slot, int B, int it0) {
    constexpr int KE = kMmaKE, KBS = kMmaKBS, PLANE = 128 * kMmaKBS;
    constexpr bool kSplit = sizeof(YT) == 4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // [1 or 2][128][KBS]: Y_r^T (and Y4_r^T), or the high and low planes of one product
    __bf16* Bs = reinterpret_cast<__bf16*>(smem_raw);
    const int f = blockIdx.y;
    if (!running(fs, f)) return;
    const int* rec = g.sym_rec + static_cast<size_t>(blockIdx.x + it0) * (kSymPairs + 4);
    const int r = rec[0], cnt = rec[1], kind = rec[2];
    const int* ent = rec + 4;
    const int N = g.N, NN = g.NN;
    const size_t N3 = static_cast<size_t>(NN) * N;
    float* Kf = K + ((static_cast<size_t>(slot) * B + f) * 3 + kind) * N3;
    const unsigned bit = kind == 0 ? FM_CH_PP : (kind == 1 ? FM_CH_CR : FM_CH_D);
    if (!(ch & bit)) {   // a channel that is switched off contributes zero
        for (int e = threadIdx.x; e < cnt * N; e += blockDim.x) {
            const int i = e / N, n = e - i * N;
            Kf[static_cast<size_t>(ent[i] >> 3) * N + n] = 0.f;
        }
        return;
    }
    // perm_o of every operation in LDS (a wave's pairs may belong to different operations),
    // operation 0 as the identity
    __shared__ int pms[8 * 128];
    {
        int pv[4];                                     // loads first (valid addresses), then stores
#pragma unroll
        for (int v = 0; v < 4; ++v) pv[v] = g.perm[min(static_cast<int>(threadIdx.x) + 256 * v, 8 * N - 1)];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = threadIdx.x + 256 * v;
            if (i < 8 * N) pms[i] = i < N ? i : pv[v];
        }
    }
    const int nq = kind == 0 ? g.nP : g.nD;
    const YT* Ya = (kind == 0 ? y1 : (kind == 1 ? y2 : y3)) + (static_cast<size_t>(f) * nq + r) * NN;
    const YT* Yb = y4 + (static_cast<size_t>(f) * nq + r) * NN;
    // stage Y_r^T: a task is 8 consecutive n' of one row x' (16-byte loads), written as 8
    // values down the staged columns (consecutive lanes, consecutive x'); zero past N
    // (N % 16 == 0: a task lies wholly below N or at or above it)
    auto stage = [&](const YT* Y0, const YT* Y1, bool both) {
#pragma unroll
        for (int task = threadIdx.x; task < 128 * (128 / 8); task += 256) {   // 8 rounds
            const int x = task & 127, nb = 8 * (task >> 7);
            const bool ok = x < N && nb < N;
            const size_t ix = static_cast<size_t>(min(x, N - 1)) * N + min(nb, N - 8);
            if constexpr (kSplit) {
                const float4 p0 = *reinterpret_cast<const float4*>(Y0 + ix);
                const float4 p1 = *reinterpret_cast<const float4*>(Y0 + ix + 4);
                const float v[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const __bf16 hi = static_cast<__bf16>(v[e]);
                    const __bf16 lo = static_cast<__bf16>(v[e] - static_cast<float>(hi));
                    Bs[(nb + e) * KBS + x] = ok ? hi : static_cast<__bf16>(0.f);
                    Bs[PLANE + (nb + e) * KBS + x] = ok ? lo : static_cast<__bf16>(0.f);
                }
            } else {
                const fm_bf8 h0 = *reinterpret_cast<const fm_bf8*>(Y0 + ix);
                fm_bf8 h1 = h0;
                if (both) h1 = *reinterpret_cast<const fm_bf8*>(Y1 + ix);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    Bs[(nb + e) * KBS + x] = ok ? h0[e] : static_cast<__bf16>(0.f);
                    if (both) Bs[PLANE + (nb + e) * KBS + x] = ok ? h1[e] : static_cast<__bf16>(0.f);
                }
            }
        }
    };
    // bf16: every task's loads first (8 rounds of 16 bytes per product, valid addresses), then
    // the LDS writes, so the block waits for one memory round trip
    auto stage_bf16 = [&](const YT* Y0, const YT* Y1) {
        constexpr int kR = 128 * (128 / 8) / 256;
        fm_bf8 h0[kR], h1[TWO ? kR : 1];
#pragma unroll
        for (int k = 0; k < kR; ++k) {
            const int task = threadIdx.x + 256 * k, x = task & 127, nb = 8 * (task >> 7);
            const size_t ix = static_cast<size_t>(min(x, N - 1)) * N + min(nb, N - 8);
            h0[k] = *reinterpret_cast<const fm_bf8*>(Y0 + ix);
            if constexpr (TWO) h1[k] = *reinterpret_cast<const fm_bf8*>(Y1 + ix);
        }
#pragma unroll
        for (int k = 0; k < kR; ++k) {
            const int task = threadIdx.x + 256 * k, x = task & 127, nb = 8 * (task >> 7);
            const bool ok = x < N && nb < N;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                Bs[(nb + e) * KBS + x] = ok ? h0[k][e] : static_cast<__bf16>(0.f);
                if constexpr (TWO) Bs[PLANE + (nb + e) * KBS + x] = ok ? h1[k][e] : static_cast<__bf16>(0.f);
            }
        }
    };
    if constexpr (!kSplit) stage_bf16(Ya, Yb);
    else stage(Ya, Ya, false);
    // the wave's tile rows: pairs 16 w .. 16 w + 15 of the record; lane % 16 the row
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));
    const int pi = 16 * wv + (lane & 15);
    const int en = pi < cnt ? ent[pi] : -1;
    const int o = en >= 0 ? (en & 7) : 0, xy = en >= 0 ? (en >> 3) : 0;
    const int u = xy / N, w = xy - u * N;
    // contiguous in x: V(u,w,x) = v0[u][w][x], V(x,u,w) = vc[w][u][x], V(u,x,w) = va[w][u][x]
    const size_t base = static_cast<size_t>(f) * N3 +
                        (kind == 0 ? static_cast<size_t>(xy) * N : static_cast<size_t>(w) * NN + static_cast<size_t>(u) * N);
    const int* pm = pms + o * N;
    __syncthreads();                                   // perm_o in LDS; every thread
    float a1[KE], a2[TWO ? KE : 1];
#pragma unroll
    for (int e = 0; e < KE; ++e) {
        const int xr = mfma_k<1>(e, lane);              // x' of the lane's e-th value
        const bool ok = en >= 0 && xr < N;
        const int x = pm[min(xr, N - 1)];
        // every address is valid (x < N, and a padding lane reads pair 0), so the loads are
        // issued unconditionally and the values selected
        if constexpr (TWO) {
            const float c = vc[base + x], b = va[base + x];
            a1[e] = ok ? c - 2.f * b : 0.f;
            a2[e] = ok ? b : 0.f;
        } else {
            const float c = (kind == 0 ? v0 : vc)[base + x];
            a1[e] = ok ? c : 0.f;
        }
    }
    const AFrag<2, KE> A1 = make_afrag<2, KE>(a1);
    AFrag<2, KE> A2;
    if constexpr (TWO) A2 = make_afrag<2, KE>(a2);
    __syncthreads();                                   // Y_r^T staged; every thread
    const bool active = 16 * wv < cnt;                 // a wave with pairs (uniform)
    const int col = lane & 15;
    // a lane's four consecutive n' go to columns perm_o n'; where those are four consecutive
    // columns starting at a multiple of 4 (ascending, or descending for a reflection) they are
    // one 16-byte store, else four
    auto store = [&](int t, const fm_f4& c) {
        if (en < 0) return;
        const int n = 16 * t + 4 * (lane >> 4);
        const fm_f4 v = kind == 0 ? -c : c;
        const int c0 = pm[n], c3 = pm[n + 3];
        float* row = Kf + static_cast<size_t>(xy) * N;
        if (c3 == c0 + 3 && (c0 & 3) == 0 && pm[n + 1] == c0 + 1 && pm[n + 2] == c0 + 2) {
            *reinterpret_cast<fm_f4*>(row + c0) = v;
        } else if (c0 == c3 + 3 && (c3 & 3) == 0 && pm[n + 1] == c3 + 2 && pm[n + 2] == c3 + 1) {
            *reinterpret_cast<fm_f4*>(row + c3) = fm_f4{v[3], v[2], v[1], v[0]};
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) row[pm[n + q]] = v[q];
        }
    };
    if constexpr (!kSplit) {
        if (!active) return;
        for (int t = 0; t < N / 16; ++t) {
            fm_f4 c = fm_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < KE / 8; ++s) {
                const int ob = (16 * t + col) * KBS + 32 * s + 8 * (lane >> 4);
                const fm_bf8 b3 = *reinterpret_cast<const fm_bf8*>(Bs + ob);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b3, A1.l[s], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b3, A1.h[s], c, 0, 0, 0);
                if constexpr (TWO) {
                    const fm_bf8 b4 = *reinterpret_cast<const fm_bf8*>(Bs + PLANE + ob);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b4, A2.l[s], c, 0, 0, 0);
                    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b4, A2.h[s], c, 0, 0, 0);
                }
            }
            store(t, c);
        }
    } else {
        // every tile's accumulators held across the passes (N <= 128: at most 8 tiles)
        fm_f4 c[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) c[t] = fm_f4{0.f, 0.f, 0.f, 0.f};
        auto products = [&](const AFrag<2, KE>& A) {
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if (t >= N / 16) break;
#pragma unroll
                for (int s = 0; s < KE / 8; ++s) {
                    const int ob = (16 * t + col) * KBS + 32 * s + 8 * (lane >> 4);
                    const fm_bf8 bh = *reinterpret_cast<const fm_bf8*>(Bs + ob);
                    const fm_bf8 bl = *reinterpret_cast<const fm_bf8*>(Bs + PLANE + ob);
                    c[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, A.l[s], c[t], 0, 0, 0);
                    c[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl, A.h[s], c[t], 0, 0, 0);
                    c[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, A.h[s], c[t], 0, 0, 0);
                }
            }
        };
        if (active) products(A1);
        if constexpr (TWO) {
            __syncthreads();                           // the first product is consumed
            stage(Yb, Yb, false);
            __syncthreads();
            if (active) products(A2);
        }
        if (!active) return;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            if (t >= N / 16) break;
            store(t, c[t]);
        }
    }
}

// ------------------------------------------------------------------------------------
// Fused phase 2 (bf16 and split-bf16 operands, N <= 128): the grouped products and the
// contraction they feed in one kernel, so the products never leave registers (no Y buffers).
// A block takes kFusedRows rows of one channel kind, all from transfers q = o(r) of one
// operation o, and one chunk of W = 16 NT output columns n; a row is (q, up to kFusedPairs of
// the output pairs that use q), held by lane % 16 of its wavefront's 16-row tile.  For every
// bin row p of the representatives (slab g = perm_o p):
//   Y_q[g][n] = sum_k' Brep_r(p, k') B'[k'][n],
//   B'[k'][n] = Z_g Z_k (al + be (W_g + W_k)) Vsrc[g][k][n],  k = perm_o k'
// (the products of the operation-class kernel), on the matrix cores with the staged operand
// first, so that a lane holds four consecutive n of its own row; then on the vector units
//   acc[pair][n] += L(pair, g) Y_q[g][n]
// with the pair vectors of phase 2b (V(a,b,g); V(g,b,c); for the direct channel
// V(g,a,c) - 2 V(a,g,c) against the va products plus V(a,g,c) against the vc products).
// After the last p the accumulators are the channel's part of the k slot (-acc for pp).  The
// staged operand is double-buffered (single with split bf16, whose two planes fill the LDS),
// so the next slab's staging overlaps this slab's products; the next bin row and pair values
// are loaded while the current ones are used.
// ------------------------------------------------------------------------------------
template <int kM, int KE, int NT>
__device__ inline void mfma_bt(const AFrag<kM, KE>& A, const __bf16* Bh, fm_f4 (&c)[NT],
                               int lane) {
    constexpr int KBS = 4 * KE + 8, PL = 16 * NT * KBS;
    const int col = lane & 15;
#pragma unroll
    for (int s = 0; s < KE / 8; ++s) {
        const int kb = 32 * s + 8 * (lane >> 4);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int o = (16 * t + col) * KBS + kb;
            const fm_bf8 bh = *reinterpret_cast<const fm_bf8*>(Bh + o);
            if constexpr (kM == 2) {
                const fm_bf8 bl = *reinterpret_cast<const fm_bf8*>(Bh + PL + o);
                c[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl, A.h[s], c[t], 0, 0, 0);
                c[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, A.l[s], c[t], 0, 0, 0);
            }
            c[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh, A.h[s], c[t], 0, 0, 0);
        }
    }
}

template <int kM, int KE, int NT>
__global__ void __launch_bounds__(4 * kFusedRows) k_fused(
        DevGeom g, const FlowState* fs, const double* Z_stage, const double* zw,
        const float* bins, const float* binsT, const float* v0, const float* va,
        const float* vc, float* K, unsigned ch, int slot, int B, int nchunk, int nf) {
    constexpr int kT = 4 * kFusedRows;            // 16 rows per wavefront
    constexpr int KP = 4 * KE;                    // staged k' (zero from N on)
    constexpr int W = 16 * NT;
    constexpr int KBS = KP + 8;
    constexpr int PL = W * KBS;                   // bf16 per plane
    constexpr int kOp = PL * (kM == 2 ? 2 : 1);   // bf16 per staged operand
    constexpr int kBuf = kM == 2 ? 1 : 2;
    constexpr int kTasks = KP / 8 * W;            // staging: 8 consecutive k' of one column
    constexpr int kTPT = (kTasks + kT - 1) / kT;  // staging tasks per thread
    constexpr int kP = kFusedPairs;
    __shared__ __align__(16) __bf16 Bs[kBuf][2][kOp];
    __shared__ float zs[256];                     // Z and W = K Z of the stage
    __shared__ int pms[128];                      // perm_o
    __shared__ float za[128], zb[128];            // fac(g, k') = Z_g (za[k'] + zb[k'] W_g)
    __shared__ int ko[128];                       // k = perm_o k' times N (row of a slab)
    const int N = g.N, NN = g.NN;
    const size_t N3 = static_cast<size_t>(NN) * N;
    // 1D grid.  The blocks that read the same bin rows -- both column chunks, and the two
    // flows of a pair (which share bins when they step together) -- are one work group of
    // M = 2 nchunk members; work groups are dealt to the 8 XCDs round-robin and a group's
    // members get block ids 8 apart, so they run on one XCD at about the same time and read
    // the rows through its L2:
    //   id = (key / 8) 8 M + member 8 + key % 8,  key = (flow / 2) nblk + row block.
    const int nblk = g.fz_nblk[0] + g.fz_nblk[1] + g.fz_nblk[2];
    const int M = 2 * nchunk;
    const int id = blockIdx.x;
    const int key = (id / (8 * M)) * 8 + id % 8;
    const int member = (id % (8 * M)) / 8;
    if (key >= nblk * ((nf + 1) / 2)) return;     // padding of the last 8 work groups
    const int b = key % nblk;
    const int f = 2 * (key / nblk) + member / nchunk;
    const int chunk = member % nchunk;
    if (f >= nf || !running(fs, f)) return;       // uniform over the block
    const int kind = b < g.fz_nblk[0] ? 0 : (b < g.fz_nblk[0] + g.fz_nblk[1] ? 1 : 2);
    const int o = g.fz_blk[2 * b], row0 = g.fz_blk[2 * b + 1];
    const int lane = threadIdx.x & 63;
    const int row = row0 + 16 * static_cast<int>(threadIdx.x >> 6) + (lane & 15);
    const int q = g.fz_row[row];
    int pr[kP];
#pragma unroll
    for (int i = 0; i < kP; ++i) pr[i] = g.fz_pair[row * kP + i];
    const int n0 = chunk * W;
    const int nl = n0 + 4 * (lane >> 4);          // the lane's first n in tile 0
    float* Kf = K + ((static_cast<size_t>(slot) * B + f) * 3 + kind) * N3;
    const unsigned bit = kind == 0 ? FM_CH_PP : (kind == 1 ? FM_CH_CR : FM_CH_D);
    if (!(ch & bit)) {                            // a channel that is off contributes zero
#pragma unroll
        for (int i = 0; i < kP; ++i)
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int n = nl + 16 * t + r;
                    if (pr[i] >= 0 && n < N) Kf[static_cast<size_t>(pr[i]) * N + n] = 0.f;
                }
        return;
    }
    const bool two = kind == 2;                   // uniform over the block
    const int nR = g.nRp + g.nRd;
    const int fb = bin_flow(fs, f);
    const float* Bf = kind == 1 ? binsT + static_cast<size_t>(fb) * g.nRd * NN
                                : bins + static_cast<size_t>(fb) * nR * NN + (kind == 0 ? 0 : static_cast<size_t>(g.nRp) * NN);
    const int rep = q >= 0 ? (kind == 0 ? g.qrep_pp[q] : g.qrep_ph[q]) : 0;
    const float* Arow = Bf + static_cast<size_t>(rep) * NN;
    const float* S0 = (kind == 0 ? v0 : (kind == 1 ? vc : va)) + f * N3;
    const float* S1 = vc + f * N3;
    const float* L0 = (kind == 0 ? v0 : vc) + f * N3;
    const float* L1 = va + f * N3;
    size_t lb[kP];
#pragma unroll
    for (int i = 0; i < kP; ++i) {
        // pair vectors, contiguous in g: V(u,w,g) = v0[u][w][g]; V(g,u,w) = vc[w][u][g],
        // V(u,g,w) = va[w][u][g]
        const int xy = max(pr[i], 0), u = xy / N, w = xy - u * N;
        lb[i] = kind == 0 ? static_cast<size_t>(xy) * N : static_cast<size_t>(w) * NN + static_cast<size_t>(u) * N;
    }
    const double* Zf = Z_stage + static_cast<size_t>(f) * 2 * N;
    for (int k = threadIdx.x; k < 2 * N; k += kT) zs[k] = static_cast<float>(Zf[k]);
    for (int k = threadIdx.x; k < N; k += kT) pms[k] = g.perm[o * N + k];
    const float al = static_cast<float>(zw[2 * f]), be = static_cast<float>(zw[2 * f + 1]);
    __syncthreads();
    // Z_g Z_k (al + be (W_g + W_k)) = Z_g (Z_k (al + be W_k) + be Z_k W_g), k = perm_o k';
    // zero for k' >= N
    for (int kk = threadIdx.x; kk < KP; kk += kT) {
        const int k = pms[min(kk, N - 1)];
        const float zk = zs[k], wk = zs[N + k];
        za[kk] = kk < N ? zk * (al + be * wk) : 0.f;
        zb[kk] = kk < N ? be * zk : 0.f;
        ko[kk] = k * N;
    }
    __syncthreads();

    // B'[k'][n] of slab perm_o p for both operands (the second only for the direct channel),
    // bf16 transposed [n][k'] (split bf16: the low parts in a second plane).  A task is 8
    // consecutive k' of one column n: its 8 loads are coalesced over the wave's columns, and
    // its values go to LDS as one 16-byte store per plane.  The loads of a slab are issued
    // one slab ahead of its stores, so their latency is spent on the current products.
    float sx0[kTPT][8], sx1[kTPT][8];
    auto stage_load = [&](int p) {
        const int gs = pms[p];
        const float* s0 = S0 + static_cast<size_t>(gs) * NN;
        const float* s1 = S1 + static_cast<size_t>(gs) * NN;
#pragma unroll
        for (int j = 0; j < kTPT; ++j) {
            const int task = min(static_cast<int>(threadIdx.x) + j * kT, kTasks - 1);
            const int n = task % W, kb = 8 * (task / W);
            const int nc = min(n0 + n, N - 1);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                sx0[j][i] = s0[ko[kb + i] + nc];
                sx1[j][i] = two ? s1[ko[kb + i] + nc] : 0.f;
            }
        }
    };
    auto stage_store = [&](int p, int buf) {
        const int gs = pms[p];
        const float zg = zs[gs], wg = zs[N + gs];
#pragma unroll
        for (int j = 0; j < kTPT; ++j) {
            const int task = static_cast<int>(threadIdx.x) + j * kT;
            if (task >= kTasks) break;
            const int n = task % W, kb = 8 * (task / W);
            const float nok = n0 + n < N ? zg : 0.f;
            fm_bf8 h0, h1, l0, l1;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const float fac = nok * (za[kb + i] + zb[kb + i] * wg);
                const float y0 = fac * sx0[j][i], y1 = fac * sx1[j][i];
                h0[i] = static_cast<__bf16>(y0);
                h1[i] = static_cast<__bf16>(y1);
                if constexpr (kM == 2) {
                    l0[i] = static_cast<__bf16>(y0 - static_cast<float>(h0[i]));
                    l1[i] = static_cast<__bf16>(y1 - static_cast<float>(h1[i]));
                }
            }
            *reinterpret_cast<fm_bf8*>(&Bs[buf][0][n * KBS + kb]) = h0;
            if constexpr (kM == 2) *reinterpret_cast<fm_bf8*>(&Bs[buf][0][PL + n * KBS + kb]) = l0;
            if (two) {
                *reinterpret_cast<fm_bf8*>(&Bs[buf][1][n * KBS + kb]) = h1;
                if constexpr (kM == 2) *reinterpret_cast<fm_bf8*>(&Bs[buf][1][PL + n * KBS + kb]) = l1;
            }
        }
    };
    // pair values at slab perm_o p (0 for the padding pairs)
    auto load_l = [&](int p, float (&x)[kP], float (&y)[kP]) {
        const int gs = pms[p];
#pragma unroll
        for (int i = 0; i < kP; ++i) {
            x[i] = pr[i] >= 0 ? L0[lb[i] + gs] : 0.f;
            y[i] = (two && pr[i] >= 0) ? L1[lb[i] + gs] : 0.f;
        }
    };

    fm_f4 acc[kP][NT];
#pragma unroll
    for (int i = 0; i < kP; ++i)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[i][t] = fm_f4{0.f, 0.f, 0.f, 0.f};
    float a[KE], lc[kP], wc[kP];
    stage_load(0);
    stage_store(0, 0);
    if (N > 1) stage_load(1);
    gather_a<kM, KE>(a, Arow, N, lane);
    load_l(0, lc, wc);
    __syncthreads();                              // slab 0 staged; every thread
    for (int p = 0; p < N; ++p) {
        const int cur = kBuf == 2 ? (p & 1) : 0;
        if constexpr (kBuf == 2) {
            if (p + 1 < N) stage_store(p + 1, cur ^ 1);   // loaded during the last slab
            if (p + 2 < N) stage_load(p + 2);
        } else {
            if (p + 1 < N && p > 0) stage_load(p + 1);
        }
        const AFrag<kM, KE> A = make_afrag<kM, KE>(a);
        float ln[kP], wn[kP];
        if (p + 1 < N) {
            gather_a<kM, KE>(a, Arow + static_cast<size_t>(p + 1) * N, N, lane);
            load_l(p + 1, ln, wn);
        }
        {
            fm_f4 c[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) c[t] = fm_f4{0.f, 0.f, 0.f, 0.f};
            mfma_bt<kM, KE, NT>(A, Bs[cur][0], c, lane);
#pragma unroll
            for (int i = 0; i < kP; ++i) {
                const float s = two ? lc[i] - 2.f * wc[i] : lc[i];
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[i][t] += s * c[t];
            }
        }
        if (two) {
            fm_f4 c[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) c[t] = fm_f4{0.f, 0.f, 0.f, 0.f};
            mfma_bt<kM, KE, NT>(A, Bs[cur][1], c, lane);
#pragma unroll
            for (int i = 0; i < kP; ++i)
#pragma unroll
                for (int t = 0; t < NT; ++t) acc[i][t] += wc[i] * c[t];
        }
        if (p + 1 < N) {
#pragma unroll
            for (int i = 0; i < kP; ++i) { lc[i] = ln[i]; wc[i] = wn[i]; }
        }
        if constexpr (kBuf == 1) {
            if (p + 1 < N) {
                __syncthreads();                  // every wave is done with the buffer
                stage_store(p + 1, 0);
            }
        }
        __syncthreads();                          // next slab staged; every thread
    }
    const float sg = kind == 0 ? -1.f : 1.f;
#pragma unroll
    for (int i = 0; i < kP; ++i) {
        if (pr[i] < 0) continue;
        float* dst = Kf + static_cast<size_t>(pr[i]) * N;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = nl + 16 * t + r;
                if (n < N) dst[n] = sg * acc[i][t][r];
            }
    }
}

// ------------------------------------------------------------------------------------
// Direct double-precision path.
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_wtable(DevGeom g, const FlowState* fs,
                                                     const double* T_stage,
                                                     const double* Z_stage, const double* zw,
                                                     double* W) {
    const int f = blockIdx.z;
    if (!running(fs, f)) return;
    const int q = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.np) return;
    const bool pp = q < g.nP;
    const int m = pp ? g.q_pp[q] : g.q_ph[q - g.nP];
    const int jp = pp ? partner_pp(m, j, g.L) : partner_ph(m, j, g.L);
    const double T = T_stage[f];
    double w;
    if (g.gflow) {
        w = pair_chi(g.xi[j], g.xi[jp], 2.0 * T, pp) / (4.0 * T * g.np);
    } else {
        const double a = g.xi[j] / (2.0 * T);
        double b = g.xi[jp] / (2.0 * T);
        if (pp) b = -b;
        w = -phi_dd<double>(a, phi_d(a), b, phi_d(b)) / (4.0 * T * g.np);
    }
    const double* Z = Z_stage + static_cast<size_t>(f) * 2 * g.N;
    const double za = Z[g.patch[j]], zb = Z[g.patch[jp]];
    const double wa = Z[g.N + g.patch[j]], wb = Z[g.N + g.patch[jp]];
    W[(static_cast<size_t>(f) * (g.nP + g.nD) + q) * g.np + j] =
        za * zb * (zw[2 * f] + zw[2 * f + 1] * (wa + wb)) * w;
}

__global__ void __launch_bounds__(kThreads) k_direct(DevGeom g, const FlowState* fs,
                                                     const double* W, const double* v0,
                                                     double* K, unsigned ch) {
    const int f = blockIdx.y;
    if (!running(fs, f)) return;
    const int N = g.N, NN = g.NN, L = g.L, np = g.np;
    const int a = blockIdx.x / N, b = blockIdx.x - (blockIdx.x / N) * N;
    const size_t N3 = static_cast<size_t>(NN) * N;
    for (int c = threadIdx.x; c < N; c += blockDim.x) {
    const double* V = v0 + f * N3;
    const double* Wf = W + static_cast<size_t>(f) * (g.nP + g.nD) * np;
    const int q1 = g.map_pp[a * N + b], q2 = g.map_cr[b * N + c], q3 = g.map_d[a * N + c];
    const int m1 = g.q_pp[q1], m2 = g.q_ph[q2], m3 = g.q_ph[q3];
    const double* W1 = Wf + static_cast<size_t>(q1) * np;
    const double* W2 = Wf + static_cast<size_t>(g.nP + q2) * np;
    const double* W3 = Wf + static_cast<size_t>(g.nP + q3) * np;
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int j = 0; j < np; ++j) {
        const int pj = g.patch[j];
        if (ch & FM_CH_PP) {
            const int pq = g.patch[partner_pp(m1, j, L)];
            s1 += W1[j] * V[static_cast<size_t>(a) * NN + b * N + pj] * V[static_cast<size_t>(pj) * NN + pq * N + c];
        }
        if (ch & FM_CH_CR) {
            const int pq = g.patch[partner_ph(m2, j, L)];
            s2 += W2[j] * V[static_cast<size_t>(a) * NN + pj * N + pq] * V[static_cast<size_t>(pq) * NN + b * N + c];
        }
        if (ch & FM_CH_D) {
            const int pq = g.patch[partner_ph(m3, j, L)];
            const double vajc = V[static_cast<size_t>(a) * NN + pj * N + c];
            s3 += W3[j] * (-2.0 * vajc * V[static_cast<size_t>(pq) * NN + b * N + pj]
                           + V[static_cast<size_t>(pj) * NN + a * N + c] * V[static_cast<size_t>(pq) * NN + b * N + pj]
                           + vajc * V[static_cast<size_t>(b) * NN + pq * N + pj]);
        }
    }
    double* Kf = K + f * 3 * N3;                       // slot parts, phase-2b order
    Kf[kpos(0, N, a, b, c)] = -s1;
    Kf[N3 + kpos(1, N, a, b, c)] = s2;
    Kf[2 * N3 + kpos(2, N, a, b, c)] = s3;
    }
}

// ------------------------------------------------------------------------------------
// Integrator kernels (double precision).
// ------------------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(kThreads) k_to_f64(const FlowState* fs, const R* K, double* out,
                                                     int N) {
    const int f = blockIdx.y;
    if (!running(fs, f)) return;
    const size_t N3 = static_cast<size_t>(N) * N * N;
    const double sg = fs[f].gflow ? -1.0 : 1.0;
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < N3;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const int x = static_cast<int>(i / (static_cast<size_t>(N) * N));
        const int y = static_cast<int>((i / N) % N), z = static_cast<int>(i % N);
        out[f * N3 + i] = sg * static_cast<double>(kval_at(K, 0, 0, f, N3, N, x, y, z));
    }
}

__global__ void __launch_bounds__(kThreads) k_fill_u(double* V, const double* U, size_t N3) {
    const int f = blockIdx.y;
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < N3;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        V[f * N3 + i] = U[f];
}

__device__ inline double block_max(double v) {
    __shared__ double red[1024 / 64];
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = red[0];
        for (int i = 1; i < static_cast<int>(blockDim.x / 64); ++i) r = fmax(r, red[i]);
        red[0] = r;
    }
    __syncthreads();
    const double r = red[0];
    __syncthreads();
    return r;
}

// V += h/6 (k0 + 2 k1 + 2 k2 + k3); partial max|V| (inf if non-finite).
template <typename R>
__global__ void __launch_bounds__(kStepThreads) k_rk4_update(const FlowState* fs, const R* K,
                                                             const R* KS, double* V,
                                                             double* part, int nblk, int N,
                                                             int B) {
    __shared__ double p1[stage_tile_lds(3)], p2[stage_tile_lds(3)];
    const int f = blockIdx.y;
    if (!running(fs, f)) return;
    const double h = fs[f].ht;
    const size_t N3 = static_cast<size_t>(N) * N * N;
    const size_t ks = static_cast<size_t>(B) * N3;
    const R* K3 = K + ((3 * static_cast<size_t>(B) + f) * 3) * N3;   // slot 3 (parts)
    const R* KSf = KS + static_cast<size_t>(f) * N3;                 // sums of slots 0..2
    constexpr int tsx = 8 * kTSY + 1, tile_n = kTZ * 64, EPT = tile_n / kStepThreads;
    double mx = 0.0;
    const int ntile = stage_tiles(N, 3);
    for (int t = blockIdx.x; t < ntile; t += gridDim.x) {   // uniform over the block
        int x0, y0, z0;
        tile_origin(t, N, 3, x0, y0, z0);
        // this thread's slot sums, slot-3 pp parts and V first (in registers across the barrier)
        R kv[EPT][4];
        double vo[EPT];
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            const int e = threadIdx.x + r * kStepThreads;
            const int lz = e & (kTZ - 1), ly = (e >> 4) & 7, lx = e >> 7;
            const int x = x0 + lx, y = y0 + ly, zz = z0 + lz;
            const size_t i =
                x < N && y < N && zz < N ? (static_cast<size_t>(x) * N + y) * N + zz : 0;
#pragma unroll
            for (int l = 0; l < 3; ++l) kv[r][l] = KSf[l * ks + i];
            kv[r][3] = K3[i];
            vo[r] = V[f * N3 + i];
        }
        tile_parts<3>(K3, N3, N, x0, y0, z0, p1, p2);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            const int e = threadIdx.x + r * kStepThreads;
            const int lz = e & (kTZ - 1), ly = (e >> 4) & 7, lx = e >> 7;
            const int x = x0 + lx, y = y0 + ly, zz = z0 + lz;
            if (x >= N || y >= N || zz >= N) continue;
            const size_t i = (static_cast<size_t>(x) * N + y) * N + zz;
            const int j = lx * tsx + ly * kTSY + lz;
            const double k0 = static_cast<double>(kv[r][0]);
            const double k1 = static_cast<double>(kv[r][1]);
            const double k2 = static_cast<double>(kv[r][2]);
            const double k3 = static_cast<double>(part_sum(kv[r][3], p1[j], p2[j]));
            const double v = vo[r] + h / 6.0 * (k0 + 2.0 * k1 + 2.0 * k2 + k3);
            V[f * N3 + i] = v;
            mx = fmax(mx, isfinite(v) ? fabs(v) : INFINITY);
        }
        __syncthreads();
    }
    mx = block_max(mx);
    if (threadIdx.x == 0) {
        part[(static_cast<size_t>(f) * nblk + blockIdx.x) * 2] = mx;
        part[(static_cast<size_t>(f) * nblk + blockIdx.x) * 2 + 1] = mx;
    }
}
template <typename R>
__global__ void __launch_bounds__(kStepThreads) k_dopri_err(const FlowState* fs, const R* K,
                                                            const R* KS, const double* V,
                                                            const double* Vnew, double rtol,
                                                            ErrWeights ew, double* part, int nblk,
                                                            int N, int B) {
    __shared__ double p1[stage_tile_lds(3)], p2[stage_tile_lds(3)];
    const int f = blockIdx.y;
    if (!running(fs, f)) return;
    const double h = fs[f].ht;
    const double at = fs[f].atol;
    const size_t N3 = static_cast<size_t>(N) * N * N;
    const size_t ks = static_cast<size_t>(B) * N3;
    const R* K6 = K + ((6 * static_cast<size_t>(B) + f) * 3) * N3;   // slot 6 (parts)
    const R* KSf = KS + static_cast<size_t>(f) * N3;                 // sums of slots 0..5
    constexpr int tsx = 8 * kTSY + 1, tile_n = kTZ * 64, EPT = tile_n / kStepThreads;
    double emax = 0.0, vmax = 0.0;
    const int ntile = stage_tiles(N, 3);
    for (int t = blockIdx.x; t < ntile; t += gridDim.x) {   // uniform over the block
        int x0, y0, z0;
        tile_origin(t, N, 3, x0, y0, z0);
        // this thread's slot sums, slot-6 pp parts, V and Vnew first (held across the barrier)
        R kv[EPT][7];
        double vop[EPT], vnp[EPT];
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            const int e = threadIdx.x + r * kStepThreads;
            const int lz = e & (kTZ - 1), ly = (e >> 4) & 7, lx = e >> 7;
            const int x = x0 + lx, y = y0 + ly, zz = z0 + lz;
            const size_t i =
                x < N && y < N && zz < N ? (static_cast<size_t>(x) * N + y) * N + zz : 0;
#pragma unroll
            for (int l = 0; l < 6; ++l) kv[r][l] = KSf[l * ks + i];
            kv[r][6] = K6[i];
            vop[r] = V[f * N3 + i];
            vnp[r] = Vnew[f * N3 + i];
        }
        tile_parts<3>(K6, N3, N, x0, y0, z0, p1, p2);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < EPT; ++r) {
            const int e = threadIdx.x + r * kStepThreads;
            const int lz = e & (kTZ - 1), ly = (e >> 4) & 7, lx = e >> 7;
            const int x = x0 + lx, y = y0 + ly, zz = z0 + lz;
            if (x >= N || y >= N || zz >= N) continue;
            const int j = lx * tsx + ly * kTSY + lz;
            const double vo = vop[r], vn = vnp[r];
            kv[r][6] = part_sum(kv[r][6], p1[j], p2[j]);
            double es = 0.0;
#pragma unroll
            for (int l = 0; l < 7; ++l) es += ew.e[l] * static_cast<double>(kv[r][l]);
            es = fabs(h * es);
            const double sc = at + rtol * fmax(fabs(vo), fabs(vn));
            const double q = es / sc;
            if (!isfinite(q) || !isfinite(vn)) { emax = INFINITY; vmax = INFINITY; }
            else { emax = fmax(emax, q); vmax = fmax(vmax, fabs(vn)); }
        }
        __syncthreads();
    }
    emax = block_max(emax);
    vmax = block_max(vmax);
    if (threadIdx.x == 0) {
        part[(static_cast<size_t>(f) * nblk + blockIdx.x) * 2] = emax;
        part[(static_cast<size_t>(f) * nblk + blockIdx.x) * 2 + 1] = vmax;
    }
}

// The crossing max|V| = v_max inside the last accepted step, on 1/max|V| as a function of
// x = ln T (temperature flow) or x = g^2 (interaction flow), where the coupling grows like a
// simple pole (1/max|V| smooth and nearly linear): the root of the parabola through the
// last three accepted points (x0, m0), (x1, m1), (x2, m2) that lies in [x1, x2], found by
// Newton's method from the straight line through the last two; the straight line itself
// when there is no earlier point (m0 = 0) or the parabola has no root in the step.
__device__ inline double crossing(double x0, double m0, double x1, double m1, double x2,
                                  double m2, double v_max) {
    if (!(m1 > 0.0) || m2 == m1) return x2;
    const double y1 = 1.0 / m1, y2 = 1.0 / m2, ys = 1.0 / v_max;
    const double d1 = (y2 - y1) / (x2 - x1);
    const double lin = x1 + (ys - y1) / d1;
    if (!(m0 > 0.0) || x0 == x1) return lin;
    const double d2 = (d1 - (y1 - 1.0 / m0) / (x1 - x0)) / (x2 - x0);
    double x = lin;
    for (int it = 0; it < 8; ++it) {
        const double r = (x - x1) * d1 + (x - x1) * (x - x2) * d2 - (ys - y1);
        const double d = d1 + (2.0 * x - x1 - x2) * d2;
        x -= r / d;
    }
    const bool inside = x1 < x2 ? (x >= x1 && x <= x2) : (x >= x2 && x <= x1);
    return isfinite(x) && inside ? x : lin;
}
// Interaction flow (s = -g): in g^2, since 1/v = 1/U - g^2 c for one patch.
__device__ inline double crossing_at(const FlowState& st, double s_new, double mv, double v_max) {
    if (!st.gflow) return crossing(st.sp, st.mp, st.lnT, st.m, s_new, mv, v_max);
    return -sqrt(crossing(st.sp * st.sp, st.mp, st.lnT * st.lnT, st.m, s_new * s_new, mv,
                          v_max));
}

__device__ inline double step_factor(double err) {
    if (err == 0.0) return 5.0;
    return fmin(5.0, fmax(0.2, 0.9 * pow(err, -0.2)));
}

// Accept/reject, stop rule and the next attempted step of one flow: e is its own error norm
// (kept in st.err), ed the norm that decides acceptance and the next step (its own, or the
// largest of its step-sharing group), mv its max|V| after the attempt.
__device__ inline void finish_flow(FlowState& st, double e, double ed, double mv, int rk45,
                                   int fixed_steps) {
    const double s = st.lnT, ht = st.ht, v_max = st.vmax;
    const bool last = ht != st.h;
    if (!rk45) {
        st.err = 0.0;
        double s_new;
        if (fixed_steps > 0)
            s_new = (st.n_acc + 1 == fixed_steps) ? st.lnT_end : st.s0 + (st.n_acc + 1) * ht;
        else
            s_new = s + ht;
        st.accepted = 1;
        st.n_acc += 1;
        st.n_rhs += 4;
        const bool finite = isfinite(mv);
        if (!finite) { st.status = FM_FLOW_NONFINITE; st.lnTc = s_new; }
        else if (mv > v_max) {
            st.status = FM_FLOW_DIVERGED;
            st.lnTc = crossing_at(st, s_new, mv, v_max);
        }
        st.sp = st.lnT;
        st.mp = st.m;
        st.lnT = s_new;
        st.m = mv;
        if (st.status == FM_FLOW_RUNNING && fixed_steps > 0 && st.n_acc >= fixed_steps)
            st.status = FM_FLOW_REACHED_TEND;
    } else {
        st.err = e;
        st.n_rhs += 6;
        if (ed <= 1.0) {
            const double s_new = last ? st.lnT_end : s + ht;
            st.accepted = 1;
            st.n_acc += 1;
            if (mv > v_max) {
                st.status = FM_FLOW_DIVERGED;
                st.lnTc = crossing_at(st, s_new, mv, v_max);
            }
            st.sp = st.lnT;
            st.mp = st.m;
            st.lnT = s_new;
            st.m = mv;
            st.h = ht * step_factor(ed);
        } else {
            st.accepted = 0;
            st.n_rej += 1;
            st.h = isfinite(ed) ? ht * step_factor(ed) : 0.5 * ht;
        }
        if (st.status == FM_FLOW_RUNNING && st.lnT <= st.lnT_end) st.status = FM_FLOW_REACHED_TEND;
        if (st.status == FM_FLOW_RUNNING && fabs(st.h) < st.hmin) st.status = FM_FLOW_STEPFAIL;
        st.ht = (st.lnT + st.h <= st.lnT_end) ? st.lnT_end - st.lnT : st.h;
    }
}

// Largest error norm and max|V| of flow f's partials (every thread returns both).
__device__ inline void flow_partials(const FlowState* fs, const double* part, int nblk, int f,
                                     double& e, double& mv) {
    e = 0.0;
    mv = 0.0;
    if (fs[f].status == FM_FLOW_RUNNING)
        for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
            e = fmax(e, part[(static_cast<size_t>(f) * nblk + i) * 2]);
            mv = fmax(mv, part[(static_cast<size_t>(f) * nblk + i) * 2 + 1]);
        }
    e = block_max(e);
    mv = block_max(mv);
}

// One workgroup per flow.
__global__ void __launch_bounds__(kThreads) k_finish(FlowState* fs, const double* part, int nblk,
                                                     int rk45, int fixed_steps) {
    const int f = blockIdx.x;
    double e, mv;
    flow_partials(fs, part, nblk, f, e, mv);
    if (threadIdx.x != 0) return;
    FlowState st = fs[f];
    if (st.status != FM_FLOW_RUNNING) { st.accepted = 0; fs[f] = st; return; }
    finish_flow(st, e, e, mv, rk45, fixed_steps);
    fs[f] = st;
}

// Flows on one step schedule, one workgroup per group (members[off[g] .. off[g+1]), which
// all hold the same ln T, h and attempted step): the group's step is decided on the largest
// error norm of its running members (accepted only if every member accepts; the next step is
// the smallest any member proposes), each member keeps its own stop rule, T_c and counters.
// The first member still running then bins for the group.  Shared memory: 2 doubles per member.
__global__ void __launch_bounds__(kThreads) k_finish_sync(FlowState* fs, const double* part,
                                                          int nblk, const int* members,
                                                          const int* off, int rk45,
                                                          int fixed_steps, int rebind) {
    extern __shared__ double sm[];
    const int i0 = off[blockIdx.x], n = off[blockIdx.x + 1] - i0;
    double* se = sm;
    double* sv = sm + n;
    for (int i = 0; i < n; ++i) {      // uniform over the block
        double e, mv;
        flow_partials(fs, part, nblk, members[i0 + i], e, mv);
        if (threadIdx.x == 0) { se[i] = e; sv[i] = mv; }
    }
    if (threadIdx.x != 0) return;
    double eg = 0.0;
    for (int i = 0; i < n; ++i)
        if (fs[members[i0 + i]].status == FM_FLOW_RUNNING) eg = fmax(eg, se[i]);
    int lead = -1;
    for (int i = 0; i < n; ++i) {
        const int f = members[i0 + i];
        FlowState st = fs[f];
        if (st.status != FM_FLOW_RUNNING) {
            st.accepted = 0;
        } else {
            finish_flow(st, se[i], eg, sv[i], rk45, fixed_steps);
            if (st.status == FM_FLOW_RUNNING && lead < 0) lead = f;
        }
        fs[f] = st;
    }
    if (!rebind || lead < 0) return;
    for (int i = 0; i < n; ++i) {
        const int f = members[i0 + i];
        if (fs[f].status == FM_FLOW_RUNNING) fs[f].bshare = lead + 1;
    }
}

// After an accepted Dormand-Prince step: V = Vnew and k0 = k6 (first same as last), all
// three channel parts.
template <typename R>
__global__ void __launch_bounds__(kThreads) k_commit(const FlowState* fs, double* V,
                                                     const double* Vnew, R* K, size_t N3, int B) {
    const int f = blockIdx.y;
    if (!fs[f].accepted) return;
    R* k0 = K + static_cast<size_t>(f) * 3 * N3;
    const R* k6 = K + (6 * static_cast<size_t>(B) + f) * 3 * N3;
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < N3;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        V[f * N3 + i] = Vnew[f * N3 + i];
        k0[i] = k6[i];
        k0[N3 + i] = k6[N3 + i];
        k0[2 * N3 + i] = k6[2 * N3 + i];
    }
}

__global__ void k_copy_state(const double* from, double* to, size_t n) {
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        to[i] = from[i];
}

}  // namespace
}  // namespace fm

// ======================================================================================
// Launchers.  nf = flows launched (grid y); buffers are strided by b.bstride flows.
// ======================================================================================
namespace fm {
namespace {

inline dim3 grid_for(size_t n, int nf, int cap = 2048) {
    size_t g = (n + kThreads - 1) / kThreads;
    if (g > static_cast<size_t>(cap)) g = cap;
    if (g == 0) g = 1;
    return dim3(static_cast<unsigned>(g), static_cast<unsigned>(nf));
}

template <typename R>
R* kslot_ptr(const Buffers& b, int slot, size_t N3) {   // slot base: [flow][channel][N^3]
    return static_cast<R*>(b.k) + static_cast<size_t>(slot) * b.bstride * 3 * N3;
}

template <typename R>
int bins_mode(const DevGeom& g) {
    // LDS bins where one padded bin matrix fits in a work group's LDS (160 KB on gfx950)
    return bins_lds_bytes(g.N, sizeof(R)) <= static_cast<size_t>(g.lds_max) ? 0 : 1;
}

// Stage argument plus, when the plan has nodes, their phase 1 in one launch.
template <typename R, int BT, int kG, int NODES>
void stage_go(hipStream_t s, const DevGeom& g, const DevZ& z, const Buffers& b, int nf,
              const StageCoef& sc, const BinPlan& bp, int write_new, const double* Vbase,
              int nRb) {
    static_assert(BT <= 1024, "a stage block covers one tile (at least 1024 elements) at a time");
    const int nbin = nRb * ((bp.n + NODES - 1) / NODES);
    const bool lds = nbin > 0 && bins_mode<R>(g) == 0;
    const int per_block = bp.n < NODES ? bp.n : NODES;   // bin matrices a block holds
    const size_t shm_bins = lds ? per_block * bins_lds_bytes(g.N, sizeof(R)) : 0;
    // stage tiles 16 x 16 x 16 (64-byte runs in all three layouts) where they give about one
    // block per CU or more and do not raise the LDS of phase-1 blocks, else 8 x 8 x 16
    // (measured: 16 wide for one flow at N = 48, 27 tiles, is 25% slower than 8 wide)
    const size_t lds16 = 2 * static_cast<size_t>(stage_tile_lds(4)) * sizeof(double);
    const int tl = static_cast<long>(stage_tiles(g.N, 4)) * nf >= 192 &&
                           (nbin == 0 || shm_bins >= lds16) ? 4 : 3;
    const int ns = std::min(stage_tiles(g.N, tl), 1024);  // one stage tile per block round
    // LDS: the block's bin matrices, or the two double tiles of a stage block
    const size_t shm =
        std::max(shm_bins, 2 * static_cast<size_t>(stage_tile_lds(tl)) * sizeof(double));
    const dim3 grid(static_cast<unsigned>(nbin + ns), nf);
    R* bins = static_cast<R*>(b.bins);
    R* binsT = static_cast<R*>(b.binsT);
    if (nbin == 0)
        hipLaunchKernelGGL(k_stage<R>, dim3(static_cast<unsigned>(ns), nf), dim3(1024), shm, s,
                           g, z, b.fs, sc, write_new, Vbase, static_cast<const R*>(b.k),
                           static_cast<R*>(b.ksum), b.Vnew,
                           static_cast<R*>(b.v0), static_cast<R*>(b.va), static_cast<R*>(b.vc),
                           b.T_stage, b.Z_stage, b.zw_stage, b.bstride, tl);
    else if (lds)
        hipLaunchKernelGGL((k_stage_bins<R, 0, BT, kG, NODES>), grid, dim3(BT), shm, s, g, z, b.fs,
                           sc, bp, write_new, Vbase, static_cast<const R*>(b.k),
                           static_cast<R*>(b.ksum), b.Vnew,
                           static_cast<R*>(b.v0), static_cast<R*>(b.va), static_cast<R*>(b.vc),
                           b.T_stage, b.Z_stage, b.zw_stage, bins, binsT, nRb, b.bstride, tl);
    else if constexpr (NODES == 1)
        hipLaunchKernelGGL((k_stage_bins<R, 1, BT, kG, 1>), grid, dim3(BT), shm, s, g, z, b.fs, sc,
                           bp, write_new, Vbase, static_cast<const R*>(b.k),
                           static_cast<R*>(b.ksum), b.Vnew,
                           static_cast<R*>(b.v0), static_cast<R*>(b.va), static_cast<R*>(b.vc),
                           b.T_stage, b.Z_stage, b.zw_stage, bins, binsT, nRb, b.bstride, tl);
}

// Stage nodes one phase-1 block bins together: two where a node's LDS bins exceed 40 KB
// (single-node blocks are then limited by LDS to two per CU anyway) and two fit in LDS,
// given many (representative, flow) pairs; else one.  Measured: two nodes per block at
// N = 128 save 5% of phase 1; five per block at N = 48 (more blocks per CU without them)
// cost 27-33%.
template <typename R>
int nodes_per_block(const DevGeom& g, const BinPlan& bp, int nRb, int nf) {
    const size_t per = bins_lds_bytes(g.N, sizeof(R));
    if (g.gflow || bp.n <= 1 || bins_mode<R>(g) != 0) return 1;
    if (static_cast<long>(nRb) * nf < 4096) return 1;
    return per > 40960 && 2 * per <= static_cast<size_t>(g.lds_max) ? 2 : 1;
}

// Stage argument plus the plan's phase 1 in one launch (without phase 1: k_stage).  Few
// (flow, node, representative) triples (at most one per CU): 1024-thread blocks; many:
// 256-thread blocks.
template <typename R, int kG, int NODES>
void stage_nodes(hipStream_t s, const DevGeom& g, const DevZ& z, const Buffers& b, int nf,
                 const StageCoef& sc, const BinPlan& bp, int write_new, const double* Vbase,
                 int wide_force) {
    const int nRb = b.bins ? g.nRp + g.nRd : 0;
    const int per_block = bp.n < NODES ? bp.n : NODES;
    // bins in LDS above 40 KB leave room for at most three blocks per CU: 256-thread blocks
    // would keep three waves or fewer per SIMD to hide the scan's dependent steps
    const bool big = nRb > 0 && bins_mode<R>(g) == 0 &&
                     per_block * bins_lds_bytes(g.N, sizeof(R)) > 40960;
    const long nblk = static_cast<long>(nRb) * ((bp.n + NODES - 1) / NODES) * nf;
    const bool wide = nblk <= 256 || (big && bp.n > 0);
    if (wide_force >= 0 && bp.n > 0) {       // a fixed launch shape (timing, or the caller's)
        if (wide_force) stage_go<R, 1024, kG, NODES>(s, g, z, b, nf, sc, bp, write_new, Vbase, nRb);
        else stage_go<R, 256, kG, NODES>(s, g, z, b, nf, sc, bp, write_new, Vbase, nRb);
        return;
    }
    if (wide) stage_go<R, 1024, kG, NODES>(s, g, z, b, nf, sc, bp, write_new, Vbase, nRb);
    else stage_go<R, 256, kG, NODES>(s, g, z, b, nf, sc, bp, write_new, Vbase, nRb);
}

template <typename R>
void stage_t(hipStream_t s, const DevGeom& g, const DevZ& z, const Buffers& b, int nf,
             const StageCoef& sc, const BinPlan& bp, int write_new, const double* Vbase) {
    if (g.gflow && bp.n > 0) {
        stage_nodes<R, 1, 1>(s, g, z, b, nf, sc, bp, write_new, Vbase, -1);
        return;
    }
    // a fixed shape (b.ph1var 1..4: 256 or 1024 threads, one or two nodes per block) where
    // it applies (two nodes need several nodes and two bin matrices within the LDS),
    // else the rule
    const int v = b.ph1var;
    int nodes = b.bins ? nodes_per_block<R>(g, bp, g.nRp + g.nRd, nf) : 1;
    int wide = -1;
    if (v >= 1 && v <= 4 && b.bins && bp.n > 0) {
        wide = (v - 1) % 2;
        nodes = (v >= 3 && bp.n > 1 && 2 * bins_lds_bytes(g.N, sizeof(R)) <= static_cast<size_t>(g.lds_max)) ? 2 : 1;
    }
    if (nodes == 2) stage_nodes<R, 0, 2>(s, g, z, b, nf, sc, bp, write_new, Vbase, wide);
    else stage_nodes<R, 0, 1>(s, g, z, b, nf, sc, bp, write_new, Vbase, wide);
}

// Matrix-core phase 2a: operand widths by patch count (KE k-values per lane, NT column
// tiles per wave); row tiles per wavefront `tpw` is a tuning choice (0: one).
template <int kM, int KE, int NT>
void y_mfma_rows(hipStream_t s, const DevGeom& g, const Buffers& b, int nf,
                const YArgs<float>& a, int tpw) {
    const int mmax = g.nP > g.nD ? g.nP : g.nD;
    const int ntiles = (mmax + 15) / 16;
    const int maxt = (ntiles + 3) / 4;
    tpw = tpw <= 0 ? 1 : (tpw > maxt ? maxt : tpw);
    const int nchunk = (g.N + 16 * NT - 1) / (16 * NT);
    const int bx = (ntiles + 4 * tpw - 1) / (4 * tpw);
    const long nwork = static_cast<long>(bx) * g.N * 3 * nf;
    const long nblocks = (nwork + 7) / 8 * 8 * nchunk;
    hipLaunchKernelGGL((k_y_mfma_rows<kM, KE, NT>), dim3(static_cast<unsigned>(nblocks)),
                       dim3(kThreads), 0, s, g, b.fs, b.Z_stage, b.zw_stage,
                       static_cast<const float*>(b.bins),
                       static_cast<const float*>(b.binsT), a, nchunk, tpw, bx,
                       static_cast<int>(nwork));
}

template <int kM, int KE, int NT>
void y_mfma_cls(hipStream_t s, const DevGeom& g, const Buffers& b, int nf,
                const YArgs<float>& a, int tpw) {
    const int maxt = y_max_tpw(g);
    tpw = tpw <= 0 ? 1 : (tpw > maxt ? maxt : tpw);
    YRuns runs{};
    for (int c = 0; c < 2; ++c)
        for (int o = 0; o < (g.sym ? 1 : 8); ++o) {   // symmetric states: class 0 only
            const int nt = (g.cls[c][o + 1] - g.cls[c][o] + 15) / 16;
            runs.nr[c][o] = (nt + 4 * tpw - 1) / (4 * tpw);
            runs.tot[c] += runs.nr[c][o];
        }
    const int nchunk = (g.N + 16 * NT - 1) / (16 * NT);
    const int bx = runs.tot[0] > runs.tot[1] ? runs.tot[0] : runs.tot[1];
    const long nwork = static_cast<long>(bx) * g.N * 3 * nf;
    const long nblocks = (nwork + 7) / 8 * 8 * nchunk;
    if (nblocks == 0) return;
    hipLaunchKernelGGL((k_y_mfma_cls<kM, KE, NT>), dim3(static_cast<unsigned>(nblocks)),
                       dim3(kThreads), 0, s, g, b.fs, b.Z_stage, b.zw_stage,
                       static_cast<const float*>(b.bins),
                       static_cast<const float*>(b.binsT), a, runs, nchunk, tpw, bx,
                       static_cast<int>(nwork));
}

template <int kM, int KE, int NT, int TPW>
void y_mfma_orb_go(hipStream_t s, const DevGeom& g, const Buffers& b, int nf,
                   const YArgs<float>& a) {
    if constexpr (kM == 1) {
        if (g.sym) {                                   // operation 0 only: one staging per unit
            const int nchunk = (g.N + 16 * NT - 1) / (16 * NT);
            const long nu = 3L * g.N * nf;
            if (nu == 0) return;
            hipLaunchKernelGGL((k_y_orb_sym<KE, NT>), dim3(static_cast<unsigned>(nu)),
                               dim3(kSymThreads), 0, s, g, b.fs, b.Z_stage, b.zw_stage,
                               static_cast<const float*>(b.bins),
                               static_cast<const float*>(b.binsT), a, nchunk,
                               static_cast<int>(nu));
            return;
        }
    }
    const int ntmax = g.orb_nt[0] > g.orb_nt[1] ? g.orb_nt[0] : g.orb_nt[1];
    const int bx = (ntmax + 4 * TPW - 1) / (4 * TPW);
    const int nchunk = (g.N + 16 * NT - 1) / (16 * NT);
    const long ngw = 3L * g.nG * nf;
    const long nblocks = (ngw + 7) / 8 * 8 * (8L * bx * nchunk);
    if (nblocks == 0) return;
    hipLaunchKernelGGL((k_y_mfma_orb<kM, KE, NT, TPW>), dim3(static_cast<unsigned>(nblocks)),
                       dim3(kThreads), 0, s, g, b.fs, b.Z_stage, b.zw_stage,
                       static_cast<const float*>(b.bins),
                       static_cast<const float*>(b.binsT), a, nchunk, bx,
                       static_cast<int>(ngw));
}

// Orbit kernel: tiles per wavefront 1, 2 or (bf16 operands) 4; A stays in registers across
// the operations.
template <int kM, int KE, int NT>
void y_mfma_orb(hipStream_t s, const DevGeom& g, const Buffers& b, int nf,
                const YArgs<float>& a, int tpw) {
    if constexpr (kM == 1) {
        if (tpw >= 4) { y_mfma_orb_go<kM, KE, NT, 4>(s, g, b, nf, a); return; }
    }
    if (tpw >= 2) y_mfma_orb_go<kM, KE, NT, 2>(s, g, b, nf, a);
    else y_mfma_orb_go<kM, KE, NT, 1>(s, g, b, nf, a);
}

// yvar 2: the operation-class kernel, 3: the orbit kernel, else the per-row one.
template <int kM, int KE, int NT>
void y_mfma_tpw(hipStream_t s, const DevGeom& g, const Buffers& b, int nf,
                const YArgs<float>& a, int tpw, int yvar) {
    if (yvar == 2) y_mfma_cls<kM, KE, NT>(s, g, b, nf, a, tpw);
    else if (yvar == 3) y_mfma_orb<kM, KE, NT>(s, g, b, nf, a, tpw);
    else y_mfma_rows<kM, KE, NT>(s, g, b, nf, a, tpw);
}

inline void y_mfma_launch(hipStream_t s, const DevGeom& g, const Buffers& b, int nf,
                          const YArgs<float>& a, int mode, int tpw, int yvar) {
    const int N = g.N;
    if (mode == 2) {         // bf16 operands
        if (N <= 16) y_mfma_tpw<1, 8, 1>(s, g, b, nf, a, tpw, yvar);
        else if (N <= 32) y_mfma_tpw<1, 8, 2>(s, g, b, nf, a, tpw, yvar);
        else if (N <= 48) y_mfma_tpw<1, 16, 3>(s, g, b, nf, a, tpw, yvar);
        else if (N <= 64) y_mfma_tpw<1, 16, 4>(s, g, b, nf, a, tpw, yvar);
        else if (N <= 96) y_mfma_tpw<1, 24, 3>(s, g, b, nf, a, tpw, yvar);
        else y_mfma_tpw<1, 32, 4>(s, g, b, nf, a, tpw, yvar);
    } else if (mode == 3) {  // split bf16 operands (two planes in LDS)
        if (N <= 16) y_mfma_tpw<2, 8, 1>(s, g, b, nf, a, tpw, yvar);
        else if (N <= 32) y_mfma_tpw<2, 8, 2>(s, g, b, nf, a, tpw, yvar);
        else if (N <= 48) y_mfma_tpw<2, 16, 3>(s, g, b, nf, a, tpw, yvar);
        else if (N <= 64) y_mfma_tpw<2, 16, 4>(s, g, b, nf, a, tpw, yvar);
        else if (N <= 96) y_mfma_tpw<2, 24, 3>(s, g, b, nf, a, tpw, yvar);
        else y_mfma_tpw<2, 32, 2>(s, g, b, nf, a, tpw, yvar);
    } else {
        if (N <= 16) y_mfma_tpw<0, 4, 1>(s, g, b, nf, a, tpw, yvar);
        else if (N <= 32) y_mfma_tpw<0, 8, 2>(s, g, b, nf, a, tpw, yvar);
        else if (N <= 48) y_mfma_tpw<0, 12, 3>(s, g, b, nf, a, tpw, yvar);
        else if (N <= 64) y_mfma_tpw<0, 16, 2>(s, g, b, nf, a, tpw, yvar);
        else if (N <= 96) y_mfma_tpw<0, 24, 2>(s, g, b, nf, a, tpw, yvar);
        else y_mfma_tpw<0, 32, 2>(s, g, b, nf, a, tpw, yvar);
    }
}

template <typename R>
void y_t(hipStream_t s, const DevGeom& g, const Buffers& b, int nf, unsigned ch, int mma,
         int tpw, int yvar) {
    YArgs<R> a;
    a.Vs[0] = static_cast<const R*>(b.v0);
    a.Vs[1] = static_cast<const R*>(b.vc);
    a.Vs[2] = static_cast<const R*>(b.va);
    a.Vs[3] = static_cast<const R*>(b.vc);
    a.Y[0] = static_cast<R*>(b.y1); a.Y[1] = static_cast<R*>(b.y2);
    a.Y[2] = static_cast<R*>(b.y3); a.Y[3] = static_cast<R*>(b.y4);
    a.on[0] = (ch & FM_CH_PP) != 0;
    a.on[1] = (ch & FM_CH_CR) != 0;
    a.on[2] = a.on[3] = (ch & FM_CH_D) != 0;
    const int mmax = g.nP > g.nD ? g.nP : g.nD;
    if constexpr (sizeof(R) == 4) {
        if (mma > 0 && g.N <= 128) {
            y_mfma_launch(s, g, b, nf, reinterpret_cast<const YArgs<float>&>(a), mma, tpw, yvar);
            return;
        }
    }
    const int tiles = ((mmax + 63) / 64) * ((g.N + 63) / 64);
    hipLaunchKernelGGL(k_y<R>, dim3(tiles, g.N, 4 * nf), dim3(kThreads), 0, s, g, b.fs,
                       b.Z_stage, b.zw_stage, static_cast<const R*>(b.bins),
                       static_cast<const R*>(b.binsT), a);
}

template <typename R, typename YT>
void contract_go(hipStream_t s, const DevGeom& g, const Buffers& b, int nf, unsigned ch, int slot) {
    if constexpr (sizeof(R) == 4) {
        // symmetric states on the matrix cores: bf16 products, or split-bf16 products (f32 Y
        // of the split mode; the f32 mode keeps its f32 phase 2b)
        if (g.sym && g.N % 16 == 0 && g.N <= 128 && (sizeof(YT) == 2 || b.y_split)) {
            // bf16: the pp and crossed items stage one product (more blocks per CU), the
            // direct items two; split: two planes of one product at a time
            const size_t one = 128 * static_cast<size_t>(kMmaKBS) * sizeof(__bf16);
            const int n01 = g.n_sym_items[0] + g.n_sym_items[1], n2 = g.n_sym_items[2];
            for (int part = 0; part < 2; ++part) {
                const int items = part ? n2 : n01;
                if (items == 0) continue;
                const size_t lds = (sizeof(YT) == 4 || part) ? 2 * one : one;
                auto kern = part ? k_contract_mma<YT, true> : k_contract_mma<YT, false>;
                hipLaunchKernelGGL(kern, dim3(items, nf), dim3(256), lds, s,
                                   g, b.fs, static_cast<const float*>(b.v0),
                                   static_cast<const float*>(b.va), static_cast<const float*>(b.vc),
                                   static_cast<const YT*>(b.y1), static_cast<const YT*>(b.y2),
                                   static_cast<const YT*>(b.y3), static_cast<const YT*>(b.y4),
                                   static_cast<float*>(b.k), ch, slot, b.bstride, part ? n01 : 0);
            }
            return;
        }
    }
    const size_t lds = 2 * static_cast<size_t>(kChunk) * g.N * sizeof(R);
    const int items = g.n_items[0] + g.n_items[1] + g.n_items[2];
    hipLaunchKernelGGL((k_contract<R, YT>), dim3(items, nf), dim3(64), lds, s, g, b.fs,
                       static_cast<const R*>(b.v0), static_cast<const R*>(b.va),
                       static_cast<const R*>(b.vc), static_cast<const YT*>(b.y1),
                       static_cast<const YT*>(b.y2), static_cast<const YT*>(b.y3),
                       static_cast<const YT*>(b.y4), static_cast<R*>(b.k), ch, slot, b.bstride);
}

template <typename R>
void contract_t(hipStream_t s, const DevGeom& g, const Buffers& b, int nf, unsigned ch, int slot) {
    if constexpr (sizeof(R) == 4) {
        if (b.y_bf16) { contract_go<float, __bf16>(s, g, b, nf, ch, slot); return; }
    }
    contract_go<R, R>(s, g, b, nf, ch, slot);
}

template <int kM, int KE, int NT>
void fused_go(hipStream_t s, const DevGeom& g, const Buffers& b, int nf, unsigned ch, int slot) {
    const int nchunk = (g.N + 16 * NT - 1) / (16 * NT);
    const int nblk = g.fz_nblk[0] + g.fz_nblk[1] + g.fz_nblk[2];
    const int keys = nblk * ((nf + 1) / 2);
    const int blocks = (keys + 7) / 8 * 8 * 2 * nchunk;
    hipLaunchKernelGGL((k_fused<kM, KE, NT>), dim3(blocks), dim3(4 * kFusedRows), 0, s, g,
                       b.fs, b.Z_stage, b.zw_stage, static_cast<const float*>(b.bins),
                       static_cast<const float*>(b.binsT), static_cast<const float*>(b.v0),
                       static_cast<const float*>(b.va), static_cast<const float*>(b.vc),
                       static_cast<float*>(b.k), ch, slot, b.bstride, nchunk, nf);
}

template <int kM>
void fused_m(hipStream_t s, const DevGeom& g, const Buffers& b, int nf, unsigned ch, int slot) {
    // k padded to whole 32-wide steps; columns in chunks of at most 64
    if (g.N <= 16) fused_go<kM, 8, 1>(s, g, b, nf, ch, slot);
    else if (g.N <= 32) fused_go<kM, 8, 2>(s, g, b, nf, ch, slot);
    else if (g.N <= 48) fused_go<kM, 16, 3>(s, g, b, nf, ch, slot);
    else if (g.N <= 64) fused_go<kM, 16, 4>(s, g, b, nf, ch, slot);
    else if (g.N <= 96) fused_go<kM, 24, 4>(s, g, b, nf, ch, slot);
    else fused_go<kM, 32, 4>(s, g, b, nf, ch, slot);
}

}  // namespace

int y_max_tpw(const DevGeom& g) {
    int most = 1;
    for (int c = 0; c < 2; ++c)
        for (int o = 0; o < 8; ++o) {
            const int nt = (g.cls[c][o + 1] - g.cls[c][o] + 15) / 16;
            most = nt > most ? nt : most;
        }
    return (most + 3) / 4;
}

void launch_stage(hipStream_t s, bool dbl, const DevGeom& g, const DevZ& z, const Buffers& b,
                  int nf, const StageCoef& sc, const BinPlan& bp, int write_new,
                  const double* Vbase) {
    if (dbl) stage_t<double>(s, g, z, b, nf, sc, bp, write_new, Vbase);
    else stage_t<float>(s, g, z, b, nf, sc, bp, write_new, Vbase);
}

Buffers with_bin_set(const Buffers& b, const DevGeom& g, bool dbl, int set) {
    Buffers o = b;
    if (b.bins && set > 0) {
        const size_t rs = dbl ? sizeof(double) : sizeof(float);
        const size_t NN = static_cast<size_t>(g.NN), B = static_cast<size_t>(b.bstride);
        o.bins = static_cast<char*>(b.bins) + set * B * (g.nRp + g.nRd) * NN * rs;
        o.binsT = static_cast<char*>(b.binsT) + set * B * g.nRd * NN * rs;
    }
    return o;
}

void launch_y(hipStream_t s, bool dbl, const DevGeom& g, const Buffers& b, int nf, unsigned ch,
              int mma, int tpw, int yvar) {
    if (dbl) y_t<double>(s, g, b, nf, ch, 0, 0, 0);
    else y_t<float>(s, g, b, nf, ch, mma, tpw, yvar);
}

int y_rows_max_tpw(const DevGeom& g) {
    const int mmax = g.nP > g.nD ? g.nP : g.nD;
    return ((mmax + 15) / 16 + 3) / 4;
}

int y_orb_max_tpw(const DevGeom& g, int mma) {
    const int ntmax = g.orb_nt[0] > g.orb_nt[1] ? g.orb_nt[0] : g.orb_nt[1];
    const int cap = mma == 2 ? 4 : 2;
    int t = 1;
    while (t < cap && 4 * t < ntmax) t *= 2;
    return t;
}

void launch_contract(hipStream_t s, bool dbl, const DevGeom& g, const Buffers& b, int nf,
                     unsigned ch, int slot) {
    if (dbl) contract_t<double>(s, g, b, nf, ch, slot);
    else contract_t<float>(s, g, b, nf, ch, slot);
}

void launch_fused(hipStream_t s, const DevGeom& g, const Buffers& b, int nf, unsigned ch,
                  int slot, int mma) {
    if (mma == 3) fused_m<2>(s, g, b, nf, ch, slot);
    else fused_m<1>(s, g, b, nf, ch, slot);
}

void launch_wtable(hipStream_t s, const DevGeom& g, const Buffers& b, int nf) {
    hipLaunchKernelGGL(k_wtable, dim3((g.np + kThreads - 1) / kThreads, g.nP + g.nD, nf),
                       dim3(kThreads), 0, s, g, b.fs, b.T_stage, b.Z_stage, b.zw_stage, b.wtab);
}

void launch_direct(hipStream_t s, const DevGeom& g, const Buffers& b, int nf, unsigned ch,
                   int slot) {
    const size_t N3 = static_cast<size_t>(g.NN) * g.N;
    const int threads = std::min(((g.N + 63) / 64) * 64, kThreads);   // a thread per c, looped
    hipLaunchKernelGGL(k_direct, dim3(g.NN, nf), dim3(threads), 0, s, g, b.fs, b.wtab,
                       static_cast<const double*>(b.v0), kslot_ptr<double>(b, slot, N3), ch);
}

void launch_k_to_f64(hipStream_t s, bool dbl, const Buffers& b, int nf, int N, int slot,
                     double* out) {
    const size_t N3 = static_cast<size_t>(N) * N * N;
    if (dbl)
        hipLaunchKernelGGL(k_to_f64<double>, grid_for(N3, nf), dim3(kThreads), 0, s, b.fs,
                           kslot_ptr<double>(b, slot, N3), out, N);
    else
        hipLaunchKernelGGL(k_to_f64<float>, grid_for(N3, nf), dim3(kThreads), 0, s, b.fs,
                           kslot_ptr<float>(b, slot, N3), out, N);
}

void launch_fill_u(hipStream_t s, const Buffers& b, int nf, size_t N3, const double* U) {
    hipLaunchKernelGGL(k_fill_u, grid_for(N3, nf), dim3(kThreads), 0, s, b.V, U, N3);
}

// (b.nblk blocks per flow, one per tile up to 512, each writing its partial maxima)
void launch_rk4_update(hipStream_t s, bool dbl, const Buffers& b, int nf, int N, double* V) {
    const dim3 grid(b.nblk, nf);
    if (dbl)
        hipLaunchKernelGGL(k_rk4_update<double>, grid, dim3(kStepThreads), 0, s, b.fs,
                           static_cast<const double*>(b.k),
                           static_cast<const double*>(b.ksum), V, b.part, b.nblk, N, b.bstride);
    else
        hipLaunchKernelGGL(k_rk4_update<float>, grid, dim3(kStepThreads), 0, s, b.fs,
                           static_cast<const float*>(b.k),
                           static_cast<const float*>(b.ksum), V, b.part, b.nblk, N, b.bstride);
}

void launch_dopri_err(hipStream_t s, bool dbl, const Buffers& b, int nf, int N,
                      const double* V, double rtol, const ErrWeights& ew) {
    const dim3 grid(b.nblk, nf);
    if (dbl)
        hipLaunchKernelGGL(k_dopri_err<double>, grid, dim3(kStepThreads), 0, s, b.fs,
                           static_cast<const double*>(b.k),
                           static_cast<const double*>(b.ksum), V, b.Vnew, rtol, ew, b.part, b.nblk,
                           N, b.bstride);
    else
        hipLaunchKernelGGL(k_dopri_err<float>, grid, dim3(kStepThreads), 0, s, b.fs,
                           static_cast<const float*>(b.k),
                           static_cast<const float*>(b.ksum), V, b.Vnew, rtol, ew, b.part, b.nblk,
                           N, b.bstride);
}

void launch_finish(hipStream_t s, const Buffers& b, int nf, int rk45, int fixed_steps) {
    hipLaunchKernelGGL(k_finish, dim3(nf), dim3(kThreads), 0, s, b.fs, b.part, b.nblk, rk45,
                       fixed_steps);
}

void launch_finish_sync(hipStream_t s, const Buffers& b, int ngroups, int max_members, int rk45,
                        int fixed_steps, int rebind) {
    hipLaunchKernelGGL(k_finish_sync, dim3(ngroups), dim3(kThreads),
                       2 * static_cast<size_t>(max_members) * sizeof(double), s, b.fs, b.part,
                       b.nblk, b.grp_members, b.grp_off, rk45, fixed_steps, rebind);
}

void launch_commit(hipStream_t s, bool dbl, const Buffers& b, int nf, size_t N3, double* V) {
    if (dbl)
        hipLaunchKernelGGL(k_commit<double>, grid_for(N3, nf), dim3(kThreads), 0, s, b.fs, V,
                           b.Vnew, static_cast<double*>(b.k), N3, b.bstride);
    else
        hipLaunchKernelGGL(k_commit<float>, grid_for(N3, nf), dim3(kThreads), 0, s, b.fs, V,
                           b.Vnew, static_cast<float*>(b.k), N3, b.bstride);
}

void launch_copy(hipStream_t s, const double* from, double* to, size_t n) {
    hipLaunchKernelGGL(k_copy_state, grid_for(n, 1), dim3(kThreads), 0, s, from, to, n);
}

}  // namespace fm
