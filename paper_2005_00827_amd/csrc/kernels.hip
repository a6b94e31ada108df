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
// Phase 1 (k_points, k_bins): bubble-weight derivatives on the fly for every transfer q and
//   loop point j, summed into per-transfer bin matrices held in LDS.  ALU bound.
// Phase 2a (k_y): per-transfer grouped products Y_q = B_q x V-slab, four kinds.
// Phase 2b (k_contract): the remaining contraction over one patch index per channel, all
//   three channels fused per output element.
// Integrator (k_stage, k_rk4_update, k_dopri_err, k_finish, k_commit): double precision.
// Direct path (k_wtable, k_direct): the same sums over every loop point, no bins.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "fm_internal.h"

namespace fm {
namespace {

constexpr int kThreads = 256;

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

template <typename R>
__device__ inline R phi_dd(R a, R pa, R b, R pb) {
    const R d = a - b;
    if (fabs(d) >= WeightCut<R>::v) return (pa - pb) / d;
    const R m = R(0.5) * (a + b);
    const R e = exp(R(-2) * fabs(m));
    const R den = R(1) + e;
    const R s = R(4) * e / (den * den);
    const R tau = copysign((R(1) - e) / den, m);
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

__device__ inline bool running(const FlowState* fs, int f) { return fs[f].status == FM_FLOW_RUNNING; }

// ------------------------------------------------------------------------------------
// Stage argument V_s = V + h sum_l a_l k_l (double), Z and T of the stage, operand layouts
//   v0[x][y][z] = V(x,y,z),  va[z][x][y] = V(x,y,z),  vc[z][y][x] = V(x,y,z).
// ------------------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(kThreads) k_stage(DevGeom g, DevZ z, const FlowState* fs,
                                                    StageCoef sc, int write_new,
                                                    const double* Vbase, const R* K,
                                                    double* Vnew, R* v0, R* va, R* vc,
                                                    double* T_stage, double* Z_stage, int B) {
    const int f = blockIdx.y;
    if (!running(fs, f)) return;
    const int N = g.N, NN = g.NN;
    const size_t N3 = static_cast<size_t>(NN) * N;
    const double ht = fs[f].ht;
    const double lnTs = fs[f].lnT + sc.c * ht;
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) T_stage[f] = exp(lnTs);
        for (int a = threadIdx.x; a < N; a += blockDim.x)
            Z_stage[static_cast<size_t>(f) * N + a] = z_interp(z, f, N, a, lnTs);
    }
    const double* Vf = Vbase + f * N3;
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < N3;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        double acc = 0.0;
        for (int l = 0; l < sc.ns; ++l) acc += sc.a[l] * static_cast<double>(K[(static_cast<size_t>(l) * B + f) * N3 + i]);
        const double v = Vf[i] + ht * acc;
        if (write_new) Vnew[f * N3 + i] = v;
        const int x = static_cast<int>(i / NN);
        const int y = static_cast<int>((i / N) % N);
        const int zz = static_cast<int>(i % N);
        const R r = static_cast<R>(v);
        v0[f * N3 + i] = r;
        va[f * N3 + static_cast<size_t>(zz) * NN + x * N + y] = r;
        vc[f * N3 + static_cast<size_t>(zz) * NN + y * N + x] = r;
    }
}

// Per-point quantities of the stage: a_j = xi_j / 2T and phi(a_j).
template <typename R>
__global__ void __launch_bounds__(kThreads) k_points(DevGeom g, const FlowState* fs,
                                                     const double* T_stage, R* pt) {
    const int f = blockIdx.y;
    if (!running(fs, f)) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.np) return;
    const double a = g.xi[j] / (2.0 * T_stage[f]);
    R* p = pt + (static_cast<size_t>(f) * g.np + j) * 2;
    p[0] = static_cast<R>(a);
    p[1] = static_cast<R>(phi_d(a));
}

// ------------------------------------------------------------------------------------
// Phase 1: bins.  One workgroup per (transfer, flow); the N x N bin matrix lives in LDS.
// blockIdx.x < nP: particle-particle transfer; otherwise particle-hole.
// ------------------------------------------------------------------------------------
template <typename R, bool kLds>
__global__ void __launch_bounds__(kThreads) k_bins(DevGeom g, const FlowState* fs,
                                                   const double* T_stage, const R* pt,
                                                   R* bpp, R* bph, R* bphT) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int f = blockIdx.y;
    if (!running(fs, f)) return;
    const int q = blockIdx.x;
    const int N = g.N, NN = g.NN, L = g.L, np = g.np;
    const bool pp = q < g.nP;
    const int m = pp ? g.q_pp[q] : g.q_ph[q - g.nP];
    R* out = pp ? bpp + (static_cast<size_t>(f) * g.nP + q) * NN
                : bph + (static_cast<size_t>(f) * g.nD + (q - g.nP)) * NN;
    R* bins = kLds ? reinterpret_cast<R*>(smem_raw) : out;
    if (kLds) {
        for (int i = threadIdx.x; i < NN; i += blockDim.x) bins[i] = R(0);
        __syncthreads();
    }
    const R scale = static_cast<R>(-1.0 / (4.0 * T_stage[f] * np));
    const R* P = pt + static_cast<size_t>(f) * np * 2;
    for (int j = threadIdx.x; j < np; j += blockDim.x) {
        const int jp = pp ? partner_pp(m, j, L) : partner_ph(m, j, L);
        const R a = P[2 * j], pa = P[2 * j + 1];
        R b = P[2 * jp], pb = P[2 * jp + 1];
        if (pp) { b = -b; pb = -pb; }   // chi_pp(x, y) = chi_ph(x, -y); phi is odd
        const R w = scale * phi_dd<R>(a, pa, b, pb);
        atomicAdd(&bins[g.patch[j] * N + g.patch[jp]], w);
    }
    if (!kLds) return;
    __syncthreads();
    for (int i = threadIdx.x; i < NN; i += blockDim.x) out[i] = bins[i];
    if (!pp) {
        R* outT = bphT + (static_cast<size_t>(f) * g.nD + (q - g.nP)) * NN;
        for (int i = threadIdx.x; i < NN; i += blockDim.x) {
            const int bb = i / N, aa = i - bb * N;   // outT[b'][a'] = bins[a'][b']
            outT[i] = bins[aa * N + bb];
        }
    }
}

// Transposed copy for the global-atomic fallback of k_bins.
template <typename R>
__global__ void __launch_bounds__(kThreads) k_transpose_bins(DevGeom g, const FlowState* fs,
                                                             const R* bph, R* bphT) {
    const int f = blockIdx.z;
    if (!running(fs, f)) return;
    const int q = blockIdx.y;
    const int N = g.N, NN = g.NN;
    const R* in = bph + (static_cast<size_t>(f) * g.nD + q) * NN;
    R* out = bphT + (static_cast<size_t>(f) * g.nD + q) * NN;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NN; i += gridDim.x * blockDim.x) {
        const int bb = i / N, aa = i - bb * N;
        out[i] = in[aa * N + bb];
    }
}

template <typename R>
__global__ void __launch_bounds__(kThreads) k_zero(R* p, size_t n) {
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        p[i] = R(0);
}

// ------------------------------------------------------------------------------------
// Phase 2a: grouped products.  For group g (one patch index) and kind k:
//   C[q][n] = sum_kk A[q][kk] Bm[kk][n],  A[q][kk] = Asrc[q][g][kk] Z_g Z_kk,
//   Bm[kk][n] = Vsrc[g][kk][n],
// stored as Y[q][g][n] (kind 0) or Y[q][n][g] (kinds 1..3):
//   kind 0 (pp):     Asrc = Bpp,  Vsrc = v0 -> Y1[q][a'][c]
//   kind 1 (crossed):Asrc = BphT, Vsrc = vc -> Y2[q][a][b']
//   kind 2 (direct): Asrc = Bph,  Vsrc = va -> Y3[q][b][a']
//   kind 3 (direct): Asrc = Bph,  Vsrc = vc -> Y4[q][b][a']
// 64 x 64 output tile, K in steps of 16, 4 x 4 per thread.
// ------------------------------------------------------------------------------------
template <typename R>
struct YArgs {
    const R* A[4];
    const R* Vs[4];
    R* Y[4];
    int M[4];
    int on[4];
};

template <typename R>
__global__ void __launch_bounds__(kThreads) k_y(DevGeom g, const FlowState* fs,
                                                const double* Z_stage, YArgs<R> args, int B) {
    constexpr int TM = 64, TN = 64, TK = 16;
    __shared__ R As[TK][TM + 4];
    __shared__ R Bs[TK][TN + 4];
    const int kind = blockIdx.z % 4;
    const int f = blockIdx.z / 4;
    if (!running(fs, f) || !args.on[kind]) return;
    const int N = g.N, NN = g.NN;
    const int M = args.M[kind];
    const int ntn = (N + TN - 1) / TN;
    const int tm = blockIdx.x / ntn, tn = blockIdx.x - tm * ntn;
    if (tm * TM >= M) return;
    const int grp = blockIdx.y;
    const size_t N3 = static_cast<size_t>(NN) * N;
    const R* A = args.A[kind] + static_cast<size_t>(f) * M * NN + static_cast<size_t>(grp) * N;
    const R* Vg = args.Vs[kind] + f * N3 + static_cast<size_t>(grp) * NN;
    const double* Zf = Z_stage + static_cast<size_t>(f) * N;
    const R zg = static_cast<R>(Zf[grp]);
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    R acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) acc[i][jj] = R(0);
    for (int k0 = 0; k0 < N; k0 += TK) {
        // A tile: 64 rows x 16 k
        for (int e = threadIdx.x; e < TM * TK; e += blockDim.x) {
            const int r = e / TK, kk = e - r * TK;
            const int q = tm * TM + r, k = k0 + kk;
            R v = R(0);
            if (q < M && k < N) v = A[static_cast<size_t>(q) * NN + k] * zg * static_cast<R>(Zf[k]);
            As[kk][r] = v;
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
    R* Y = args.Y[kind] + static_cast<size_t>(f) * M * NN;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int q = tm * TM + ty * 4 + i;
        if (q >= M) continue;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int n = tn * TN + tx * 4 + jj;
            if (n >= N) continue;
            const size_t o = kind == 0 ? static_cast<size_t>(q) * NN + grp * N + n
                                       : static_cast<size_t>(q) * NN + n * N + grp;
            Y[o] = acc[i][jj];
        }
    }
}

// ------------------------------------------------------------------------------------
// Phase 2b: one thread per output (a,b,c); all three channels.
// ------------------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(kThreads) k_contract(DevGeom g, const FlowState* fs,
                                                       const R* v0, const R* y1, const R* y2,
                                                       const R* y3, const R* y4, R* K,
                                                       unsigned ch) {
    const int f = blockIdx.y;
    if (!running(fs, f)) return;
    const int N = g.N, NN = g.NN;
    const size_t N3 = static_cast<size_t>(NN) * N;
    const size_t o = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
    if (o >= N3) return;
    const int a = static_cast<int>(o / NN);
    const int b = static_cast<int>((o / N) % N);
    const int c = static_cast<int>(o % N);
    const R* V = v0 + f * N3;
    R s = R(0);
    if (ch & FM_CH_PP) {
        const R* Y = y1 + (static_cast<size_t>(f) * g.nP + g.map_pp[a * N + b]) * NN;
        const R* Vab = V + static_cast<size_t>(a) * NN + b * N;
        R t = R(0);
        for (int x = 0; x < N; ++x) t += Vab[x] * Y[x * N + c];
        s -= t;
    }
    if (ch & FM_CH_CR) {
        const R* Y = y2 + (static_cast<size_t>(f) * g.nD + g.map_cr[b * N + c]) * NN + a * N;
        R t = R(0);
        for (int x = 0; x < N; ++x) t += Y[x] * V[static_cast<size_t>(x) * NN + b * N + c];
        s += t;
    }
    if (ch & FM_CH_D) {
        const size_t qo = (static_cast<size_t>(f) * g.nD + g.map_d[a * N + c]) * NN + b * N;
        const R* Y3 = y3 + qo;
        const R* Y4 = y4 + qo;
        R t = R(0);
        for (int x = 0; x < N; ++x) {
            const R vaxc = V[static_cast<size_t>(a) * NN + x * N + c];
            const R vxac = V[static_cast<size_t>(x) * NN + a * N + c];
            t += (vxac - R(2) * vaxc) * Y3[x] + vaxc * Y4[x];
        }
        s += t;
    }
    K[f * N3 + o] = s;
}

// ------------------------------------------------------------------------------------
// Direct double-precision path.
// ------------------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) k_wtable(DevGeom g, const FlowState* fs,
                                                     const double* T_stage,
                                                     const double* Z_stage, double* W) {
    const int f = blockIdx.z;
    if (!running(fs, f)) return;
    const int q = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.np) return;
    const bool pp = q < g.nP;
    const int m = pp ? g.q_pp[q] : g.q_ph[q - g.nP];
    const int jp = pp ? partner_pp(m, j, g.L) : partner_ph(m, j, g.L);
    const double T = T_stage[f];
    const double a = g.xi[j] / (2.0 * T);
    double b = g.xi[jp] / (2.0 * T);
    if (pp) b = -b;
    const double w = -phi_dd<double>(a, phi_d(a), b, phi_d(b)) / (4.0 * T * g.np);
    const double* Z = Z_stage + static_cast<size_t>(f) * g.N;
    W[(static_cast<size_t>(f) * (g.nP + g.nD) + q) * g.np + j] = Z[g.patch[j]] * Z[g.patch[jp]] * w;
}

__global__ void __launch_bounds__(kThreads) k_direct(DevGeom g, const FlowState* fs,
                                                     const double* W, const double* v0,
                                                     double* K, unsigned ch) {
    const int f = blockIdx.y;
    if (!running(fs, f)) return;
    const int N = g.N, NN = g.NN, L = g.L, np = g.np;
    const int a = blockIdx.x / N, b = blockIdx.x - (blockIdx.x / N) * N;
    const int c = threadIdx.x;
    if (c >= N) return;
    const size_t N3 = static_cast<size_t>(NN) * N;
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
    K[f * N3 + static_cast<size_t>(a) * NN + b * N + c] = -s1 + s2 + s3;
}

// ------------------------------------------------------------------------------------
// Integrator kernels (double precision).
// ------------------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(kThreads) k_to_f64(const FlowState* fs, const R* K, double* out,
                                                     size_t N3) {
    const int f = blockIdx.y;
    if (!running(fs, f)) return;
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < N3;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        out[f * N3 + i] = static_cast<double>(K[f * N3 + i]);
}

__global__ void __launch_bounds__(kThreads) k_fill_u(double* V, const double* U, size_t N3) {
    const int f = blockIdx.y;
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < N3;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        V[f * N3 + i] = U[f];
}

__device__ inline double block_max(double v) {
    __shared__ double red[kThreads / 64];
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
__global__ void __launch_bounds__(kThreads) k_rk4_update(const FlowState* fs, const R* K,
                                                         double* V, double* part, int nblk,
                                                         size_t N3, int B) {
    const int f = blockIdx.y;
    if (!running(fs, f)) return;
    const double h = fs[f].ht;
    double mx = 0.0;
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < N3;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        const double k0 = K[(0 * static_cast<size_t>(B) + f) * N3 + i];
        const double k1 = K[(1 * static_cast<size_t>(B) + f) * N3 + i];
        const double k2 = K[(2 * static_cast<size_t>(B) + f) * N3 + i];
        const double k3 = K[(3 * static_cast<size_t>(B) + f) * N3 + i];
        const double v = V[f * N3 + i] + h / 6.0 * (k0 + 2.0 * k1 + 2.0 * k2 + k3);
        V[f * N3 + i] = v;
        mx = fmax(mx, isfinite(v) ? fabs(v) : INFINITY);
    }
    mx = block_max(mx);
    if (threadIdx.x == 0) {
        part[(static_cast<size_t>(f) * nblk + blockIdx.x) * 2] = mx;
        part[(static_cast<size_t>(f) * nblk + blockIdx.x) * 2 + 1] = mx;
    }
}

// Dormand-Prince error norm max_i |h sum_l e_l k_l| / (atol + rtol max(|V|, |Vnew|)) and
// max|Vnew|; inf when anything is non-finite.
template <typename R>
__global__ void __launch_bounds__(kThreads) k_dopri_err(const FlowState* fs, const R* K,
                                                        const double* V, const double* Vnew,
                                                        double rtol, ErrWeights ew,
                                                        double* part, int nblk, size_t N3,
                                                        int B) {
    const int f = blockIdx.y;
    if (!running(fs, f)) return;
    const double h = fs[f].ht;
    const double at = fs[f].atol;
    double emax = 0.0, vmax = 0.0;
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < N3;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        double e = 0.0;
        for (int l = 0; l < 7; ++l) e += ew.e[l] * static_cast<double>(K[(static_cast<size_t>(l) * B + f) * N3 + i]);
        e = fabs(h * e);
        const double vn = Vnew[f * N3 + i];
        const double sc = at + rtol * fmax(fabs(V[f * N3 + i]), fabs(vn));
        const double r = e / sc;
        if (!isfinite(r) || !isfinite(vn)) { emax = INFINITY; vmax = INFINITY; }
        else { emax = fmax(emax, r); vmax = fmax(vmax, fabs(vn)); }
    }
    emax = block_max(emax);
    vmax = block_max(vmax);
    if (threadIdx.x == 0) {
        part[(static_cast<size_t>(f) * nblk + blockIdx.x) * 2] = emax;
        part[(static_cast<size_t>(f) * nblk + blockIdx.x) * 2 + 1] = vmax;
    }
}

__device__ inline double step_factor(double err) {
    if (err == 0.0) return 5.0;
    return fmin(5.0, fmax(0.2, 0.9 * pow(err, -0.2)));
}

// Accept/reject, stop rule and the next attempted step, one workgroup per flow.
__global__ void __launch_bounds__(kThreads) k_finish(FlowState* fs, const double* part, int nblk,
                                                     int rk45, double v_max, int fixed_steps) {
    const int f = blockIdx.x;
    const bool run = fs[f].status == FM_FLOW_RUNNING;
    double e = 0.0, mv = 0.0;
    if (run)
        for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
            e = fmax(e, part[(static_cast<size_t>(f) * nblk + i) * 2]);
            mv = fmax(mv, part[(static_cast<size_t>(f) * nblk + i) * 2 + 1]);
        }
    e = block_max(e);
    mv = block_max(mv);
    if (threadIdx.x != 0) return;
    FlowState st = fs[f];
    if (!run) { st.accepted = 0; fs[f] = st; return; }
    const double s = st.lnT, ht = st.ht;
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
            st.lnTc = (st.m > 0.0 && mv != st.m)
                          ? s + (log(v_max) - log(st.m)) * (s_new - s) / (log(mv) - log(st.m))
                          : s_new;
        }
        st.lnT = s_new;
        st.m = mv;
        if (st.status == FM_FLOW_RUNNING && fixed_steps > 0 && st.n_acc >= fixed_steps)
            st.status = FM_FLOW_REACHED_TEND;
    } else {
        st.err = e;
        st.n_rhs += 6;
        if (e <= 1.0) {
            const double s_new = last ? st.lnT_end : s + ht;
            st.accepted = 1;
            st.n_acc += 1;
            if (mv > v_max) {
                st.status = FM_FLOW_DIVERGED;
                st.lnTc = (st.m > 0.0 && mv != st.m)
                              ? s + (log(v_max) - log(st.m)) * (s_new - s) / (log(mv) - log(st.m))
                              : s_new;
            }
            st.lnT = s_new;
            st.m = mv;
            st.h = ht * step_factor(e);
        } else {
            st.accepted = 0;
            st.n_rej += 1;
            st.h = isfinite(e) ? ht * step_factor(e) : 0.5 * ht;
        }
        if (st.status == FM_FLOW_RUNNING && st.lnT <= st.lnT_end) st.status = FM_FLOW_REACHED_TEND;
        if (st.status == FM_FLOW_RUNNING && fabs(st.h) < st.hmin) st.status = FM_FLOW_STEPFAIL;
        st.ht = (st.lnT + st.h <= st.lnT_end) ? st.lnT_end - st.lnT : st.h;
    }
    fs[f] = st;
}

// After an accepted Dormand-Prince step: V = Vnew and k0 = k6 (first same as last).
template <typename R>
__global__ void __launch_bounds__(kThreads) k_commit(const FlowState* fs, double* V,
                                                     const double* Vnew, R* K, size_t N3, int B) {
    const int f = blockIdx.y;
    if (!fs[f].accepted) return;
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < N3;
         i += static_cast<size_t>(gridDim.x) * blockDim.x) {
        V[f * N3 + i] = Vnew[f * N3 + i];
        K[static_cast<size_t>(f) * N3 + i] = K[(6 * static_cast<size_t>(B) + f) * N3 + i];
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
R* kslot_ptr(const Buffers& b, int slot, size_t N3) {
    return static_cast<R*>(b.k) + static_cast<size_t>(slot) * b.bstride * N3;
}

template <typename R>
void stage_t(hipStream_t s, const DevGeom& g, const DevZ& z, const Buffers& b, int nf,
             const StageCoef& sc, int write_new, const double* Vbase) {
    const size_t N3 = static_cast<size_t>(g.NN) * g.N;
    hipLaunchKernelGGL(k_stage<R>, grid_for(N3, nf), dim3(kThreads), 0, s, g, z, b.fs, sc,
                       write_new, Vbase, static_cast<const R*>(b.k), b.Vnew,
                       static_cast<R*>(b.v0), static_cast<R*>(b.va), static_cast<R*>(b.vc),
                       b.T_stage, b.Z_stage, b.bstride);
}

template <typename R>
void bins_t(hipStream_t s, const DevGeom& g, const Buffers& b, int nf) {
    hipLaunchKernelGGL(k_points<R>, dim3((g.np + kThreads - 1) / kThreads, nf), dim3(kThreads),
                       0, s, g, b.fs, b.T_stage, static_cast<R*>(b.pt));
    const size_t lds = static_cast<size_t>(g.NN) * sizeof(R);
    const dim3 grid(g.nP + g.nD, nf);
    if (lds <= 65536) {
        hipLaunchKernelGGL((k_bins<R, true>), grid, dim3(kThreads), lds, s, g, b.fs, b.T_stage,
                           static_cast<const R*>(b.pt), static_cast<R*>(b.bpp),
                           static_cast<R*>(b.bph), static_cast<R*>(b.bphT));
    } else {
        const size_t n1 = static_cast<size_t>(nf) * g.nP * g.NN;
        const size_t n2 = static_cast<size_t>(nf) * g.nD * g.NN;
        hipLaunchKernelGGL(k_zero<R>, dim3(4096), dim3(kThreads), 0, s, static_cast<R*>(b.bpp), n1);
        hipLaunchKernelGGL(k_zero<R>, dim3(4096), dim3(kThreads), 0, s, static_cast<R*>(b.bph), n2);
        hipLaunchKernelGGL((k_bins<R, false>), grid, dim3(kThreads), 0, s, g, b.fs, b.T_stage,
                           static_cast<const R*>(b.pt), static_cast<R*>(b.bpp),
                           static_cast<R*>(b.bph), static_cast<R*>(b.bphT));
        hipLaunchKernelGGL(k_transpose_bins<R>, dim3((g.NN + kThreads - 1) / kThreads, g.nD, nf),
                           dim3(kThreads), 0, s, g, b.fs, static_cast<const R*>(b.bph),
                           static_cast<R*>(b.bphT));
    }
}

template <typename R>
void y_t(hipStream_t s, const DevGeom& g, const Buffers& b, int nf, unsigned ch) {
    YArgs<R> a;
    a.A[0] = static_cast<const R*>(b.bpp);  a.Vs[0] = static_cast<const R*>(b.v0);
    a.A[1] = static_cast<const R*>(b.bphT); a.Vs[1] = static_cast<const R*>(b.vc);
    a.A[2] = static_cast<const R*>(b.bph);  a.Vs[2] = static_cast<const R*>(b.va);
    a.A[3] = static_cast<const R*>(b.bph);  a.Vs[3] = static_cast<const R*>(b.vc);
    a.Y[0] = static_cast<R*>(b.y1); a.Y[1] = static_cast<R*>(b.y2);
    a.Y[2] = static_cast<R*>(b.y3); a.Y[3] = static_cast<R*>(b.y4);
    a.M[0] = g.nP; a.M[1] = a.M[2] = a.M[3] = g.nD;
    a.on[0] = (ch & FM_CH_PP) != 0;
    a.on[1] = (ch & FM_CH_CR) != 0;
    a.on[2] = a.on[3] = (ch & FM_CH_D) != 0;
    const int mmax = g.nP > g.nD ? g.nP : g.nD;
    const int tiles = ((mmax + 63) / 64) * ((g.N + 63) / 64);
    hipLaunchKernelGGL(k_y<R>, dim3(tiles, g.N, 4 * nf), dim3(kThreads), 0, s, g, b.fs,
                       b.Z_stage, a, nf);
}

template <typename R>
void contract_t(hipStream_t s, const DevGeom& g, const Buffers& b, int nf, unsigned ch, int slot) {
    const size_t N3 = static_cast<size_t>(g.NN) * g.N;
    hipLaunchKernelGGL(k_contract<R>, dim3((N3 + kThreads - 1) / kThreads, nf), dim3(kThreads),
                       0, s, g, b.fs, static_cast<const R*>(b.v0), static_cast<const R*>(b.y1),
                       static_cast<const R*>(b.y2), static_cast<const R*>(b.y3),
                       static_cast<const R*>(b.y4), kslot_ptr<R>(b, slot, N3), ch);
}

}  // namespace

void launch_stage(hipStream_t s, bool dbl, const DevGeom& g, const DevZ& z, const Buffers& b,
                  int nf, const StageCoef& sc, int write_new, const double* Vbase) {
    if (dbl) stage_t<double>(s, g, z, b, nf, sc, write_new, Vbase);
    else stage_t<float>(s, g, z, b, nf, sc, write_new, Vbase);
}

void launch_bins(hipStream_t s, bool dbl, const DevGeom& g, const Buffers& b, int nf) {
    if (dbl) bins_t<double>(s, g, b, nf);
    else bins_t<float>(s, g, b, nf);
}

void launch_y(hipStream_t s, bool dbl, const DevGeom& g, const Buffers& b, int nf, unsigned ch) {
    if (dbl) y_t<double>(s, g, b, nf, ch);
    else y_t<float>(s, g, b, nf, ch);
}

void launch_contract(hipStream_t s, bool dbl, const DevGeom& g, const Buffers& b, int nf,
                     unsigned ch, int slot) {
    if (dbl) contract_t<double>(s, g, b, nf, ch, slot);
    else contract_t<float>(s, g, b, nf, ch, slot);
}

void launch_wtable(hipStream_t s, const DevGeom& g, const Buffers& b, int nf) {
    hipLaunchKernelGGL(k_wtable, dim3((g.np + kThreads - 1) / kThreads, g.nP + g.nD, nf),
                       dim3(kThreads), 0, s, g, b.fs, b.T_stage, b.Z_stage, b.wtab);
}

void launch_direct(hipStream_t s, const DevGeom& g, const Buffers& b, int nf, unsigned ch,
                   int slot) {
    const size_t N3 = static_cast<size_t>(g.NN) * g.N;
    const int threads = ((g.N + 63) / 64) * 64;
    hipLaunchKernelGGL(k_direct, dim3(g.NN, nf), dim3(threads), 0, s, g, b.fs, b.wtab,
                       static_cast<const double*>(b.v0), kslot_ptr<double>(b, slot, N3), ch);
}

void launch_k_to_f64(hipStream_t s, bool dbl, const Buffers& b, int nf, size_t N3, int slot,
                     double* out) {
    if (dbl)
        hipLaunchKernelGGL(k_to_f64<double>, grid_for(N3, nf), dim3(kThreads), 0, s, b.fs,
                           kslot_ptr<double>(b, slot, N3), out, N3);
    else
        hipLaunchKernelGGL(k_to_f64<float>, grid_for(N3, nf), dim3(kThreads), 0, s, b.fs,
                           kslot_ptr<float>(b, slot, N3), out, N3);
}

void launch_fill_u(hipStream_t s, const Buffers& b, int nf, size_t N3, const double* U) {
    hipLaunchKernelGGL(k_fill_u, grid_for(N3, nf), dim3(kThreads), 0, s, b.V, U, N3);
}

void launch_rk4_update(hipStream_t s, bool dbl, const Buffers& b, int nf, size_t N3, double* V) {
    const dim3 grid(b.nblk, nf);
    if (dbl)
        hipLaunchKernelGGL(k_rk4_update<double>, grid, dim3(kThreads), 0, s, b.fs,
                           static_cast<const double*>(b.k), V, b.part, b.nblk, N3, b.bstride);
    else
        hipLaunchKernelGGL(k_rk4_update<float>, grid, dim3(kThreads), 0, s, b.fs,
                           static_cast<const float*>(b.k), V, b.part, b.nblk, N3, b.bstride);
}

void launch_dopri_err(hipStream_t s, bool dbl, const Buffers& b, int nf, size_t N3,
                      const double* V, double rtol, const ErrWeights& ew) {
    const dim3 grid(b.nblk, nf);
    if (dbl)
        hipLaunchKernelGGL(k_dopri_err<double>, grid, dim3(kThreads), 0, s, b.fs,
                           static_cast<const double*>(b.k), V, b.Vnew, rtol, ew, b.part, b.nblk,
                           N3, b.bstride);
    else
        hipLaunchKernelGGL(k_dopri_err<float>, grid, dim3(kThreads), 0, s, b.fs,
                           static_cast<const float*>(b.k), V, b.Vnew, rtol, ew, b.part, b.nblk,
                           N3, b.bstride);
}

void launch_finish(hipStream_t s, const Buffers& b, int nf, int rk45, double v_max,
                   int fixed_steps, double h_fixed) {
    (void)h_fixed;
    hipLaunchKernelGGL(k_finish, dim3(nf), dim3(kThreads), 0, s, b.fs, b.part, b.nblk, rk45,
                       v_max, fixed_steps);
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
