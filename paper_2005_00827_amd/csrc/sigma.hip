// gfx950 kernels of the quasi-particle weight provider: the second-order self-energy on the
// real axis at each patch's representative point, its real part by Kramers-Kronig, and Z from
// the slope of the real part outside the window of inverted slope (Sec. 3.1; App. A,
// Eq. definition_Z).
//
//   Im Sigma(w, k) = -pi (1/L^4) sum_{p1,p3} W F delta(w + xi(p1) - xi(p2) - xi(p3)),
//   p2 = k + p1 - p3 (off the loop grid, its energy evaluated exactly),
//   F = f1 (1 - f2)(1 - f3) + (1 - f1) f2 f3,
//   W = U^2 (bare), or V(a,b,c)^2 + (V(a,b,c) - V(b,a,c))^2 / 2 with a, b, c the patches of
//       k, p1, p3 (the static vertex summed over spins; U^2 for V = U),
// with the delta function shared linearly between the two nearest nodes of a uniform grid of
// kSigmaW frequencies on [-W0, W0].
#include <hip/hip_runtime.h>

#include <cmath>

#include "fm_internal.h"

namespace fm {
namespace {

constexpr int kSigThreads = 256;

__device__ inline double fermi_d(double x, double T) { return 0.5 * (1.0 - tanh(0.5 * x / T)); }

// One block per (patch a, run of kSigThreads hole points p1); each thread sums over every
// particle point p3 for its p1 and spreads its terms into the block's histogram in LDS, which
// the block then adds to the patch's histogram in global memory.  cos and sin of k + p1 - p3
// come from angle addition with per-block tables of the grid differences.
__global__ void __launch_bounds__(kSigThreads) k_sigma_hist(SigmaArgs s, const double* V,
                                                            double* hist) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* h = reinterpret_cast<double*>(smem_raw);            // [kSigmaW]
    double* cd = h + kSigmaW;                                    // [L] cos(2 pi d / L)
    double* sd = cd + s.L;                                       // [L]
    const int a = blockIdx.y, L = s.L, np = L * L, N = s.N;
    for (int i = threadIdx.x; i < kSigmaW; i += blockDim.x) h[i] = 0.0;
    for (int d = threadIdx.x; d < L; d += blockDim.x) {
        const double ang = 2.0 * M_PI * d / L;
        cd[d] = cos(ang);
        sd[d] = sin(ang);
    }
    __syncthreads();
    const double kx = s.kpt[2 * a], ky = s.kpt[2 * a + 1];
    const double ckx = cos(kx), skx = sin(kx), cky = cos(ky), sky = sin(ky);
    const int j1 = blockIdx.x * blockDim.x + threadIdx.x;
    if (j1 < np) {
        const int j1x = j1 % L, j1y = j1 / L;
        const double x1 = s.xi[j1], f1 = fermi_d(x1, s.T);
        const int b = s.patch[j1];
        const double inv = 1.0 / s.dw;
        for (int j3 = 0; j3 < np; ++j3) {
            const int j3x = j3 % L, j3y = j3 / L;
            // k + p1 - p3 = k + 2 pi (j1 - j3) / L per axis
            const int dx = (j1x - j3x + L) % L, dy = (j1y - j3y + L) % L;
            const double cx = ckx * cd[dx] - skx * sd[dx];
            const double cy = cky * cd[dy] - sky * sd[dy];
            const double x2 = -2.0 * s.t * (cx + cy) - 4.0 * s.tp * cx * cy - s.mu;
            const double x3 = s.xi[j3];
            const double f2 = fermi_d(x2, s.T), f3 = s.f[j3];
            const double F = f1 * (1.0 - f2) * (1.0 - f3) + (1.0 - f1) * f2 * f3;
            double W = s.U * s.U;
            if (V) {
                const int c = s.patch[j3];
                const double v = V[(static_cast<size_t>(a) * N + b) * N + c];
                const double vx = V[(static_cast<size_t>(b) * N + a) * N + c];
                W = v * v + 0.5 * (v - vx) * (v - vx);
            }
            const double x = (x2 + x3 - x1 + s.w0) * inv;   // inside (0, kSigmaW - 1) by W0
            const int i = min(max(static_cast<int>(floor(x)), 0), kSigmaW - 2);
            const double fr = x - i, wt = W * F;
            atomicAdd(&h[i], (1.0 - fr) * wt);
            atomicAdd(&h[i + 1], fr * wt);
        }
    }
    __syncthreads();
    double* hg = hist + static_cast<size_t>(a) * kSigmaW;
    for (int i = threadIdx.x; i < kSigmaW; i += blockDim.x)
        if (h[i] != 0.0) atomicAdd(&hg[i], h[i]);
}

// Per patch: Im Sigma from the histogram, Re Sigma by the principal-value Kramers-Kronig
// integral of the piecewise-linear Im Sigma (closed form per interval; the two intervals
// touching w cancel their logarithms), and Z = 1/(1 - s), s the least-squares slope of
// Re Sigma over the nodes with 2T <= |w| <= 4T (NaN below 8 such nodes).  One block per patch.
__global__ void __launch_bounds__(kSigThreads) k_sigma_finish(SigmaArgs s, const double* hist,
                                                              double* im, double* re,
                                                              double* Z) {
    __shared__ double sim[kSigmaW];
    __shared__ double red[5][kSigThreads / 64];
    const int a = blockIdx.x, np = s.L * s.L;
    const double norm = -M_PI / (static_cast<double>(np) * np * s.dw);
    for (int i = threadIdx.x; i < kSigmaW; i += blockDim.x) {
        sim[i] = norm * hist[static_cast<size_t>(a) * kSigmaW + i];
        im[static_cast<size_t>(a) * kSigmaW + i] = sim[i];
    }
    __syncthreads();
    double sx = 0.0, sy = 0.0, sxx = 0.0, sxy = 0.0, cnt = 0.0;
    for (int i = threadIdx.x; i < kSigmaW; i += blockDim.x) {
        const double w = -s.w0 + s.dw * i;
        double acc = 0.0;
        for (int j = 0; j + 1 < kSigmaW; ++j) {
            const double x0 = -s.w0 + s.dw * j, x1 = x0 + s.dw;
            const double sl = (sim[j + 1] - sim[j]) / s.dw;
            acc -= sl * s.dw;
            if (j != i && j + 1 != i)
                acc += (sim[j] + sl * (w - x0)) * log(fabs((w - x0) / (w - x1)));
        }
        const double r = -acc / M_PI;
        re[static_cast<size_t>(a) * kSigmaW + i] = r;
        if (fabs(w) >= 2.0 * s.T && fabs(w) <= 4.0 * s.T) {
            sx += w; sy += r; sxx += w * w; sxy += w * r; cnt += 1.0;
        }
    }
    double v[5] = {sx, sy, sxx, sxy, cnt};
    for (int k = 0; k < 5; ++k) {
        double x = v[k];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x / 64] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < 5; ++k) {
            double x = 0.0;
            for (int w = 0; w < static_cast<int>(blockDim.x / 64); ++w) x += red[k][w];
            v[k] = x;
        }
        const double n = v[4];
        const double slope = (n * v[3] - v[0] * v[1]) / (n * v[2] - v[0] * v[0]);
        Z[a] = n >= 8.0 ? 1.0 / (1.0 - slope) : NAN;   // an unresolved slope: no Z
    }
}

__global__ void __launch_bounds__(kSigThreads) k_sigma_fermi(SigmaArgs s) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < s.L * s.L) s.f[j] = fermi_d(s.xi[j], s.T);
}

}  // namespace

void launch_sigma(hipStream_t st, const SigmaArgs& s, const double* V, double* hist, double* im,
                  double* re, double* Z) {
    const int np = s.L * s.L;
    (void)hipMemsetAsync(hist, 0, sizeof(double) * kSigmaW * s.N, st);
    hipLaunchKernelGGL(k_sigma_fermi, dim3((np + kSigThreads - 1) / kSigThreads), dim3(kSigThreads),
                       0, st, s);
    const size_t lds = sizeof(double) * (kSigmaW + 2 * static_cast<size_t>(s.L));
    hipLaunchKernelGGL(k_sigma_hist, dim3((np + kSigThreads - 1) / kSigThreads, s.N),
                       dim3(kSigThreads), lds, st, s, V, hist);
    hipLaunchKernelGGL(k_sigma_finish, dim3(s.N), dim3(kSigThreads), 0, st, s, hist, im, re, Z);
}

}  // namespace fm
