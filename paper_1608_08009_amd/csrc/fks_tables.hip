// Device FP64 build of the kernel-mode tables (Section 3.3).
//
// For every convolution term j = (direction e, radial term r) and every
// half-spectrum wavenumber k = (kx, ky, kz), kz in [0, n/2]:
//   tab[j][k] = (omega_e * phi_r(kappa k.e), psi_r(kappa |k - (k.e) e|)),
// omega_e = 4 C_gamma w_e (eq. Btilde in 3D times the sphere weight).  The last
// term is the loss: L(k) = sum_j omega_j alpha_j(k) beta_j(k) = B_F(k, k)
// (eq. ode) stored as (-L(k), 1), so that every term contributes
// Re(z) * Im(z) with z = F^{-1}[(a + i b) fhat].
// Hard spheres: phi(s) = R^2 [2 Sinc(Rs) - Sinc^2(Rs/2)], psi(s) = 2 pi R J1(Rs)/s.
// Other gamma: phi_r(s) = 2 sum_i c_ir cos(rho_i s), psi_r(s) = 2 pi sum_i c_ir J0(rho_i s).
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "fks_internal.hpp"

namespace fks {
namespace {

constexpr double kPiD = 3.141592653589793238462643383279502884;

__device__ inline int signed_k(int i, int n) { return i < n / 2 ? i : i - n; }

__device__ inline double sinc(double x) {
    return fabs(x) < 1e-8 ? 1.0 - x * x / 6.0 : sin(x) / x;
}

// one thread per (half-spectrum point, direction); writes all K radial terms
__global__ void k_term_tables(double* __restrict__ tab64, const double* __restrict__ dirs, int M, int K,
                              const double* __restrict__ rnodes, const double* __restrict__ rcoef, int nq,
                              int n, int H, double kappa, double R, double c4) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)H * M) return;
    int d = (int)(t / H);
    int h = (int)(t - (long long)d * H);
    int ky = h % n, kx = (h / n) % n, kz = h / (n * n);
    double k1 = signed_k(kx, n), k2 = signed_k(ky, n), k3 = kz;   // kz <= n/2 (half spectrum)
    double ex = dirs[4 * d + 0], ey = dirs[4 * d + 1], ez = dirs[4 * d + 2], w = dirs[4 * d + 3];
    double kd = k1 * ex + k2 * ey + k3 * ez;
    double kk = k1 * k1 + k2 * k2 + k3 * k3;
    double kp = sqrt(fmax(kk - kd * kd, 0.0));
    double s1 = kappa * kd, s2 = kappa * kp;
    double om = c4 * w;
    if (nq == 0) {
        double a = R * R * (2.0 * sinc(R * s1) - sinc(0.5 * R * s1) * sinc(0.5 * R * s1));
        double b = (s2 < 1e-12) ? kPiD * R * R : 2.0 * kPiD * R * j1(R * s2) / s2;
        size_t o = ((size_t)d * H + h) * 2;
        tab64[o] = om * a;
        tab64[o + 1] = b;
        return;
    }
    // general gamma: K radial terms at once
    double a[64], b[64];
    for (int r = 0; r < K; ++r) { a[r] = 0.0; b[r] = 0.0; }
    for (int i = 0; i < nq; ++i) {
        double c1 = cos(rnodes[i] * s1);
        double c2 = j0(rnodes[i] * s2);
        const double* cr = rcoef + (size_t)i * K;
        for (int r = 0; r < K; ++r) {
            a[r] = fma(cr[r], c1, a[r]);
            b[r] = fma(cr[r], c2, b[r]);
        }
    }
    for (int r = 0; r < K; ++r) {
        size_t o = ((size_t)(d * K + r) * H + h) * 2;
        tab64[o] = om * 2.0 * a[r];
        tab64[o + 1] = 2.0 * kPiD * b[r];
    }
}

// loss term L(k) = sum_j omega_j alpha_j(k) beta_j(k), summed in term order j = 0..J-2
__global__ void k_loss(double* __restrict__ tab64, int J, int H) {
    int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= H) return;
    double L = 0.0;
    for (int j = 0; j < J - 1; ++j) {
        size_t o = ((size_t)j * H + h) * 2;
        L = fma(tab64[o], tab64[o + 1], L);
    }
    size_t o = ((size_t)(J - 1) * H + h) * 2;
    tab64[o] = -L;
    tab64[o + 1] = 1.0;
}

// FP32 copy with balanced pairs (s_j a, b / s_j): the product a b, which is all
// the operator uses, is unchanged, while the real and imaginary parts of each
// packed inverse transform get comparable magnitudes, so that FP32 rounding
// of the larger one does not swamp the smaller.  Gain terms use
// s_j = sqrt(pi / omega_j) (|psi(0)| = pi |phi(0)|); the loss term uses
// s = 1/sqrt(L(0)) with L(0) = max |L|.
__global__ void k_round(const double* __restrict__ tab64, float* __restrict__ tab32,
                        const double* __restrict__ gain_scale, int J, int H) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)J * H) return;
    int j = (int)(t / H);
    double s = (j < J - 1) ? gain_scale[j] : 1.0 / sqrt(-tab64[(size_t)(J - 1) * H * 2]);
    size_t o = (size_t)t * 2;
    tab32[o] = (float)(tab64[o] * s);
    tab32[o + 1] = (float)(tab64[o + 1] / s);
}

// The FP32 table's planes kz < n/2 regrouped for the fused kernels: complex element
// (j, kz, kx, ky) goes to ((j (n/4) + kz/2) n^2 + kx n + ky) 2 + kz % 2, so that the two
// planes of a kz pair sit side by side and one 16-byte load reads both.
__global__ void k_pairs(const float2* __restrict__ tab32, float2* __restrict__ tab32p, int J, int n, int H) {
    const long long nn = (long long)n * n;
    const long long per_term = (long long)(n / 2) * nn;
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long long)J * per_term) return;
    const int j = (int)(t / per_term);
    const long long r = t - j * per_term;           // r = (m nn + kxy) 2 + s
    const int s = (int)(r & 1);
    const long long m = (r >> 1) / nn, kxy = (r >> 1) - m * nn;
    tab32p[t] = tab32[(long long)j * H + (2 * m + s) * nn + kxy];
}

}  // namespace

hipError_t build_tables(fks_plan* p, hipStream_t stream) {
    const int nq = (int)p->rad_nodes.size();
    if (nq > 0 && p->K > 64) return hipErrorInvalidValue;
    double* d_dirs = nullptr;
    double* d_nodes = nullptr;
    double* d_coef = nullptr;
    hipError_t e = hipMalloc(&d_dirs, p->dirs.size() * sizeof(double));
    if (e != hipSuccess) return e;
    e = hipMemcpy(d_dirs, p->dirs.data(), p->dirs.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess && nq > 0) {
        e = hipMalloc(&d_nodes, nq * sizeof(double));
        if (e == hipSuccess) e = hipMalloc(&d_coef, p->rad_coef.size() * sizeof(double));
        if (e == hipSuccess)
            e = hipMemcpy(d_nodes, p->rad_nodes.data(), nq * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(d_coef, p->rad_coef.data(), p->rad_coef.size() * sizeof(double),
                          hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) {
        long long total = (long long)p->H * p->M;
        int bs = 256;
        unsigned grid = (unsigned)((total + bs - 1) / bs);
        k_term_tables<<<grid, bs, 0, stream>>>(p->d_tab64, d_dirs, p->M, p->K, d_nodes, d_coef, nq, p->desc.n,
                                               p->H, p->kappa, p->desc.R, 4.0 * p->desc.c_gamma);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        int bs = 256;
        k_loss<<<(p->H + bs - 1) / bs, bs, 0, stream>>>(p->d_tab64, p->J, p->H);
        e = hipGetLastError();
    }
    double* d_scale = nullptr;
    if (e == hipSuccess && p->d_tab32) {
        std::vector<double> sc((size_t)p->J - 1);
        for (int d = 0; d < p->M; ++d)
            for (int r = 0; r < p->K; ++r)
                sc[(size_t)d * p->K + r] = std::sqrt(kPiD / (4.0 * p->desc.c_gamma * p->dirs[4 * d + 3]));
        e = hipMalloc(&d_scale, sc.size() * sizeof(double));
        if (e == hipSuccess)
            e = hipMemcpy(d_scale, sc.data(), sc.size() * sizeof(double), hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            long long total = (long long)p->J * p->H;
            int bs = 256;
            k_round<<<(unsigned)((total + bs - 1) / bs), bs, 0, stream>>>(p->d_tab64, p->d_tab32, d_scale, p->J,
                                                                          p->H);
            e = hipGetLastError();
        }
        if (e == hipSuccess && p->d_tab32p) {
            const int n = p->desc.n;
            long long total = (long long)p->J * (n / 2) * n * n;
            int bs = 256;
            k_pairs<<<(unsigned)((total + bs - 1) / bs), bs, 0, stream>>>(
                reinterpret_cast<const float2*>(p->d_tab32), reinterpret_cast<float2*>(p->d_tab32p), p->J, n, p->H);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (d_dirs) (void)hipFree(d_dirs);
    if (d_nodes) (void)hipFree(d_nodes);
    if (d_coef) (void)hipFree(d_coef);
    if (d_scale) (void)hipFree(d_scale);
    return e;
}

}  // namespace fks
