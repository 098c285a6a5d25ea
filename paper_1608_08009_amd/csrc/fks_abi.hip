// C ABI, argument validation and host-side FP64 precompute of the plan.
//
// Host precompute (Section 3.3): half-sphere directions and weights, the
// separable radial expansion of the VHS Carleman kernel, and the Gram matrix
// of the collision invariants (Section 3.2).  The kernel-mode tables
// themselves are built on the device (fks_tables.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "fks_internal.hpp"

namespace fks {

namespace {
constexpr double kPi = 3.141592653589793238462643383279502884;

bool is_finite(double x) { return std::isfinite(x); }
}  // namespace

bool supported_n(int n) {
    if (n < 4 || n > 48 || (n % 2) != 0) return false;
    int m = n;
    while (m % 2 == 0) m /= 2;
    while (m % 3 == 0) m /= 3;
    return m == 1;
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n (long double).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        long double z = cosl(pi * (i + 0.75L) / (n + 0.5L));
        long double pp = 0;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1; }
            pp = n * (z * p1 - p0) / (z * z - 1);   // P_n'(z)
            long double dz = p1 / pp;
            z -= dz;
            if (fabsl(dz) < 1e-19L) break;
        }
        {   // derivative at the converged node
            long double p0 = 1, p1 = z;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1; }
            pp = n * (z * p1 - p0) / (z * z - 1);
        }
        long double wi = 2 / ((1 - z * z) * pp * pp);
        x[i] = (double)(-z);          // ascending order
        x[n - 1 - i] = (double)z;
        w[i] = w[n - 1 - i] = (double)wi;
    }
}

namespace {

// Cyclic Jacobi eigen-decomposition of a symmetric matrix a[n][n] (destroyed).
// Returns eigenvalues in lam and eigenvectors as columns of v[n][n].
void jacobi_eigen(int n, std::vector<double>& a, std::vector<double>& lam, std::vector<double>& v) {
    v.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int p = 0; p < n; ++p) {
            diag += a[(size_t)p * n + p] * a[(size_t)p * n + p];
            for (int q = p + 1; q < n; ++q) off += a[(size_t)p * n + q] * a[(size_t)p * n + q];
        }
        if (off <= 1e-32 * diag) break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                double apq = a[(size_t)p * n + q];
                if (apq == 0.0) continue;
                double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = c * akp - s * akq;
                    a[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = c * apk - s * aqk;
                    a[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = v[(size_t)k * n + p], vkq = v[(size_t)k * n + q];
                    v[(size_t)k * n + p] = c * vkp - s * vkq;
                    v[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = a[(size_t)i * n + i];
}

}  // namespace

// Separable expansion of k(rho, rho') = (rho^2 + rho'^2)^((gamma-1)/2) on [0,R]^2
// with the measure rho rho' d rho d rho' (Section 3.3, decoupling assumption
// eq. decoup, extended to K terms): nq graded Gauss-Legendre nodes rho = R u^2,
// symmetric matrix sqrt(w_i rho_i) k_ij sqrt(w_j rho_j), K leading eigenpairs.
// coef[i][r] = sqrt(w_i rho_i) U_ir sqrt(lambda_r).  Returns K.
int radial_expansion(double gamma, double R, int K, double tol, int nq, std::vector<double>& nodes,
                     std::vector<double>& coef) {
    std::vector<double> u, wu;
    gauss_legendre(nq, u, wu);
    nodes.assign(nq, 0.0);
    std::vector<double> sq(nq);
    for (int i = 0; i < nq; ++i) {
        double ui = 0.5 * (u[i] + 1.0), wi = 0.5 * wu[i];
        nodes[i] = R * ui * ui;
        double w = wi * 2.0 * R * ui;
        sq[i] = std::sqrt(w * nodes[i]);
    }
    std::vector<double> a((size_t)nq * nq);
    for (int i = 0; i < nq; ++i)
        for (int j = 0; j < nq; ++j) {
            double r2 = nodes[i] * nodes[i] + nodes[j] * nodes[j];
            a[(size_t)i * nq + j] = sq[i] * std::pow(r2, 0.5 * (gamma - 1.0)) * sq[j];
        }
    std::vector<double> lam, v;
    jacobi_eigen(nq, a, lam, v);
    std::vector<int> order(nq);
    for (int i = 0; i < nq; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int p, int q) { return lam[p] > lam[q]; });
    if (K <= 0) {
        K = nq;
        for (int r = 0; r < nq; ++r)
            if (lam[order[r]] / lam[order[0]] < tol) { K = r; break; }
        K = std::max(K, 1);
    }
    K = std::min(K, nq);
    coef.assign((size_t)nq * K, 0.0);
    for (int r = 0; r < K; ++r) {
        int c = order[r];
        double sl = std::sqrt(std::max(lam[c], 0.0));
        for (int i = 0; i < nq; ++i) coef[(size_t)i * K + r] = sq[i] * v[(size_t)i * nq + c] * sl;
    }
    return K;
}

// Half-sphere rule: theta over [0, pi] (Gauss-Legendre in cos theta or midpoint
// with the sin theta Jacobian), azimuth phi_q = q pi / n_azim.  p-major order.
static void sphere_rule(int n_polar, int n_azim, int rule, std::vector<double>& out) {
    std::vector<double> ct(n_polar), st(n_polar), wt(n_polar);
    if (rule == FKS_RULE_GAUSS) {
        std::vector<double> x, w;
        gauss_legendre(n_polar, x, w);
        for (int p = 0; p < n_polar; ++p) {
            ct[p] = x[p];
            st[p] = std::sqrt(std::max(0.0, 1.0 - x[p] * x[p]));
            wt[p] = w[p];
        }
    } else {
        for (int p = 0; p < n_polar; ++p) {
            double th = (p + 0.5) * kPi / n_polar;
            ct[p] = std::cos(th);
            st[p] = std::sin(th);
            wt[p] = st[p] * kPi / n_polar;
        }
    }
    out.assign((size_t)n_polar * n_azim * 4, 0.0);
    for (int p = 0; p < n_polar; ++p)
        for (int q = 0; q < n_azim; ++q) {
            double ph = q * kPi / n_azim;
            double* o = &out[((size_t)p * n_azim + q) * 4];
            o[0] = st[p] * std::cos(ph);
            o[1] = st[p] * std::sin(ph);
            o[2] = ct[p];
            o[3] = wt[p] * kPi / n_azim;
        }
}

// Gram matrix of the scaled invariants over the grid, inverted in long double.
GridConst grid_const(int n, double T) {
    GridConst g{};
    g.T = T;
    g.dv = 2.0 * T / n;
    // Gram matrix of the scaled basis (1, u, |u|^2), u = v/T, over the n^3 nodes.  The grid is
    // a tensor product, so every entry is a product of the 1D power sums S_k = sum_i u_i^k
    // (O(n) work: the n^3 triple loop cost about a millisecond of host time per call)
    long double S[5] = {};
    for (int i = 0; i < n; ++i) {
        const long double u = (-T + i * g.dv) / T;
        long double pw = 1.0L;
        for (int k = 0; k < 5; ++k) {
            S[k] += pw;
            pw *= u;
        }
    }
    const long double N = S[0];
    long double G[5][5] = {};
    G[0][0] = N * N * N;
    G[0][4] = G[4][0] = 3.0L * S[2] * N * N;                        // sum |u|^2
    G[4][4] = 3.0L * S[4] * N * N + 6.0L * S[2] * S[2] * N;         // sum |u|^4
    for (int a = 1; a <= 3; ++a) {
        G[0][a] = G[a][0] = S[1] * N * N;                           // sum u_a
        G[a][a] = S[2] * N * N;                                     // sum u_a^2
        G[a][4] = G[4][a] = S[3] * N * N + 2.0L * S[1] * S[2] * N;  // sum u_a |u|^2
        for (int b = 1; b <= 3; ++b)
            if (b != a) G[a][b] = S[1] * S[1] * N;                  // sum u_a u_b
    }
    long double A[5][10] = {};
    for (int a = 0; a < 5; ++a) {
        for (int b = 0; b < 5; ++b) A[a][b] = G[a][b];
        A[a][5 + a] = 1.0L;
    }
    for (int c = 0; c < 5; ++c) {
        int piv = c;
        for (int r = c + 1; r < 5; ++r)
            if (fabsl(A[r][c]) > fabsl(A[piv][c])) piv = r;
        for (int k = 0; k < 10; ++k) std::swap(A[c][k], A[piv][k]);
        long double d = A[c][c];
        for (int k = 0; k < 10; ++k) A[c][k] /= d;
        for (int r = 0; r < 5; ++r)
            if (r != c) {
                long double m = A[r][c];
                for (int k = 0; k < 10; ++k) A[r][k] -= m * A[c][k];
            }
    }
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b) g.ginv[a * 5 + b] = (double)A[a][5 + b];
    return g;
}

// Resolves defaults and checks ranges; used by fks_desc_validate and plan creation.
static fks_status resolve_desc(const fks_plan_desc* in, fks_plan_desc* out) {
    if (!in) return FKS_ERR_INVALID;
    fks_plan_desc d = *in;
    if (!is_finite(d.T) || d.T <= 0) return FKS_ERR_INVALID;
    if (!is_finite(d.gamma) || d.gamma < 0.0 || d.gamma > 1.0) return FKS_ERR_INVALID;
    if (!is_finite(d.R) || !is_finite(d.c_gamma) || !is_finite(d.radial_tol)) return FKS_ERR_INVALID;
    if (d.n_polar < 1 || d.n_azim < 1 || d.n_polar > 256 || d.n_azim > 256) return FKS_ERR_INVALID;
    if (d.rule != FKS_RULE_GAUSS && d.rule != FKS_RULE_MIDPOINT) return FKS_ERR_INVALID;
    if (d.precision != FKS_PREC_F64 && d.precision != FKS_PREC_F32_FIX64) return FKS_ERR_INVALID;
    if (d.radial_terms < 0 || d.radial_terms > 200) return FKS_ERR_INVALID;
    if ((d.flags & ~(FKS_FLAG_FORCE_GENERIC | FKS_FLAG_NUMERIC_GUARD | FKS_FLAG_DEALIAS)) != 0) return FKS_ERR_INVALID;
    if (d.n <= 0) return FKS_ERR_INVALID;
    if (d.dim == 0) d.dim = 3;
    if (d.dim != 2 && d.dim != 3) return FKS_ERR_INVALID;
    if (d.dim == 2) {
        // Maxwell molecules in two velocity dimensions (Section 3.3, eq. dfor0)
        if (d.n_azim != 1 || d.radial_terms > 1) return FKS_ERR_INVALID;
        if (d.gamma != 0.0 || (d.flags & (FKS_FLAG_FORCE_GENERIC | FKS_FLAG_DEALIAS))) return FKS_ERR_UNSUPPORTED;
        if (!supported_n_2d(d.n, d.precision)) return FKS_ERR_UNSUPPORTED;
        if (d.c_gamma <= 0) d.c_gamma = 1.0 / (2.0 * kPi);
        d.radial_terms = 1;
    } else {
        if (!supported_n(d.n)) return FKS_ERR_UNSUPPORTED;
        if ((d.flags & FKS_FLAG_DEALIAS) && !(d.n == 4 || d.n == 8 || d.n == 12 || d.n == 16 || d.n == 24 || d.n == 32))
            return FKS_ERR_UNSUPPORTED;
        if (d.c_gamma <= 0) d.c_gamma = 1.0 / (4.0 * kPi);
    }
    if (d.R <= 0) d.R = 2.0 * d.T / (3.0 + std::sqrt(2.0));
    if (d.radial_tol <= 0) d.radial_tol = 1e-4;
    if (out) *out = d;
    return FKS_OK;
}

// Workspace of fks_collide_batch_static: a file-scope device array, one copy per GPU,
// held from the code object's load until the process ends.  In host code its name is
// a host-side stand-in, not a device address: the device address comes from
// hipGetSymbolAddress, looked up once per device with that device current (at plan
// creation, this library's set-up call, else at the first static call on the device)
// and kept here; only that address is handed to kernels.
__device__ __align__(256) unsigned char scratch[FKS_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// device address of the current device's copy of `scratch`
static fks_status static_workspace(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return FKS_ERR_DEVICE;
    if (dev < 0 || dev >= kMaxDevices) return FKS_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FKS_ERR_DEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FKS_OK;
}

}  // namespace fks

using namespace fks;

extern "C" {

const char* fks_status_string(fks_status s) {
    switch (s) {
        case FKS_OK: return "FKS_OK";
        case FKS_ERR_INVALID: return "FKS_ERR_INVALID: invalid argument";
        case FKS_ERR_UNSUPPORTED: return "FKS_ERR_UNSUPPORTED: request outside the implemented set";
        case FKS_ERR_NOMEM: return "FKS_ERR_NOMEM: device allocation failed";
        case FKS_ERR_DEVICE: return "FKS_ERR_DEVICE: HIP runtime or launch failure";
        case FKS_ERR_NUMERIC: return "FKS_ERR_NUMERIC: non-finite data";
    }
    return "unknown fks_status";
}

fks_status fks_desc_validate(const fks_plan_desc* desc) { return resolve_desc(desc, nullptr); }

fks_status fks_stable_dt(double dx, double T, double tau, double R, double gamma, double c_gamma, double rho_max,
                         double* dt) {
    if (!dt) return FKS_ERR_INVALID;
    for (double v : {dx, T, tau, R, c_gamma, rho_max})
        if (!(v > 0) || !std::isfinite(v)) return FKS_ERR_INVALID;
    if (!(gamma >= 0.0 && gamma <= 1.0)) return FKS_ERR_INVALID;
    const double mu = 4.0 * kPi * c_gamma * std::pow(2.0 * R, gamma) * rho_max;
    *dt = std::min(dx / T, tau / mu);
    return FKS_OK;
}

fks_status fks_exp_euler_step(double mu, double dt_over_tau, double* h) {
    if (!h || !(mu > 0) || !std::isfinite(mu) || !(dt_over_tau >= 0) || !std::isfinite(dt_over_tau))
        return FKS_ERR_INVALID;
    *h = -std::expm1(-mu * dt_over_tau) / mu;
    return FKS_OK;
}

fks_status fks_profile_enable(int32_t enable) {
    profile_enable(enable != 0);
    return FKS_OK;
}

fks_status fks_profile_last(double* kernel_ms, int32_t capacity, int32_t* count) {
    if (!count || capacity < 0 || (capacity > 0 && !kernel_ms)) return FKS_ERR_INVALID;
    int c = 0;
    if (profile_last(kernel_ms, capacity, &c) != hipSuccess) return FKS_ERR_DEVICE;
    *count = c;
    return FKS_OK;
}

fks_status fks_host_sphere_rule(int32_t n_polar, int32_t n_azim, int32_t rule, double* e_w) {
    if (!e_w || n_polar < 1 || n_azim < 1 || n_polar > 256 || n_azim > 256) return FKS_ERR_INVALID;
    if (rule != FKS_RULE_GAUSS && rule != FKS_RULE_MIDPOINT) return FKS_ERR_INVALID;
    std::vector<double> out;
    sphere_rule(n_polar, n_azim, rule, out);
    std::memcpy(e_w, out.data(), out.size() * sizeof(double));
    return FKS_OK;
}

fks_status fks_host_radial_terms(double gamma, double R, int32_t K, double tol, int32_t nq,
                                 int32_t* K_out, double* nodes, double* coef) {
    if (!K_out || !(gamma >= 0.0 && gamma <= 1.0) || !(R > 0) || K < 0 || nq < 2 || nq > 2000)
        return FKS_ERR_INVALID;
    std::vector<double> nd, cf;
    int k = radial_expansion(gamma, R, K, tol > 0 ? tol : 1e-4, nq, nd, cf);
    *K_out = k;
    if (nodes) std::memcpy(nodes, nd.data(), nd.size() * sizeof(double));
    if (coef) std::memcpy(coef, cf.data(), cf.size() * sizeof(double));
    return FKS_OK;
}

fks_status fks_host_tables_2d(const fks_plan_desc* desc, int32_t* J_out, double* ab) {
    if (!J_out) return FKS_ERR_INVALID;
    fks_plan_desc d{};
    fks_status st = resolve_desc(desc, &d);
    if (st != FKS_OK) return st;
    if (d.dim != 2) return FKS_ERR_INVALID;
    *J_out = d.n_polar + 1;
    if (ab) {
        std::vector<double> t;
        tables_2d(d, t);
        std::memcpy(ab, t.data(), t.size() * sizeof(double));
    }
    return FKS_OK;
}

// A dim = 2 plan: host FP64 tables (closed form), uploaded in FP64 and, for
// FP32 plans, rounded to FP32; 4x4 Gram inverse of the 2D invariants.
static fks_status plan_create_2d(fks_plan* p) {
    const fks_plan_desc& d = p->desc;
    const int n = d.n, A = d.n_polar;
    p->dim = 2;
    p->M = A;
    p->K = 1;
    p->J = A + 1;
    p->H = n * n;
    p->kappa = kPi / d.T;
    p->dirs.assign((size_t)A * 4, 0.0);
    for (int q = 1; q <= A; ++q) {
        double t = kPi * q / A;
        p->dirs[(q - 1) * 4 + 0] = std::cos(t);
        p->dirs[(q - 1) * 4 + 1] = std::sin(t);
        p->dirs[(q - 1) * 4 + 3] = kPi / A;
    }
    // 2 (A + 1) real FFTs of n^2 points (A packed inverse pairs, forward, loss)
    const double nn = (double)n * n;
    p->flops_per_cell = (2.0 * A + 2.0) * 2.5 * nn * std::log2(nn) + 7.0 * A * nn + 3.0 * nn;
    std::vector<double> ab;
    tables_2d(d, ab);
    const GridConst2 g2 = grid_const2(n, d.T);
    if (hipMalloc(&p->d_tab64, ab.size() * sizeof(double)) != hipSuccess) return FKS_ERR_NOMEM;
    p->table_bytes = ab.size() * sizeof(double);
    if (hipMalloc(&p->d_gc2, sizeof(GridConst2)) != hipSuccess) return FKS_ERR_NOMEM;
    if (hipMemcpy(p->d_tab64, ab.data(), ab.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_gc2, &g2, sizeof(GridConst2), hipMemcpyHostToDevice) != hipSuccess)
        return FKS_ERR_DEVICE;
    if (d.precision == FKS_PREC_F32_FIX64) {
        // FP32 copy with kx pairs side by side: (j, kx, ky) at ((j n/2 + kx/2) n + ky) 2 + kx % 2
        std::vector<float> ab32(ab.size());
        const size_t nn = (size_t)n * n;
        for (size_t j = 0; j < (size_t)p->J; ++j)
            for (int kx = 0; kx < n; ++kx)
                for (int ky = 0; ky < n; ++ky) {
                    const size_t src = (j * nn + (size_t)kx * n + ky) * 2;
                    const size_t dst = ((j * (n / 2) + kx / 2) * n + ky) * 4 + (kx % 2) * 2;
                    ab32[dst] = (float)ab[src];
                    ab32[dst + 1] = (float)ab[src + 1];
                }
        if (hipMalloc(&p->d_tab32, ab32.size() * sizeof(float)) != hipSuccess) return FKS_ERR_NOMEM;
        p->table_bytes += ab32.size() * sizeof(float);
        if (hipMemcpy(p->d_tab32, ab32.data(), ab32.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
            return FKS_ERR_DEVICE;
    }
    return FKS_OK;
}

static void plan_free(fks_plan* p) {
    if (p->d_guard) (void)hipFree(p->d_guard);
    if (p->d_tab64) (void)hipFree(p->d_tab64);
    if (p->d_tab32) (void)hipFree(p->d_tab32);
    if (p->d_tab32p) (void)hipFree(p->d_tab32p);
    if (p->d_tab48p) (void)hipFree(p->d_tab48p);
    if (p->d_gc) (void)hipFree(p->d_gc);
    if (p->d_gc2) (void)hipFree(p->d_gc2);
    delete p;
}

fks_status fks_plan_create(const fks_plan_desc* desc, void* hip_stream, fks_plan** out) {
    if (!out) return FKS_ERR_INVALID;
    *out = nullptr;
    fks_plan_desc d{};
    fks_status st = resolve_desc(desc, &d);
    if (st != FKS_OK) return st;
    fks_plan* p = new (std::nothrow) fks_plan();
    if (!p) return FKS_ERR_NOMEM;
    p->desc = d;
    const int n = d.n;
    if (hipGetDevice(&p->device) != hipSuccess) { delete p; return FKS_ERR_DEVICE; }
    void* static_ws = nullptr;   // set-up of fks_collide_batch_static's workspace on this device
    if ((st = static_workspace(&static_ws)) != FKS_OK) {
        delete p;
        return st;
    }
    if (d.flags & FKS_FLAG_NUMERIC_GUARD) {
        const unsigned long long none = ~0ull;
        if (hipMalloc(&p->d_guard, sizeof(none)) != hipSuccess) {
            delete p;
            return FKS_ERR_NOMEM;
        }
        if (hipMemcpy(p->d_guard, &none, sizeof(none), hipMemcpyHostToDevice) != hipSuccess) {
            plan_free(p);
            return FKS_ERR_DEVICE;
        }
    }
    if (d.dim == 2) {
        st = plan_create_2d(p);
        if (st != FKS_OK) {
            plan_free(p);
            return st;
        }
        *out = p;
        return FKS_OK;
    }
    p->M = d.n_polar * d.n_azim;
    if (d.gamma == 1.0) {
        p->K = 1;   // constant Carleman kernel: closed-form phi, psi
    } else {
        p->K = radial_expansion(d.gamma, d.R, d.radial_terms, d.radial_tol, 200, p->rad_nodes, p->rad_coef);
    }
    p->J = p->M * p->K + 1;
    p->H = (n / 2 + 1) * n * n;
    p->kappa = kPi / d.T;
    p->gc = grid_const(n, d.T);
    sphere_rule(d.n_polar, d.n_azim, d.rule, p->dirs);
    // algorithmic flops: (2 J' + 2) real FFTs of n^3 points at 2.5 n log2 n,
    // J' = M K packed complex inverse transforms (two real ones each) plus the
    // forward and loss transforms; 7 flops per point and term for the products
    // and accumulation; 3 per point for the update.
    double nn = (double)n * n * n;
    p->flops_per_cell = (2.0 * p->M * p->K + 2.0) * 2.5 * nn * std::log2(nn) + 7.0 * p->M * p->K * nn + 3.0 * nn;
    if (d.flags & FKS_FLAG_DEALIAS) {
        // per term: zero-padded inverse transforms over n^2, n n' and n'^2 lines of n' points
        // (5 n' log2 n' flop each), the product with fhat and Re z Im z on the n' grid; once per
        // cell: the forward and inverse n-point transforms, the truncating forward n'-point
        // transforms and the update
        const double np = 1.5 * n, lines = (double)n * n + (double)n * np + np * np;
        const double fft_np = 5.0 * np * std::log2(np) * lines;
        p->flops_per_cell = (p->M * p->K + 1.0) * (fft_np + 6.0 * nn + 2.0 * np * np * np) + fft_np +
                            2.0 * 2.5 * nn * std::log2(nn) + 3.0 * nn;
    }
    size_t tab_elems = (size_t)p->J * p->H * 2;
    if (hipMalloc(&p->d_tab64, tab_elems * sizeof(double)) != hipSuccess) {
        plan_free(p);
        return FKS_ERR_NOMEM;
    }
    p->table_bytes = tab_elems * sizeof(double);
    if (hipMalloc(&p->d_gc, sizeof(GridConst)) != hipSuccess ||
        hipMemcpy(p->d_gc, &p->gc, sizeof(GridConst), hipMemcpyHostToDevice) != hipSuccess) {
        plan_free(p);
        return FKS_ERR_NOMEM;
    }
    if (d.precision == FKS_PREC_F32_FIX64) {
        if (hipMalloc(&p->d_tab32, tab_elems * sizeof(float)) != hipSuccess) {
            plan_free(p);
            return FKS_ERR_NOMEM;
        }
        p->table_bytes += tab_elems * sizeof(float);
        p->fused = fused_available(n) && !(d.flags & (FKS_FLAG_FORCE_GENERIC | FKS_FLAG_DEALIAS));
        if (p->fused) p->fused_grid = fused_grid_size(n, p->device);
        if (p->fused) {   // the kz-pair copy read by the fused kernels
            const size_t pair_elems = (size_t)p->J * (n / 2) * n * n * 2;
            if (hipMalloc(&p->d_tab32p, pair_elems * sizeof(float)) != hipSuccess) {
                plan_free(p);
                return FKS_ERR_NOMEM;
            }
            p->table_bytes += pair_elems * sizeof(float);
        }
    }
    hipStream_t s = (hipStream_t)hip_stream;
    if (build_tables(p, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
        plan_free(p);
        return FKS_ERR_DEVICE;
    }
    if (p->d_tab32p) {   // fused plans read only the kz-pair copy; the multi-pass path never runs them
        (void)hipFree(p->d_tab32);
        p->d_tab32 = nullptr;
        p->table_bytes -= tab_elems * sizeof(float);
    }
    if (d.precision == FKS_PREC_F32_FIX64 && (d.flags & FKS_FLAG_DEALIAS) && n == 32) {
        // the products of the 48-point grid run on the n = 48 kernel: the tables zero-padded
        // to that grid, planes kz < 24 in its kz-pair layout
        const size_t e48 = (size_t)p->J * 24 * 48 * 48 * 2;
        if (hipMalloc(&p->d_tab48p, e48 * sizeof(float)) != hipSuccess) {
            plan_free(p);
            return FKS_ERR_NOMEM;
        }
        p->table_bytes += e48 * sizeof(float);
        p->grid48 = terms48_grid(p->device);
        if (embed_tables48(p, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
            plan_free(p);
            return FKS_ERR_DEVICE;
        }
    }
    *out = p;
    return FKS_OK;
}

fks_status fks_plan_destroy(fks_plan* p) {
    if (!p) return FKS_OK;
    // the plan's memory lives on the device it was created on; hipFree itself waits for
    // work still pending on that device
    int cur = 0;
    const bool switch_dev = hipGetDevice(&cur) == hipSuccess && cur != p->device;
    if (switch_dev && hipSetDevice(p->device) != hipSuccess) return FKS_ERR_DEVICE;
    plan_free(p);
    if (switch_dev) (void)hipSetDevice(cur);
    return FKS_OK;
}

fks_status fks_plan_query(const fks_plan* p, fks_plan_info* info) {
    if (!p || !info) return FKS_ERR_INVALID;
    info->n = p->desc.n;
    info->M = p->M;
    info->K = p->K;
    info->J = p->J;
    info->R = p->desc.R;
    info->c_gamma = p->desc.c_gamma;
    info->precision = p->desc.precision;
    info->fused = p->fused ? 1 : 0;
    info->table_bytes = p->table_bytes;
    info->flops_per_cell = p->flops_per_cell;
    info->dim = p->dim;
    info->fused_grid = p->fused ? p->fused_grid : 0;
    info->queue_items_per_wg = p->queue_ipw;
    return FKS_OK;
}

fks_status fks_numeric_status(const fks_plan* p, int64_t* first_bad_cell, int32_t reset) {
    if (!p || !first_bad_cell || !p->d_guard) return FKS_ERR_INVALID;
    unsigned long long v = 0;
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(&v, p->d_guard, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess)
        return FKS_ERR_DEVICE;
    if (reset) {
        const unsigned long long none = ~0ull;
        if (hipMemcpy(p->d_guard, &none, sizeof(none), hipMemcpyHostToDevice) != hipSuccess) return FKS_ERR_DEVICE;
    }
    *first_bad_cell = v == ~0ull ? -1 : (int64_t)v;
    return v == ~0ull ? FKS_OK : FKS_ERR_NUMERIC;
}

fks_status fks_plan_copy_tables(const fks_plan* p, double* ab_host, double* dirs_host) {
    if (!p) return FKS_ERR_INVALID;
    if (ab_host) {
        size_t bytes = (size_t)p->J * p->H * 2 * sizeof(double);
        if (hipMemcpy(ab_host, p->d_tab64, bytes, hipMemcpyDeviceToHost) != hipSuccess) return FKS_ERR_DEVICE;
    }
    if (dirs_host) std::memcpy(dirs_host, p->dirs.data(), p->dirs.size() * sizeof(double));
    return FKS_OK;
}

static fks_status check_segment(const fks_segment& s) {
    if (!s.plan) return FKS_ERR_INVALID;
    if (s.ncell < 0) return FKS_ERR_INVALID;
    if (s.ncell == 0) return FKS_OK;
    if (!s.f || (!s.q_out && !s.f_out)) return FKS_ERR_INVALID;
    if (!std::isfinite(s.dt_over_tau)) return FKS_ERR_INVALID;
    // the kernels move f, q_out, f_out and f_base in 16-byte vectors
    if (((uintptr_t)s.f | (uintptr_t)s.q_out | (uintptr_t)s.f_out | (uintptr_t)s.f_base) & 15u)
        return FKS_ERR_INVALID;
    size_t bytes = (size_t)s.ncell * s.plan->desc.n * s.plan->desc.n * sizeof(double);
    if (s.plan->dim == 3) bytes *= (size_t)s.plan->desc.n;
    if (s.q_out && s.f_out) {
        const char* a = (const char*)s.q_out;
        const char* b = (const char*)s.f_out;
        if (a < b + bytes && b < a + bytes) return FKS_ERR_INVALID;
    }
    if (s.q_out) {
        const char* a = (const char*)s.q_out;
        const char* b = (const char*)s.f;
        if (a < b + bytes && b < a + bytes) return FKS_ERR_INVALID;
    }
    if (s.f_out && s.f_out != s.f) {
        const char* a = (const char*)s.f_out;
        const char* b = (const char*)s.f;
        if (a < b + bytes && b < a + bytes) return FKS_ERR_INVALID;
    }
    if (s.f_base && s.f_base != s.f) {
        const char* a = (const char*)s.f_base;
        if (s.q_out) {
            const char* b = (const char*)s.q_out;
            if (a < b + bytes && b < a + bytes) return FKS_ERR_INVALID;
        }
        if (s.f_out && s.f_out != s.f_base) {
            const char* b = (const char*)s.f_out;
            if (a < b + bytes && b < a + bytes) return FKS_ERR_INVALID;
        }
    }
    return FKS_OK;
}

static size_t segment_ws(const fks_segment& s) {
    if (s.ncell == 0 || s.plan->dim == 2) return 0;
    return s.plan->fused ? fused_workspace_bytes(s.plan, s.ncell) : generic_workspace_bytes(s.plan, s.ncell);
}


// Launch groups of one call.  Fused 3D segments that share n, two or more of them, go
// through one work queue (up to fused_queue_max_segments() per queue; at n = 48 the
// three-workgroup kernel over all their cells), so that small segments fill the device
// together; every other segment runs alone, in call order.  Groups run one after another on the call's stream and share the
// workspace.
struct LaunchGroup {
    std::vector<const fks_segment*> segs;
    bool queue = false;
};

static bool queueable(const fks_segment& g) {
    return g.ncell > 0 && g.plan->dim == 3 && g.plan->fused;
}

static std::vector<LaunchGroup> batch_groups(const fks_segment* segs, int32_t nseg) {
    std::vector<LaunchGroup> out;
    std::vector<bool> done(nseg, false);
    for (int i = 0; i < nseg; ++i) {
        if (done[i] || segs[i].ncell == 0) continue;
        done[i] = true;
        LaunchGroup g;
        g.segs.push_back(&segs[i]);
        if (queueable(segs[i])) {
            for (int k = i + 1; k < nseg && (int)g.segs.size() < fused_queue_max_segments(); ++k) {
                if (!done[k] && queueable(segs[k]) && segs[k].plan->desc.n == segs[i].plan->desc.n) {
                    g.segs.push_back(&segs[k]);
                    done[k] = true;
                }
            }
            g.queue = g.segs.size() > 1;
        }
        out.push_back(std::move(g));
    }
    return out;
}

static size_t group_ws(const LaunchGroup& g) {
    return g.queue ? fused_queue_workspace_bytes(g.segs.data(), (int)g.segs.size()) : segment_ws(*g.segs[0]);
}

// Segments of one call, validated; the workspace the largest launch group needs.
static fks_status batch_need(const fks_segment* segs, int32_t nseg, size_t* need) {
    if (nseg < 0 || (nseg > 0 && !segs)) return FKS_ERR_INVALID;
    *need = 0;
    for (int i = 0; i < nseg; ++i) {
        fks_status st = check_segment(segs[i]);
        if (st != FKS_OK) return st;
    }
    for (const LaunchGroup& g : batch_groups(segs, nseg)) *need = std::max(*need, group_ws(g));
    return FKS_OK;
}

static fks_status batch_launch(const fks_segment* segs, int32_t nseg, void* workspace, size_t ws_bytes,
                               hipStream_t s) {
    for (const LaunchGroup& grp : batch_groups(segs, nseg)) {
        hipError_t e = hipSuccess;
        if (grp.queue) {
            e = collide_fused_queue(grp.segs.data(), (int)grp.segs.size(), workspace, ws_bytes, s);
        } else {
            const fks_segment& g = *grp.segs[0];
            e = g.plan->dim == 2 ? collide_2d(g.plan, g, s)
                : g.plan->fused  ? collide_fused(g.plan, g, workspace, ws_bytes, s)
                                 : collide_generic(g.plan, g, workspace, ws_bytes, s);
        }
        if (e != hipSuccess) return FKS_ERR_DEVICE;
    }
    return FKS_OK;
}

fks_status fks_workspace_size(const fks_segment* segs, int32_t nseg, size_t* bytes) {
    if (!bytes) return FKS_ERR_INVALID;
    return batch_need(segs, nseg, bytes);
}

fks_status fks_collide_batch(const fks_segment* segs, int32_t nseg, void* workspace, size_t ws_bytes,
                             void* hip_stream) {
    size_t need = 0;
    fks_status st = batch_need(segs, nseg, &need);
    if (st != FKS_OK) return st;
    if (need > 0 && (!workspace || ws_bytes < need || ((uintptr_t)workspace & 255u))) return FKS_ERR_INVALID;
    return batch_launch(segs, nseg, workspace, ws_bytes, (hipStream_t)hip_stream);
}

fks_status fks_collide_batch_static(const fks_segment* segs, int32_t nseg, void* hip_stream) {
    size_t need = 0;
    fks_status st = batch_need(segs, nseg, &need);
    if (st != FKS_OK) return st;
    if (need > FKS_STATIC_WORKSPACE_BYTES) return FKS_ERR_INVALID;
    void* ws = nullptr;
    if (need > 0 && (st = static_workspace(&ws)) != FKS_OK) return st;
    return batch_launch(segs, nseg, ws, need > 0 ? FKS_STATIC_WORKSPACE_BYTES : 0, (hipStream_t)hip_stream);
}

// Candidate schedules of one segment: the two fused decompositions, or cells per
// pass batch of the multi-pass path.  Empty when nothing is to be chosen.
static std::vector<Schedule> schedule_candidates(const fks_segment& s) {
    std::vector<Schedule> c;
    if (s.ncell <= 0 || s.plan->dim == 2) return c;
    if (s.plan->fused) {
        if (s.plan->desc.n == 48) return c;   // one decomposition (three workgroups per cell)
        c.push_back(Schedule{1, 0});
        c.push_back(Schedule{0, 0});
        return c;
    }
    // the de-aliased variant and FP64 at n = 48 have no terms-per-launch knob
    const bool multi = generic_multi_terms(s.plan);
    for (int chunk : {32, 64, 128, 256, 512}) {
        const int ch = chunk >= s.ncell ? (int)s.ncell : chunk;
        for (int terms : {1, 2, 4}) {
            if (!multi && terms > 1) break;
            c.push_back(Schedule{-1, ch, multi ? terms : 0});
        }
        if (chunk >= s.ncell) break;
    }
    return c;
}

// Transport step shared by the whole-grid and the slab entry points: validation, the
// per-axis displacement update and integer shifts (host, FP64), then the shift kernel.
// A slab reads its z neighbours from their messages, so its z shift must be -1, 0 or 1.
static fks_status transport_step(const double* f_in, double* f_out, const fks_space_desc* sp, int32_t n, double T,
                                 double dt, double* offsets, const double* bc_f, void* hip_stream,
                                 const double* from_below, const double* from_above) {
    const bool slab = from_below != nullptr || from_above != nullptr;
    if (!f_in || !f_out || !sp || !offsets) return FKS_ERR_INVALID;
    if (slab && !(from_below && from_above)) return FKS_ERR_INVALID;
    if (n < 2 || n > 64 || !(T > 0) || !std::isfinite(T) || !std::isfinite(dt)) return FKS_ERR_INVALID;
    if (sp->nx < 1 || sp->ny < 1 || sp->nz < 1 || !(sp->dx > 0) || !std::isfinite(sp->dx)) return FKS_ERR_INVALID;
    bool any_dirichlet = false;
    for (int a = 0; a < (slab ? 2 : 3); ++a) {
        if (sp->bc[a] != FKS_BC_PERIODIC && sp->bc[a] != FKS_BC_DIRICHLET) return FKS_ERR_INVALID;
        any_dirichlet |= sp->bc[a] == FKS_BC_DIRICHLET;
    }
    if (any_dirichlet && !bc_f) return FKS_ERR_INVALID;
    const size_t bytes = (size_t)sp->nx * sp->ny * sp->nz * n * n * n * sizeof(double);
    const char* a = (const char*)f_in;
    const char* b = (const char*)f_out;
    if (a < b + bytes && b < a + bytes) return FKS_ERR_INVALID;
    ShiftTable sh{};
    const double dv = 2.0 * T / n;
    double next[3][64];
    for (int ax = 0; ax < 3; ++ax)
        for (int k = 0; k < n; ++k) {
            double v = -T + k * dv;
            double s0 = offsets[ax * n + k];
            double s1 = s0 + v * dt;
            if (!std::isfinite(s1)) return FKS_ERR_INVALID;
            double d0 = std::floor(s0 / sp->dx + 0.5), d1 = std::floor(s1 / sp->dx + 0.5);
            double dd = d1 - d0;
            if (dd > 127 || dd < -127) return FKS_ERR_INVALID;
            // a slab's messages hold only what crosses its faces: a z shift of +1 is allowed
            // for the velocities sent up (v_z > 0), -1 for those sent down (v_z < 0)
            if (slab && ax == 2 && dd != 0 && !(dd == 1 && 2 * k > n) && !(dd == -1 && 2 * k < n))
                return FKS_ERR_INVALID;
            sh.s[ax][k] = (int8_t)dd;
            next[ax][k] = s1;
        }
    hipError_t e = transport(f_in, f_out, *sp, n, sh, bc_f, (hipStream_t)hip_stream, from_below, from_above);
    if (e != hipSuccess) return FKS_ERR_DEVICE;
    for (int ax = 0; ax < 3; ++ax)
        for (int k = 0; k < n; ++k) offsets[ax * n + k] = next[ax][k];
    return FKS_OK;
}

static bool slab_valid(const fks_space_desc* sp, int32_t n) {
    return sp && n >= 2 && n <= 64 && sp->nx >= 1 && sp->ny >= 1 && sp->nz >= 1;
}

// Velocities that leave a slab through a z face: v_z < 0 (kz < n/2) through z-, v_z > 0
// (kz > n/2) through z+; v_z = 0 never crosses.  Their kz form one range [k0, k0 + h).
static bool halo_range(int32_t n, int32_t face, int* k0, int* h) {
    if (face == FKS_FACE_ZLO) {
        *k0 = 0;
        *h = (n + 1) / 2;
    } else if (face == FKS_FACE_ZHI) {
        *k0 = n / 2 + 1;
        *h = n - 1 - n / 2;
    } else {
        return false;
    }
    return true;
}

// sets (or with erase, removes) the measured schedule of (plan, ncell)
static void set_schedule(fks_plan* p, int64_t ncell, const Schedule* sc) {
    for (size_t i = 0; i < p->tuned.size(); ++i) {
        if (p->tuned[i].first == ncell) {
            if (sc) p->tuned[i].second = *sc;
            else p->tuned.erase(p->tuned.begin() + i);
            return;
        }
    }
    if (sc) p->tuned.emplace_back(ncell, *sc);
}

static hipError_t collide_one(const fks_segment& g, void* ws, size_t ws_bytes, hipStream_t s) {
    return g.plan->fused ? collide_fused(g.plan, g, ws, ws_bytes, s) : collide_generic(g.plan, g, ws, ws_bytes, s);
}

// Work-queue candidates of fks_autotune: items per resident workgroup (the direction batch
// of an item is about J over the items per cell).  Queues at n = 48 have no such knob.
static const int kQueueIpw[] = {1, 2, 4, 8};
static bool tunable_queue(const LaunchGroup& g) { return g.queue && g.segs[0]->plan->desc.n != 48; }
static void set_queue_ipw(const LaunchGroup& g, int ipw) {
    for (const fks_segment* s : g.segs) const_cast<fks_plan*>(s->plan)->queue_ipw = ipw;
}

fks_status fks_autotune_workspace_size(const fks_segment* segs, int32_t nseg, size_t* bytes) {
    if (!bytes || nseg < 0 || (nseg > 0 && !segs)) return FKS_ERR_INVALID;
    size_t mx = 0;
    for (int i = 0; i < nseg; ++i) {
        fks_status st = check_segment(segs[i]);
        if (st != FKS_OK) return st;
        fks_plan* p = const_cast<fks_plan*>(segs[i].plan);
        const auto saved = p->tuned;
        for (const Schedule& c : schedule_candidates(segs[i])) {
            set_schedule(p, segs[i].ncell, &c);
            mx = std::max(mx, segment_ws(segs[i]));
        }
        p->tuned = saved;
        mx = std::max(mx, segment_ws(segs[i]));
    }
    for (const LaunchGroup& g : batch_groups(segs, nseg)) {
        if (!tunable_queue(g)) continue;
        const int saved = g.segs[0]->plan->queue_ipw;
        for (int ipw : kQueueIpw) {
            set_queue_ipw(g, ipw);
            mx = std::max(mx, group_ws(g));
        }
        set_queue_ipw(g, saved);
        mx = std::max(mx, group_ws(g));
    }
    *bytes = mx;
    return FKS_OK;
}

fks_status fks_autotune(const fks_segment* segs, int32_t nseg, void* workspace, size_t ws_bytes, void* hip_stream,
                        int32_t* choice_out) {
    if (nseg < 0 || (nseg > 0 && !segs)) return FKS_ERR_INVALID;
    if (workspace && ((uintptr_t)workspace & 255u)) return FKS_ERR_INVALID;
    for (int i = 0; i < nseg; ++i) {
        const fks_segment& g = segs[i];
        fks_status st = check_segment(g);
        if (st != FKS_OK) return st;
        // the segment is evaluated several times: its outputs must not feed its inputs
        const size_t bytes = (size_t)g.ncell * g.plan->desc.n * g.plan->desc.n * (g.plan->dim == 2 ? 1 : g.plan->desc.n) *
                             sizeof(double);
        const double* in[2] = {g.f, g.f_base ? g.f_base : g.f};
        for (const double* a : in) {
            if (g.f_out && (const char*)a < (const char*)g.f_out + bytes && (const char*)g.f_out < (const char*)a + bytes)
                return FKS_ERR_INVALID;
        }
    }
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t ev[2];
    if (hipEventCreate(&ev[0]) != hipSuccess) return FKS_ERR_DEVICE;
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return FKS_ERR_DEVICE;
    }
    fks_status result = FKS_OK;
    for (int i = 0; i < nseg && result == FKS_OK; ++i) {
        const fks_segment& g = segs[i];
        fks_plan* p = const_cast<fks_plan*>(g.plan);
        if (choice_out) {
            choice_out[3 * i] = -1;
            choice_out[3 * i + 1] = 0;
            choice_out[3 * i + 2] = 0;
        }
        const std::vector<Schedule> cand = schedule_candidates(g);
        if (cand.empty()) continue;
        set_schedule(p, g.ncell, nullptr);
        int best = -1;
        float best_ms = 0.0f;
        for (size_t k = 0; k < cand.size(); ++k) {
            set_schedule(p, g.ncell, &cand[k]);
            const size_t need = segment_ws(g);
            if (need > ws_bytes || (need > 0 && !workspace)) continue;
            float ms = 0.0f;
            if (collide_one(g, workspace, ws_bytes, s) != hipSuccess ||            // warm-up
                hipEventRecord(ev[0], s) != hipSuccess ||
                collide_one(g, workspace, ws_bytes, s) != hipSuccess ||
                collide_one(g, workspace, ws_bytes, s) != hipSuccess ||
                hipEventRecord(ev[1], s) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
                hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) {
                result = FKS_ERR_DEVICE;
                break;
            }
            if (best < 0 || ms < best_ms) {
                best = (int)k;
                best_ms = ms;
            }
        }
        if (best < 0 || result != FKS_OK) {
            set_schedule(p, g.ncell, nullptr);   // nothing fitted the workspace: keep the defaults
            continue;
        }
        set_schedule(p, g.ncell, &cand[best]);
        if (choice_out) {
            choice_out[3 * i] = cand[best].one;
            choice_out[3 * i + 1] = cand[best].chunk;
            choice_out[3 * i + 2] = cand[best].terms;
        }
    }
    // work queues (the launch groups fks_collide_batch forms from these segments): items per
    // resident workgroup, kept in every plan of the group
    for (const LaunchGroup& grp : batch_groups(segs, nseg)) {
        if (result != FKS_OK) break;
        if (!tunable_queue(grp)) continue;
        int best = 0;
        float best_ms = 0.0f;
        for (int ipw : kQueueIpw) {
            set_queue_ipw(grp, ipw);
            const size_t need = group_ws(grp);
            if (need > ws_bytes || !workspace) continue;
            const int ns = (int)grp.segs.size();
            float ms = 0.0f;
            if (collide_fused_queue(grp.segs.data(), ns, workspace, ws_bytes, s) != hipSuccess ||   // warm-up
                hipEventRecord(ev[0], s) != hipSuccess ||
                collide_fused_queue(grp.segs.data(), ns, workspace, ws_bytes, s) != hipSuccess ||
                collide_fused_queue(grp.segs.data(), ns, workspace, ws_bytes, s) != hipSuccess ||
                hipEventRecord(ev[1], s) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
                hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) {
                result = FKS_ERR_DEVICE;
                break;
            }
            if (best == 0 || ms < best_ms) {
                best = ipw;
                best_ms = ms;
            }
        }
        set_queue_ipw(grp, best);   // 0 (the cost model) if no candidate fitted the workspace
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    return result;
}

fks_status fks_moments(const double* f, int64_t ncell, int32_t n, double T, double* U, void* hip_stream) {
    if (ncell < 0 || !(T > 0) || !std::isfinite(T) || n < 2 || n > 64) return FKS_ERR_INVALID;
    if (ncell == 0) return FKS_OK;
    if (!f || !U) return FKS_ERR_INVALID;
    return moments(f, ncell, n, T, U, (hipStream_t)hip_stream) == hipSuccess ? FKS_OK : FKS_ERR_DEVICE;
}

fks_status fks_conserve(double* f, const double* U, int64_t ncell, int32_t n, double T, void* hip_stream) {
    if (ncell < 0 || !(T > 0) || !std::isfinite(T) || n < 2 || n > 64) return FKS_ERR_INVALID;
    if (ncell == 0) return FKS_OK;
    if (!f || !U) return FKS_ERR_INVALID;
    return conserve(f, U, ncell, n, T, (hipStream_t)hip_stream) == hipSuccess ? FKS_OK : FKS_ERR_DEVICE;
}

fks_status fks_spectrum_workspace_size(int64_t ncell, int32_t n, size_t* bytes) {
    if (!bytes || ncell < 0 || !supported_n(n)) return !bytes || ncell < 0 ? FKS_ERR_INVALID : FKS_ERR_UNSUPPORTED;
    *bytes = ncell == 0 ? 0 : spectrum_workspace_bytes(n, ncell);
    return FKS_OK;
}

fks_status fks_spectrum(const double* x, double* xhat, int64_t ncell, int32_t n, int32_t zero_nyquist,
                        void* workspace, size_t ws_bytes, void* hip_stream) {
    if (ncell < 0 || (zero_nyquist != 0 && zero_nyquist != 1)) return FKS_ERR_INVALID;
    if (!supported_n(n)) return n > 0 ? FKS_ERR_UNSUPPORTED : FKS_ERR_INVALID;
    if (ncell == 0) return FKS_OK;
    if (!x || !xhat || !workspace || ((uintptr_t)workspace & 255u)) return FKS_ERR_INVALID;
    const size_t one = (size_t)n * n * n * 16;   // one cell of complex FP64 work
    if (ws_bytes < one) return FKS_ERR_INVALID;
    const size_t in_bytes = (size_t)ncell * n * n * n * sizeof(double);
    const size_t out_bytes = (size_t)ncell * n * n * (n / 2 + 1) * 2 * sizeof(double);
    const char* a = (const char*)x;
    const char* b = (const char*)xhat;
    const char* w = (const char*)workspace;
    if ((a < b + out_bytes && b < a + in_bytes) || (w < b + out_bytes && b < w + ws_bytes) ||
        (w < a + in_bytes && a < w + ws_bytes))
        return FKS_ERR_INVALID;
    return spectrum(x, xhat, ncell, n, zero_nyquist, workspace, ws_bytes, (hipStream_t)hip_stream) == hipSuccess
               ? FKS_OK
               : FKS_ERR_DEVICE;
}

fks_status fks_bgk(const fks_bgk_desc* d, const double* f, double* q_out, double* f_out, int64_t ncell,
                   double dt_over_tau, void* hip_stream) {
    if (!d || ncell < 0 || !std::isfinite(dt_over_tau)) return FKS_ERR_INVALID;
    if (d->dim != 2 && d->dim != 3) return FKS_ERR_INVALID;
    if (d->n < 2 || d->n > (d->dim == 3 ? 64 : 512)) return FKS_ERR_INVALID;
    if (!(d->T > 0) || !std::isfinite(d->T) || !(d->nu >= 0) || !std::isfinite(d->nu)) return FKS_ERR_INVALID;
    if ((d->nu_rho != 0 && d->nu_rho != 1) || (d->step != FKS_BGK_EULER && d->step != FKS_BGK_EXACT))
        return FKS_ERR_INVALID;
    if (ncell == 0) return FKS_OK;
    if (!f || (!q_out && !f_out)) return FKS_ERR_INVALID;
    size_t bytes = (size_t)ncell * d->n * d->n * sizeof(double);
    if (d->dim == 3) bytes *= (size_t)d->n;
    auto overlap = [bytes](const void* x, const void* y) {
        const char* a = (const char*)x;
        const char* b = (const char*)y;
        return x && y && a < b + bytes && b < a + bytes;
    };
    if (overlap(q_out, f) || overlap(q_out, f_out)) return FKS_ERR_INVALID;
    if (f_out && f_out != f && overlap(f_out, f)) return FKS_ERR_INVALID;
    return bgk(*d, f, q_out, f_out, ncell, dt_over_tau, (hipStream_t)hip_stream) == hipSuccess ? FKS_OK
                                                                                             : FKS_ERR_DEVICE;
}

fks_status fks_transport_shift(const double* f_in, double* f_out, const fks_space_desc* sp, int32_t n,
                               double T, double dt, double* offsets, const double* bc_f, void* hip_stream) {
    return transport_step(f_in, f_out, sp, n, T, dt, offsets, bc_f, hip_stream, nullptr, nullptr);
}

fks_status fks_transport_shift_slab(const double* f_in, double* f_out, const fks_space_desc* slab, int32_t n,
                                    double T, double dt, double* offsets, const double* from_below,
                                    const double* from_above, const double* bc_f, void* hip_stream) {
    if (!from_below || !from_above) return FKS_ERR_INVALID;
    return transport_step(f_in, f_out, slab, n, T, dt, offsets, bc_f, hip_stream, from_below, from_above);
}

fks_status fks_halo_size(const fks_space_desc* slab, int32_t n, int32_t face, size_t* bytes) {
    if (!bytes) return FKS_ERR_INVALID;
    int k0 = 0, h = 0;
    if (!slab_valid(slab, n) || !halo_range(n, face, &k0, &h)) return FKS_ERR_INVALID;
    *bytes = (size_t)slab->nx * slab->ny * n * n * h * sizeof(double);
    return FKS_OK;
}

fks_status fks_halo_pack(const double* f, const fks_space_desc* slab, int32_t n, int32_t face, double* buf,
                         void* hip_stream) {
    int k0 = 0, h = 0;
    if (!f || !buf || !slab_valid(slab, n) || !halo_range(n, face, &k0, &h)) return FKS_ERR_INVALID;
    // the outgoing velocities of the first (z-) or last (z+) plane
    const int64_t plane = face == FKS_FACE_ZLO ? 0 : slab->nz - 1;
    hipError_t e = halo_pack(f, buf, plane, (int64_t)slab->nx * slab->ny, n, k0, h, (hipStream_t)hip_stream);
    return e == hipSuccess ? FKS_OK : FKS_ERR_DEVICE;
}

}  // extern "C"
