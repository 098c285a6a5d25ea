// Host check of the register FFT templates against a direct DFT in long double.
#include <cmath>
#include <cstdio>
#include <random>
#include "../../paper_1608_08009_amd/csrc/fks_fft.hpp"

template <typename T, int N, int SIGN>
static double check(std::mt19937_64& g) {
    std::uniform_real_distribution<double> u(-1, 1);
    fks::cx<T> x[N];
    long double xr[N], xi[N];
    for (int i = 0; i < N; ++i) {
        x[i] = {T(u(g)), T(u(g))};
        xr[i] = x[i].x; xi[i] = x[i].y;
    }
    fks::fft<T, N, SIGN>(x);
    double err = 0, nrm = 0;
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < N; ++k) {
        long double sr = 0, si = 0;
        for (int m = 0; m < N; ++m) {
            long double a = SIGN * 2 * pi * (long double)((long)m * k % N) / N;
            sr += xr[m] * cosl(a) - xi[m] * sinl(a);
            si += xr[m] * sinl(a) + xi[m] * cosl(a);
        }
        err = std::fmax(err, (double)std::hypot((double)(x[k].x - sr), (double)(x[k].y - si)));
        nrm = std::fmax(nrm, (double)std::hypot((double)sr, (double)si));
    }
    return err / nrm;
}

template <int N>
static int run(std::mt19937_64& g) {
    double e64 = std::fmax(check<double, N, 1>(g), check<double, N, -1>(g));
    double e32 = std::fmax(check<float, N, 1>(g), check<float, N, -1>(g));
    int bad = !(e64 < 4e-15 * std::log2(2.0 * N)) || !(e32 < 2e-7 * std::log2(2.0 * N));
    std::printf("N=%2d  fp64 rel err %.2e   fp32 rel err %.2e  %s\n", N, e64, e32, bad ? "FAIL" : "ok");
    return bad;
}

int main() {
    std::mt19937_64 g(1608080090ull);
    int bad = 0;
    bad += run<2>(g); bad += run<3>(g); bad += run<4>(g); bad += run<6>(g);
    bad += run<8>(g); bad += run<12>(g); bad += run<16>(g); bad += run<24>(g);
    bad += run<32>(g); bad += run<48>(g); bad += run<64>(g);
    // twiddle constants against libm in long double
    double worst = 0;
    for (int den = 1; den <= 64; ++den)
        for (int num = 0; num < den; ++num) {
            fks::ct::sc w = fks::ct::sincos2pi(num, den);
            long double a = 2 * 3.141592653589793238462643383279502884L * num / den;
            worst = std::fmax(worst, std::fabs((double)(w.s - sinl(a))));
            worst = std::fmax(worst, std::fabs((double)(w.c - cosl(a))));
        }
    std::printf("twiddle max abs err %.2e %s\n", worst, worst < 3e-16 ? "ok" : "FAIL");
    bad += !(worst < 3e-16);
    return bad ? 1 : 0;
}
