// Device helpers shared by the HIP kernels of the library.
#pragma once

#include <hip/hip_runtime.h>

namespace rom {
namespace dev {

typedef float f4 __attribute__((ext_vector_type(4)));

// s_waitcnt immediate for vmcnt(0) with expcnt and lgkmcnt left free (gfx9
// encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
constexpr int kWaitVm0 = 0x0F70;

// Error-free sum: s + e == a + b exactly (Knuth's two-sum, 6 flops, no
// assumption on magnitudes).  Built with -ffp-contract=off so nothing here
// is fused or reassociated.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Ricker wavelet with centre frequency mu and delay 1.5/mu (Sec. 3.2 names
// the signal; unit-peak form): u = (1 - 2a) exp(-a), a = pi^2 (mu t - 1.5)^2.
__device__ __forceinline__ double ricker(double t, double mu) {
    const double pi = 3.141592653589793238462643383279502884;
    double x = pi * (mu * t - 1.5);
    double a = x * x;
    return (1.0 - 2.0 * a) * exp(-a);
}

// d u / d mu of the wavelet above, including the mu-dependence of the delay.
__device__ __forceinline__ double ricker_dmu(double t, double mu) {
    const double pi = 3.141592653589793238462643383279502884;
    double x = mu * t - 1.5;
    double a = pi * pi * x * x;
    return (2.0 * a - 3.0) * exp(-a) * (2.0 * pi * pi * t * x);
}

// First derivative of a Gaussian, the second source signal (Sec. 3.2; the
// appendix's FOM runs use it), with period 1/mu and delay 3/mu, unit peak:
// u = -sqrt(2e) x exp(-x^2), x = pi (mu t - 3).
__device__ __forceinline__ double gauss1(double t, double mu) {
    const double pi = 3.141592653589793238462643383279502884;
    const double s2e = 2.331643981597124;      // sqrt(2 e)
    const double x = pi * (mu * t - 3.0);
    return -s2e * x * exp(-x * x);
}

// d u / d mu of gauss1 (the delay moves with mu): dx/dmu = pi t.
__device__ __forceinline__ double gauss1_dmu(double t, double mu) {
    const double pi = 3.141592653589793238462643383279502884;
    const double s2e = 2.331643981597124;
    const double x = pi * (mu * t - 3.0);
    return -s2e * (1.0 - 2.0 * x * x) * exp(-x * x) * (pi * t);
}

// Source kinds (rom_config.flags ROM_SOURCE_GAUSS1 selects the second).
enum Source { kRicker = 0, kGauss1 = 1 };

// Both signals are a polynomial times exp(-x^2) in x = pi (mu t - d):
// Ricker d = 1.5, (1 - 2 x^2); gauss1 d = 3, -sqrt(2e) x.  One expression
// with the coefficients chosen per kind (scalar selects, a single exp) gives
// each signal exactly as ricker() and gauss1() above compute it: the zero
// coefficients add exact zeros.
__device__ __forceinline__ double forcing(int src, double t, double mu) {
    const double pi = 3.141592653589793238462643383279502884;
    const bool g = src == kGauss1;
    const double d = g ? 3.0 : 1.5, c0 = g ? 0.0 : 1.0, c1 = g ? -2.331643981597124 : 0.0, c2 = g ? 0.0 : -2.0;
    const double x = pi * (mu * t - d);
    const double a = x * x;
    return ((c0 + c1 * x) + c2 * a) * exp(-a);
}

__device__ __forceinline__ double forcing_dmu(int src, double t, double mu) {
    return src == kGauss1 ? gauss1_dmu(t, mu) : ricker_dmu(t, mu);
}

// State increment in double-float arithmetic, one element:
//   (vh, vl) += d * ((H + L) + (F + Fe))
// where (H, L) is the compensated product row, (F, Fe) the forcing term and d
// the FP32 step.  Every rounding error of the increment is carried into the
// low word; (vh, vl) is renormalised so |vl| <= ulp(vh)/2.
__device__ __forceinline__ void comp_update(float &vh, float &vl, float H, float L, float F,
                                            float Fe, float d) {
    float s1, e1;
    two_sum(H, F, s1, e1);
    float tlo = (L + Fe) + e1;
    float p = d * s1;
    float pe = fmaf(d, s1, -p);
    float inclo = fmaf(d, tlo, pe);
    float s2, e2;
    two_sum(vh, p, s2, e2);
    float lo = (vl + e2) + inclo;
    float s3, e3;
    two_sum(s2, lo, s3, e3);
    vh = s3;
    vl = e3;
}

}  // namespace dev
}  // namespace rom
