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
