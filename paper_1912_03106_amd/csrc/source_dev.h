// Device-side evaluation of the PWM current-density source (Sec. 3.2, 3.3),
// shared by the stepping kernels and the learned coarse propagator.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace mg {

// PWM signal b_p(t) = sgn(sin(2 pi f t + phi_p) - c(t)) (Sec. 3.2, 3.3).
// A difference within 1e-12 of zero is a tie (sgn = 0): the time grids hit
// r = c exactly (reference and carrier both at their peak 1 at t = T/4), and
// the last ulp of the sine must not decide the sign there.  With
// s.signal = 1 the coils follow the sine reference itself (the smooth
// source of the nested-iteration start, Sec. 4.1).
__device__ __forceinline__ double pwm(double t_rel, const SourceDev& s, int p) {
  const double t = t_rel + s.t0;
  const double two_pi = 6.283185307179586;  // 2*pi rounded to double
  const double ref = sin(two_pi * s.freq * t + s.phi[p]);
  if (s.signal == 1) return ref;
  const double x = s.f_carrier * t;
  const double c = (s.carrier == 0) ? 1.0 - 4.0 * fabs(x - floor(x + 0.5))
                                    : 2.0 * (x - floor(x)) - 1.0;
  const double d = ref - c;
  return d > 1e-12 ? 1.0 : (d < -1e-12 ? -1.0 : 0.0);
}

// Amplitude of the coil current density at time t: J0 * amplitude, times the
// start-up factor (1 - cos(pi t / span)) / 2 while t < span (nonlinear
// model, Sec. 3.3); t = t0 + t_rel.
__device__ __forceinline__ double source_scale(double t_rel, const SourceDev& s) {
  const double t = t_rel + s.t0;
  if (s.ramp_span > 0.0 && t < s.ramp_span)
    return s.scale * (0.5 * (1.0 - cos(3.141592653589793 * t / s.ramp_span)));
  return s.scale;
}

}  // namespace mg
