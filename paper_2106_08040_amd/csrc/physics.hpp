// Particle scalars of the Neel rotation model (arXiv 2106.08040, constants listed after
// Eq. convection; beta and V_C as in model M0).  Host and device.
#pragma once
#include <cmath>

#if defined(__HIP__)
#include <hip/hip_runtime.h>
#define FPN_HD __host__ __device__
#else
#define FPN_HD
#endif

namespace fpn {

constexpr double kPi = 3.14159265358979323846;
constexpr double kBoltzmann = 1.380649e-23;     // J/K (exact SI)
constexpr double kGammaE = 1.76085963023e11;    // rad/(s T), electron gyromagnetic ratio

// inv2tau = 1/(2 tau), tau = V_C M_S / (2 k_B T gamma~ alpha), gamma~ = gamma/(1+alpha^2)
// beta_T  = V_C M_S / (k_B T): beta * H for H = B/mu0, per tesla of B
// sigma   = K V_C / (k_B T)
struct ParticleScalars {
  double inv2tau, sigma, beta_T, alpha;
};

FPN_HD inline ParticleScalars particle_scalars(double D, double Ms, double K, double alpha, double T) {
  const double V = kPi * D * D * D / 6.0;
  const double gt = kGammaE / (1.0 + alpha * alpha);
  const double tau = V * Ms / (2.0 * kBoltzmann * T * gt * alpha);
  ParticleScalars s;
  s.inv2tau = 0.5 / tau;
  s.beta_T = V * Ms / (kBoltzmann * T);
  s.sigma = K * V / (kBoltzmann * T);
  s.alpha = alpha;
  return s;
}

}  // namespace fpn
