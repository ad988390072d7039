// Pointwise compressible Navier-Stokes fluxes (paper eq. C4-C6) for device
// code, templated on the scalar so that forward-mode derivatives come from a
// one-direction dual number.  Acoustic scaling: gamma P = rho T,
// P = (gamma-1)(rhoE - |m|^2/(2 rho)), tau = (mu/Re_c)(grad v + grad v^T -
// (2/d) div v I), heat flux -kappa grad T with kappa = mu/(Re_c Pr (gamma-1)).
#pragma once
#include "internal.h"

struct Dl {
  double v, d;
};
__device__ __forceinline__ Dl operator+(Dl a, Dl b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dl operator-(Dl a, Dl b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dl operator-(Dl a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dl operator*(Dl a, Dl b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dl operator/(Dl a, Dl b) {
  double inv = 1.0 / b.v;
  return {a.v * inv, (a.d - a.v * inv * b.d) * inv};
}
__device__ __forceinline__ Dl operator+(Dl a, double b) { return {a.v + b, a.d}; }
__device__ __forceinline__ Dl operator+(double b, Dl a) { return {a.v + b, a.d}; }
__device__ __forceinline__ Dl operator-(Dl a, double b) { return {a.v - b, a.d}; }
__device__ __forceinline__ Dl operator-(double b, Dl a) { return {b - a.v, -a.d}; }
__device__ __forceinline__ Dl operator*(Dl a, double b) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ Dl operator*(double b, Dl a) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ Dl operator/(Dl a, double b) { return {a.v / b, a.d / b}; }

__device__ __forceinline__ double val(double x) { return x; }
__device__ __forceinline__ double val(Dl x) { return x.v; }

// F_k (inviscid) and/or G_k (viscous) of eq. (C5): out[k * NS + c] += ...
template <int D, class S>
__device__ __forceinline__ void ns_flux(const S* u, const S* q, const PhysDev& ph, S* out, bool inv, bool vis) {
  constexpr int NS = D + 2;
  const S rho = u[0];
  const S irho = S{1.0} / rho;
  S v[D];
#pragma unroll
  for (int j = 0; j < D; ++j) v[j] = u[j + 1] * irho;
  S ke = v[0] * u[1];
#pragma unroll
  for (int j = 1; j < D; ++j) ke = ke + v[j] * u[j + 1];
  const S P = (ph.gamma - 1.0) * (u[D + 1] - 0.5 * ke);
  if (inv) {
#pragma unroll
    for (int k = 0; k < D; ++k) {
      out[k * NS + 0] = out[k * NS + 0] + u[k + 1];
#pragma unroll
      for (int j = 0; j < D; ++j) {
        S t = u[j + 1] * v[k];
        if (j == k) t = t + P;
        out[k * NS + j + 1] = out[k * NS + j + 1] + t;
      }
      out[k * NS + D + 1] = out[k * NS + D + 1] + (u[D + 1] + P) * v[k];
    }
  }
  if (vis) {
    const S E = u[D + 1] * irho;
    S dv[D][D], dE[D], dT[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
#pragma unroll
      for (int j = 0; j < D; ++j) dv[j][k] = (q[k * NS + j + 1] - v[j] * q[k * NS + 0]) * irho;
      dE[k] = (q[k * NS + D + 1] - E * q[k * NS + 0]) * irho;
    }
    const double gg = ph.gamma * (ph.gamma - 1.0);
#pragma unroll
    for (int k = 0; k < D; ++k) {
      S s = v[0] * dv[0][k];
#pragma unroll
      for (int j = 1; j < D; ++j) s = s + v[j] * dv[j][k];
      dT[k] = gg * (dE[k] - s);
    }
    S div = dv[0][0];
#pragma unroll
    for (int j = 1; j < D; ++j) div = div + dv[j][j];
    const double cm = ph.mu / ph.Re_c, lam = -2.0 / D;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      S tv = S{0.0};
#pragma unroll
      for (int j = 0; j < D; ++j) {
        S tjk = cm * (dv[j][k] + dv[k][j]);
        if (j == k) tjk = tjk + (cm * lam) * div;
        out[k * NS + j + 1] = out[k * NS + j + 1] - tjk;
        tv = tv + tjk * v[j];
      }
      out[k * NS + D + 1] = out[k * NS + D + 1] - (tv + ph.kappa * dT[k]);
    }
  }
}

template <int D>
__device__ __forceinline__ double pressure(const double* u, const PhysDev& ph) {
  double ke = 0.0;
#pragma unroll
  for (int j = 0; j < D; ++j) ke += u[j + 1] * u[j + 1];
  return (ph.gamma - 1.0) * (u[D + 1] - 0.5 * ke / u[0]);
}
