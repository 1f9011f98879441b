// Broken power-law CR spectrum: the table of incomplete synchrotron moments
// that the march kernels interpolate, and its host-side builder.
//
// Electrons of the spectrum N(gamma) = C gamma^-a1 (gamma < gamma_b),
// C gamma_b^(a2 - a1) gamma^-a2 (gamma >= gamma_b) emit at frequency nu the
// single-electron spectrum integrated over gamma; in x = nu / nu_c(gamma) the
// electrons below the break emit at x > xb = 4 pi nu m c / (3 q B_perp gamma_b^2).
// For one power law of index a the gamma-integral is the complete x-moment of
// order mu = (a - 3) / 2 of F(x) = x int_x^inf K_5/3 (of G(x) = x K_2/3(x) for
// the polarised part), i.e. Eqs. ji and jp; for the broken law each side of the
// break takes the part of its moment on its side of xb:
//
//   j_I = j_I(a1) (1 - S_F(a1, xb)) + gamma_b^(a2 - a1) j_I(a2) S_F(a2, xb),
//
// S(a, xb) = int_0^xb x^mu F dx / int_0^inf x^mu F dx, and the same for j_P with
// G.  The table holds, at t = log2 xb on a uniform grid, g = S 2^(-p t) with
// p = mu + 4/3 = a/2 - 1/6 (the power S falls off with at small xb, so g tends
// to a constant there and keeps its relative accuracy) and h dg/dt, for
// (F, a1), (G, a1), (F, a2), (G, a2): a cubic Hermite interpolant in t per
// function.  Below the first node g is held constant (the leading power law,
// next order ~ xb^(2/3) ~ 1e-8 there); above the last S = 1 to ~e^-128.
//
// A second part of the table, for the gradient in the indices, holds per node
// dg/da (each function's derivative in its own index) and h d2g/da dt, laid
// out like the first part and interpolated the same way.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

namespace sm {

constexpr double kBpT0 = -40.0;                 // log2 xb of node 0
constexpr int kBpPerOctave = 16;                // nodes per unit of t
constexpr int kBpNodes = 47 * kBpPerOctave + 1;  // t in [-40, 7]
constexpr size_t kBpPartFloats = (size_t)kBpNodes * 8;  // one part: nodes x two float4
constexpr size_t kBpTableBytes = 2 * kBpPartFloats * sizeof(float);
// the indices the table is built for: above the pole of Eq. ji's Gamma
// function at 1/3, and up to 6 (the FP32 powers of the kernels stay in range)
constexpr double kBpAlphaMin = 1.0 / 3.0, kBpAlphaMax = 6.0;

// Fills nodes[2][kBpNodes][8]: part 0 (g_F1, g_G1, g_F2, g_G2, h dg_F1/dt, ..),
// part 1 (dg_F1/da1, dg_G1/da1, dg_F2/da2, dg_G2/da2, h d2g_F1/da1 dt, ..) for
// indices a1, a2.  Returns false with a message if the moments it integrates
// do not reach their closed forms (a self-check of the quadrature).
bool bp_build_table(double a1, double a2, float* nodes, std::string* err);

// p = a/2 - 1/6 of an index
inline double bp_power(double a) { return 0.5 * a - 1.0 / 6.0; }

}  // namespace sm
