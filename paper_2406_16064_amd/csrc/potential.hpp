// Launch-side view of the scalar-potential demag route (potential.hip).
#pragma once

#include "kernels.hpp"

namespace mmx {

// Tables of a group's potential route: the folded real kernel spectrum
// kp[3][Kz][Xp][Ky] (S^_a = -i Phi C_a), the half-cell phase factors
// phx[kx] = exp(-i pi kx / Px) (Xp entries), phy (Py), phz (Pz), and the edge
// difference factors -1 / (4 d_a).
template <typename T> struct PotTab {
  const T* kp;
  const Cx<T>* phx;
  const Cx<T>* phy;
  const Cx<T>* phz;
  double gdx, gdy, gdz;
};

// Launch shapes of the potential passes (derived from the plan's tuning).
struct PotShape {
  int qz, tpc_z;          // z pass: (kx, ky) points per workgroup, threads per transform
  int cb_y, tpc_y;        // y inverse: kx columns per workgroup, threads per transform
  int nt_x, tpc_x;        // x inverse: threads, threads per transform
  int cpt_x;              // x inverse: epilogue cells per thread (0: a loop)
  size_t lds_x;           // x inverse LDS bytes
  int sl_y, cb_ys;        // y inverse compiled for Py = sl_y (0: general): columns per workgroup
};

template <typename T>
PotShape pot_shape(const HotPlan<T>& h);

// The route's launch shapes fit the group (nz >= 2, LDS, threads per transform
// at least tpc_x_min).
template <typename T>
bool pot_supported(const HotPlan<T>& h, int tpc_x_min);

// One evaluation (single group): x and y forward (the Newell route's passes),
// z with the potential product, y inverse, x inverse with the edge
// differences and the epilogue `mode` (MODE_FIELD, MODE_RHS, MODE_ENERGY, or
// the Runge-Kutta MODE_STAGE / MODE_ERROR: no fused forward pass, the error
// pass's last workgroup of an instance takes the step decision).
// pass_mask bit p launches pass p (0 x, 1 y, 2 z, 3 y inverse, 4 x inverse).
template <typename T>
hipError_t launch_potential(const GroupSet<T>& gs, const Epi<T>* epis, const PotTab<T>& pt, int mode,
                            hipStream_t s, unsigned pass_mask = ~0u);

}  // namespace mmx
