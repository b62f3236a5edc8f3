// Internal types shared by the HIP kernels and the host runtime of the
// micromagnetics hot path (gfx950).  Not part of the C interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mm.h"

namespace mmx {

constexpr double kMu0 = 4e-7 * 3.14159265358979323846264338327950288;
constexpr int kMaxFFT = 2048;     // longest 1-D transform supported
constexpr int kMaxStages = 12;    // radix stages of one transform

// Aligned to its full size so that one complex moves in one 8- or 16-byte access.
template <typename T> struct alignas(2 * sizeof(T)) Cx { T x, y; };

template <typename T> __device__ __forceinline__ Cx<T> cadd(Cx<T> a, Cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ Cx<T> csub(Cx<T> a, Cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ Cx<T> cconj(Cx<T> a) { return {a.x, -a.y}; }
template <typename T> __device__ __forceinline__ Cx<T> cscale(Cx<T> a, T s) { return {a.x * s, a.y * s}; }

// Radix plan of one transform length: L = prod(rad[s]); stage s has span ns[s]
// (product of the radices before it).  tw points at exp(-2 pi i m / L), m < L.
template <typename T> struct FftPlan {
  int L;
  int nst;
  int rad[kMaxStages];
  int ns[kMaxStages];
  const Cx<T>* tw;
};

// The same plan in the form the kernels take: the radices packed three bits a
// stage (0: 2, 1: 3, 2: 4, 3: 8, 4: 16; at most 10 stages), first stage in the
// lowest bits, and two flags above them (first / last radix even, so that a
// half-length input / output end can be specialised); the spans follow as
// running products.  psh: the LDS padding shift (3: one slot every 8
// elements; 31: none), 3 only where every stage's strides keep LDS addresses
// linear.  Scalars only, so it lives in scalar registers.
// Radices of a power-of-two length 2^a, as plans take them (radix-3 stages,
// for 3-smooth lengths, are inserted after the first stage by the host):
// with a16 and a > 9, sixteens then the remainder 2^(a mod 4); otherwise
// eights, then the remainder as 4 (a mod 3 = 2), 4 + 4 in place of one 8
// (a mod 3 = 1, a > 3) or 2 (a = 1).  Shared by the host plans and the
// kernels compiled for one fixed length.
__host__ __device__ constexpr int p2_nst(int a, bool a16) {
  if (a16 && a > 9) return a / 4 + (a % 4 != 0 ? 1 : 0);
  const int n8 = a / 3, rem = a % 3;
  if (rem == 1 && n8 > 0) return n8 + 1;
  return n8 + (rem != 0 ? 1 : 0);
}
__host__ __device__ constexpr int p2_radix(int a, bool a16, int s) {
  if (a16 && a > 9) return s < a / 4 ? 16 : 1 << (a % 4);
  int n8 = a / 3;
  const int rem = a % 3;
  int t0 = 0, t1 = 0;
  if (rem == 1 && n8 > 0) { --n8; t0 = 4; t1 = 4; }
  else if (rem == 1) t0 = 2;
  else if (rem == 2) t0 = 4;
  return s < n8 ? 8 : s == n8 ? t0 : t1;
}
__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }
// Largest radix of that plan
__host__ __device__ constexpr int p2_maxradix(int L, bool a16) {
  int r = 1;
  for (int s = 0; s < p2_nst(ilog2c(L), a16); ++s) r = p2_radix(ilog2c(L), a16, s) > r ? p2_radix(ilog2c(L), a16, s) : r;
  return r;
}
// LDS padding shift of the plan of a power-of-two length (the rule of
// describe() below: 3 when every stage keeps LDS addresses linear)
__host__ __device__ constexpr int p2_psh(int L, bool a16) {
  const int a = ilog2c(L);
  int ns = 1;
  bool lin = a > 0;
  for (int s = 0; s < p2_nst(a, a16); ++s) {
    const int R = p2_radix(a, a16, s);
    if ((L / R) % 8 != 0) lin = false;
    if (s > 0 && ns % 8 != 0) lin = false;
    ns *= R;
  }
  return lin ? 3 : 31;
}

constexpr uint32_t kFftFirstEven = 1u << 30;
constexpr uint32_t kFftLastEven = 1u << 31;

template <typename T> struct FftDesc {
  int L;
  int nst;
  uint32_t code;
  int psh;
  const Cx<T>* tw;
};

__host__ __device__ inline int radix_of(uint32_t code, int s) {
  const uint32_t c = (code >> (3 * s)) & 7u;
  return c == 0 ? 2 : c == 1 ? 3 : c == 2 ? 4 : c == 3 ? 8 : 16;
}

template <typename T> inline FftDesc<T> describe(const FftPlan<T>& p) {
  FftDesc<T> d{};
  d.L = p.L;
  d.nst = p.nst;
  d.tw = p.tw;
  // padding keeps addresses linear when the reads' stride L/R and (after the
  // first stage) the span are multiples of 8 and the first radix divides 16
  bool lin = p.nst > 0;
  for (int s = 0; s < p.nst; ++s) {
    const int R = p.rad[s];
    const uint32_t c = R == 2 ? 0u : R == 3 ? 1u : R == 4 ? 2u : R == 8 ? 3u : 4u;
    d.code |= c << (3 * s);
    if ((p.L / R) % 8 != 0) lin = false;
    if (s == 0 ? R == 3 : p.ns[s] % 8 != 0) lin = false;
  }
  if (p.nst > 0 && p.rad[0] % 2 == 0) d.code |= kFftFirstEven;
  if (p.nst > 0 && p.rad[p.nst - 1] % 2 == 0) d.code |= kFftLastEven;
  d.psh = lin ? 3 : 31;
  return d;
}

// Per-instance coefficients, precomputed in FP64 on the host.
struct DevParams {
  double Ms;
  double cex[3];     // 2A / (mu0 Ms d_a^2) for a = x, y, z
  double cdmi[3];    // D / (mu0 Ms d_a) for a = x, y, z
  double can;        // 2 Ku / (mu0 Ms)
  double u[3];       // easy axis, normalised
  double H[3];       // applied field
  double g1, g2;     // -gamma/(1+alpha^2), -alpha gamma/(1+alpha^2)
  double demag_scale;  // -Ms / (Px Py Pz)  (cell-based Ms: -1 / (Px Py Pz), Ms inside M)
  uint32_t terms;
  uint32_t pad;
  // general-material form (cell arrays, interlayer coupling, spin torques);
  // there cex = 2/(mu0 d^2), cdmi = 1/(mu0 d), can = 2 Ku / mu0 and each cell
  // applies its own Ms, A_ij, D_ij
  double Mu, Au, Du;   // uniform Ms, A, D (instances without cell arrays)
  double crk;          // J_rkky / (mu0 dz)
  double cdi[3];       // D_int / (mu0 dz)
  double sa, sb;       // a_J / gamma, b_J / gamma
  double sp[3];        // polarisation p, normalised
  double zu[3];        // u_zl[a] / (gamma d_a)
  double zbeta;        // beta
  int32_t k_lo, k_hi;  // interlayer layers
};

// Per-instance Dormand-Prince controller state in device memory.
struct DevCtl {
  double t, h, t_end, rtol, h_min, h_max;
  double h_att;           // step size of the attempt in flight
  double last_err;        // err / rtol of the last attempt
  unsigned long long err_bits;  // running max of ||e_i|| (bits of a non-negative double)
  double stop_dmdt;       // relaxation: stop once the largest |dm/dt| (rad/s) is below; 0 = off
  double last_dmdt;       // largest |dm/dt| (rad/s) at the last check
  unsigned long long dmdt_bits;  // running max of |k_7,i| in the error pass (bits, as err_bits)
  long long n_accept, n_reject, n_attempt, max_attempt;
  long long replay_pos, replay_n;
  int pending_finish;     // 1: the last attempt was accepted and m not yet projected
  int after_reject;
  int done;
  int status;             // mm_status of this instance
  int last_accepted;
  int nonfinite;          // consecutive attempts with a non-finite error norm
  int arrive;             // workgroups of the error pass done with this instance's norm
  int pad;
};

}  // namespace mmx
