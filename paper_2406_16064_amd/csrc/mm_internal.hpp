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
// lowest bits; the spans follow as running products.  Scalars only, so it
// lives in scalar registers.
template <typename T> struct FftDesc {
  int L;
  int nst;
  uint32_t code;
  uint32_t pad;
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
  for (int s = 0; s < p.nst; ++s) {
    const uint32_t c = p.rad[s] == 2 ? 0u : p.rad[s] == 3 ? 1u : p.rad[s] == 4 ? 2u : p.rad[s] == 8 ? 3u : 4u;
    d.code |= c << (3 * s);
  }
  return d;
}

// Per-instance coefficients, precomputed in FP64 on the host.
struct DevParams {
  double Ms;
  double cex[3];     // 2A / (mu0 Ms d_a^2) for a = x, y, z
  double cdmi[2];    // D / (mu0 Ms d_a) for a = x, y
  double can;        // 2 Ku / (mu0 Ms)
  double u[3];       // easy axis, normalised
  double H[3];       // applied field
  double g1, g2;     // -gamma/(1+alpha^2), -alpha gamma/(1+alpha^2)
  double demag_scale;  // -Ms / (Px Py Pz)
  uint32_t terms;
  uint32_t pad;
};

// Per-instance Dormand-Prince controller state in device memory.
struct DevCtl {
  double t, h, t_end, rtol, h_min, h_max;
  double h_att;           // step size of the attempt in flight
  double last_err;        // err / rtol of the last attempt
  unsigned long long err_bits;  // running max of ||e_i|| (bits of a non-negative double)
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
