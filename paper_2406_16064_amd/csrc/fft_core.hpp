// LDS-resident mixed-radix Stockham FFT for gfx950 workgroups.
//
// A workgroup holds `ncol` complex columns of length L in LDS (column c starts
// at c*cs, element i sits at pidx(i) -- one padding slot every 8 elements
// breaks the power-of-two strides of the first stages across the LDS banks).
// Threads are split into ncol groups of tpc threads; each group transforms its
// own column, stage by stage, with the butterflies of radix 2, 3, 4 or 8 held
// in registers.  Stockham autosort: the output comes out in natural order.
// Twiddles come from a table exp(-2 pi i m / L) computed in FP64 on the host.
#pragma once

#include "mm_internal.hpp"

namespace mmx {

__device__ __forceinline__ int pidx(int i) { return i + (i >> 3); }
__host__ __device__ inline int col_stride(int L) { return L + (L >> 3) + 1; }

template <typename T, bool INV>
__device__ __forceinline__ Cx<T> mul_mi(Cx<T> a) {  // a * (-i) forward, a * (+i) inverse
  return INV ? Cx<T>{-a.y, a.x} : Cx<T>{a.y, -a.x};
}

template <typename T, bool INV>
__device__ __forceinline__ void dft2(Cx<T>* v) {
  Cx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft3(Cx<T>* v) {
  const T c = T(-0.5);
  const T s = T(0.86602540378443864676372317075294);  // sin(2 pi / 3)
  Cx<T> t = cadd(v[1], v[2]);
  Cx<T> d = csub(v[1], v[2]);
  Cx<T> m = {v[0].x + c * t.x, v[0].y + c * t.y};
  Cx<T> r = mul_mi<T, INV>(Cx<T>{s * d.x, s * d.y});  // -i s d (fwd), +i s d (inv)
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, r);
  v[2] = csub(m, r);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(Cx<T>* v) {
  Cx<T> t0 = cadd(v[0], v[2]);
  Cx<T> t1 = csub(v[0], v[2]);
  Cx<T> t2 = cadd(v[1], v[3]);
  Cx<T> t3 = mul_mi<T, INV>(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(Cx<T>* v) {
  Cx<T> e[4] = {v[0], v[2], v[4], v[6]};
  Cx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, INV>(e);
  dft4<T, INV>(o);
  const T r = T(0.70710678118654752440084436210485);
  // o[k] *= W8^k, W8 = exp(-+ i pi/4)
  Cx<T> o1 = INV ? Cx<T>{r * (o[1].x - o[1].y), r * (o[1].x + o[1].y)}
                 : Cx<T>{r * (o[1].x + o[1].y), r * (o[1].y - o[1].x)};
  Cx<T> o2 = mul_mi<T, INV>(o[2]);
  Cx<T> o3 = INV ? Cx<T>{-r * (o[3].x + o[3].y), r * (o[3].x - o[3].y)}
                 : Cx<T>{r * (o[3].y - o[3].x), -r * (o[3].x + o[3].y)};
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], o1);
  v[5] = csub(e[1], o1);
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = cadd(e[3], o3);
  v[7] = csub(e[3], o3);
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dftR(Cx<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 3) dft3<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else dft8<T, INV>(v);
}

// One Stockham stage of radix R on every column of the workgroup.
// Per thread at most NB = 16/R butterflies (host guarantees L/R <= NB*tpc).
template <typename T, int R, bool INV>
__device__ __forceinline__ void fft_stage(Cx<T>* __restrict__ col, int L, int Ns, int lane, int tpc,
                                          bool active, const Cx<T>* __restrict__ tw) {
  constexpr int NB = 16 / R;
  const int nbf = L / R;
  Cx<T> v[NB][R];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int j = lane + k * tpc;
    if (active && j < nbf) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[k][r] = col[pidx(j + r * nbf)];
    }
  }
  __syncthreads();
  const int tstep = L / (Ns * R);
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int j = lane + k * tpc;
    if (active && j < nbf) {
      const int kk = j % Ns;
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          Cx<T> w = tw[r * kk * tstep];
          if (INV) w.y = -w.y;
          v[k][r] = cmul(v[k][r], w);
        }
      }
      dftR<T, R, INV>(v[k]);
      const int base = (j / Ns) * Ns * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) col[pidx(base + r * Ns)] = v[k][r];
    }
  }
  __syncthreads();
}

// Full transform of every column.  Must be called by all threads of the
// workgroup (it contains barriers); threads with active == false only sync.
template <typename T, bool INV>
__device__ void fft_columns(Cx<T>* lds, const FftPlan<T>& p, int cs, int ncol, int tpc) {
  const int c = threadIdx.x / tpc;
  const int lane = threadIdx.x % tpc;
  const bool active = c < ncol;
  Cx<T>* col = lds + (active ? c : 0) * cs;
  for (int s = 0; s < p.nst; ++s) {
    switch (p.rad[s]) {
      case 8: fft_stage<T, 8, INV>(col, p.L, p.ns[s], lane, tpc, active, p.tw); break;
      case 4: fft_stage<T, 4, INV>(col, p.L, p.ns[s], lane, tpc, active, p.tw); break;
      case 3: fft_stage<T, 3, INV>(col, p.L, p.ns[s], lane, tpc, active, p.tw); break;
      default: fft_stage<T, 2, INV>(col, p.L, p.ns[s], lane, tpc, active, p.tw); break;
    }
  }
}

}  // namespace mmx
