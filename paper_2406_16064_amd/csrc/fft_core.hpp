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

#include "gmem.hpp"

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

// 16 points as 4 x 4: length-4 transforms over n1 of x[4 n1 + n2], twiddles
// W16^(n2 k1), length-4 transforms over n2; output in natural order.
template <typename T, bool INV>
__device__ __forceinline__ void dft16(Cx<T>* v) {
  Cx<T> a[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    a[n2][0] = v[n2]; a[n2][1] = v[4 + n2]; a[n2][2] = v[8 + n2]; a[n2][3] = v[12 + n2];
    dft4<T, INV>(a[n2]);
  }
  const T c1 = T(0.92387953251128675612818318939679);  // cos(pi/8)
  const T s1 = T(0.38268343236508977172845998403040);  // sin(pi/8)
  const T r2 = T(0.70710678118654752440084436210485);  // cos(pi/4)
  // W16^m = exp(-+ 2 pi i m / 16) for the products m = n2 k1 (n2, k1 = 1..3)
  auto tw = [&](Cx<T> x, int m) -> Cx<T> {
    T c, s;
    switch (m) {
      case 1: c = c1; s = s1; break;
      case 2: c = r2; s = r2; break;
      case 3: c = s1; s = c1; break;
      case 4: c = T(0); s = T(1); break;
      case 6: c = -r2; s = r2; break;
      default: c = -c1; s = -s1; break;  // m = 9: cos(9 pi/8), sin(9 pi/8) -> (-c1, -s1)
    }
    if (!INV) s = -s;  // forward: exp(-i theta)
    return Cx<T>{x.x * c - x.y * s, x.x * s + x.y * c};
  };
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) a[n2][k1] = tw(a[n2][k1], n2 * k1);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    Cx<T> b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
    dft4<T, INV>(b);
    v[k1] = b[0]; v[k1 + 4] = b[1]; v[k1 + 8] = b[2]; v[k1 + 12] = b[3];
  }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dftR(Cx<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 3) dft3<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else if constexpr (R == 8) dft8<T, INV>(v);
  else dft16<T, INV>(v);
}


// One Stockham stage of radix R (2, 3, 4, 8, 16) on every column of the
// workgroup.  Per thread at most NB = max(1, 16/R) butterflies (host
// guarantees L/R <= NB*tpc).
// Twiddle read: from a table in LDS (TWL, copied there by the kernel) or in
// global memory.
template <typename T, bool TWL>
__device__ __forceinline__ Cx<T> twiddle(const Cx<T>* tw, int i) {
  if constexpr (TWL) return tw[i];
  else return gld(tw + i);
}

// v[r] *= w^r, r = 1..R-1, with w = table[i] (conjugated for INV): one table
// read per butterfly, the powers by products (r < 8: a chain of at most 6;
// R = 16 also reads w^4 = table[4 i] so that every power is within 5 products)
template <typename T, int R, bool INV, bool TWL>
__device__ __forceinline__ void twiddle_powers(Cx<T>* v, const Cx<T>* tw, int i) {
  Cx<T> w1 = twiddle<T, TWL>(tw, i);
  if (INV) w1.y = -w1.y;
  if constexpr (R == 16) {
    Cx<T> w4 = twiddle<T, TWL>(tw, 4 * i);
    if (INV) w4.y = -w4.y;
    const Cx<T> w2 = cmul(w1, w1), w3 = cmul(w2, w1);
    const Cx<T> w8 = cmul(w4, w4), w12 = cmul(w8, w4);
    const Cx<T> lo[4] = {Cx<T>{T(1), T(0)}, w1, w2, w3};
    const Cx<T> hi[4] = {Cx<T>{T(1), T(0)}, w4, w8, w12};
#pragma unroll
    for (int r = 1; r < 16; ++r) {
      const int a = r >> 2, b = r & 3;
      const Cx<T> w = a == 0 ? lo[b] : (b == 0 ? hi[a] : cmul(hi[a], lo[b]));
      v[r] = cmul(v[r], w);
    }
  } else {
    Cx<T> w = w1;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      v[r] = cmul(v[r], w);
      if (r + 1 < R) w = cmul(w, w1);
    }
  }
}

struct NoHook {
  __device__ __forceinline__ void operator()() const {}
};

template <typename T, int R, bool INV, bool TWL = false>
__device__ __forceinline__ void fft_stage(Cx<T>* __restrict__ col, int L, int Ns, int lane, int tpc,
                                          bool active, const Cx<T>* __restrict__ tw) {
  constexpr int NB = R >= 16 ? 1 : 16 / R;
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
      if (Ns > 1) twiddle_powers<T, R, INV, TWL>(v[k], tw, kk * tstep);
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
// tw: the twiddle table to use (p.tw, or its copy in LDS when TWL).
// R16: the plan may hold radix-16 stages (otherwise their code is left out,
// which keeps the register count of kernels that never need them lower).
template <typename T, bool INV, bool TWL = false, bool R16 = false>
__device__ __forceinline__ void fft_columns(Cx<T>* lds, const FftDesc<T>& p, int cs, int ncol, int tpc,
                                            const Cx<T>* tw) {
  const int c = threadIdx.x / tpc;
  const int lane = threadIdx.x % tpc;
  const bool active = c < ncol;
  Cx<T>* col = lds + (active ? c : 0) * cs;
  int ns = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int R = radix_of(p.code, s);
    switch (R) {
      case 16:
        if constexpr (R16) fft_stage<T, 16, INV, TWL>(col, p.L, ns, lane, tpc, active, tw);
        break;
      case 8: fft_stage<T, 8, INV, TWL>(col, p.L, ns, lane, tpc, active, tw); break;
      case 4: fft_stage<T, 4, INV, TWL>(col, p.L, ns, lane, tpc, active, tw); break;
      case 3: fft_stage<T, 3, INV, TWL>(col, p.L, ns, lane, tpc, active, tw); break;
      default: fft_stage<T, 2, INV, TWL>(col, p.L, ns, lane, tpc, active, tw); break;
    }
    ns *= R;
  }
}

template <typename T, bool INV, bool R16 = false>
__device__ __forceinline__ void fft_columns(Cx<T>* lds, const FftDesc<T>& p, int cs, int ncol, int tpc) {
  fft_columns<T, INV, false, R16>(lds, p, cs, ncol, tpc, p.tw);
}

// ---------------------------------------------------------------------------
// Same transform with the first stage reading its inputs straight from global
// memory (ld(c, e) -> element e of column c, zero padding included) and/or the
// last stage writing straight to global memory (st(c, e, v)); the stages in
// between go through LDS.  Saves one LDS round trip and one barrier at each
// end.  The caller makes sure LDS is free before the call when GIN, and syncs
// before reusing LDS after the call when GOUT.
// ---------------------------------------------------------------------------
template <typename T, int R, bool INV, bool GIN, bool GOUT, bool TWL, class Load, class Store, class Hook>
__device__ __forceinline__ void fft_stage_io(Cx<T>* __restrict__ col, int c, int L, int Ns, int lane, int tpc,
                                             bool active, const Cx<T>* __restrict__ tw, Load& ld, Store& st,
                                             Hook& hook) {
  constexpr int NB = R >= 16 ? 1 : 16 / R;
  const int nbf = L / R;
  Cx<T> v[NB][R];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int j = lane + k * tpc;
    if (active && j < nbf) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (GIN) v[k][r] = ld(c, j + r * nbf);
        else v[k][r] = col[pidx(j + r * nbf)];
      }
    }
  }
  if constexpr (!GIN) __syncthreads();
  if constexpr (GIN) hook();  // runs with this stage's global loads in flight
  const int tstep = L / (Ns * R);
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int j = lane + k * tpc;
    if (active && j < nbf) {
      const int kk = j % Ns;
      if (Ns > 1) twiddle_powers<T, R, INV, TWL>(v[k], tw, kk * tstep);
      dftR<T, R, INV>(v[k]);
      const int base = (j / Ns) * Ns * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (GOUT) st(c, base + r * Ns, v[k][r]);
        else col[pidx(base + r * Ns)] = v[k][r];
      }
    }
  }
  if constexpr (!GOUT) __syncthreads();
}

template <typename T, bool INV, bool GIN, bool GOUT, bool TWL, bool R16, class Load, class Store, class Hook>
__device__ __forceinline__ void fft_stage_any(Cx<T>* col, int c, const FftDesc<T>& p, const Cx<T>* tw, int s,
                                              int ns, int lane, int tpc, bool active, Load& ld, Store& st,
                                              Hook& hook) {
  switch (radix_of(p.code, s)) {
    case 16:
      if constexpr (R16) fft_stage_io<T, 16, INV, GIN, GOUT, TWL>(col, c, p.L, ns, lane, tpc, active, tw, ld, st, hook);
      break;
    case 8: fft_stage_io<T, 8, INV, GIN, GOUT, TWL>(col, c, p.L, ns, lane, tpc, active, tw, ld, st, hook); break;
    case 4: fft_stage_io<T, 4, INV, GIN, GOUT, TWL>(col, c, p.L, ns, lane, tpc, active, tw, ld, st, hook); break;
    case 3: fft_stage_io<T, 3, INV, GIN, GOUT, TWL>(col, c, p.L, ns, lane, tpc, active, tw, ld, st, hook); break;
    default: fft_stage_io<T, 2, INV, GIN, GOUT, TWL>(col, c, p.L, ns, lane, tpc, active, tw, ld, st, hook); break;
  }
}

// hook(): called once by every thread inside the first stage, after that
// stage's global loads are issued (GIN only) -- e.g. to copy a twiddle table
// into LDS while the data loads are in flight.  tw as for fft_columns.
template <typename T, bool INV, bool GIN, bool GOUT, bool TWL, class Load, class Store, class Hook,
          bool R16 = false>
__device__ __forceinline__ void fft_columns_io(Cx<T>* lds, const FftDesc<T>& p, const Cx<T>* tw, int cs, int ncol,
                                               int tpc, Load ld, Store st, Hook hook) {
  const int c = threadIdx.x / tpc;
  const int lane = threadIdx.x % tpc;
  const bool active = c < ncol;
  Cx<T>* col = lds + (active ? c : 0) * cs;
  if (p.nst == 0) {  // length 1: identity
    if constexpr (GIN) hook();
    if (active && lane == 0) {
      Cx<T> v;
      if constexpr (GIN) v = ld(c, 0);
      else v = col[0];
      if constexpr (GOUT) st(c, 0, v);
      else col[0] = v;
    }
    if constexpr (!GOUT) __syncthreads();
    return;
  }
  if (p.nst == 1) {
    fft_stage_any<T, INV, GIN, GOUT, TWL, R16>(col, c, p, tw, 0, 1, lane, tpc, active, ld, st, hook);
    return;
  }
  fft_stage_any<T, INV, GIN, false, TWL, R16>(col, c, p, tw, 0, 1, lane, tpc, active, ld, st, hook);
  int ns = radix_of(p.code, 0);
  for (int s = 1; s + 1 < p.nst; ++s) {
    fft_stage_any<T, INV, false, false, TWL, R16>(col, c, p, tw, s, ns, lane, tpc, active, ld, st, hook);
    ns *= radix_of(p.code, s);
  }
  fft_stage_any<T, INV, false, GOUT, TWL, R16>(col, c, p, tw, p.nst - 1, ns, lane, tpc, active, ld, st, hook);
}

template <typename T, bool INV, bool GIN, bool GOUT, bool R16 = false, class Load, class Store>
__device__ __forceinline__ void fft_columns_io(Cx<T>* lds, const FftDesc<T>& p, int cs, int ncol, int tpc, Load ld,
                                               Store st) {
  fft_columns_io<T, INV, GIN, GOUT, false, Load, Store, NoHook, R16>(lds, p, p.tw, cs, ncol, tpc, ld, st, NoHook{});
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Remap so that consecutive tiles -- which share cache lines and halo
// rows -- run on the same XCD.  Identity when the grid is not a multiple of 8.
__device__ __forceinline__ long long xcd_tile(long long bid, long long nblk) {
  if (nblk % 8 != 0) return bid;
  return (bid % 8) * (nblk / 8) + bid / 8;
}

// ---------------------------------------------------------------------------
// Register-resident transform of compile-time length L held by one thread
// (Stockham stages unrolled at compile time; radices 8/4/2/3).  Twiddles come
// from the uniform table tw[TS * m] = exp(-2 pi i m / L): TS = 1 for a table
// of length L, TS = 2 when the table belongs to a transform twice as long.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int reg_radix(int rem) {
  return (rem % 8 == 0 && rem != 16) ? 8 : (rem % 4 == 0) ? 4 : (rem % 2 == 0) ? 2 : 3;
}

template <typename T, int L, int Ns, bool INV, int TS = 1>
struct RegFft {
  static __device__ __forceinline__ void run(Cx<T>* v, const Cx<T>* __restrict__ tw) {
    constexpr int R = reg_radix(L / Ns);
    constexpr int NB = L / R;
    Cx<T> o[L];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int kk = j % Ns;
      Cx<T> a[R];
#pragma unroll
      for (int r = 0; r < R; ++r) a[r] = v[j + r * NB];
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          Cx<T> w = ldu(tw + TS * (r * kk * (L / (Ns * R))));  // same entry in every lane
          if (INV) w.y = -w.y;
          a[r] = cmul(a[r], w);
        }
      }
      dftR<T, R, INV>(a);
      const int base = (j / Ns) * Ns * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) o[base + r * Ns] = a[r];
    }
#pragma unroll
    for (int i = 0; i < L; ++i) v[i] = o[i];
    RegFft<T, L, Ns * R, INV, TS>::run(v, tw);
  }
};

template <typename T, int L, bool INV, int TS>
struct RegFft<T, L, L, INV, TS> {
  static __device__ __forceinline__ void run(Cx<T>*, const Cx<T>*) {}
};

}  // namespace mmx
