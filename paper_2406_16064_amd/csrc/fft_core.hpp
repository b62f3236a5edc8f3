// LDS-resident mixed-radix Stockham FFT for gfx950 workgroups.
//
// A workgroup holds `ncol` complex columns of length L in LDS (column c starts
// at c*cs, element i sits at pidx(i, sh): with sh = 3 one padding slot every 8
// elements breaks the power-of-two strides across the LDS banks; sh = 31 is
// no padding, for the plans whose strides would not keep addresses linear).
// Threads are split into ncol groups of tpc threads; each group transforms its
// own column, stage by stage, with the butterflies of radix 2, 3, 4, 8 or 16
// held in registers.  Stockham autosort: the output comes out in natural order.
// Twiddles come from a table exp(-2 pi i m / L) computed in FP64 on the host.
#pragma once

#include "gmem.hpp"

namespace mmx {

__device__ __forceinline__ int pidx(int i, int sh) { return i + (i >> sh); }
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

// v[r] *= w^r, r = 1..R-1, with w^r = table[r i] (conjugated for INV).
// Table in LDS (TWL): every power is read (LDS reads instead of the products,
// which would occupy the vector ALU).  Table in global memory: one read, the
// powers by products (r < 8: a chain of at most 6; R = 16 also reads
// w^4 = table[4 i] so that every power is within 5 products).
template <typename T, int R, bool INV, bool TWL>
__device__ __forceinline__ void twiddle_powers(Cx<T>* v, const Cx<T>* tw, int i) {
  if constexpr (TWL) {
#pragma unroll
    for (int r = 1; r < R; ++r) {
      Cx<T> w = tw[r * i];
      if (INV) w.y = -w.y;
      v[r] = cmul(v[r], w);
    }
    return;
  }
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

// Quotient of small non-negative integers by a divisor that is the same in
// every lane, from one float product.  With r = 1/d rounded to nearest and
// h = r/2, fma(n, r, h) = (n + 1/2)/d (1 + e) with |e| < 2^-22.9; for
// n < 2^21 that is off by less than 1/(2d), while (n + 1/2)/d is at least
// 1/(2d) away from the integers on either side, so truncation gives floor(n/d).
// Five full-rate instructions per quotient and remainder instead of the
// integer division sequence (two of whose multiplies issue at quarter rate).
struct FDiv {
  int d;
  float r, h;
};
__device__ __forceinline__ FDiv fdiv_of(int d) {
  const float r = 1.0f / (float)d;
  return FDiv{d, r, 0.5f * r};
}
__device__ __forceinline__ int fdiv_q(int n, const FDiv& D) { return (int)__builtin_fmaf((float)n, D.r, D.h); }
// a * b for operands below 2^24 (full-rate 24-bit multiply)
__device__ __forceinline__ int mul24(int a, int b) { return (int)__umul24((unsigned)a, (unsigned)b); }

// One Stockham stage of radix R on one column per thread group (tpc threads;
// each thread at most NB = max(1, 16/R) butterflies, the host guarantees
// L/R <= NB tpc).  Source and destination are the LDS column (element i at
// pidx(i, sh)) or, with GIN / GOUT, the caller's global loads and stores:
// ld.template get<CHK>(column, index), st.template put<CHK>(column, index, v),
// CHK = false where the index is known to be inside the data.
// FIRST: the span-1 stage (no twiddles; outputs j R + r).
// HIN: inputs at index >= L/2 are zero and the ones below are all present
// (read without checks, the upper half not at all); HOUT: outputs at index
// >= L/2 are not needed.  Both need an even R.
// LDS addresses are linear in r: with padding (sh = 3) the host keeps every
// stride (L/R for the reads, the span for the writes) a multiple of 8 and
// the first radix a power of two, without padding (sh = 31) anything goes.
template <typename T, int R, bool INV, bool GIN, bool GOUT, bool TWL, bool FIRST, bool HIN, bool HOUT, class Load,
          class Store, class Hook>
__device__ __forceinline__ void fft_stage(Cx<T>* __restrict__ col, int c, int L, int Ns, int lane, int tpc,
                                          bool active, int sh, const Cx<T>* __restrict__ tw, Load& ld, Store& st,
                                          Hook& hook) {
  static_assert(!(HIN || HOUT) || R % 2 == 0, "half-length ends need an even radix");
  constexpr int NB = R >= 16 ? 1 : 16 / R;
  constexpr int RI = HIN ? R / 2 : R;
  constexpr int RO = HOUT ? R / 2 : R;
  const int nbf = L / R;
  Cx<T> v[NB][R];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int j = lane + k * tpc;
    if (active && j < nbf) {
      if constexpr (GIN) {
#pragma unroll
        for (int r = 0; r < RI; ++r) v[k][r] = ld.template get<!HIN>(c, j + r * nbf);
      } else {
        const int a = j + (j >> sh);
        const int nbp = nbf + (nbf >> sh);
#pragma unroll
        for (int r = 0; r < RI; ++r) v[k][r] = col[a + r * nbp];
      }
#pragma unroll
      for (int r = RI; r < R; ++r) v[k][r] = Cx<T>{T(0), T(0)};
    }
  }
  if constexpr (!GIN) __syncthreads();
  if constexpr (GIN) hook();  // runs with this stage's global loads in flight
  FDiv dn{1, 1.0f, 0.5f};
  int tstep = 0;
  if constexpr (!FIRST) {
    dn = fdiv_of(Ns);
    tstep = fdiv_q(nbf, dn);  // L / (Ns R)
  }
  const int span = Ns * R;
  const int nsp = Ns + (Ns >> sh);
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int j = lane + k * tpc;
    if (active && j < nbf) {
      int q = j, kk = 0;
      if constexpr (!FIRST) {
        q = fdiv_q(j, dn);
        kk = j - mul24(q, Ns);
        twiddle_powers<T, R, INV, TWL>(v[k], tw, mul24(kk, tstep));
      }
      dftR<T, R, INV>(v[k]);
      const int base = mul24(q, span) + kk;
      if constexpr (GOUT) {
#pragma unroll
        for (int r = 0; r < RO; ++r) st.template put<!HOUT>(c, base + r * Ns, v[k][r]);
      } else if constexpr (FIRST) {
        const int a = base + (base >> sh);
        const int hi = 8 >> sh;  // radix 16: one more padding slot from r = 8 on
#pragma unroll
        for (int r = 0; r < RO; ++r) col[a + r + (r >= 8 ? hi : 0)] = v[k][r];
      } else {
        const int a = base + (base >> sh);
#pragma unroll
        for (int r = 0; r < RO; ++r) col[a + r * nsp] = v[k][r];
      }
    }
  }
  if constexpr (!GOUT) __syncthreads();
}

// The stage of radix radix_of(code, s).  EVEN: only even radices can occur
// (a half-length end).
template <typename T, bool INV, bool GIN, bool GOUT, bool TWL, bool R16, bool FIRST, bool HIN, bool HOUT, class Load,
          class Store, class Hook>
__device__ __forceinline__ void fft_stage_any(Cx<T>* col, int c, const FftDesc<T>& p, const Cx<T>* tw, int s, int ns,
                                              int lane, int tpc, bool active, Load& ld, Store& st, Hook& hook) {
  constexpr bool EVEN = HIN || HOUT;
#define MMX_STAGE(R) \
  fft_stage<T, R, INV, GIN, GOUT, TWL, FIRST, HIN, HOUT>(col, c, p.L, ns, lane, tpc, active, p.psh, tw, ld, st, hook)
  switch (radix_of(p.code, s)) {
    case 16:
      if constexpr (R16) MMX_STAGE(16);
      break;
    case 8: MMX_STAGE(8); break;
    case 4: MMX_STAGE(4); break;
    case 3:
      if constexpr (!EVEN) MMX_STAGE(3);
      break;
    default: MMX_STAGE(2); break;
  }
#undef MMX_STAGE
}

// Transform of ncol columns, column c = threadIdx.x / tpc.  Without GIN the
// input is the LDS column, without GOUT the output is (natural order).
// hin / hout as HIN / HOUT above; the caller passes them only where the data
// lengths allow (exactly L/2 inputs / outputs), and they are dropped unless the
// plan's end radix is even.  The first stage's loads are issued before hook().
template <typename T, bool INV, bool GIN, bool GOUT, bool TWL, bool R16 = false, class Load, class Store,
          class Hook>
__device__ __forceinline__ void fft_run(Cx<T>* lds, const FftDesc<T>& p, const Cx<T>* tw, int cs, int ncol, int tpc,
                                        bool hin, bool hout, Load ld, Store st, Hook hook) {
  const int c = threadIdx.x / tpc;
  const int lane = threadIdx.x - c * tpc;
  const bool active = c < ncol;
  Cx<T>* col = lds + (active ? c : 0) * cs;
  hin = hin && (p.code & kFftFirstEven) && p.nst > 1;
  hout = hout && (p.code & kFftLastEven) && p.nst > 1;
  if (p.nst == 0) {  // length 1: identity
    if constexpr (GIN) hook();
    if (active && lane == 0) {
      Cx<T> v;
      if constexpr (GIN) v = ld.template get<true>(c, 0);
      else v = col[0];
      if constexpr (GOUT) st.template put<true>(c, 0, v);
      else col[0] = v;
    }
    if constexpr (!GOUT) __syncthreads();
    return;
  }
  if (p.nst == 1) {
    fft_stage_any<T, INV, GIN, GOUT, TWL, R16, true, false, false>(col, c, p, tw, 0, 1, lane, tpc, active, ld, st,
                                                                   hook);
    return;
  }
  if (hin)
    fft_stage_any<T, INV, GIN, false, TWL, R16, true, true, false>(col, c, p, tw, 0, 1, lane, tpc, active, ld, st,
                                                                   hook);
  else
    fft_stage_any<T, INV, GIN, false, TWL, R16, true, false, false>(col, c, p, tw, 0, 1, lane, tpc, active, ld, st,
                                                                    hook);
  NoHook nh;
  int ns = radix_of(p.code, 0);
  for (int s = 1; s + 1 < p.nst; ++s) {
    fft_stage_any<T, INV, false, false, TWL, R16, false, false, false>(col, c, p, tw, s, ns, lane, tpc, active, ld,
                                                                       st, nh);
    ns *= radix_of(p.code, s);
  }
  if (hout)
    fft_stage_any<T, INV, false, GOUT, TWL, R16, false, false, true>(col, c, p, tw, p.nst - 1, ns, lane, tpc, active,
                                                                     ld, st, nh);
  else
    fft_stage_any<T, INV, false, GOUT, TWL, R16, false, false, false>(col, c, p, tw, p.nst - 1, ns, lane, tpc,
                                                                      active, ld, st, nh);
}

// The same transform for one length L fixed at compile time (a power of two,
// the plan p2_radix(log2 L, A16, s)) with EPT entries per thread and stage
// (16, or 8 for plans without radix 16: L/EPT threads per column, which
// shortens each stage where a transform has few columns to share the CU):
// every index, stride and LDS offset is a constant and no butterfly is
// predicated, which keeps the kernels that use it small in registers.
template <typename T, int R, int L, int NS, int SH, int EPT, bool INV, bool GIN, bool GOUT, bool TWL, bool HIN,
          bool HOUT, class Load, class Store, class Hook>
__device__ __forceinline__ void fft_stage_s(Cx<T>* __restrict__ col, int c, int lane, bool active,
                                            const Cx<T>* __restrict__ tw, Load& ld, Store& st, Hook& hook) {
  static_assert(!(HIN || HOUT) || R % 2 == 0, "half-length ends need an even radix");
  constexpr bool FIRST = NS == 1;
  static_assert(R <= EPT, "a butterfly fits the entries of one thread");
  constexpr int TPC = L / EPT;
  constexpr int NB = EPT / R;
  constexpr int NBF = L / R;
  static_assert(NB * TPC == NBF, "L/EPT threads cover every butterfly");
  constexpr int RI = HIN ? R / 2 : R;
  constexpr int RO = HOUT ? R / 2 : R;
  constexpr int NBP = NBF + (NBF >> SH);
  constexpr int NSP = NS + (NS >> SH);
  constexpr int TSTEP = L / (NS * R);
  Cx<T> v[NB][R];
  if (active) {
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int j = lane + k * TPC;
      if constexpr (GIN) {
#pragma unroll
        for (int r = 0; r < RI; ++r) v[k][r] = ld.template get<!HIN>(c, j + r * NBF);
      } else {
        const int a = j + (j >> SH);
#pragma unroll
        for (int r = 0; r < RI; ++r) v[k][r] = col[a + r * NBP];
      }
#pragma unroll
      for (int r = RI; r < R; ++r) v[k][r] = Cx<T>{T(0), T(0)};
    }
  }
  if constexpr (!GIN) __syncthreads();
  if constexpr (GIN) hook();
  if (active) {
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      const int j = lane + k * TPC;
      const int q = j / NS, kk = j % NS;
      if constexpr (!FIRST) twiddle_powers<T, R, INV, TWL>(v[k], tw, kk * TSTEP);
      dftR<T, R, INV>(v[k]);
      const int base = q * NS * R + kk;
      if constexpr (GOUT) {
#pragma unroll
        for (int r = 0; r < RO; ++r) st.template put<!HOUT>(c, base + r * NS, v[k][r]);
      } else if constexpr (FIRST) {
        const int a = base + (base >> SH);
#pragma unroll
        for (int r = 0; r < RO; ++r) col[a + r + (r >= 8 ? (8 >> SH) : 0)] = v[k][r];
      } else {
        const int a = base + (base >> SH);
#pragma unroll
        for (int r = 0; r < RO; ++r) col[a + r * NSP] = v[k][r];
      }
    }
  }
  if constexpr (!GOUT) __syncthreads();
}

template <typename T, int L, bool A16, int EPT, bool INV, bool GIN, bool GOUT, bool TWL, bool HIN, bool HOUT, int S,
          int NS, class Load, class Store, class Hook>
__device__ __forceinline__ void fft_static_from(Cx<T>* col, int c, int lane, bool active, const Cx<T>* tw, Load& ld,
                                                Store& st, Hook& hook) {
  constexpr int A = ilog2c(L);
  constexpr int NST = p2_nst(A, A16);
  constexpr int R = p2_radix(A, A16, S);
  constexpr int SH = p2_psh(L, A16);
  constexpr bool FIRST = S == 0, LAST = S == NST - 1;
  fft_stage_s<T, R, L, NS, SH, EPT, INV, GIN && FIRST, GOUT && LAST, TWL, HIN && FIRST, HOUT && LAST>(
      col, c, lane, active, tw, ld, st, hook);
  if constexpr (!LAST) {
    NoHook nh;
    fft_static_from<T, L, A16, EPT, INV, false, GOUT, TWL, false, HOUT, S + 1, NS * R>(col, c, lane, active, tw, ld,
                                                                                      st, nh);
  }
}

// Column c = threadIdx.x / (L/EPT) of ncol; ends as for fft_run (HIN / HOUT
// compile-time here: exactly L/2 inputs / outputs).
template <typename T, int L, bool A16, bool INV, bool GIN, bool GOUT, bool TWL, bool HIN, bool HOUT, int EPT = 16,
          class Load, class Store, class Hook>
__device__ __forceinline__ void fft_static(Cx<T>* lds, const Cx<T>* tw, int cs, int ncol, Load ld, Store st,
                                           Hook hook) {
  static_assert((L & (L - 1)) == 0 && L >= 16, "power-of-two lengths of 16 and more");
  constexpr int TPC = L / EPT;
  const int c = (int)threadIdx.x / TPC;
  const int lane = (int)threadIdx.x & (TPC - 1);
  const bool active = c < ncol;
  Cx<T>* col = lds + (active ? c : 0) * cs;
  fft_static_from<T, L, A16, EPT, INV, GIN, GOUT, TWL, HIN, HOUT, 0, 1>(col, c, lane, active, tw, ld, st, hook);
}

// Loads / stores that are never called (LDS input or output)
template <typename T>
struct NoLoad {
  template <bool CHK>
  __device__ __forceinline__ Cx<T> get(int, int) const { return Cx<T>{T(0), T(0)}; }
};
template <typename T>
struct NoStore {
  template <bool CHK>
  __device__ __forceinline__ void put(int, int, Cx<T>) const {}
};

// LDS to LDS transform of ncol columns
template <typename T, bool INV, bool TWL, bool R16 = false>
__device__ __forceinline__ void fft_columns(Cx<T>* lds, const FftDesc<T>& p, int cs, int ncol, int tpc,
                                            const Cx<T>* tw, bool hin = false, bool hout = false) {
  fft_run<T, INV, false, false, TWL, R16>(lds, p, tw, cs, ncol, tpc, hin, hout, NoLoad<T>{}, NoStore<T>{}, NoHook{});
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
