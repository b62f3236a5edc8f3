// Hot-path kernels for gfx950: demag FFT passes, Fourier-space tensor product,
// fused local-field + Landau-Lifshitz + Dormand-Prince epilogue, controller,
// reductions, NEB passes.
//
// Effective field per cell (paper, section "Micromagnetics"):
//   exchange  H = 2A/(mu0 Ms) sum_j (m_j - m_i)/D_ij^2      (open boundaries)
//   DMI       H = -(D/(mu0 Ms)) sum_j (e_ij x m_j)/D_ij, e_ij = {-e_y,+e_y,+e_x,-e_x,0,0}
//   anis.     H = 2Ku/(mu0 Ms) (m.u) u
//   Zeeman    H = H_app
//   demag     H_i = -sum_j N_{i-j} M_j (eq_hd1), by the convolution theorem on a
//             zero-padded grid.
// LL right-hand side (eq_llg2): dm/dt = g1 m x H + g2 m x (m x H).
//
// Demag data flow for one evaluation (all FP32 or all FP64):
//   x pass   m[3][nz][ny][nx] -> real-to-complex along x (two reals packed per
//            complex, half-length transform) -> Sx[3][nz][Xp][ny] (transposed,
//            so the y transform reads contiguous rows)
//   y pass   3-D: Sx -> Sy[3][nz][Xp][Py];  2-D: forward y, tensor product,
//            inverse y fused, in place in Sx
//   z pass   3-D: forward z (zero padded in registers or LDS), tensor product,
//            inverse z, in place in Sy (only the nz physical planes are stored)
//   y inv    3-D: Sy -> Sx (only the ny physical rows)
//   x inv    complex-to-real along x for the 3 components of TY rows, then the
//            local fields, H_eff, LL and the integrator epilogue per cell.
//
// Every launch covers a set of groups (instances sharing a mesh): workgroup
// ranges per group come with the launch, each group's geometry, tables and
// buffers from device memory, so instances of different meshes advance in one
// launch per pass.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>

#include "fft_core.hpp"
#include "kernels.hpp"

namespace mmx {

constexpr int kNT = 256;   // threads of the pointwise kernels and the register z pass
constexpr int kUnroll = 8; // global loads kept in flight per thread when filling LDS

template <typename T> __device__ __forceinline__ T rsqrt_t(T v);
template <> __device__ __forceinline__ float rsqrt_t<float>(float v) { return 1.0f / sqrtf(v); }
template <> __device__ __forceinline__ double rsqrt_t<double>(double v) { return 1.0 / sqrt(v); }

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Copy of small read-only tables (twiddles, post-processing factors) into LDS:
// issue() starts the global loads into registers, store() writes them to LDS
// (and copies any entries beyond NPER per thread directly).  Issuing before
// a pass's data loads and storing after them lets one memory latency cover both.
template <typename T, int NPER>
struct TableCopy {
  Cx<T> r[NPER];
  const Cx<T>* a;
  const Cx<T>* b;
  int na, nb;
  __device__ __forceinline__ Cx<T> src(int i) const { return i < na ? gld(a + i) : gld(b + (i - na)); }
  __device__ __forceinline__ void issue(const Cx<T>* a_, int na_, const Cx<T>* b_, int nb_) {
    a = a_; b = b_; na = na_; nb = nb_;
#pragma unroll
    for (int j = 0; j < NPER; ++j) {
      const int i = threadIdx.x + j * blockDim.x;
      if (i < na + nb) r[j] = src(i);
    }
  }
  __device__ __forceinline__ void store(Cx<T>* dst) const {
#pragma unroll
    for (int j = 0; j < NPER; ++j) {
      const int i = threadIdx.x + j * blockDim.x;
      if (i < na + nb) dst[i] = r[j];
    }
    for (int i = threadIdx.x + NPER * blockDim.x; i < na + nb; i += blockDim.x) dst[i] = src(i);
  }
};

// The same for nseg segments of a real array: segment k is seg_len entries
// starting at src + k * seg_stride, stored one after the other in LDS.
template <typename T, int NPER>
struct SegTableCopy {
  T r[NPER];
  const T* src;
  size_t stride;
  int len, n;
  __device__ __forceinline__ T at(int i) const {
    const int k = i / len, e = i - k * len;
    return gld(src + k * stride + e);
  }
  __device__ __forceinline__ void issue(const T* src_, size_t stride_, int len_, int nseg) {
    src = src_; stride = stride_; len = len_; n = len_ * nseg;
#pragma unroll
    for (int j = 0; j < NPER; ++j) {
      const int i = threadIdx.x + j * blockDim.x;
      if (i < n) r[j] = at(i);
    }
  }
  __device__ __forceinline__ void store(T* dst) const {
#pragma unroll
    for (int j = 0; j < NPER; ++j) {
      const int i = threadIdx.x + j * blockDim.x;
      if (i < n) dst[i] = r[j];
    }
    for (int i = threadIdx.x + NPER * blockDim.x; i < n; i += blockDim.x) dst[i] = at(i);
  }
};

// Plan of group gi of a launch (group 0 from the kernel arguments).
template <typename T>
__device__ __forceinline__ HotPlan<T> hot_plan(const Launch<T>& L, int gi) {
  return gi == 0 ? L.h0 : ldu(L.hps + gi);
}

// Group of this workgroup and its index inside the group (XCD-ordered).
template <typename T>
__device__ __forceinline__ int group_of(const Launch<T>& L, long long& lb) {
  int gi = 0;
  while (gi + 1 < L.ngroups && (long long)blockIdx.x >= L.off[gi + 1]) ++gi;
  const long long nb = L.off[gi + 1] - L.off[gi];
  lb = xcd_tile((long long)blockIdx.x - L.off[gi], nb);
  return gi;
}

// ---------------------------------------------------------------------------
// x forward: real-to-complex of TY rows (fixed b, c, z), transposed store.
// ---------------------------------------------------------------------------
__host__ __device__ inline long long fwd_blocks(const Geo& g, const Tuning& tu, int batch) {
  return (long long)batch * 3 * g.nz * ((g.ny + tu.ty_f - 1) / tu.ty_f);
}

// Row loads of the forward x transform: element n of column r packs
// x[2n] + i x[2n+1] of row y0 + r (zero beyond nx).  Offsets in bytes from
// the z plane's first row.
// ms (nullable): per-cell saturation magnetisation at the same offsets (cell-based
// material), by which each m component is scaled (M = Ms m).
template <typename T>
struct XRowLoad {
  const T* src;
  int nx;
  bool pairs;  // nx even: rows start 8-byte aligned, x[2n] and x[2n+1] in one load
  const T* ms;
  template <bool CHK>
  __device__ __forceinline__ Cx<T> raw(const T* a, int r, int n) const {
    const uint32_t row = (uint32_t)(r * nx);
    const int i0 = 2 * n;
    Cx<T> v = {T(0), T(0)};
    if (!CHK) return gldo(reinterpret_cast<const Cx<T>*>(a), (row + (uint32_t)i0) * (uint32_t)sizeof(T));
    if (pairs) {
      if (i0 < nx) v = gldo(reinterpret_cast<const Cx<T>*>(a), (row + (uint32_t)i0) * (uint32_t)sizeof(T));
    } else {
      if (i0 < nx) v.x = gldo(a, (row + (uint32_t)i0) * (uint32_t)sizeof(T));
      if (i0 + 1 < nx) v.y = gldo(a, (row + (uint32_t)i0 + 1) * (uint32_t)sizeof(T));
    }
    return v;
  }
  template <bool CHK>
  __device__ __forceinline__ Cx<T> get(int r, int n) const {
    Cx<T> v = raw<CHK>(src, r, n);
    if (ms) {
      const Cx<T> w = raw<CHK>(ms, r, n);
      v.x *= w.x;
      v.y *= w.y;
    }
    return v;
  }
};

// SLX: 0 for any group, else the one length Lx of every group, all with an
// even nx = Lx (a kernel holding one static transform keeps fewer registers).
template <typename T, int SLX>
__global__ void __launch_bounds__(512) k_fwd_x(Launch<T> L) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  long long bid0;
  const int gi = group_of(L, bid0);
  const HotPlan<T> hp = hot_plan(L, gi);
  const Geo& g = hp.g;
  if (bid0 >= fwd_blocks(g, hp.tu, hp.batch)) return;
  const int TY = hp.tu.ty_f;  // a power of two
  const int lty = __builtin_ctz((unsigned)TY);
  const unsigned tiles = (unsigned)((g.ny + TY - 1) >> lty);
  unsigned bid = (unsigned)bid0;
  const int tile = (int)(bid % tiles); bid /= tiles;
  const int z = (int)(bid % (unsigned)g.nz); bid /= (unsigned)g.nz;
  const int c = (int)(bid % 3u);
  const int b = (int)(bid / 3u);
  DevCtl* const ctl = ldu(&L.epis[gi].ctl);
  if (ctl && ldu(&ctl[b].done)) return;
  const int y0 = tile * TY;
  const int nrow = g.ny - y0 < TY ? g.ny - y0 : TY;
  const int cs = col_stride(g.Lx);
  const int sh = hp.fd[0].psh;
  // LDS: TY columns, then the twiddle table (Lx) and the post factors (Lx + 1)
  Cx<T>* const twl = lds + TY * cs;
  Cx<T>* const postl = twl + g.Lx;
  TableCopy<T, 4> tab;
  tab.issue(hp.fd[0].tw, g.Lx, hp.post, g.Lx + 1);
  const T* in = ldu(&L.epis[gi].in);
  const size_t rows0 = ((size_t)z * g.ny + y0) * g.nx;
  const bool cellarr = hp.cells && (ldu(&hp.prm[b].terms) & MM_CELLS);
  XRowLoad<T> ld{in + ((size_t)b * 3 + c) * g.N + rows0, g.nx, (g.nx & 1) == 0,
                 cellarr ? hp.cells + (size_t)b * 3 * g.N + rows0 : nullptr};
  auto hook = [&]() { tab.store(twl); };
  // all nx / 2 packed inputs present and the rest zero when nx = Lx (even)
  const bool hin = ld.pairs && g.nx == g.Lx;
  const NoStore<T> nst;
  // compiled for the power-of-two lengths (L/8 threads a row where the
  // workgroup has them, else L/16)
  const bool e8 = nrow * (g.Lx / 8) <= (int)blockDim.x;
#define MMX_FS(LL)                                                                                             \
  case LL:                                                                                                     \
    if (e8) fft_static<T, LL, false, false, true, false, true, true, false, 8>(lds, twl, cs, nrow, ld, nst, hook); \
    else fft_static<T, LL, false, false, true, false, true, true, false, 16>(lds, twl, cs, nrow, ld, nst, hook);   \
    break;
  switch (SLX != 0 ? SLX : hin ? g.Lx : 0) {
    MMX_FS(128)
    MMX_FS(256)
    MMX_FS(512)
    MMX_FS(1024)
    default:
      if constexpr (SLX == 0)
        fft_run<T, false, true, false, true>(lds, hp.fd[0], twl, cs, nrow, (int)blockDim.x >> lty, hin, false, ld,
                                             nst, hook);
  }
#undef MMX_FS
  // real-to-complex post-processing: X[k] of row r
  auto post = [&](int r, int k) -> Cx<T> {
    const Cx<T> Zk = lds[r * cs + pidx(k == g.Lx ? 0 : k, sh)];
    const Cx<T> Zc = cconj(lds[r * cs + pidx(k == 0 ? 0 : g.Lx - k, sh)]);
    const Cx<T> E = cscale(cadd(Zk, Zc), T(0.5));
    const Cx<T> D = cscale(csub(Zk, Zc), T(0.5));
    const Cx<T> O = {D.y, -D.x};  // D / i
    return cadd(E, cmul(postl[k], O));
  };
  if (g.nz > 1) {  // 3-D: Sx [3][nz][XB][ny][kSxB], kSxB TY contiguous entries per block
    const int lq = lty + 2;  // kSxB = 4
    Cx<T>* dst = hp.Sx + (size_t)b * g.sx + ((size_t)c * g.nz + z) * g.XB * kSxB * g.ny + kSxB * y0;
    for (int t = threadIdx.x; t < (g.XB << lq); t += blockDim.x) {
      const int kb = t >> lq, q = t & ((1 << lq) - 1);
      const int r = q >> 2, k = kb * kSxB + (q & 3);
      if (r < nrow && k < g.Xp)
        gsto(dst, (uint32_t)(kb * kSxB * g.ny + q) * (uint32_t)sizeof(Cx<T>), post(r, k));
    }
  } else {  // 2-D: Sx transposed [3][Xp][ny] (the fused y pass reads columns)
    Cx<T>* dst = hp.Sx + (size_t)b * g.sx + (size_t)c * g.Xp * g.ny + y0;
    const int tot2 = g.Xp << lty;
    for (int t = threadIdx.x; t < tot2; t += blockDim.x) {
      const int k = t >> lty, r = t & (TY - 1);
      if (r >= nrow) continue;
      gsto(dst, (uint32_t)(k * g.ny + r) * (uint32_t)sizeof(Cx<T>), post(r, k));
    }
  }
}

// ---------------------------------------------------------------------------
// Tensor product at one spectral point: H_a = s * sum_b K_ab M_b (K real).
// ---------------------------------------------------------------------------
// The six (or four, nz = 1) entries at one point, scaled by s, with the
// parity signs of the folded spectrum applied.
template <typename T>
struct Ten {
  T xx, yy, zz, xy, xz, yz;
};
template <typename T>
__device__ __forceinline__ Ten<T> tensor_load(const HotPlan<T>& hp, int kx, int ky, int kz, T s) {
  const Geo& g = hp.g;
  const int kyf = ky <= g.Py - ky ? ky : g.Py - ky;
  const int kzf = kz <= g.Pz - kz ? kz : g.Pz - kz;
  const T sy = ky > g.Py - ky ? T(-1) : T(1);
  const T sz = kz > g.Pz - kz ? T(-1) : T(1);
  const size_t cstride = (size_t)g.Kz * g.Xp * g.Ky;
  const size_t off = ((size_t)kzf * g.Xp + kx) * g.Ky + kyf;
  Ten<T> t;
  t.xx = gld(hp.kt + off) * s;
  t.yy = gld(hp.kt + cstride + off) * s;
  t.zz = gld(hp.kt + 2 * cstride + off) * s;
  t.xy = gld(hp.kt + 3 * cstride + off) * (s * sy);
  t.xz = T(0);
  t.yz = T(0);
  if (hp.ncomp == 6) {
    t.xz = gld(hp.kt + 4 * cstride + off) * (s * sz);
    t.yz = gld(hp.kt + 5 * cstride + off) * (s * sy * sz);
  }
  return t;
}
template <typename T>
__device__ __forceinline__ void tensor_mul(const Ten<T>& t, Cx<T>& m0, Cx<T>& m1, Cx<T>& m2) {
  const Cx<T> a = m0, b = m1, c = m2;
  m0 = {t.xx * a.x + t.xy * b.x + t.xz * c.x, t.xx * a.y + t.xy * b.y + t.xz * c.y};
  m1 = {t.xy * a.x + t.yy * b.x + t.yz * c.x, t.xy * a.y + t.yy * b.y + t.yz * c.y};
  m2 = {t.xz * a.x + t.yz * b.x + t.zz * c.x, t.xz * a.y + t.yz * b.y + t.zz * c.y};
}
template <typename T>
__device__ __forceinline__ void tensor_apply(const HotPlan<T>& hp, int kx, int ky, int kz, T s,
                                             Cx<T>& m0, Cx<T>& m1, Cx<T>& m2) {
  tensor_mul(tensor_load(hp, kx, ky, kz, s), m0, m1, m2);
}

// ---------------------------------------------------------------------------
// y pass.  2-D groups (nz = 1): forward y, tensor product, inverse y for cb_y2
// kx values and the 3 components, in place in Sx.  3-D groups: rows of fixed
// (b, c, z, kx); forward Sx(ny) -> Sy(Py) or inverse Sy(Py) -> Sx(ny).
// ---------------------------------------------------------------------------
__host__ __device__ inline long long y2d_blocks(const Geo& g, const Tuning& tu, int batch) {
  const int slots = y2d_packed(g) ? g.Lx : g.Xp;  // packed: kx = 0 and Lx share a slot
  return (long long)batch * ((slots + tu.cb_y2 - 1) / tu.cb_y2);
}
// 3-D groups: tiles of cb_y consecutive kx inside one (component, z) plane
__host__ __device__ inline long long y3d_blocks(const Geo& g, const Tuning& tu, int batch) {
  return (long long)batch * 3 * g.nz * ((g.Xp + tu.cb_y - 1) / tu.cb_y);
}

// Global column access of the y passes: this thread's column starts coff
// bytes after base and holds n elements (every thread only touches its own
// column, so the offset is formed once).
template <typename T>
struct ColLoad {
  const Cx<T>* base;
  uint32_t coff;
  int n;
  template <bool CHK>
  __device__ __forceinline__ Cx<T> get(int, int e) const {
    if (CHK && e >= n) return Cx<T>{T(0), T(0)};
    return gldo(base, coff + (uint32_t)e * (uint32_t)sizeof(Cx<T>));
  }
};
template <typename T>
struct ColStore {
  Cx<T>* base;
  uint32_t coff;
  int n;
  template <bool CHK>
  __device__ __forceinline__ void put(int, int e, Cx<T> v) const {
    if (CHK && e >= n) return;
    gsto(base, coff + (uint32_t)e * (uint32_t)sizeof(Cx<T>), v);
  }
};

// A column of the 2-D y pass.  The kx = 0 and kx = Lx (Nyquist) columns of a
// real field's x spectrum are real in y; the pass carries them as one complex
// column (kx = 0 in the real part, kx = Lx in the imaginary part): coff2 is
// the kx = Lx column for that packed column, ~0u for every other one.
template <typename T>
struct ColLoad2 {
  const Cx<T>* base;
  uint32_t coff, coff2;
  int n;
  template <bool CHK>
  __device__ __forceinline__ Cx<T> get(int, int e) const {
    if (CHK && e >= n) return Cx<T>{T(0), T(0)};
    const uint32_t eo = (uint32_t)e * (uint32_t)sizeof(Cx<T>);
    const Cx<T> v = gldo(base, coff + eo);
    if (coff2 == ~0u) return v;
    return Cx<T>{v.x, gldo(base, coff2 + eo).x};
  }
};
template <typename T>
struct ColStore2 {
  Cx<T>* base;
  uint32_t coff, coff2;
  int n;
  template <bool CHK>
  __device__ __forceinline__ void put(int, int e, Cx<T> v) const {
    if (CHK && e >= n) return;
    const uint32_t eo = (uint32_t)e * (uint32_t)sizeof(Cx<T>);
    if (coff2 == ~0u) {
      gsto(base, coff + eo, v);
    } else {
      gsto(base, coff + eo, Cx<T>{v.x, T(0)});
      gsto(base, coff2 + eo, Cx<T>{v.y, T(0)});
    }
  }
};

// The same with entries sb bytes apart (a column inside the x-pass buffer's
// kx blocks).
template <typename T>
struct ColLoadS {
  const Cx<T>* base;
  uint32_t coff, sb;
  int n;
  template <bool CHK>
  __device__ __forceinline__ Cx<T> get(int, int e) const {
    if (CHK && e >= n) return Cx<T>{T(0), T(0)};
    return gldo(base, coff + (uint32_t)e * sb);
  }
};
template <typename T>
struct ColStoreS {
  Cx<T>* base;
  uint32_t coff, sb;
  int n;
  template <bool CHK>
  __device__ __forceinline__ void put(int, int e, Cx<T> v) const {
    if (CHK && e >= n) return;
    gsto(base, coff + (uint32_t)e * sb, v);
  }
};

// SL > 0: compiled for Py = SL = 2 ny (fft_static, SL/EPT threads a column).
template <typename T, bool R16, int SL = 0, int EPT = 16>
__device__ __forceinline__ void y_fused2d(const HotPlan<T>& hp, const Epi<T>& ep, long long bid0, Cx<T>* lds) {
  const Geo& g = hp.g;
  const int CB = hp.tu.cb_y2;
  // column slots: slot k the column kx = k; packed (y2d_packed), Lx slots
  // with kx = 0 and kx = Lx together in slot 0, else Lx + 1
  const int L = g.Lx;
  const bool pk = SL > 0 ? SL >= 1024 : y2d_packed(g);  // the same predicate (Py = SL)
  const int nslot = pk ? L : L + 1;
  const unsigned tiles = (unsigned)((nslot + CB - 1) / CB);
  const unsigned bid = (unsigned)bid0;
  const int tile = (int)(bid % tiles);
  const int b = (int)(bid / tiles);
  if (ep.ctl && ldu(&ep.ctl[b].done)) return;
  const int kx0 = tile * CB;
  const int ncb = nslot - kx0 < CB ? nslot - kx0 : CB;  // slots of this tile
  const int ncol = 3 * ncb;                     // column c * ncb + j: component c of slot kx0 + j
  const int cs = col_stride(g.Py);
  const int sh = hp.fd[1].psh;
  const int Xp = g.Xp, ny = g.ny;
  const int tpc = SL > 0 ? SL / EPT : blockDim.x / (3 * CB);
  // this thread's column, in Sx = [3][1][Xp][ny] of the instance
  const int mc = (int)threadIdx.x / tpc;
  const int cc = mc < ncol ? mc : 0;
  const int c = cc / ncb, j = cc - c * ncb;
  const uint32_t coff = (uint32_t)((c * Xp + kx0 + j) * ny) * (uint32_t)sizeof(Cx<T>);
  const uint32_t coff2 = pk && kx0 + j == 0 ? (uint32_t)((c * Xp + L) * ny) * (uint32_t)sizeof(Cx<T>) : ~0u;
  Cx<T>* base = hp.Sx + (size_t)b * g.sx;
  // LDS after the columns: the twiddle table (Py) and the tensor rows of this
  // tile, kt[a][j][ky] for the components a = xx, yy, zz, xy and the ncb kx
  // (nz = 1: one kz plane), both copied while the first stage's loads fly
  Cx<T>* const twl = lds + 3 * CB * cs;
  T* const ktl = reinterpret_cast<T*>(twl + g.Py);
  const bool ktlds = SL > 0 ? SL <= 1024 : y2d_tensor_in_lds(g);  // the same predicate (Py = SL)
  TableCopy<T, 4> tab;
  tab.issue(hp.fd[1].tw, g.Py, nullptr, 0);
  SegTableCopy<T, 8> ktab;
  if (ktlds) ktab.issue(hp.kt + (size_t)kx0 * g.Ky, (size_t)g.Kz * g.Xp * g.Ky, ncb * g.Ky, 4);
  // the packed slot's tile also takes the tensor rows of kx = Lx, after the
  // rows of a full tile (4 (Py/2 + 1) values: compiled lengths hold them all
  // in registers while the first stage runs, 2 EPT / 3 + 1 a thread)
  const bool packed = pk && kx0 == 0;
  T* const ktlN = ktl + 4 * CB * g.Ky;
  SegTableCopy<T, (SL > 0 ? 2 * EPT / 3 + 1 : 8)> ktabN;
  if (ktlds && packed) ktabN.issue(hp.kt + (size_t)L * g.Ky, (size_t)g.Kz * g.Xp * g.Ky, g.Ky, 4);
  auto hook = [&]() {
    tab.store(twl);
    if (ktlds) ktab.store(ktl);
    if (ktlds && packed) ktabN.store(ktlN);
  };
  const bool half = g.Py == 2 * ny;  // ny inputs / outputs of Py points
  if constexpr (SL > 0)
    fft_static<T, SL, (EPT > 8), false, true, false, true, true, false, EPT>(
        lds, twl, cs, ncol, ColLoad2<T>{base, coff, coff2, ny}, NoStore<T>{}, hook);
  else
    fft_run<T, false, true, false, true, R16>(lds, hp.fd[1], twl, cs, ncol, tpc, half, false,
                                              ColLoad2<T>{base, coff, coff2, ny}, NoStore<T>{}, hook);
  Cx<T>* const spec = lds;
  const T s = T(ldu(&hp.prm[b].demag_scale));
  // tensor entry of component a at o = jj Ky + ky (kx0 + jj): from the LDS
  // rows, or from global memory (component stride Kz Xp Ky)
  const int seg = ncb * g.Ky;
  const T* const ktg = hp.kt + (size_t)kx0 * g.Ky;
  const size_t kgs = (size_t)g.Kz * g.Xp * g.Ky;
  auto kent = [&](int a, int o) -> T { return ktlds ? ktl[a * seg + o] : gld(ktg + a * kgs + o); };
  const FDiv dpy = fdiv_of(g.Py);
  const int psh = SL > 0 ? p2_psh(SL, EPT > 8) : sh;
  for (int t = threadIdx.x; t < ncb * g.Py; t += blockDim.x) {
    const int jj = fdiv_q(t, dpy), ky = t - mul24(jj, g.Py);
    if (packed && jj == 0) continue;  // below
    const int kyf = ky <= g.Py - ky ? ky : g.Py - ky;
    const T sy = ky > g.Py - ky ? T(-1) : T(1);
    const int o = jj * g.Ky + kyf;
    const T kxx = kent(0, o) * s, kyy = kent(1, o) * s, kzz = kent(2, o) * s;
    const T kxy = kent(3, o) * (s * sy);
    const int p = pidx(ky, SL > 0 ? p2_psh(SL, EPT > 8) : sh);
    Cx<T>& m0 = spec[(0 * ncb + jj) * cs + p];
    Cx<T>& m1 = spec[(1 * ncb + jj) * cs + p];
    Cx<T>& m2 = spec[(2 * ncb + jj) * cs + p];
    const Cx<T> a = m0, bq = m1, cq = m2;
    m0 = {kxx * a.x + kxy * bq.x, kxx * a.y + kxy * bq.y};
    m1 = {kxy * a.x + kyy * bq.x, kxy * a.y + kyy * bq.y};
    m2 = {kzz * cq.x, kzz * cq.y};
  }
  if (packed) {
    // the packed slot: Z = A + i B with A (kx = 0) and B (kx = Lx) the spectra
    // of real sequences, so A(k) = (Z(k) + conj Z(-k)) / 2 and
    // B(k) = (Z(k) - conj Z(-k)) / 2i; each takes the product with the tensor
    // of its own kx, and W = H_A + i H_B goes back (its inverse transform
    // holds the two real fields in its real and imaginary parts).  One thread
    // a pair (k, Py - k).
    const T* const ktL = hp.kt + (size_t)L * g.Ky;
    auto kentN = [&](int a, int kyf) -> T { return ktlds ? ktlN[a * g.Ky + kyf] : gld(ktL + a * kgs + kyf); };
    for (int k1 = threadIdx.x; k1 <= g.Py / 2; k1 += blockDim.x) {
      const int k2 = k1 == 0 ? 0 : g.Py - k1;
      Cx<T> A1[3], B1[3];
#pragma unroll
      for (int cp = 0; cp < 3; ++cp) {
        const Cx<T> z1 = spec[(cp * ncb) * cs + pidx(k1, psh)];
        const Cx<T> z2 = spec[(cp * ncb) * cs + pidx(k2, psh)];
        A1[cp] = {T(0.5) * (z1.x + z2.x), T(0.5) * (z1.y - z2.y)};
        const Cx<T> d = {T(0.5) * (z1.x - z2.x), T(0.5) * (z1.y + z2.y)};
        B1[cp] = {d.y, -d.x};
      }
      for (int side = 0; side < (k2 == k1 ? 1 : 2); ++side) {
        const int ky = side == 0 ? k1 : k2;
        const int kyf = ky <= g.Py - ky ? ky : g.Py - ky;
        const T sy = ky > g.Py - ky ? T(-1) : T(1);
        // A(-k) = conj A(k), B(-k) = conj B(k)
        Cx<T> A[3], B[3];
#pragma unroll
        for (int cp = 0; cp < 3; ++cp) {
          A[cp] = side == 0 ? A1[cp] : cconj(A1[cp]);
          B[cp] = side == 0 ? B1[cp] : cconj(B1[cp]);
        }
        const T axx = kent(0, kyf) * s, ayy = kent(1, kyf) * s, azz = kent(2, kyf) * s;
        const T axy = kent(3, kyf) * (s * sy);
        const T bxx = kentN(0, kyf) * s, byy = kentN(1, kyf) * s, bzz = kentN(2, kyf) * s;
        const T bxy = kentN(3, kyf) * (s * sy);
        const Cx<T> ha[3] = {{axx * A[0].x + axy * A[1].x, axx * A[0].y + axy * A[1].y},
                             {axy * A[0].x + ayy * A[1].x, axy * A[0].y + ayy * A[1].y},
                             {azz * A[2].x, azz * A[2].y}};
        const Cx<T> hb[3] = {{bxx * B[0].x + bxy * B[1].x, bxx * B[0].y + bxy * B[1].y},
                             {bxy * B[0].x + byy * B[1].x, bxy * B[0].y + byy * B[1].y},
                             {bzz * B[2].x, bzz * B[2].y}};
#pragma unroll
        for (int cp = 0; cp < 3; ++cp)
          spec[(cp * ncb) * cs + pidx(ky, psh)] = Cx<T>{ha[cp].x - hb[cp].y, ha[cp].y + hb[cp].x};
      }
    }
  }
  __syncthreads();
  if constexpr (SL > 0)
    fft_static<T, SL, (EPT > 8), true, false, true, true, false, true, EPT>(
        lds, twl, cs, ncol, NoLoad<T>{}, ColStore2<T>{base, coff, coff2, ny}, NoHook{});
  else
    fft_run<T, true, false, true, true, R16>(lds, hp.fd[1], twl, cs, ncol, tpc, false, half, NoLoad<T>{},
                                             ColStore2<T>{base, coff, coff2, ny}, NoHook{});
}

// 3-D groups keep Sx in kx blocks, [3][nz][XB][ny][kSxB].  A y tile is cb_y
// consecutive kx of one (component, z) plane.  cb_y up to kSxB (columns of
// one block): the transform reads and writes its column straight from the
// block, entries kSxB apart.  cb_y a larger multiple of kSxB: whole blocks,
// staged through LDS on the Sx side (the forward pass copies the contiguous
// blocks into the LDS columns and transforms from there; the inverse
// transforms into LDS and copies the first ny entries of each column back the
// same way).  Sy [3][nz][Xp][Py] is read and written
// row by row by the transform itself.
template <typename T, bool INV, bool R16, int SL = 0, int EPT = 16>
__device__ __forceinline__ void y_rows3d(const HotPlan<T>& hp, const Epi<T>& ep, long long bid0, Cx<T>* lds) {
  const Geo& g = hp.g;
  const int CB = hp.tu.cb_y;
  const unsigned tiles = (unsigned)((g.Xp + CB - 1) / CB);  // per (component, z) plane
  unsigned bid = (unsigned)bid0;
  const int tile = (int)(bid % tiles); bid /= tiles;
  const int cz = (int)(bid % (3u * (unsigned)g.nz));
  const int b = (int)(bid / (3u * (unsigned)g.nz));
  if (ep.ctl && ldu(&ep.ctl[b].done)) return;
  const int kx0 = tile * CB;
  const int ncol = g.Xp - kx0 < CB ? g.Xp - kx0 : CB;
  const int cs = col_stride(g.Py);
  const int sh = hp.fd[1].psh;
  const int ny = g.ny;
  // Sx blocks kx0 / kSxB ... of this plane; Sy rows cz Xp + kx0 + i
  Cx<T>* const sx = hp.Sx + (size_t)b * g.sx + (size_t)cz * g.XB * kSxB * ny + (size_t)kx0 * ny;
  Cx<T>* const sy = hp.Sy + (size_t)b * g.sy + ((size_t)cz * g.Xp + kx0) * g.Py;
  const int tpc = SL > 0 ? SL / EPT : (int)blockDim.x / CB;
  const int c = (int)threadIdx.x / tpc;
  const int cc = c < ncol ? c : 0;
  const bool half = g.Py == 2 * ny;
  if (CB <= kSxB) {
    Cx<T>* const sxp = hp.Sx + (size_t)b * g.sx + (size_t)cz * g.XB * kSxB * ny;  // plane
    const int kxc = kx0 + cc;
    const uint32_t coff = (uint32_t)((kxc >> 2) * kSxB * ny + (kxc & 3)) * (uint32_t)sizeof(Cx<T>);
    constexpr uint32_t sb = kSxB * sizeof(Cx<T>);
    const uint32_t yoff = (uint32_t)(cc * g.Py) * (uint32_t)sizeof(Cx<T>);
    if constexpr (!INV) {
      const ColLoadS<T> ld{sxp, coff, sb, ny};
      const ColStore<T> st{sy, yoff, g.Py};
      if constexpr (SL > 0)
        fft_static<T, SL, (EPT > 8), false, true, true, false, true, false, EPT>(lds, hp.fd[1].tw, cs, ncol, ld, st, NoHook{});
      else
        fft_run<T, false, true, true, false, R16>(lds, hp.fd[1], hp.fd[1].tw, cs, ncol, tpc, half, false, ld, st,
                                                  NoHook{});
    } else {
      const ColLoad<T> ld{sy, yoff, g.Py};
      const ColStoreS<T> st{sxp, coff, sb, ny};
      if constexpr (SL > 0)
        fft_static<T, SL, (EPT > 8), true, true, true, false, false, true, EPT>(lds, hp.fd[1].tw, cs, ncol, ld, st, NoHook{});
      else
        fft_run<T, true, true, true, false, R16>(lds, hp.fd[1], hp.fd[1].tw, cs, ncol, tpc, false, half, ld, st,
                                                 NoHook{});
    }
    return;
  }
  // entry t of the staged blocks: column i = kSxB (t / (kSxB ny)) + t % kSxB, row
  // (t / kSxB) % ny; the tile's blocks (ncol rounded up) are contiguous from sx
  const int nblk = (ncol + kSxB - 1) / kSxB;
  const FDiv dbl = fdiv_of(kSxB * ny);
  auto ent = [&](int t, int& i, int& y) {
    const int q = fdiv_q(t, dbl), e = t - mul24(q, kSxB * ny);
    y = e >> 2;
    i = q * kSxB + (e & 3);
  };
  if constexpr (!INV) {
    for (int t = threadIdx.x; t < nblk * kSxB * ny; t += blockDim.x) {  // stage in
      int i, y;
      ent(t, i, y);
      if (i < ncol) lds[i * cs + pidx(y, sh)] = gldo(sx, (uint32_t)t * (uint32_t)sizeof(Cx<T>));
    }
    // zero padding of the columns, unless the transform leaves the upper half unread
    const bool hin = SL > 0 || (half && (hp.fd[1].code & kFftFirstEven) && hp.fd[1].nst > 1);
    if (!hin) {
      const int nz0 = g.Py - ny;
      const FDiv dz = fdiv_of(nz0);
      for (int t = threadIdx.x; t < CB * nz0; t += blockDim.x) {
        const int i = fdiv_q(t, dz), y = ny + (t - mul24(i, nz0));
        lds[i * cs + pidx(y, sh)] = Cx<T>{T(0), T(0)};
      }
    }
    __syncthreads();
    const ColStore<T> st{sy, (uint32_t)(cc * g.Py) * (uint32_t)sizeof(Cx<T>), g.Py};
    if constexpr (SL > 0)
      fft_static<T, SL, (EPT > 8), false, false, true, false, true, false, EPT>(lds, hp.fd[1].tw, cs, ncol, NoLoad<T>{}, st,
                                                                      NoHook{});
    else
      fft_run<T, false, false, true, false, R16>(lds, hp.fd[1], hp.fd[1].tw, cs, ncol, tpc, half, false, NoLoad<T>{},
                                                 st, NoHook{});
  } else {
    const ColLoad<T> ld{sy, (uint32_t)(cc * g.Py) * (uint32_t)sizeof(Cx<T>), g.Py};
    if constexpr (SL > 0)
      fft_static<T, SL, (EPT > 8), true, true, false, false, false, true, EPT>(lds, hp.fd[1].tw, cs, ncol, ld, NoStore<T>{},
                                                                     NoHook{});
    else
      fft_run<T, true, true, false, false, R16>(lds, hp.fd[1], hp.fd[1].tw, cs, ncol, tpc, false, half, ld,
                                                NoStore<T>{}, NoHook{});
    for (int t = threadIdx.x; t < nblk * kSxB * ny; t += blockDim.x) {  // stage out
      int i, y;
      ent(t, i, y);
      if (i < ncol) gsto(sx, (uint32_t)t * (uint32_t)sizeof(Cx<T>), lds[i * cs + pidx(y, sh)]);
    }
  }
}

// Forward y pass of every group: fused 2-D or 3-D forward rows.
// R16: the y plans hold radix-16 stages (lengths beyond 512 points).
template <typename T, bool R16>
__global__ void __launch_bounds__(512) k_ypass(Launch<T> L) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  long long bid;
  const int gi = group_of(L, bid);
  const HotPlan<T> hp = hot_plan(L, gi);
  if (hp.g.nz == 1) {
    if (bid >= y2d_blocks(hp.g, hp.tu, hp.batch)) return;
    y_fused2d<T, R16>(hp, ldu(L.epis + gi), bid, lds);
  } else {
    if (bid >= y3d_blocks(hp.g, hp.tu, hp.batch)) return;
    y_rows3d<T, false, R16>(hp, ldu(L.epis + gi), bid, lds);
  }
}

template <typename T, bool R16>
__global__ void __launch_bounds__(512) k_yinv(Launch<T> L) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  long long bid;
  const int gi = group_of(L, bid);
  const HotPlan<T> hp = hot_plan(L, gi);
  if (bid >= y3d_blocks(hp.g, hp.tu, hp.batch)) return;
  y_rows3d<T, true, R16>(hp, ldu(L.epis + gi), bid, lds);
}

// The y passes compiled for one length: every group of the launch has
// Py = SL = 2 ny (the host checks), SL/EPT threads per column.
template <typename T, int SL, int EPT>
__global__ void __launch_bounds__(512) k_ypass_s(Launch<T> L) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  long long bid;
  const int gi = group_of(L, bid);
  const HotPlan<T> hp = hot_plan(L, gi);
  if (hp.g.nz == 1) {
    if (bid >= y2d_blocks(hp.g, hp.tu, hp.batch)) return;
    y_fused2d<T, false, SL, EPT>(hp, ldu(L.epis + gi), bid, lds);
  } else {
    if (bid >= y3d_blocks(hp.g, hp.tu, hp.batch)) return;
    y_rows3d<T, false, false, SL, EPT>(hp, ldu(L.epis + gi), bid, lds);
  }
}

template <typename T, int SL, int EPT>
__global__ void __launch_bounds__(512) k_yinv_s(Launch<T> L) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  long long bid;
  const int gi = group_of(L, bid);
  const HotPlan<T> hp = hot_plan(L, gi);
  if (bid >= y3d_blocks(hp.g, hp.tu, hp.batch)) return;
  y_rows3d<T, true, false, SL, EPT>(hp, ldu(L.epis + gi), bid, lds);
}

// ---------------------------------------------------------------------------
// 3-D z pass (LDS version, any Pz): forward z, tensor product, inverse z for
// qz consecutive (kx,ky) points and the 3 components, in place in Sy.
// ---------------------------------------------------------------------------
__host__ __device__ inline long long zlds_blocks(const Geo& g, const Tuning& tu, int batch) {
  return (long long)batch * (((long long)g.Xp * g.Py + tu.qz - 1) / tu.qz);
}

template <typename T>
__global__ void __launch_bounds__(512) k_z3d(Launch<T> L) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  long long bid;
  const int gi = group_of(L, bid);
  const HotPlan<T> hp = hot_plan(L, gi);
  const Epi<T> ep = ldu(L.epis + gi);
  const Geo& g = hp.g;
  if (bid >= zlds_blocks(g, hp.tu, hp.batch)) return;
  const int QZ = hp.tu.qz;
  const long long nq = (long long)g.Xp * g.Py;
  const long long tiles = (nq + QZ - 1) / QZ;
  const long long tile = bid % tiles;
  const int b = (int)(bid / tiles);
  if (ep.ctl && ldu(&ep.ctl[b].done)) return;
  const long long q0 = tile * QZ;
  const int nqt = (int)((nq - q0) < QZ ? (nq - q0) : QZ);
  const int cs = col_stride(g.Pz);
  const int sh = hp.fd[2].psh;
  Cx<T>* base = hp.Sy + (size_t)b * g.sy;  // [3][nz][Xp*Py]
  const size_t plane = (size_t)nq;
  // column col = c*QZ + j, element z
  for (int t0 = threadIdx.x; t0 < 3 * g.Pz * QZ; t0 += kUnroll * blockDim.x) {
    Cx<T> v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int t = t0 + u * blockDim.x;
      const int j = t % QZ;
      const int cz = t / QZ;
      const int c = cz / g.Pz, z = cz - c * g.Pz;
      v[u] = {T(0), T(0)};
      if (t < 3 * g.Pz * QZ && z < g.nz && j < nqt) v[u] = gld(base + ((size_t)c * g.nz + z) * plane + q0 + j);
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int t = t0 + u * blockDim.x;
      if (t < 3 * g.Pz * QZ) {
        const int j = t % QZ;
        const int cz = t / QZ;
        const int c = cz / g.Pz, z = cz - c * g.Pz;
        lds[(c * QZ + j) * cs + pidx(z, sh)] = v[u];
      }
    }
  }
  __syncthreads();
  const int tpc = blockDim.x / (3 * QZ);
  fft_columns<T, false, false>(lds, hp.fd[2], cs, 3 * QZ, tpc, hp.fd[2].tw);
  const T s = T(ldu(&hp.prm[b].demag_scale));
  for (int t = threadIdx.x; t < QZ * g.Pz; t += blockDim.x) {
    const int j = t % QZ, kz = t / QZ;
    if (j >= nqt) continue;
    const long long q = q0 + j;
    const int kx = (int)(q / g.Py), ky = (int)(q - (long long)kx * g.Py);
    tensor_apply(hp, kx, ky, kz, s, lds[(0 * QZ + j) * cs + pidx(kz, sh)],
                 lds[(1 * QZ + j) * cs + pidx(kz, sh)], lds[(2 * QZ + j) * cs + pidx(kz, sh)]);
  }
  __syncthreads();
  fft_columns<T, true, false>(lds, hp.fd[2], cs, 3 * QZ, tpc, hp.fd[2].tw);
  for (int t = threadIdx.x; t < 3 * g.nz * QZ; t += blockDim.x) {
    const int j = t % QZ;
    const int cz = t / QZ;
    const int c = cz / g.nz, z = cz - c * g.nz;
    if (j < nqt) gst(base + ((size_t)c * g.nz + z) * plane + q0 + j, lds[(c * QZ + j) * cs + pidx(z, sh)]);
  }
}

// ---------------------------------------------------------------------------
// 3-D z pass with nz = PZ/2 and PZ a power of two, through LDS with a
// transform compiled for PZ: Q consecutive (kx,ky) points of one instance,
// the 3 components' nz planes loaded as Q-long contiguous runs, forward z
// (upper half zero, not read), tensor product, inverse z (only the nz
// physical planes formed), stored the same way.  For FP64, whose 32-point
// columns do not fit one lane's registers.
// ---------------------------------------------------------------------------
__host__ __device__ inline long long zs_blocks(const Geo& g, int batch, int Q) {
  return (long long)batch * (((long long)g.Xp * g.Py + Q - 1) / Q);
}

template <typename T, int PZ, int Q, int EPT>
__global__ void __launch_bounds__(512) k_z3d_s(Launch<T> L) {
  constexpr int NZ = PZ / 2;
  constexpr int LQ = ilog2c(Q), LNZ = ilog2c(NZ);
  static_assert((1 << LQ) == Q && (1 << LNZ) == NZ, "powers of two");
  constexpr int SH = p2_psh(PZ, false);
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  long long bid0;
  const int gi = group_of(L, bid0);
  const HotPlan<T> hp = hot_plan(L, gi);
  const Geo& g = hp.g;
  if (bid0 >= zs_blocks(g, hp.batch, Q)) return;
  const int nq = g.Xp * g.Py;
  const unsigned tiles = (unsigned)((nq + Q - 1) / Q);
  const unsigned bid = (unsigned)bid0;
  const int tile = (int)(bid % tiles);
  const int b = (int)(bid / tiles);
  DevCtl* const ctl = ldu(&L.epis[gi].ctl);
  if (ctl && ldu(&ctl[b].done)) return;
  const int q0 = tile * Q;
  const int nqt = nq - q0 < Q ? nq - q0 : Q;
  const int cs = col_stride(PZ);
  // Sy [3][nz][Xp Py] of the instance, from point q0 on: entry (c, z, j) at
  // (c nz + z) nq + j
  const Cx<T>* src = hp.Sy + (size_t)b * g.sy + q0;
  Cx<T>* dst = hp.Sy + (size_t)b * g.sy + q0;
  constexpr int NE = 3 * NZ * Q;
  constexpr int U = 4;
  for (int t0 = threadIdx.x; t0 < NE; t0 += U * blockDim.x) {  // column (c, j) = c Q + j, entry z
    Cx<T> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * blockDim.x, j = t & (Q - 1), cz = t >> LQ;
      v[u] = Cx<T>{T(0), T(0)};
      if (t < NE && j < nqt) v[u] = gldo(src, (uint32_t)(cz * nq + j) * (uint32_t)sizeof(Cx<T>));
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * blockDim.x, j = t & (Q - 1), cz = t >> LQ;
      if (t < NE) lds[((cz >> LNZ) * Q + j) * cs + pidx(cz & (NZ - 1), SH)] = v[u];
    }
  }
  // this thread's tensor points (t = threadIdx.x + i NTH, the kernel runs NTH
  // threads), loaded before the transform so that their latency overlaps it
  constexpr int NTH = 3 * Q * (PZ / EPT);
  constexpr int IT = (Q * PZ + NTH - 1) / NTH;
  const T s = T(ldu(&hp.prm[b].demag_scale));
  const FDiv dpy = fdiv_of(g.Py);
  Ten<T> ten[IT];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int t = threadIdx.x + i * NTH, j = t & (Q - 1), kz = t >> LQ;
    const int q = q0 + (j < nqt ? j : 0);
    const int kx = fdiv_q(q, dpy), ky = q - mul24(kx, g.Py);
    if (t < Q * PZ) ten[i] = tensor_load(hp, kx, ky, kz < PZ ? kz : 0, s);
  }
  __syncthreads();
  const NoLoad<T> nl;
  const NoStore<T> nst;
  const NoHook nh;
  fft_static<T, PZ, false, false, false, false, false, true, false, EPT>(lds, hp.fd[2].tw, cs, 3 * Q, nl, nst, nh);
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int t = threadIdx.x + i * NTH, j = t & (Q - 1), kz = t >> LQ;
    if (t >= Q * PZ || j >= nqt) continue;
    const int o = pidx(kz, SH);
    tensor_mul(ten[i], lds[(0 * Q + j) * cs + o], lds[(1 * Q + j) * cs + o], lds[(2 * Q + j) * cs + o]);
  }
  __syncthreads();
  fft_static<T, PZ, false, true, false, false, false, false, true, EPT>(lds, hp.fd[2].tw, cs, 3 * Q, nl, nst, nh);
  for (int t = threadIdx.x; t < NE; t += blockDim.x) {
    const int j = t & (Q - 1), cz = t >> LQ;
    if (j < nqt)
      gsto(dst, (uint32_t)(cz * nq + j) * (uint32_t)sizeof(Cx<T>),
           lds[((cz >> LNZ) * Q + j) * cs + pidx(cz & (NZ - 1), SH)]);
  }
}

// ---------------------------------------------------------------------------
// 3-D z pass with the transform in registers: one thread owns the Pz-point
// columns of the 3 components at one (kx, ky); no LDS, no barriers.
// ---------------------------------------------------------------------------
__host__ __device__ inline long long zreg_blocks(const Geo& g, int batch) {
  return (long long)batch * (((long long)g.Xp * g.Py + kNT - 1) / kNT);
}

// HALF: nz == Pz / 2 (the usual padding), so the upper half of every input
// column is a compile-time zero and only the lower half of the output is kept.
template <typename T, int PZ, bool HALF>
__device__ __forceinline__ void z3d_reg_body(const Launch<T>& L) {
  long long bid;
  const int gi = group_of(L, bid);
  const HotPlan<T> hp = hot_plan(L, gi);
  const Epi<T> ep = ldu(L.epis + gi);
  const Geo& g = hp.g;
  if (bid >= zreg_blocks(g, hp.batch)) return;
  const long long nq = (long long)g.Xp * g.Py;
  const long long qb = (nq + kNT - 1) / kNT;
  const int b = (int)(bid / qb);
  if (ep.ctl && ldu(&ep.ctl[b].done)) return;
  const long long q = (bid % qb) * kNT + threadIdx.x;
  if (q >= nq) return;
  Cx<T>* base = hp.Sy + (size_t)b * g.sy + q;
  const size_t plane = (size_t)nq;
  Cx<T> v[3][PZ];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int z = 0; z < PZ; ++z) {
      v[c][z] = {T(0), T(0)};
      if (HALF ? z < PZ / 2 : z < g.nz) v[c][z] = gld(base + ((size_t)c * g.nz + z) * plane);
    }
  // the stores recompute their addresses from an opaque copy of the column
  // pointer: keeping the 3 nz load addresses alive through the transforms
  // would cost two registers each
  asm volatile("" : "+v"(base));
#pragma unroll
  for (int c = 0; c < 3; ++c) RegFft<T, PZ, 1, false>::run(v[c], hp.twz);
  const int kx = (int)q / g.Py, ky = (int)q - kx * g.Py;
  const int kyf = ky <= g.Py - ky ? ky : g.Py - ky;
  const T sy = ky > g.Py - ky ? T(-1) : T(1);
  const size_t cstride = (size_t)g.Kz * g.Xp * g.Ky;
  const T s = T(ldu(&hp.prm[b].demag_scale));
#pragma unroll
  for (int kz = 0; kz < PZ; ++kz) {
    const int kzf = kz <= PZ - kz ? kz : PZ - kz;
    const T sz = kz > PZ - kz ? T(-1) : T(1);
    const size_t off = ((size_t)kzf * g.Xp + kx) * g.Ky + kyf;
    const T kxx = gld(hp.kt + off) * s;
    const T kyy = gld(hp.kt + cstride + off) * s;
    const T kzz = gld(hp.kt + 2 * cstride + off) * s;
    const T kxy = gld(hp.kt + 3 * cstride + off) * (s * sy);
    const T kxz = gld(hp.kt + 4 * cstride + off) * (s * sz);
    const T kyz = gld(hp.kt + 5 * cstride + off) * (s * sy * sz);
    const Cx<T> a = v[0][kz], bb = v[1][kz], cc = v[2][kz];
    v[0][kz] = {kxx * a.x + kxy * bb.x + kxz * cc.x, kxx * a.y + kxy * bb.y + kxz * cc.y};
    v[1][kz] = {kxy * a.x + kyy * bb.x + kyz * cc.x, kxy * a.y + kyy * bb.y + kyz * cc.y};
    v[2][kz] = {kxz * a.x + kyz * bb.x + kzz * cc.x, kxz * a.y + kyz * bb.y + kzz * cc.y};
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) RegFft<T, PZ, 1, true>::run(v[c], hp.twz);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int z = 0; z < PZ; ++z)
      if (HALF ? z < PZ / 2 : z < g.nz) gst(base + ((size_t)c * g.nz + z) * plane, v[c][z]);
}

// Two waves per SIMD fit the half-zero columns (up to 32 points in FP32)
// without spilling; the general columns keep the default register budget.
template <typename T, int PZ>
__global__ void __launch_bounds__(kNT, 2) k_z3d_reg_half(Launch<T> L) {
  z3d_reg_body<T, PZ, true>(L);
}

template <typename T, int PZ>
__global__ void __launch_bounds__(kNT) k_z3d_reg(Launch<T> L) {
  z3d_reg_body<T, PZ, false>(L);
}

// ---------------------------------------------------------------------------
// 3-D z pass for even Pz = 2M, one (kx, ky) column per lane pair.  The input
// is zero beyond z = M - 1 (nz <= M), so the even outputs of the length-2M
// transform are the length-M transform of x and the odd ones that of
// x[z] exp(-2 pi i z / 2M).  Lane p of the pair computes the outputs with
// kz = 2k + p, multiplies by the tensor there and transforms back over M
// points; the inverse over 2M points is the sum of the two halves, the odd
// half multiplied by exp(+2 pi i z / 2M).  Each lane ends with the z of its
// parity, after one exchange with its partner.  Half the registers of the
// one-lane version, so twice to four times the waves per SIMD.
// ---------------------------------------------------------------------------
__host__ __device__ inline long long zpair_blocks(const Geo& g, int batch) {
  return (long long)batch * (((long long)g.Xp * g.Py + kNT / 2 - 1) / (kNT / 2));
}

// value of the partner lane (lane ^ 1), within a quad
__device__ __forceinline__ float pair_swap(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double pair_swap(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename T, int M>
__global__ void __launch_bounds__(kNT) k_z3d_pair(Launch<T> L) {
  constexpr int PZ = 2 * M;
  long long bid;
  const int gi = group_of(L, bid);
  const HotPlan<T> hp = hot_plan(L, gi);
  const Geo& g = hp.g;
  if (bid >= zpair_blocks(g, hp.batch)) return;
  const long long nq = (long long)g.Xp * g.Py;
  const long long qb = (nq + kNT / 2 - 1) / (kNT / 2);
  const int b = (int)(bid / qb);
  DevCtl* const ctl = ldu(&L.epis[gi].ctl);
  if (ctl && ldu(&ctl[b].done)) return;
  const int p = threadIdx.x & 1;
  const long long q = (bid % qb) * (kNT / 2) + (threadIdx.x >> 1);
  // both lanes of a pair are in range or out of range together (the exchange
  // below needs the partner); out-of-range pairs compute on zeros and store nothing
  const bool live = q < nq;
  const int ql = live ? (int)q : 0;  // out-of-range lanes read element 0 and store nothing
  const uint32_t qoff = (uint32_t)ql * (uint32_t)sizeof(Cx<T>);
  Cx<T>* const Syb = hp.Sy + (size_t)b * g.sy;  // plane (c, z) starts at Syb + (c nz + z) nq
  const int nz = g.nz;
  Cx<T> v[3][M];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int z = 0; z < M; ++z) {
      v[c][z] = {T(0), T(0)};
      if (z < nz) v[c][z] = gldo(Syb + ((size_t)c * nz + z) * nq, qoff);  // uniform branch
    }
  // odd lanes: pre-multiply by exp(-2 pi i z / 2M)
#pragma unroll
  for (int z = 1; z < M; ++z) {
    Cx<T> w = ldu(hp.twz + z);
    if (!p) w = Cx<T>{T(1), T(0)};
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c][z] = cmul(v[c][z], w);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) RegFft<T, M, 1, false, 2>::run(v[c], hp.twz);
  const int kx = ql / g.Py, ky = ql - kx * g.Py;
  const int kyf = ky <= g.Py - ky ? ky : g.Py - ky;
  const T sy = ky > g.Py - ky ? T(-1) : T(1);
  const size_t cstride = (size_t)g.Kz * g.Xp * g.Ky;
  const T s = T(ldu(&hp.prm[b].demag_scale));
  const uint32_t XK = (uint32_t)g.Xp * (uint32_t)g.Ky;
  const uint32_t kxy0 = (uint32_t)kx * (uint32_t)g.Ky + (uint32_t)kyf;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const int kz = 2 * k + p;
    const int kzf = kz <= PZ - kz ? kz : PZ - kz;
    const T sz = kz > PZ - kz ? T(-1) : T(1);
    const uint32_t ko = ((uint32_t)kzf * XK + kxy0) * (uint32_t)sizeof(T);
    const T kxx = gldo(hp.kt, ko) * s;
    const T kyy = gldo(hp.kt + cstride, ko) * s;
    const T kzz = gldo(hp.kt + 2 * cstride, ko) * s;
    const T kxy = gldo(hp.kt + 3 * cstride, ko) * (s * sy);
    const T kxz = gldo(hp.kt + 4 * cstride, ko) * (s * sz);
    const T kyz = gldo(hp.kt + 5 * cstride, ko) * (s * sy * sz);
    const Cx<T> a = v[0][k], bb = v[1][k], cc = v[2][k];
    v[0][k] = {kxx * a.x + kxy * bb.x + kxz * cc.x, kxx * a.y + kxy * bb.y + kxz * cc.y};
    v[1][k] = {kxy * a.x + kyy * bb.x + kyz * cc.x, kxy * a.y + kyy * bb.y + kyz * cc.y};
    v[2][k] = {kxz * a.x + kyz * bb.x + kzz * cc.x, kxz * a.y + kyz * bb.y + kzz * cc.y};
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) RegFft<T, M, 1, true, 2>::run(v[c], hp.twz);
  // odd lanes: post-multiply by exp(+2 pi i z / 2M)
#pragma unroll
  for (int z = 1; z < M; ++z) {
    Cx<T> w = ldu(hp.twz + z);
    w.y = -w.y;
    if (!p) w = Cx<T>{T(1), T(0)};
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c][z] = cmul(v[c][z], w);
  }
  // z of parity p: own half + partner's half.  Lane p sends the partner the
  // value at the partner's parity.
#pragma unroll
  for (int z0 = 0; z0 < M; z0 += 2) {
    const int ze = z0, zo = z0 + 1 < M ? z0 + 1 : z0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const Cx<T> send = p ? v[c][ze] : v[c][zo];
      const Cx<T> got = {pair_swap(send.x), pair_swap(send.y)};
      const Cx<T> mine = p ? v[c][zo] : v[c][ze];
      const Cx<T> sum = cadd(mine, got);
      const int zz = p ? zo : ze;
      if (live && zz < nz && (p == 0 || z0 + 1 < M)) gsto(Syb + ((size_t)c * nz + zz) * nq, qoff, sum);
    }
  }
}

// ---------------------------------------------------------------------------
// Local fields at one cell.  Returns the separate terms when ENERGY is set.
// ---------------------------------------------------------------------------
template <typename T> struct V3 { T x, y, z; };

template <typename T>
__device__ __forceinline__ V3<T> ld3(const T* __restrict__ p, long long N, long long i) {
  return {gld(p + i), gld(p + N + i), gld(p + 2 * N + i)};
}

// Byte offsets of one cell in an instance's [3][N] array (component c at
// o[c]; the host keeps 3 N sizeof(T) below 2^32).  Neighbours and the other
// arrays of the same layout use the same offsets from a shifted base pointer
// (a scalar add), so that every access is one vector offset plus a scalar base.
struct COff {
  uint32_t o[3];
};
template <typename T>
__device__ __forceinline__ COff coff_of(long long N, int i) {
  const uint32_t nb = (uint32_t)N * (uint32_t)sizeof(T);
  const uint32_t o0 = (uint32_t)i * (uint32_t)sizeof(T);
  return COff{{o0, o0 + nb, o0 + 2 * nb}};
}
template <typename T>
__device__ __forceinline__ V3<T> ld3o(const T* base, const COff& c) {
  return {gldo(base, c.o[0]), gldo(base, c.o[1]), gldo(base, c.o[2])};
}
template <typename T>
__device__ __forceinline__ void st3o(T* base, const COff& c, V3<T> v) {
  gsto(base, c.o[0], v.x);
  gsto(base, c.o[1], v.y);
  gsto(base, c.o[2], v.z);
}

struct LocalTerms {
  double ex, dmi, an, ze;  // m . H_term (FP64), for energies
};

// Coefficients of the local terms in the working precision (kept in scalar
// registers for the whole epilogue).
template <typename T> struct LocalCoef {
  T cex[3], cdmi[3], can, u[3], H[3];
  uint32_t terms;
};

template <typename T>
__device__ __forceinline__ LocalCoef<T> local_coef(const DevParams& P) {
  LocalCoef<T> c;
  for (int a = 0; a < 3; ++a) {
    c.cex[a] = T(P.cex[a]);
    c.u[a] = T(P.u[a]);
    c.H[a] = T(P.H[a]);
  }
  c.cdmi[0] = T(P.cdmi[0]);
  c.cdmi[1] = T(P.cdmi[1]);
  c.cdmi[2] = T(P.cdmi[2]);
  c.can = T(P.can);
  c.terms = P.terms;
  return c;
}

// m at a cell and its six neighbours (zero where the mesh ends or no term needs them)
template <typename T> struct Nbr { V3<T> mi, xm, xp, ym, yp, zm, zp; };

template <typename T>
__device__ __forceinline__ Nbr<T> load_nbr(const Geo& g, uint32_t terms, const T* __restrict__ mb, const COff& co,
                                           int x, int y, int z) {
  Nbr<T> n;
  n.mi = ld3o(mb, co);
  n.xm = {T(0), T(0), T(0)};
  n.xp = n.xm; n.ym = n.xm; n.yp = n.xm; n.zm = n.xm; n.zp = n.xm;
  if (terms & (MM_EXCHANGE | MM_DMI_INTERFACIAL | MM_DMI_BULK | MM_DMI_D2D | MM_STT_ZL)) {
    const long long nxy = (long long)g.nx * g.ny;
    if (x > 0) n.xm = ld3o(mb - 1, co);
    if (x + 1 < g.nx) n.xp = ld3o(mb + 1, co);
    if (y > 0) n.ym = ld3o(mb - g.nx, co);
    if (y + 1 < g.ny) n.yp = ld3o(mb + g.nx, co);
    if (z > 0) n.zm = ld3o(mb - nxy, co);
    if (z + 1 < g.nz) n.zp = ld3o(mb + nxy, co);
  }
  return n;
}

template <typename T, bool ENERGY>
__device__ __forceinline__ V3<T> local_field(const Geo& g, const LocalCoef<T>& P, const Nbr<T>& nb, int x, int y,
                                             int z, LocalTerms* lt) {
  const V3<T> mi = nb.mi;
  V3<T> H = {T(0), T(0), T(0)};
  const V3<T> xm = nb.xm, xp = nb.xp, ym = nb.ym, yp = nb.yp, zm = nb.zm, zp = nb.zp;
  const bool hxm = x > 0, hxp = x + 1 < g.nx, hym = y > 0, hyp = y + 1 < g.ny;
  const bool hzm = z > 0, hzp = z + 1 < g.nz;
  if (P.terms & MM_EXCHANGE) {
    const T cx = P.cex[0], cy = P.cex[1], cz = P.cex[2];
    V3<T> e = {T(0), T(0), T(0)};
    auto acc = [&](bool has, V3<T> nb, T c) {
      if (has) {
        e.x += c * (nb.x - mi.x);
        e.y += c * (nb.y - mi.y);
        e.z += c * (nb.z - mi.z);
      }
    };
    acc(hxm, xm, cx); acc(hxp, xp, cx);
    acc(hym, ym, cy); acc(hyp, yp, cy);
    acc(hzm, zm, cz); acc(hzp, zp, cz);
    H.x += e.x; H.y += e.y; H.z += e.z;
    if (ENERGY) lt->ex = (double)mi.x * e.x + (double)mi.y * e.y + (double)mi.z * e.z;
  }
  if (P.terms & MM_DMI_INTERFACIAL) {
    // x neighbours: -(D/mu0Ms dx) e_y x (m_{+x} - m_{-x});  e_y x v = (v_z, 0, -v_x)
    // y neighbours: -(D/mu0Ms dy) e_x x (m_{-y} - m_{+y});  e_x x v = (0, -v_z, v_y)
    const T cx = P.cdmi[0], cy = P.cdmi[1];
    const V3<T> dx = {xp.x - xm.x, xp.y - xm.y, xp.z - xm.z};
    const V3<T> dy = {ym.x - yp.x, ym.y - yp.y, ym.z - yp.z};
    V3<T> d = {-cx * dx.z, cy * dy.z, cx * dx.x - cy * dy.y};
    H.x += d.x; H.y += d.y; H.z += d.z;
    if (ENERGY) lt->dmi += (double)mi.x * d.x + (double)mi.y * d.y + (double)mi.z * d.z;
  }
  if (P.terms & (MM_DMI_BULK | MM_DMI_D2D)) {
    // a = m_{+x} - m_{-x}, b = m_{+y} - m_{-y}, c = m_{+z} - m_{-z} (missing neighbours are zero);
    // e_x x v = (0, -v_z, v_y), e_y x v = (v_z, 0, -v_x), e_z x v = (-v_y, v_x, 0)
    const T cx = P.cdmi[0], cy = P.cdmi[1], cz = P.cdmi[2];
    const V3<T> a = {xp.x - xm.x, xp.y - xm.y, xp.z - xm.z};
    const V3<T> b = {yp.x - ym.x, yp.y - ym.y, yp.z - ym.z};
    V3<T> d = {T(0), T(0), T(0)};
    if (P.terms & MM_DMI_BULK) {  // -(cx e_x x a + cy e_y x b + cz e_z x c)
      const V3<T> c = {zp.x - zm.x, zp.y - zm.y, zp.z - zm.z};
      d.x += cz * c.y - cy * b.z;
      d.y += cx * a.z - cz * c.x;
      d.z += cy * b.x - cx * a.y;
    }
    if (P.terms & MM_DMI_D2D) {  // cx e_x x a - cy e_y x b
      d.x -= cy * b.z;
      d.y -= cx * a.z;
      d.z += cx * a.y + cy * b.x;
    }
    H.x += d.x; H.y += d.y; H.z += d.z;
    if (ENERGY) lt->dmi += (double)mi.x * d.x + (double)mi.y * d.y + (double)mi.z * d.z;
  }
  if (P.terms & MM_ANIS_UNIAXIAL) {
    const T ux = P.u[0], uy = P.u[1], uz = P.u[2];
    const T s = P.can * (mi.x * ux + mi.y * uy + mi.z * uz);
    H.x += s * ux; H.y += s * uy; H.z += s * uz;
    if (ENERGY) lt->an = (double)s * ((double)mi.x * ux + (double)mi.y * uy + (double)mi.z * uz);
  }
  if (P.terms & MM_ZEEMAN) {
    H.x += P.H[0]; H.y += P.H[1]; H.z += P.H[2];
    if (ENERGY) lt->ze = (double)mi.x * P.H[0] + (double)mi.y * P.H[1] + (double)mi.z * P.H[2];
  }
  return H;
}

// General-material form of the local field (instances with cell-based
// material, interlayer coupling or spin torques).  Material per cell: with
// MM_CELLS each instance's cells carry Ms, A and D in a [3][N] array laid out
// like m (the same byte offsets reach them), else the instance's uniform
// values stand for every cell.  Pair couplings are the harmonic means of the
// exchange and DMI sections, A_ij = 2 A_i A_j / (A_i + A_j) and
// D_ij = 2 D_i D_j / (D_i + D_j) (0 unless D_i D_j > 0); a neighbour that is
// missing or empty (Ms = 0) couples with 0.  Neighbour order: -x, +x, -y, +y,
// -z, +z.
template <typename T> struct CellNbr {
  T ms;       // Ms of the cell (0: empty)
  T a[6];     // A_ij
  T d[6];     // D_ij
  uint32_t nbm;  // bit k: neighbour k present and magnetic
  int il;     // interlayer partner: +1 (this is layer k_lo), -1 (k_hi), 0 none
  V3<T> mo;   // the partner's m
};

// What the material loads need of the instance (scalar registers).
template <typename T> struct CellCtx {
  uint32_t terms;
  T Mu, Au, Du;
  int k_lo, k_hi;
};
template <typename T>
__device__ __forceinline__ CellCtx<T> cell_ctx(const DevParams* p) {
  CellCtx<T> c;
  c.terms = ldu(&p->terms);
  c.Mu = T(ldu(&p->Mu));
  c.Au = T(ldu(&p->Au));
  c.Du = T(ldu(&p->Du));
  c.k_lo = ldu(&p->k_lo);
  c.k_hi = ldu(&p->k_hi);
  return c;
}

template <typename T>
__device__ __forceinline__ T harmonic_a(T ai, T aj) {
  const T s = ai + aj;
  return s > T(0) ? T(2) * ai * aj / s : T(0);
}
template <typename T>
__device__ __forceinline__ T harmonic_d(T di, T dj) {
  return di * dj > T(0) ? T(2) * di * dj / (di + dj) : T(0);
}

// cb: the instance's cell arrays (read only with MM_CELLS); mb: its m
template <typename T>
__device__ __forceinline__ CellNbr<T> load_cells(const Geo& g, const CellCtx<T>& cx, const T* __restrict__ cb,
                                                 const T* __restrict__ mb, const COff& co, int x, int y, int z) {
  CellNbr<T> c;
  const bool arr = (cx.terms & MM_CELLS) != 0;
  const V3<T> me = arr ? ld3o(cb, co) : V3<T>{cx.Mu, cx.Au, cx.Du};
  c.ms = me.x;
  c.nbm = 0u;
  c.il = 0;
  c.mo = {T(0), T(0), T(0)};
#pragma unroll
  for (int k = 0; k < 6; ++k) { c.a[k] = T(0); c.d[k] = T(0); }
  const long long nxy = (long long)g.nx * g.ny;
  if (cx.terms & (MM_EXCHANGE | MM_DMI_INTERFACIAL | MM_DMI_BULK | MM_DMI_D2D | MM_STT_ZL)) {
    const bool in[6] = {x > 0, x + 1 < g.nx, y > 0, y + 1 < g.ny, z > 0, z + 1 < g.nz};
    const long long off[6] = {-1, 1, -(long long)g.nx, (long long)g.nx, -nxy, nxy};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      V3<T> o = {T(0), T(0), T(0)};
      if (in[k]) o = arr ? ld3o(cb + off[k], co) : me;
      const bool on = me.x > T(0) && o.x > T(0);
      c.a[k] = on ? harmonic_a(me.y, o.y) : T(0);
      c.d[k] = on ? harmonic_d(me.z, o.z) : T(0);
      c.nbm |= on ? (1u << k) : 0u;
    }
  }
  if ((cx.terms & MM_INTERLAYER) && (z == cx.k_lo || z == cx.k_hi)) {
    const long long off = (long long)((z == cx.k_lo ? cx.k_hi : cx.k_lo) - z) * nxy;
    const T mso = arr ? gldo(cb + off, co.o[0]) : cx.Mu;
    c.mo = ld3o(mb + off, co);
    c.il = me.x > T(0) && mso > T(0) ? (z == cx.k_lo ? 1 : -1) : 0;
  }
  return c;
}

// Coefficients of the general form beyond LocalCoef (interlayer, torques).
template <typename T> struct GenCoef {
  T crk, cdi[3], sa, sb, sp[3], zu[3], zbeta;
};
template <typename T>
__device__ __forceinline__ GenCoef<T> gen_coef(const DevParams& P) {
  GenCoef<T> q;
  q.crk = T(P.crk);
  q.sa = T(P.sa);
  q.sb = T(P.sb);
  q.zbeta = T(P.zbeta);
  for (int a = 0; a < 3; ++a) {
    q.cdi[a] = T(P.cdi[a]);
    q.sp[a] = T(P.sp[a]);
    q.zu[a] = T(P.zu[a]);
  }
  return q;
}

// Local field of a cell in the general form.  P holds the unit coefficients
// cex[a] = 2/(mu0 d_a^2), cdmi[a] = 1/(mu0 d_a), can = 2 Ku / mu0; each term
// carries the cell's own 1/Ms_i.  An empty cell has no field.  Missing or
// empty neighbours have zero couplings (their m, zero where the mesh ends,
// drops out).  Interlayer: (J m_o +- D_int x m_o)/(mu0 Ms dz) (+ at layer
// k_lo); spin-orbit torque: (b_J p + a_J m x p)/gamma; Zhang-Li:
// -(m x v + beta v)/gamma with v = (u . grad) m (central differences, one-sided
// next to a missing neighbour).
template <typename T, bool ENERGY>
__device__ __forceinline__ V3<T> local_field_cells(const LocalCoef<T>& P, const GenCoef<T>& Q, const Nbr<T>& nb,
                                                   const CellNbr<T>& cn, LocalTerms* lt) {
  V3<T> H = {T(0), T(0), T(0)};
  if (!(cn.ms > T(0))) return H;
  const T inv = T(1) / cn.ms;
  const V3<T> mi = nb.mi;
  const V3<T> xm = nb.xm, xp = nb.xp, ym = nb.ym, yp = nb.yp, zm = nb.zm, zp = nb.zp;
  if (P.terms & MM_EXCHANGE) {
    V3<T> e = {T(0), T(0), T(0)};
    auto acc = [&](V3<T> v, T c) {
      e.x += c * (v.x - mi.x);
      e.y += c * (v.y - mi.y);
      e.z += c * (v.z - mi.z);
    };
    acc(xm, P.cex[0] * cn.a[0]); acc(xp, P.cex[0] * cn.a[1]);
    acc(ym, P.cex[1] * cn.a[2]); acc(yp, P.cex[1] * cn.a[3]);
    acc(zm, P.cex[2] * cn.a[4]); acc(zp, P.cex[2] * cn.a[5]);
    e.x *= inv; e.y *= inv; e.z *= inv;
    H.x += e.x; H.y += e.y; H.z += e.z;
    if (ENERGY) lt->ex = (double)mi.x * e.x + (double)mi.y * e.y + (double)mi.z * e.z;
  }
  if (P.terms & (MM_DMI_INTERFACIAL | MM_DMI_BULK | MM_DMI_D2D)) {
    // weighted differences: a along x, b along y, c along z (+ neighbour minus - neighbour)
    const T cx = P.cdmi[0] * inv, cy = P.cdmi[1] * inv, cz = P.cdmi[2] * inv;
    const V3<T> a = {cx * (cn.d[1] * xp.x - cn.d[0] * xm.x), cx * (cn.d[1] * xp.y - cn.d[0] * xm.y),
                     cx * (cn.d[1] * xp.z - cn.d[0] * xm.z)};
    const V3<T> b = {cy * (cn.d[3] * yp.x - cn.d[2] * ym.x), cy * (cn.d[3] * yp.y - cn.d[2] * ym.y),
                     cy * (cn.d[3] * yp.z - cn.d[2] * ym.z)};
    V3<T> d = {T(0), T(0), T(0)};
    if (P.terms & MM_DMI_INTERFACIAL) {  // e_ij = {-e_y, e_y, e_x, -e_x}: -(e_y x a - e_x x b)
      d.x -= a.z;
      d.y -= b.z;
      d.z += a.x + b.y;
    }
    if (P.terms & MM_DMI_BULK) {  // e_ij = r_ij: -(e_x x a + e_y x b + e_z x c)
      const V3<T> c = {cz * (cn.d[5] * zp.x - cn.d[4] * zm.x), cz * (cn.d[5] * zp.y - cn.d[4] * zm.y),
                       cz * (cn.d[5] * zp.z - cn.d[4] * zm.z)};
      d.x += c.y - b.z;
      d.y += a.z - c.x;
      d.z += b.x - a.y;
    }
    if (P.terms & MM_DMI_D2D) {  // e_ij = {e_x, -e_x, -e_y, e_y}: -(-e_x x a + e_y x b)
      d.x -= b.z;
      d.y -= a.z;
      d.z += a.y + b.x;
    }
    H.x += d.x; H.y += d.y; H.z += d.z;
    if (ENERGY) lt->dmi = (double)mi.x * d.x + (double)mi.y * d.y + (double)mi.z * d.z;
  }
  if (P.terms & MM_ANIS_UNIAXIAL) {
    const T ux = P.u[0], uy = P.u[1], uz = P.u[2];
    const T s = P.can * inv * (mi.x * ux + mi.y * uy + mi.z * uz);
    H.x += s * ux; H.y += s * uy; H.z += s * uz;
    if (ENERGY) lt->an = (double)s * ((double)mi.x * ux + (double)mi.y * uy + (double)mi.z * uz);
  }
  if (P.terms & MM_ZEEMAN) {
    H.x += P.H[0]; H.y += P.H[1]; H.z += P.H[2];
    if (ENERGY) lt->ze = (double)mi.x * P.H[0] + (double)mi.y * P.H[1] + (double)mi.z * P.H[2];
  }
  if (cn.il != 0) {  // interlayer exchange and DMI with the partner layer
    const V3<T> mo = cn.mo;
    const T cj = Q.crk * inv, sg = cn.il > 0 ? inv : -inv;
    const V3<T> hj = {cj * mo.x, cj * mo.y, cj * mo.z};
    const V3<T> hd = {sg * (Q.cdi[1] * mo.z - Q.cdi[2] * mo.y), sg * (Q.cdi[2] * mo.x - Q.cdi[0] * mo.z),
                      sg * (Q.cdi[0] * mo.y - Q.cdi[1] * mo.x)};
    H.x += hj.x + hd.x; H.y += hj.y + hd.y; H.z += hj.z + hd.z;
    if (ENERGY) {
      lt->ex += (double)mi.x * hj.x + (double)mi.y * hj.y + (double)mi.z * hj.z;
      lt->dmi += (double)mi.x * hd.x + (double)mi.y * hd.y + (double)mi.z * hd.z;
    }
  }
  if (P.terms & MM_STT_SOT) {  // (b_J p + a_J m x p) / gamma
    const T px = Q.sp[0], py = Q.sp[1], pz = Q.sp[2];
    H.x += Q.sb * px + Q.sa * (mi.y * pz - mi.z * py);
    H.y += Q.sb * py + Q.sa * (mi.z * px - mi.x * pz);
    H.z += Q.sb * pz + Q.sa * (mi.x * py - mi.y * px);
  }
  if (P.terms & MM_STT_ZL) {  // -(m x v + beta v) / gamma, v = (u . grad) m
    V3<T> v = {T(0), T(0), T(0)};
    auto axis = [&](V3<T> p_, V3<T> m_, uint32_t bp, uint32_t bm, T c) {
      const bool hp = (cn.nbm & bp) != 0, hm = (cn.nbm & bm) != 0;
      V3<T> g_ = {T(0), T(0), T(0)};
      if (hp && hm) g_ = {T(0.5) * (p_.x - m_.x), T(0.5) * (p_.y - m_.y), T(0.5) * (p_.z - m_.z)};
      else if (hp) g_ = {p_.x - mi.x, p_.y - mi.y, p_.z - mi.z};
      else if (hm) g_ = {mi.x - m_.x, mi.y - m_.y, mi.z - m_.z};
      v.x += c * g_.x; v.y += c * g_.y; v.z += c * g_.z;
    };
    axis(xp, xm, 2u, 1u, Q.zu[0]);
    axis(yp, ym, 8u, 4u, Q.zu[1]);
    axis(zp, zm, 32u, 16u, Q.zu[2]);
    H.x -= (mi.y * v.z - mi.z * v.y) + Q.zbeta * v.x;
    H.y -= (mi.z * v.x - mi.x * v.z) + Q.zbeta * v.y;
    H.z -= (mi.x * v.y - mi.y * v.x) + Q.zbeta * v.z;
  }
  return H;
}

template <typename T>
__device__ __forceinline__ V3<T> ll_rhs(V3<T> m, V3<T> H, T g1, T g2) {
  const V3<T> a = {m.y * H.z - m.z * H.y, m.z * H.x - m.x * H.z, m.x * H.y - m.y * H.x};
  const V3<T> b = {m.y * a.z - m.z * a.y, m.z * a.x - m.x * a.z, m.x * a.y - m.y * a.x};
  return {g1 * a.x + g2 * b.x, g1 * a.y + g2 * b.y, g1 * a.z + g2 * b.z};
}

// x transform of the inverse-x kernel, LDS to LDS, TWL table twl: compiled for
// the power-of-two lengths 128 to 1024 (L/16 threads a column; the host's
// launch shapes give every column that many), the general plan otherwise.
// Inverse: only the first half of the output is kept; forward: hin as for
// fft_run (the input's upper half is zero and not read).
template <typename T, bool INV>
__device__ __forceinline__ void x_columns(Cx<T>* lds, const FftDesc<T>& p, int cs, int ncol, const Cx<T>* twl,
                                          bool hin) {
  constexpr bool HIN = !INV, HOUT = INV;
  const NoLoad<T> nl;
  const NoStore<T> nst;
  const NoHook nh;
  if (INV || hin) {
    // 8 entries per thread where the workgroup has the threads (shorter stages)
    const bool e8 = ncol * (p.L / 8) <= (int)blockDim.x;
#define MMX_XS(LL)                                                                                      \
  case LL:                                                                                              \
    if (e8) fft_static<T, LL, false, INV, false, false, true, HIN, HOUT, 8>(lds, twl, cs, ncol, nl, nst, nh); \
    else fft_static<T, LL, false, INV, false, false, true, HIN, HOUT, 16>(lds, twl, cs, ncol, nl, nst, nh);   \
    return;
    switch (p.L) {
      MMX_XS(128)
      MMX_XS(256)
      MMX_XS(512)
      MMX_XS(1024)
      default: break;
    }
#undef MMX_XS
  }
  fft_columns<T, INV, true>(lds, p, cs, ncol, (int)blockDim.x / ncol, twl, hin, INV);
}

// ---------------------------------------------------------------------------
// x inverse (complex-to-real) + local fields + LL + epilogue.  One workgroup:
// TY rows of one z plane of one instance.  The 3 x TY spectra are loaded
// together, transformed together (one column per component and row) and left
// in LDS, where the epilogue picks H_d up cell by cell.  DEMAG = false skips
// the transform (H_d = 0) and uses no LDS for it.  MODE is the epilogue.
// ---------------------------------------------------------------------------
__host__ __device__ inline long long inv_blocks(const Geo& g, const Tuning& tu, int batch) {
  return (long long)batch * g.nz * ((g.ny + tu.ty_x - 1) / tu.ty_x);
}


// ---------------------------------------------------------------------------
// Device-side Dormand-Prince controller, one thread per instance (FP64).
// ---------------------------------------------------------------------------
__device__ inline void control_step(DevCtl& C, const double* __restrict__ replay_h) {
  if (C.done) {
    C.pending_finish = 0;
    C.err_bits = 0ull;
    return;
  }
  const double h = C.h_att;
  const double err = __longlong_as_double((long long)C.err_bits) / C.rtol;
  const double dmdt = __longlong_as_double((long long)C.dmdt_bits);
  C.err_bits = 0ull;
  C.dmdt_bits = 0ull;
  C.last_err = err;
  C.n_attempt += 1;
  bool accept;
  const bool finite_err = err <= DBL_MAX;  // false for NaN and Inf
  if (!finite_err) {
    // overflowed stages or NaN in m: reject with the smallest factor; give up
    // after ten in a row
    C.nonfinite += 1;
    if (C.nonfinite >= 10 || C.replay_n > 0) {
      C.status = MM_E_NONFINITE;
      C.done = 1;
      C.pending_finish = 0;
      C.last_accepted = 0;
      return;
    }
    accept = false;
  } else {
    C.nonfinite = 0;
    accept = C.replay_n > 0 ? true : err <= 1.0;
  }
  if (accept) {
    C.t = (h == C.t_end - C.t) ? C.t_end : C.t + h;
    C.n_accept += 1;
    double fac = err == 0.0 ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(err, -0.2)));
    if (C.after_reject) fac = fmin(fac, 1.0);
    C.after_reject = 0;
    C.h = fmin(h * fac, C.h_max);
  } else {
    C.n_reject += 1;
    C.after_reject = 1;
    C.h = finite_err ? h * fmax(0.2, 0.9 * pow(err, -0.2)) : h * 0.2;
  }
  C.pending_finish = accept ? 1 : 0;
  C.last_accepted = accept ? 1 : 0;
  if (accept && C.stop_dmdt > 0.0) {  // relaxation: the new state's slope is k_7
    C.last_dmdt = dmdt;
    if (dmdt < C.stop_dmdt) {
      C.done = 1;
      return;
    }
  }
  // next attempt
  double hn;
  if (C.replay_n > 0) {
    C.replay_pos += 1;
    if (C.replay_pos >= C.replay_n) {
      C.done = 1;
      return;
    }
    hn = replay_h[C.replay_pos];
  } else {
    if (!(C.t_end - C.t > C.h_min)) {  // arrived; a remainder below h_min counts as arrived
      C.t = C.t_end;
      C.done = 1;
      return;
    }
    hn = fmin(fmin(C.h, C.h_max), C.t_end - C.t);
    if (hn < C.h_min) {
      C.status = MM_E_STEP_UNDERFLOW;
      C.done = 1;
      return;
    }
  }
  if (C.n_attempt >= C.max_attempt) {
    C.status = MM_E_MAXSTEPS;
    C.done = 1;
    return;
  }
  C.h_att = hn;
}

// End of an error pass in one workgroup: the largest error norm emax (and,
// for relaxations, the largest |k_7|^2 kmax) of its cells go into the
// instance's running maxima; the last of the instance's bpi workgroups to
// arrive takes the step decision.  The arrival uses the maxima's returned
// values (their top bits, always 0 for non-negative doubles), so it is issued
// only once the maxima are complete; the atomics are performed where every
// XCD sees them, so no fence (an L2 write-back on this part) is needed.
// red: the workgroup's LDS scratch, at least [2][waves].
__device__ __forceinline__ void error_pass_end(double emax, double kmax, DevCtl* ctl, int b, int bpi,
                                               const double* replay, double (*red)[512 / 64]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool relax = ldu(&ctl[b].stop_dmdt) > 0.0;
  const double w = wave_max(emax);
  if (lane == 0) red[0][wave] = w;
  if (relax) {
    const double wk = wave_max(kmax);
    if (lane == 0) red[1][wave] = wk;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = red[0][0];
    for (int j = 1; j < (int)(blockDim.x >> 6); ++j) v = fmax(v, red[0][j]);
    const unsigned long long prev = atomicMax(&ctl[b].err_bits, (unsigned long long)__double_as_longlong(v));
    unsigned long long prevk = 0ull;
    if (relax) {
      double vk = red[1][0];
      for (int j = 1; j < (int)(blockDim.x >> 6); ++j) vk = fmax(vk, red[1][j]);
      prevk = atomicMax(&ctl[b].dmdt_bits, (unsigned long long)__double_as_longlong(sqrt(vk)));
    }
    const int inc = 1 + (int)(prev >> 63) + (int)(prevk >> 63);
    if (atomicAdd(&ctl[b].arrive, inc) == bpi - 1) {
      ctl[b].arrive = 0;
      ctl[b].err_bits = atomicOr(&ctl[b].err_bits, 0ull);  // the complete maxima
      if (relax) ctl[b].dmdt_bits = atomicOr(&ctl[b].dmdt_bits, 0ull);
      control_step(ctl[b], replay);
    }
  }
}

// Runge-Kutta combination of one cell: base + sum_j hc_j kb_j + hl kk (hc_j,
// hl: h times the coefficients, zero where a slope is not used), projected
// back onto |m| = 1 when `project` (the end of a fixed step).
template <typename T>
__device__ __forceinline__ V3<T> rk_combine(V3<T> base, const V3<T> (&kb)[6], const T (&hc)[7], T hl, V3<T> kk,
                                            bool project) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    base.x += hc[j] * kb[j].x; base.y += hc[j] * kb[j].y; base.z += hc[j] * kb[j].z;
  }
  base.x += hl * kk.x; base.y += hl * kk.y; base.z += hl * kk.z;
  if (project) {
    const T s = rsqrt_t<T>(base.x * base.x + base.y * base.y + base.z * base.z);
    base.x *= s; base.y *= s; base.z *= s;
  }
  return base;
}

// Embedded error of one cell, |sum_j hc_j kb_j + hl kk| (the products in the
// plan precision, their sum in FP64), and |kk|^2, into running maxima; NaN or
// Inf count as +Inf.
template <typename T>
__device__ __forceinline__ void rk_error(const V3<T> (&kb)[6], const T (&hc)[7], T hl, V3<T> kk, double& emax,
                                         double& kmax) {
  double ex = 0, ey = 0, ez = 0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    ex += (double)(hc[j] * kb[j].x); ey += (double)(hc[j] * kb[j].y); ez += (double)(hc[j] * kb[j].z);
  }
  ex += (double)(hl * kk.x); ey += (double)(hl * kk.y); ez += (double)(hl * kk.z);
  double en = sqrt(ex * ex + ey * ey + ez * ez);
  if (!(en <= DBL_MAX)) en = HUGE_VAL;
  emax = fmax(emax, en);
  double kn = (double)kk.x * kk.x + (double)kk.y * kk.y + (double)kk.z * kk.z;
  if (!(kn <= DBL_MAX)) kn = HUGE_VAL;
  kmax = fmax(kmax, kn);
}

// End of an energy pass in one workgroup: its five FP64 sums (exchange, demag,
// DMI, anisotropy, Zeeman) to partial[(b bpi + lb) 5 + q], summed later in a
// fixed order.  red: the workgroup's LDS scratch, [5][waves].
__device__ __forceinline__ void energy_pass_end(const double (&esum)[5], double* partial, int b, int bpi, int lb,
                                                double (*red)[512 / 64]) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int q = 0; q < 5; ++q) {
    const double w = wave_sum(esum[q]);
    if (lane == 0) red[q][wave] = w;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    double v = 0;
    for (int j = 0; j < (int)(blockDim.x >> 6); ++j) v += red[threadIdx.x][j];
    gst(partial + ((size_t)b * bpi + lb) * 5 + threadIdx.x, v);
  }
}



// CPT > 0: every thread owns at most CPT cells (the host checks TY nx <= CPT
// threads) and the cell loop is unrolled; CPT == 1 also loads the cell's
// epilogue inputs (m and neighbours, the step's m and slopes) before the
// transform, so their latency overlaps it.  CPT == 0: any number of cells.
// FUSE (MODE_STAGE, DEMAG, CPT > 0): the next stage input just formed for
// these rows is transformed forward along x here, into the same Sx rows this
// workgroup read (no other workgroup touches them), which takes the forward x
// pass of the next evaluation off the critical path.
// CELLS: the general-material form (cell-based material, interlayer
// coupling, spin torques; local_field_cells): every cell's terms carry its own
// Ms, A_ij, D_ij, an empty cell gets no demag field either, energies weight
// each cell by its Ms, and with cell arrays the fused forward transform takes
// Ms m.
template <typename T, bool DEMAG, int MODE, int CPT, bool FUSE, bool CELLS>
__global__ void __launch_bounds__(512) k_inv_x(Launch<T> L) {
  constexpr bool PREF = CPT == 1;
  static_assert(!FUSE || (MODE == MODE_STAGE && DEMAG && CPT > 0), "fused forward pass needs a stage epilogue");
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  __shared__ double red[5][512 / 64];
  constexpr bool energy = MODE == MODE_ENERGY || MODE == MODE_FIELD_ENERGY;
  long long bid0;
  const int gi = group_of(L, bid0);
  const HotPlan<T> hp = hot_plan(L, gi);
  const Geo& g = hp.g;
  if (bid0 >= inv_blocks(g, hp.tu, hp.batch)) return;
  const int TY = hp.tu.ty_x;  // a power of two
  const int lty = __builtin_ctz((unsigned)TY);
  const int tiles = (g.ny + TY - 1) >> lty;
  unsigned bid = (unsigned)bid0;
  // z varies fastest: the workgroups of planes z - 1, z, z + 1 of a tile (which
  // read each other's m as the z halo) are neighbours in the XCD-ordered grid
  const int z = (int)(bid % (unsigned)g.nz); bid /= (unsigned)g.nz;
  const int tile = (int)(bid % (unsigned)tiles);
  const int b = (int)(bid / (unsigned)tiles);
  const int y0 = tile * TY;
  const int nrow = g.ny - y0 < TY ? g.ny - y0 : TY;
  const int cs = col_stride(g.Lx);
  const int sh = hp.fd[0].psh;

  // Spectrum tile: column c * TY + r holds component c of row y0 + r (rows past
  // the mesh are left out: only the epilogue's rows are read back).
  // 3-D groups: Sx [3][nz][XB][ny][kSxB], the tile of a component is XB runs
  // of kSxB TY entries; 2-D groups: Sx [3][Xp][ny], TY entries of each kx
  // column.  Its first batch of loads is issued before anything else waits
  // (the controller flag, the epilogue's arguments and prefetch).
  const int ncol = 3 * TY;
  const bool blk = g.nz > 1;
  const size_t plane = blk ? (size_t)g.XB * kSxB * g.ny : (size_t)g.Xp * g.ny;
  const size_t cstride = (size_t)g.nz * plane;
  const Cx<T>* src0 = hp.Sx + (size_t)b * g.sx + (size_t)z * plane + (blk ? kSxB * y0 : y0);
  const int lq = lty + 2;  // kSxB = 4
  const int tot = DEMAG ? (blk ? g.XB << lq : g.Xp << lty) : 0;
  // entry t of a component's tile: row r, kx k; returns its offset from src0
  auto tile_ent = [&](int t, int& r, int& k) -> uint32_t {
    if (blk) {
      const int kb = t >> lq, q = t & ((1 << lq) - 1);
      r = q >> 2;
      k = kb * kSxB + (q & 3);
      return (uint32_t)(kb * kSxB * g.ny + q);
    }
    r = t & (TY - 1);
    k = t >> lty;
    return (uint32_t)(k * g.ny + r);
  };
  constexpr int U = 4;
  auto load_batch = [&](int t0, Cx<T> (&v)[U][3]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * blockDim.x;
      int r, k;
      const uint32_t off = tile_ent(t, r, k) * (uint32_t)sizeof(Cx<T>);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        v[u][c] = {T(0), T(0)};
        if (t < tot && r < nrow && k < g.Xp) v[u][c] = gldo(src0 + c * cstride, off);
      }
    }
  };
  auto store_batch = [&](int t0, const Cx<T> (&v)[U][3]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = t0 + u * blockDim.x;
      int r, k;
      (void)tile_ent(t, r, k);
      if (t < tot && k < g.Xp) {
#pragma unroll
        for (int c = 0; c < 3; ++c) lds[(c * TY + r) * cs + pidx(k, sh)] = v[u][c];
      }
    }
  };
  Cx<T> v0[U][3];
  if constexpr (DEMAG) load_batch((int)threadIdx.x, v0);

  DevCtl* const ctl = ldu(&L.epis[gi].ctl);
  if (ctl && ldu(&ctl[b].done)) return;
  const bool add_hd = DEMAG && (ldu(&hp.prm[b].terms) & MM_DEMAG);
  const int ncell = nrow * g.nx;
  const long long N = g.N;
  const FDiv dnx = fdiv_of(g.nx);

  // prefetch of the single cell's epilogue inputs (PREF)
  Nbr<T> pnb;
  CellNbr<T> pcn;
  V3<T> pbase = {T(0), T(0), T(0)};
  V3<T> pk[6];
  if constexpr (PREF) {
    const Epi<T>* ep = L.epis + gi;
    const int e = threadIdx.x;
    const int ec = e < ncell ? e : 0;  // idle lanes read the first cell and drop it
    const int rc = fdiv_q(ec, dnx), xc = ec - mul24(rc, g.nx);
    const size_t ib = (size_t)b * ldu(&ep->inst_stride);
    const COff co = coff_of<T>(N, (z * g.ny + y0 + rc) * g.nx + xc);
    pnb = load_nbr<T>(g, ldu(&hp.prm[b].terms), ldu(&ep->in) + ib, co, xc, y0 + rc, z);
    if constexpr (CELLS)
      pcn = load_cells<T>(g, cell_ctx<T>(hp.prm + b), hp.cells + (size_t)b * 3 * N, ldu(&ep->in) + ib, co, xc,
                          y0 + rc, z);
    if constexpr (MODE == MODE_STAGE) pbase = ld3o(ldu(&ep->mbase) + ib, co);
    if constexpr (MODE == MODE_STAGE || MODE == MODE_ERROR) {
      const int nk = ldu(&ep->nk);
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        pk[j] = {T(0), T(0), T(0)};
        if (j + 1 < nk && ldu(&ep->coef[j]) != 0.0) pk[j] = ld3o(ldu(&ep->kprev[j]) + ib, co);
      }
    }
  }

  // LDS: 3 TY columns, then the twiddle table (Lx) and the post factors (Lx + 1)
  Cx<T>* const twl = lds + 3 * TY * cs;
  Cx<T>* const postl = twl + g.Lx;
  if (DEMAG) {
    TableCopy<T, 4> tab;
    tab.issue(hp.fd[0].tw, g.Lx, hp.post, g.Lx + 1);
    store_batch((int)threadIdx.x, v0);
    for (int t0 = threadIdx.x + U * blockDim.x; t0 < tot; t0 += U * blockDim.x) {
      Cx<T> v[U][3];
      load_batch(t0, v);
      store_batch(t0, v);
    }
    tab.store(twl);
    __syncthreads();
    // Z2[k] = (X[k] + conj X[Lx-k]) + i (X[k] - conj X[Lx-k]) conj(W^k), k in [0, Lx)
    const int half = g.Lx / 2;
    const FDiv dh = fdiv_of(half + 1);
    for (int t = threadIdx.x; t < ncol * (half + 1); t += blockDim.x) {
      const int col = fdiv_q(t, dh), k = t - mul24(col, half + 1);
      Cx<T>* cp = lds + col * cs;
      const int k2 = g.Lx - k;
      const Cx<T> Xa = cp[pidx(k, sh)], Xb = cp[pidx(k2, sh)];
      {
        const Cx<T> s = cadd(Xa, cconj(Xb));
        const Cx<T> d = cmul(csub(Xa, cconj(Xb)), cconj(postl[k]));
        cp[pidx(k, sh)] = Cx<T>{s.x - d.y, s.y + d.x};
      }
      if (k > 0 && k < k2) {
        const Cx<T> s = cadd(Xb, cconj(Xa));
        const Cx<T> d = cmul(csub(Xb, cconj(Xa)), cconj(postl[k2]));
        cp[pidx(k2, sh)] = Cx<T>{s.x - d.y, s.y + d.x};
      }
    }
    __syncthreads();
    // the epilogue reads complex entries below ceil(nx / 2) <= Lx / 2 only
    x_columns<T, true>(lds, hp.fd[0], cs, ncol, twl, false);
  }

  // ----- epilogue ----- (its arguments are read only now, which keeps the
  // scalar registers free during the transform)
  const Epi<T> epi = ldu(L.epis + gi);
  const DevParams Pd = ldu(hp.prm + b);
  const LocalCoef<T> P = local_coef<T>(Pd);
  GenCoef<T> Q;
  CellCtx<T> ccx;
  if constexpr (CELLS) {
    Q = gen_coef<T>(Pd);
    ccx = cell_ctx<T>(hp.prm + b);
  }
  const T g1 = T(Pd.g1), g2 = T(Pd.g2);
  const T* mb = epi.in + (size_t)b * epi.inst_stride;
  double esum[5] = {0, 0, 0, 0, 0};
  double emax = 0.0;
  double kmax = 0.0;  // MODE_ERROR: largest |k_7|^2 (relaxations)
  // h * coefficients; hlast multiplies the k of this stage (entry nk - 1).
  // Loops over the 7 slots are unrolled so that every index is a constant.
  T hcoef[7] = {0, 0, 0, 0, 0, 0, 0};
  T hlast = T(0);
  if constexpr (MODE == MODE_STAGE || MODE == MODE_ERROR) {
    const double h = ldu(&ctl[b].h_att);
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      hcoef[j] = j + 1 < epi.nk ? T(h * epi.coef[j]) : T(0);
      if (j + 1 == epi.nk) hlast = T(h * epi.coef[j]);
    }
  }
  V3<T> mnext[CPT > 0 ? CPT : 1];
  // CPT > 1: the cells' results are stored after all of them are computed, so
  // that no store sits between one cell's loads and the next (the compiler
  // may then issue the loads of every cell of the thread together)
  constexpr bool DEFER = CPT > 1;
  constexpr int NS = DEFER ? CPT : 1;
  V3<T> res1[NS], res2[NS];
  COff cos[NS];
  auto cell = [&](int e, int slot) {
    const int r = fdiv_q(e, dnx), x = e - mul24(r, g.nx);
    const int y = y0 + r;
    const COff co = coff_of<T>(N, (z * g.ny + y) * g.nx + x);
    const Nbr<T> nb = PREF ? pnb : load_nbr<T>(g, P.terms, mb, co, x, y, z);
    CellNbr<T> cn;
    if constexpr (CELLS) cn = PREF ? pcn : load_cells<T>(g, ccx, hp.cells + (size_t)b * 3 * N, mb, co, x, y, z);
    const size_t ib = (size_t)b * epi.inst_stride;
    // the stage's earlier slopes (and m for the stage input), all issued
    // before any of them is used: one memory round trip per cell, not one per
    // slope
    V3<T> kb[6];
    V3<T> mbv = {T(0), T(0), T(0)};
    if constexpr (MODE == MODE_STAGE || MODE == MODE_ERROR) {
      if constexpr (PREF) {
        mbv = pbase;
#pragma unroll
        for (int j = 0; j < 6; ++j) kb[j] = pk[j];
      } else {
        if constexpr (MODE == MODE_STAGE) mbv = ld3o(epi.mbase + ib, co);
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          if (hcoef[j] != T(0)) kb[j] = ld3o(epi.kprev[j] + ib, co);
          else kb[j] = {T(0), T(0), T(0)};
        }
      }
    }
    const V3<T> mi = nb.mi;
    LocalTerms lt = {0, 0, 0, 0};
    V3<T> H;
    if constexpr (CELLS) {
      if constexpr (energy) H = local_field_cells<T, true>(P, Q, nb, cn, &lt);
      else H = local_field_cells<T, false>(P, Q, nb, cn, nullptr);
    } else {
      if constexpr (energy) H = local_field<T, true>(g, P, nb, x, y, z, &lt);
      else H = local_field<T, false>(g, P, nb, x, y, z, nullptr);
    }
    V3<T> hd = {T(0), T(0), T(0)};
    bool cell_hd = add_hd;
    if constexpr (CELLS) cell_hd = add_hd && cn.ms > T(0);
    if (cell_hd) {
      const int kk = pidx(x >> 1, sh);
      const Cx<T> a = lds[(0 * TY + r) * cs + kk], bq = lds[(1 * TY + r) * cs + kk];
      const Cx<T> cq = lds[(2 * TY + r) * cs + kk];
      hd = (x & 1) ? V3<T>{a.y, bq.y, cq.y} : V3<T>{a.x, bq.x, cq.x};
      H.x += hd.x; H.y += hd.y; H.z += hd.z;
    }
    if constexpr (DEFER) cos[slot] = co;
    if constexpr (MODE == MODE_FIELD || MODE == MODE_FIELD_ENERGY) {
      if constexpr (DEFER) res1[slot] = H;
      else st3o(epi.out + ib, co, H);
    }
    if constexpr (energy) {
      double wms = 1.0;  // cell-based material: each cell weighs with its own Ms
      if constexpr (CELLS) wms = (double)cn.ms;
      esum[0] += wms * lt.ex;
      if (cell_hd) esum[1] += wms * ((double)mi.x * hd.x + (double)mi.y * hd.y + (double)mi.z * hd.z);
      esum[2] += wms * lt.dmi;
      esum[3] += wms * lt.an;
      esum[4] += wms * lt.ze;
    }
    if constexpr (MODE == MODE_RHS || MODE == MODE_STAGE || MODE == MODE_ERROR) {
      const V3<T> kk = ll_rhs(mi, H, g1, g2);
      if constexpr (DEFER) res1[slot] = kk;
      else st3o(epi.out + ib, co, kk);
      if constexpr (MODE == MODE_STAGE) {
        // next stage input: m + h sum_j a_j k_j (k of this stage is the last term;
        // slots with a zero coefficient hold zeros)
        const V3<T> acc = rk_combine(mbv, kb, hcoef, hlast, kk, epi.project != 0);
        if constexpr (DEFER) res2[slot] = acc;
        else st3o(epi.msn + ib, co, acc);
        if constexpr (FUSE) {
          mnext[slot] = acc;
          if constexpr (CELLS)  // cell arrays: the transform takes M = Ms m
            if (P.terms & MM_CELLS) mnext[slot] = {acc.x * cn.ms, acc.y * cn.ms, acc.z * cn.ms};
        }
      } else if constexpr (MODE == MODE_ERROR) {
        rk_error(kb, hcoef, hlast, kk, emax, kmax);
      }
    }
    (void)slot;
  };
  if constexpr (CPT == 0) {
    for (int e = threadIdx.x; e < ncell; e += blockDim.x) cell(e, 0);
  } else {
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int e = threadIdx.x + k * blockDim.x;
      if (e < ncell) cell(e, k);
    }
    if constexpr (DEFER && MODE != MODE_ENERGY) {
      const size_t ib = (size_t)b * epi.inst_stride;
#pragma unroll
      for (int k = 0; k < CPT; ++k) {
        const int e = threadIdx.x + k * blockDim.x;
        if (e < ncell) {
          st3o(epi.out + ib, cos[k], res1[k]);
          if constexpr (MODE == MODE_STAGE) st3o(epi.msn + ib, cos[k], res2[k]);
        }
      }
    }
  }

  if constexpr (FUSE) {
    // forward x transform of the next stage input of these rows, into Sx
    const int ncol = 3 * TY;
    __syncthreads();  // every thread is done reading H_d from the columns
    // real view of column col: x -> 2 pidx(x >> 1) + (x & 1); zero from nx
    // to the end of the part the transform reads (Lx reals with a
    // half-length input end, else 2 Lx)
    T* const re = reinterpret_cast<T*>(lds);
    const int rcs = 2 * cs;
    const bool hin = (hp.fd[0].code & kFftFirstEven) && hp.fd[0].nst > 1;
    const int nz0 = (hin ? g.Lx : 2 * g.Lx) - g.nx;
    if (nz0 > 0) {
      const FDiv dz = fdiv_of(nz0);
      for (int t = threadIdx.x; t < ncol * nz0; t += blockDim.x) {
        const int col = fdiv_q(t, dz), x = g.nx + (t - mul24(col, nz0));
        re[col * rcs + 2 * pidx(x >> 1, sh) + (x & 1)] = T(0);
      }
    }
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int e = threadIdx.x + k * blockDim.x;
      if (e < ncell) {
        const int r = fdiv_q(e, dnx), x = e - mul24(r, g.nx);
        const int off = 2 * pidx(x >> 1, sh) + (x & 1);
        re[(0 * TY + r) * rcs + off] = mnext[k].x;
        re[(1 * TY + r) * rcs + off] = mnext[k].y;
        re[(2 * TY + r) * rcs + off] = mnext[k].z;
      }
    }
    __syncthreads();
    x_columns<T, false>(lds, hp.fd[0], cs, ncol, twl, hin);
    // real-to-complex post-processing and transposed store (the rows this
    // workgroup read at the start)
    // layouts as for the load at the start
    const bool blk = g.nz > 1;
    const size_t plane = blk ? (size_t)g.XB * kSxB * g.ny : (size_t)g.Xp * g.ny;
    const size_t cstride = (size_t)g.nz * plane;
    Cx<T>* dst0 = hp.Sx + (size_t)b * g.sx + (size_t)z * plane + (blk ? kSxB * y0 : y0);
    const int lq = lty + 2;
    const int tot = blk ? g.XB << lq : g.Xp << lty;
    for (int t = threadIdx.x; t < tot; t += blockDim.x) {
      int r, k;
      uint32_t o;
      if (blk) {
        const int kb = t >> lq, q = t & ((1 << lq) - 1);
        r = q >> 2;
        k = kb * kSxB + (q & 3);
        o = (uint32_t)(kb * kSxB * g.ny + q);
      } else {
        r = t & (TY - 1);
        k = t >> lty;
        o = (uint32_t)(k * g.ny + r);
      }
      if (r >= nrow || k >= g.Xp) continue;
      const uint32_t off = o * (uint32_t)sizeof(Cx<T>);
      const Cx<T> pk = postl[k];
      const int ka = pidx(k == g.Lx ? 0 : k, sh), kb = pidx(k == 0 ? 0 : g.Lx - k, sh);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const Cx<T>* cp = lds + (c * TY + r) * cs;
        const Cx<T> Zk = cp[ka];
        const Cx<T> Zc = cconj(cp[kb]);
        const Cx<T> E = cscale(cadd(Zk, Zc), T(0.5));
        const Cx<T> D = cscale(csub(Zk, Zc), T(0.5));
        const Cx<T> O = {D.y, -D.x};  // D / i
        gsto(dst0 + c * cstride, off, cadd(E, cmul(pk, O)));
      }
    }
  }
  if constexpr (MODE == MODE_ERROR) {
    error_pass_end(emax, kmax, ctl, b, tiles * g.nz, epi.replay, red);
  } else if constexpr (energy) {
    energy_pass_end(esum, epi.partial, b, tiles * g.nz, (int)(bid0 % (tiles * g.nz)), red);
  }
}

template <typename T, bool DEMAG, int CPT, bool CELLS>
void inv_x_launch_c(int mode, bool fuse, const Launch<T>& L, long long total, int nt, size_t lds, hipStream_t s) {
  const dim3 grid((unsigned)total);
  switch (mode) {
    case MODE_FIELD: k_inv_x<T, DEMAG, MODE_FIELD, CPT, false, CELLS><<<grid, nt, lds, s>>>(L); break;
    case MODE_RHS: k_inv_x<T, DEMAG, MODE_RHS, CPT, false, CELLS><<<grid, nt, lds, s>>>(L); break;
    case MODE_STAGE:
      if constexpr (DEMAG && CPT > 0) {
        if (fuse) {
          k_inv_x<T, DEMAG, MODE_STAGE, CPT, true, CELLS><<<grid, nt, lds, s>>>(L);
          break;
        }
      }
      k_inv_x<T, DEMAG, MODE_STAGE, CPT, false, CELLS><<<grid, nt, lds, s>>>(L);
      break;
    case MODE_ERROR: k_inv_x<T, DEMAG, MODE_ERROR, CPT, false, CELLS><<<grid, nt, lds, s>>>(L); break;
    case MODE_ENERGY: k_inv_x<T, DEMAG, MODE_ENERGY, CPT, false, CELLS><<<grid, nt, lds, s>>>(L); break;
    default: k_inv_x<T, DEMAG, MODE_FIELD_ENERGY, CPT, false, CELLS><<<grid, nt, lds, s>>>(L); break;
  }
}

// cpt: cells per thread of the unrolled epilogue (1, 2, 4, 8) or 0 (loop);
// CELLS: the launch's instances use cell-based material
template <typename T, bool DEMAG, bool CELLS>
void inv_x_launch(int mode, int cpt, bool fuse, const Launch<T>& L, long long total, int nt, size_t lds,
                  hipStream_t s) {
  switch (cpt) {
    case 1: inv_x_launch_c<T, DEMAG, 1, CELLS>(mode, fuse, L, total, nt, lds, s); break;
    case 2: inv_x_launch_c<T, DEMAG, 2, CELLS>(mode, fuse, L, total, nt, lds, s); break;
    case 4: inv_x_launch_c<T, DEMAG, 4, CELLS>(mode, fuse, L, total, nt, lds, s); break;
    case 8: inv_x_launch_c<T, DEMAG, 8, CELLS>(mode, fuse, L, total, nt, lds, s); break;
    default: inv_x_launch_c<T, DEMAG, 0, CELLS>(mode, false, L, total, nt, lds, s); break;
  }
}


}  // namespace mmx
