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
//   z pass   3-D: forward z (zero padded in LDS), tensor product, inverse z,
//            in place in Sy (only the nz physical planes are stored)
//   y inv    3-D: Sy -> Sx (only the ny physical rows)
//   x inv    complex-to-real along x for the 3 components of TY rows, then the
//            local fields, H_eff, LL and the integrator epilogue per cell.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "fft_core.hpp"
#include "kernels.hpp"

namespace mmx {

constexpr int kNT = 256;   // threads of the forward x pass and pointwise kernels
constexpr int kNTI = 512;  // threads of the fused x-inverse epilogue
constexpr int kCPT = 8;    // cells owned by one thread in the fused x-inverse epilogue
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

// ---------------------------------------------------------------------------
// x forward: real-to-complex of TY rows (fixed b, c, z), transposed store.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(512) k_fwd_x(HotPlan<T> hp, const T* __restrict__ m,
                                               const DevCtl* __restrict__ ctl) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  const Geo& g = hp.g;
  const int TY = hp.tu.ty_f;
  const int tiles = (g.ny + TY - 1) / TY;
  long long bid = xcd_tile(blockIdx.x, gridDim.x);
  const int tile = bid % tiles; bid /= tiles;
  const int z = bid % g.nz; bid /= g.nz;
  const int c = bid % 3;
  const int b = bid / 3;
  if (ctl && ctl[b].done) return;
  const int y0 = tile * TY;
  const int cs = col_stride(g.Lx);
  const T* src = m + ((size_t)b * 3 + c) * g.N + (size_t)z * g.ny * g.nx;
  // element n of row r packs x[2n] + i x[2n+1] (zero beyond nx and past the last row)
  auto ld = [&](int r, int n) -> Cx<T> {
    Cx<T> v = {T(0), T(0)};
    const int y = y0 + r;
    if (y < g.ny) {
      const T* row = src + (size_t)y * g.nx;
      const int i0 = 2 * n;
      if (i0 < g.nx) v.x = row[i0];
      if (i0 + 1 < g.nx) v.y = row[i0 + 1];
    }
    return v;
  };
  auto st = [](int, int, Cx<T>) {};
  fft_columns_io<T, false, true, false>(lds, hp.fp[0], cs, TY, hp.tu.tpc_f, ld, st);
  Cx<T>* dst = hp.Sx + (size_t)b * g.sx + ((size_t)c * g.nz + z) * g.Xp * g.ny;
  const int tot2 = TY * g.Xp;
  for (int t = threadIdx.x; t < tot2; t += blockDim.x) {
    const int k = t / TY, r = t - k * TY;
    const int y = y0 + r;
    if (y >= g.ny) continue;
    const Cx<T> Zk = lds[r * cs + pidx(k == g.Lx ? 0 : k)];
    const Cx<T> Zc = cconj(lds[r * cs + pidx(k == 0 ? 0 : g.Lx - k)]);
    const Cx<T> E = cscale(cadd(Zk, Zc), T(0.5));
    const Cx<T> D = cscale(csub(Zk, Zc), T(0.5));
    const Cx<T> O = {D.y, -D.x};  // D / i
    dst[(size_t)k * g.ny + y] = cadd(E, cmul(hp.post[k], O));
  }
}

// ---------------------------------------------------------------------------
// Tensor product at one spectral point: H_a = s * sum_b K_ab M_b (K real).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void tensor_apply(const HotPlan<T>& hp, int kx, int ky, int kz, T s,
                                             Cx<T>& m0, Cx<T>& m1, Cx<T>& m2) {
  const Geo& g = hp.g;
  const int kyf = ky <= g.Py - ky ? ky : g.Py - ky;
  const int kzf = kz <= g.Pz - kz ? kz : g.Pz - kz;
  const T sy = ky > g.Py - ky ? T(-1) : T(1);
  const T sz = kz > g.Pz - kz ? T(-1) : T(1);
  const size_t cstride = (size_t)g.Kz * g.Xp * g.Ky;
  const size_t off = ((size_t)kzf * g.Xp + kx) * g.Ky + kyf;
  const T kxx = hp.kt[off] * s;
  const T kyy = hp.kt[cstride + off] * s;
  const T kzz = hp.kt[2 * cstride + off] * s;
  const T kxy = hp.kt[3 * cstride + off] * (s * sy);
  T kxz = T(0), kyz = T(0);
  if (hp.ncomp == 6) {
    kxz = hp.kt[4 * cstride + off] * (s * sz);
    kyz = hp.kt[5 * cstride + off] * (s * sy * sz);
  }
  const Cx<T> a = m0, b = m1, c = m2;
  m0 = {kxx * a.x + kxy * b.x + kxz * c.x, kxx * a.y + kxy * b.y + kxz * c.y};
  m1 = {kxy * a.x + kyy * b.x + kyz * c.x, kxy * a.y + kyy * b.y + kyz * c.y};
  m2 = {kxz * a.x + kyz * b.x + kzz * c.x, kxz * a.y + kyz * b.y + kzz * c.y};
}

// ---------------------------------------------------------------------------
// 2-D (nz = 1): forward y, tensor product, inverse y for cb_y2 kx values and
// the 3 components, in place in Sx.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(512) k_y_fused2d(HotPlan<T> hp, const DevCtl* __restrict__ ctl) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  const Geo& g = hp.g;
  const int CB = hp.tu.cb_y2;
  const int tiles = (g.Xp + CB - 1) / CB;
  const int tile = blockIdx.x % tiles;
  const int b = blockIdx.x / tiles;
  if (ctl && ctl[b].done) return;
  const int kx0 = tile * CB;
  const int ncol = 3 * CB;
  const int cs = col_stride(g.Py);
  Cx<T>* base = hp.Sx + (size_t)b * g.sx;  // [3][1][Xp][ny]
  // column col = c*CB + j holds component c of kx = kx0 + j
  const int Xp = g.Xp, ny = g.ny;
  auto ld = [=](int col, int y) -> Cx<T> {
    const int c = col / CB, j = col - c * CB;
    const bool ok = y < ny && kx0 + j < Xp;
    return ok ? base[((size_t)c * Xp + kx0 + j) * ny + y] : Cx<T>{T(0), T(0)};
  };
  auto st = [=](int col, int y, Cx<T> v) {
    const int c = col / CB, j = col - c * CB;
    if (y < ny && kx0 + j < Xp) base[((size_t)c * Xp + kx0 + j) * ny + y] = v;
  };
  fft_columns_io<T, false, true, false>(lds, hp.fp[1], cs, ncol, hp.tu.tpc_y2, ld, st);
  const T s = T(hp.prm[b].demag_scale);
  for (int t = threadIdx.x; t < CB * g.Py; t += blockDim.x) {
    const int j = t / g.Py, ky = t - j * g.Py;
    const int kx = kx0 + j;
    if (kx >= g.Xp) continue;
    tensor_apply(hp, kx, ky, 0, s, lds[(0 * CB + j) * cs + pidx(ky)], lds[(1 * CB + j) * cs + pidx(ky)],
                 lds[(2 * CB + j) * cs + pidx(ky)]);
  }
  __syncthreads();
  fft_columns_io<T, true, false, true>(lds, hp.fp[1], cs, ncol, hp.tu.tpc_y2, ld, st);
}

// ---------------------------------------------------------------------------
// 3-D y passes: rows of fixed (b, c, z, kx).  INV = false: Sx(ny) -> Sy(Py);
// INV = true: Sy(Py) -> Sx(ny).
// ---------------------------------------------------------------------------
template <typename T, bool INV>
__global__ void __launch_bounds__(512) k_y3d(HotPlan<T> hp, const DevCtl* __restrict__ ctl) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  const Geo& g = hp.g;
  const int CB = hp.tu.cb_y;
  const long long rows_per_inst = 3LL * g.nz * g.Xp;
  const long long tiles = (rows_per_inst + CB - 1) / CB;
  const long long tile = blockIdx.x % tiles;
  const int b = blockIdx.x / tiles;
  if (ctl && ctl[b].done) return;
  const long long row0 = tile * CB;
  const int ncol = (int)((rows_per_inst - row0) < CB ? (rows_per_inst - row0) : CB);
  const int cs = col_stride(g.Py);
  const Cx<T>* src = (INV ? hp.Sy + (size_t)b * g.sy : hp.Sx + (size_t)b * g.sx) + (size_t)row0 * (INV ? g.Py : g.ny);
  Cx<T>* dst = (INV ? hp.Sx + (size_t)b * g.sx : hp.Sy + (size_t)b * g.sy) + (size_t)row0 * (INV ? g.ny : g.Py);
  const int nin = INV ? g.Py : g.ny;
  const int nout = INV ? g.ny : g.Py;
  auto ld = [&](int c, int e) -> Cx<T> {
    return e < nin ? src[(size_t)c * nin + e] : Cx<T>{T(0), T(0)};
  };
  auto st = [&](int c, int e, Cx<T> v) {
    if (e < nout) dst[(size_t)c * nout + e] = v;
  };
  fft_columns_io<T, INV, true, true>(lds, hp.fp[1], cs, ncol, hp.tu.tpc_y, ld, st);
}

// ---------------------------------------------------------------------------
// 3-D z pass: forward z, tensor product, inverse z for qz consecutive (kx,ky)
// points and the 3 components, in place in Sy (nz physical planes).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(512) k_z3d(HotPlan<T> hp, const DevCtl* __restrict__ ctl) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  const Geo& g = hp.g;
  const int QZ = hp.tu.qz;
  const long long nq = (long long)g.Xp * g.Py;
  const long long tiles = (nq + QZ - 1) / QZ;
  const long long tile = blockIdx.x % tiles;
  const int b = blockIdx.x / tiles;
  if (ctl && ctl[b].done) return;
  const long long q0 = tile * QZ;
  const int nqt = (int)((nq - q0) < QZ ? (nq - q0) : QZ);
  const int cs = col_stride(g.Pz);
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
      if (t < 3 * g.Pz * QZ && z < g.nz && j < nqt) v[u] = base[((size_t)c * g.nz + z) * plane + q0 + j];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int t = t0 + u * blockDim.x;
      if (t < 3 * g.Pz * QZ) {
        const int j = t % QZ;
        const int cz = t / QZ;
        const int c = cz / g.Pz, z = cz - c * g.Pz;
        lds[(c * QZ + j) * cs + pidx(z)] = v[u];
      }
    }
  }
  __syncthreads();
  fft_columns<T, false>(lds, hp.fp[2], cs, 3 * QZ, hp.tu.tpc_z);
  const T s = T(hp.prm[b].demag_scale);
  for (int t = threadIdx.x; t < QZ * g.Pz; t += blockDim.x) {
    const int j = t % QZ, kz = t / QZ;
    if (j >= nqt) continue;
    const long long q = q0 + j;
    const int kx = (int)(q / g.Py), ky = (int)(q - (long long)kx * g.Py);
    tensor_apply(hp, kx, ky, kz, s, lds[(0 * QZ + j) * cs + pidx(kz)],
                 lds[(1 * QZ + j) * cs + pidx(kz)], lds[(2 * QZ + j) * cs + pidx(kz)]);
  }
  __syncthreads();
  fft_columns<T, true>(lds, hp.fp[2], cs, 3 * QZ, hp.tu.tpc_z);
  for (int t = threadIdx.x; t < 3 * g.nz * QZ; t += blockDim.x) {
    const int j = t % QZ;
    const int cz = t / QZ;
    const int c = cz / g.nz, z = cz - c * g.nz;
    if (j < nqt) base[((size_t)c * g.nz + z) * plane + q0 + j] = lds[(c * QZ + j) * cs + pidx(z)];
  }
}

// ---------------------------------------------------------------------------
// 3-D z pass with the transform in registers: one thread owns the Pz-point
// columns of the 3 components at one (kx, ky); no LDS, no barriers.
// ---------------------------------------------------------------------------
template <typename T, int PZ>
__global__ void __launch_bounds__(256) k_z3d_reg(HotPlan<T> hp, const DevCtl* __restrict__ ctl) {
  const Geo& g = hp.g;
  const int b = blockIdx.y;
  if (ctl && ctl[b].done) return;
  const long long nq = (long long)g.Xp * g.Py;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  Cx<T>* base = hp.Sy + (size_t)b * g.sy + q;
  const size_t plane = (size_t)nq;
  Cx<T> v[3][PZ];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int z = 0; z < PZ; ++z) {
      v[c][z] = {T(0), T(0)};
      if (z < g.nz) v[c][z] = base[((size_t)c * g.nz + z) * plane];
    }
#pragma unroll
  for (int c = 0; c < 3; ++c) RegFft<T, PZ, 1, false>::run(v[c], hp.twz);
  const int kx = (int)(q / g.Py), ky = (int)(q - (long long)kx * g.Py);
  const int kyf = ky <= g.Py - ky ? ky : g.Py - ky;
  const T sy = ky > g.Py - ky ? T(-1) : T(1);
  const size_t cstride = (size_t)g.Kz * g.Xp * g.Ky;
  const T s = T(hp.prm[b].demag_scale);
#pragma unroll
  for (int kz = 0; kz < PZ; ++kz) {
    constexpr int half = PZ / 2;
    const int kzf = kz <= PZ - kz ? kz : PZ - kz;
    const T sz = kz > PZ - kz ? T(-1) : T(1);
    (void)half;
    const size_t off = ((size_t)kzf * g.Xp + kx) * g.Ky + kyf;
    const T kxx = hp.kt[off] * s;
    const T kyy = hp.kt[cstride + off] * s;
    const T kzz = hp.kt[2 * cstride + off] * s;
    const T kxy = hp.kt[3 * cstride + off] * (s * sy);
    const T kxz = hp.kt[4 * cstride + off] * (s * sz);
    const T kyz = hp.kt[5 * cstride + off] * (s * sy * sz);
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
      if (z < g.nz) base[((size_t)c * g.nz + z) * plane] = v[c][z];
}

template <typename T, int PZ>
static bool z_reg(const HotPlan<T>& hp, dim3 grid, const DevCtl* ctl, hipStream_t s) {
  if constexpr (sizeof(T) == 8 && PZ > 16) {
    return false;  // FP64 columns beyond 16 points do not fit in registers
  } else {
    k_z3d_reg<T, PZ><<<grid, 256, 0, s>>>(hp, ctl);
    return true;
  }
}

template <typename T>
static bool launch_z_reg(const HotPlan<T>& hp, int batch, const DevCtl* ctl, hipStream_t s) {
  const long long nq = (long long)hp.g.Xp * hp.g.Py;
  const dim3 grid((unsigned)((nq + 255) / 256), (unsigned)batch);
  switch (hp.g.Pz) {
    case 2: return z_reg<T, 2>(hp, grid, ctl, s);
    case 3: return z_reg<T, 3>(hp, grid, ctl, s);
    case 4: return z_reg<T, 4>(hp, grid, ctl, s);
    case 6: return z_reg<T, 6>(hp, grid, ctl, s);
    case 8: return z_reg<T, 8>(hp, grid, ctl, s);
    case 9: return z_reg<T, 9>(hp, grid, ctl, s);
    case 12: return z_reg<T, 12>(hp, grid, ctl, s);
    case 16: return z_reg<T, 16>(hp, grid, ctl, s);
    case 18: return z_reg<T, 18>(hp, grid, ctl, s);
    case 24: return z_reg<T, 24>(hp, grid, ctl, s);
    case 27: return z_reg<T, 27>(hp, grid, ctl, s);
    case 32: return z_reg<T, 32>(hp, grid, ctl, s);
    default: return false;
  }
}

// ---------------------------------------------------------------------------
// Local fields at one cell.  Returns the separate terms when ENERGY is set.
// ---------------------------------------------------------------------------
template <typename T> struct V3 { T x, y, z; };

template <typename T>
__device__ __forceinline__ V3<T> ld3(const T* __restrict__ p, long long N, long long i) {
  return {p[i], p[N + i], p[2 * N + i]};
}

struct LocalTerms {
  double ex, dmi, an, ze;  // m . H_term (FP64), for energies
};

template <typename T, bool ENERGY>
__device__ __forceinline__ V3<T> local_field(const Geo& g, const DevParams& P, const T* __restrict__ mb,
                                             int x, int y, int z, V3<T> mi, LocalTerms* lt) {
  const long long N = g.N;
  const long long i = ((long long)z * g.ny + y) * g.nx + x;
  V3<T> H = {T(0), T(0), T(0)};
  const bool need_nb = (P.terms & (MM_EXCHANGE | MM_DMI_INTERFACIAL)) != 0;
  V3<T> xm = {T(0), T(0), T(0)}, xp = xm, ym = xm, yp = xm, zm = xm, zp = xm;
  const bool hxm = x > 0, hxp = x + 1 < g.nx, hym = y > 0, hyp = y + 1 < g.ny;
  const bool hzm = z > 0, hzp = z + 1 < g.nz;
  if (need_nb) {
    if (hxm) xm = ld3(mb, N, i - 1);
    if (hxp) xp = ld3(mb, N, i + 1);
    if (hym) ym = ld3(mb, N, i - g.nx);
    if (hyp) yp = ld3(mb, N, i + g.nx);
    if (hzm) zm = ld3(mb, N, i - (long long)g.nx * g.ny);
    if (hzp) zp = ld3(mb, N, i + (long long)g.nx * g.ny);
  }
  if (P.terms & MM_EXCHANGE) {
    const T cx = T(P.cex[0]), cy = T(P.cex[1]), cz = T(P.cex[2]);
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
    const T cx = T(P.cdmi[0]), cy = T(P.cdmi[1]);
    const V3<T> dx = {xp.x - xm.x, xp.y - xm.y, xp.z - xm.z};
    const V3<T> dy = {ym.x - yp.x, ym.y - yp.y, ym.z - yp.z};
    V3<T> d = {-cx * dx.z, cy * dy.z, cx * dx.x - cy * dy.y};
    H.x += d.x; H.y += d.y; H.z += d.z;
    if (ENERGY) lt->dmi = (double)mi.x * d.x + (double)mi.y * d.y + (double)mi.z * d.z;
  }
  if (P.terms & MM_ANIS_UNIAXIAL) {
    const T ux = T(P.u[0]), uy = T(P.u[1]), uz = T(P.u[2]);
    const T s = T(P.can) * (mi.x * ux + mi.y * uy + mi.z * uz);
    H.x += s * ux; H.y += s * uy; H.z += s * uz;
    if (ENERGY) lt->an = (double)s * ((double)mi.x * ux + (double)mi.y * uy + (double)mi.z * uz);
  }
  if (P.terms & MM_ZEEMAN) {
    H.x += T(P.H[0]); H.y += T(P.H[1]); H.z += T(P.H[2]);
    if (ENERGY) lt->ze = (double)mi.x * P.H[0] + (double)mi.y * P.H[1] + (double)mi.z * P.H[2];
  }
  return H;
}

template <typename T>
__device__ __forceinline__ V3<T> ll_rhs(V3<T> m, V3<T> H, T g1, T g2) {
  const V3<T> a = {m.y * H.z - m.z * H.y, m.z * H.x - m.x * H.z, m.x * H.y - m.y * H.x};
  const V3<T> b = {m.y * a.z - m.z * a.y, m.z * a.x - m.x * a.z, m.x * a.y - m.y * a.x};
  return {g1 * a.x + g2 * b.x, g1 * a.y + g2 * b.y, g1 * a.z + g2 * b.z};
}

// ---------------------------------------------------------------------------
// x inverse (complex-to-real) + local fields + LL + epilogue.  One workgroup:
// TY rows of one z plane of one instance, 3 components.  DEMAG = false skips
// the transform (H_d = 0) and uses no LDS for it.
// ---------------------------------------------------------------------------
template <typename T, bool DEMAG>
__global__ void __launch_bounds__(kNTI) k_inv_x(HotPlan<T> hp, const T* __restrict__ ms, Epi<T> epi) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  __shared__ double red[5][kNTI / 64];
  const Geo& g = hp.g;
  const int TY = hp.tu.ty_x;
  const int tiles = (g.ny + TY - 1) / TY;
  const long long bid0 = xcd_tile(blockIdx.x, gridDim.x);
  long long bid = bid0;
  const int tile = bid % tiles; bid /= tiles;
  const int z = bid % g.nz;
  const int b = bid / g.nz;
  if (epi.ctl && epi.ctl[b].done) return;
  const int y0 = tile * TY;
  const int ncell = TY * g.nx;
  T Hd[3][kCPT];
#pragma unroll
  for (int k = 0; k < kCPT; ++k) Hd[0][k] = Hd[1][k] = Hd[2][k] = T(0);

  if (DEMAG) {
    const int cs = col_stride(g.Lx);
    for (int c = 0; c < 3; ++c) {
      const Cx<T>* src = hp.Sx + (size_t)b * g.sx + ((size_t)c * g.nz + z) * g.Xp * g.ny;
      for (int t0 = threadIdx.x; t0 < TY * g.Xp; t0 += kUnroll * blockDim.x) {
        Cx<T> v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int t = t0 + u * blockDim.x;
          const int k = t / TY, r = t - k * TY;
          const int y = y0 + r;
          v[u] = {T(0), T(0)};
          if (t < TY * g.Xp && y < g.ny) v[u] = src[(size_t)k * g.ny + y];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          const int t = t0 + u * blockDim.x;
          if (t < TY * g.Xp) {
            const int k = t / TY, r = t - k * TY;
            lds[r * cs + pidx(k)] = v[u];
          }
        }
      }
      __syncthreads();
      // Z2[k] = (X[k] + conj X[Lx-k]) + i (X[k] - conj X[Lx-k]) conj(W^k), k in [0, Lx)
      const int half = g.Lx / 2;
      for (int t = threadIdx.x; t < TY * (half + 1); t += blockDim.x) {
        const int r = t / (half + 1), k = t - r * (half + 1);
        Cx<T>* col = lds + r * cs;
        const int k2 = g.Lx - k;
        const Cx<T> Xa = col[pidx(k)], Xb = col[pidx(k2)];
        // value at k
        {
          const Cx<T> s = cadd(Xa, cconj(Xb));
          const Cx<T> d = cmul(csub(Xa, cconj(Xb)), cconj(hp.post[k]));
          const Cx<T> v = {s.x - d.y, s.y + d.x};
          if (k < g.Lx) col[pidx(k)] = v;
        }
        // value at Lx - k (for 0 < k < Lx - k)
        if (k > 0 && k < k2) {
          const Cx<T> s = cadd(Xb, cconj(Xa));
          const Cx<T> d = cmul(csub(Xb, cconj(Xa)), cconj(hp.post[k2]));
          const Cx<T> v = {s.x - d.y, s.y + d.x};
          col[pidx(k2)] = v;
        }
      }
      __syncthreads();
      fft_columns<T, true>(lds, hp.fp[0], cs, TY, hp.tu.tpc_x);
#pragma unroll
      for (int k = 0; k < kCPT; ++k) {
        const int e = threadIdx.x + k * blockDim.x;
        if (e < ncell) {
          const int r = e / g.nx, x = e - r * g.nx;
          const Cx<T> v = lds[r * cs + pidx(x >> 1)];
          Hd[c][k] = (x & 1) ? v.y : v.x;
        }
      }
      __syncthreads();
    }
  }

  // ----- epilogue -----
  const DevParams P = hp.prm[b];
  const bool add_hd = DEMAG && (P.terms & MM_DEMAG);
  const T g1 = T(P.g1), g2 = T(P.g2);
  const long long N = g.N;
  const T* mb = ms + (size_t)b * epi.inst_stride;
  const bool energy = epi.mode == MODE_ENERGY || epi.mode == MODE_FIELD_ENERGY;
  double esum[5] = {0, 0, 0, 0, 0};
  double emax = 0.0;
  double hcoef[7];
  if (epi.mode == MODE_STAGE || epi.mode == MODE_ERROR) {
    const double h = epi.ctl[b].h_att;
    for (int j = 0; j < 7; ++j) hcoef[j] = h * epi.coef[j];
  }
#pragma unroll
  for (int k = 0; k < kCPT; ++k) {
    const int e = threadIdx.x + k * blockDim.x;
    if (e >= ncell) continue;
    const int r = e / g.nx, x = e - r * g.nx;
    const int y = y0 + r;
    if (y >= g.ny) continue;
    const long long i = ((long long)z * g.ny + y) * g.nx + x;
    const V3<T> mi = ld3(mb, N, i);
    LocalTerms lt = {0, 0, 0, 0};
    V3<T> H;
    if (energy) H = local_field<T, true>(g, P, mb, x, y, z, mi, &lt);
    else H = local_field<T, false>(g, P, mb, x, y, z, mi, nullptr);
    if (add_hd) {
      H.x += Hd[0][k]; H.y += Hd[1][k]; H.z += Hd[2][k];
    }
    const size_t o = (size_t)b * epi.inst_stride + i;
    if (epi.mode == MODE_FIELD || epi.mode == MODE_FIELD_ENERGY) {
      epi.out[o] = H.x; epi.out[o + N] = H.y; epi.out[o + 2 * N] = H.z;
    }
    if (energy) {
      esum[0] += lt.ex;
      if (add_hd) esum[1] += (double)mi.x * Hd[0][k] + (double)mi.y * Hd[1][k] + (double)mi.z * Hd[2][k];
      esum[2] += lt.dmi;
      esum[3] += lt.an;
      esum[4] += lt.ze;
      continue;
    }
    if (epi.mode == MODE_FIELD) continue;
    const V3<T> kk = ll_rhs(mi, H, g1, g2);
    epi.out[o] = kk.x; epi.out[o + N] = kk.y; epi.out[o + 2 * N] = kk.z;
    if (epi.mode == MODE_STAGE) {
      // next stage input: m + h sum_j a_j k_j (k of this stage is the last term)
      V3<T> acc = ld3(epi.mbase + (size_t)b * epi.inst_stride, N, i);
      for (int j = 0; j + 1 < epi.nk; ++j) {
        if (hcoef[j] == 0.0) continue;
        const V3<T> kj = ld3(epi.kprev[j] + (size_t)b * epi.inst_stride, N, i);
        const T cj = T(hcoef[j]);
        acc.x += cj * kj.x; acc.y += cj * kj.y; acc.z += cj * kj.z;
      }
      const T cl = T(hcoef[epi.nk - 1]);
      acc.x += cl * kk.x; acc.y += cl * kk.y; acc.z += cl * kk.z;
      epi.msn[o] = acc.x; epi.msn[o + N] = acc.y; epi.msn[o + 2 * N] = acc.z;
    } else if (epi.mode == MODE_ERROR) {
      double ex = 0, ey = 0, ez = 0;
      for (int j = 0; j + 1 < epi.nk; ++j) {
        if (hcoef[j] == 0.0) continue;
        const V3<T> kj = ld3(epi.kprev[j] + (size_t)b * epi.inst_stride, N, i);
        const T cj = T(hcoef[j]);
        ex += (double)(cj * kj.x); ey += (double)(cj * kj.y); ez += (double)(cj * kj.z);
      }
      const T cl = T(hcoef[epi.nk - 1]);
      ex += (double)(cl * kk.x); ey += (double)(cl * kk.y); ez += (double)(cl * kk.z);
      double en = sqrt(ex * ex + ey * ey + ez * ez);
      if (!(en <= DBL_MAX)) en = HUGE_VAL;  // NaN or Inf -> +Inf (kept by max)
      emax = fmax(emax, en);
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (epi.mode == MODE_ERROR) {
    const double w = wave_max(emax);
    if (lane == 0) red[0][wave] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
      double v = red[0][0];
      for (int j = 1; j < (int)(blockDim.x >> 6); ++j) v = fmax(v, red[0][j]);
      atomicMax(&epi.ctl[b].err_bits, (unsigned long long)__double_as_longlong(v));
    }
  } else if (energy) {
    for (int q = 0; q < 5; ++q) {
      const double w = wave_sum(esum[q]);
      if (lane == 0) red[q][wave] = w;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
      double v = 0;
      for (int j = 0; j < (int)(blockDim.x >> 6); ++j) v += red[threadIdx.x][j];
      const int bpi = tiles * g.nz;
      const int lb = (int)(bid0 % bpi);
      epi.partial[((size_t)b * bpi + lb) * 5 + threadIdx.x] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Step begin: finish the previous accepted attempt (project y5, FSAL copy),
// then form the stage-2 input m + h a21 k1.  One thread per cell.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kNT) k_begin(Geo g, T* __restrict__ m, T* __restrict__ ms0,
                                               const T* __restrict__ ms1, T* __restrict__ k1,
                                               const T* __restrict__ k7, double a21,
                                               const DevCtl* __restrict__ ctl) {
  const long long N = g.N;
  const long long blocks_per = (N + kNT - 1) / kNT;
  const int b = blockIdx.x / blocks_per;
  const long long i = (blockIdx.x % blocks_per) * kNT + threadIdx.x;
  if (i >= N) return;
  const DevCtl& C = ctl[b];
  const size_t o = (size_t)b * 3 * N + i;
  V3<T> mi;
  V3<T> kv;
  if (C.pending_finish) {
    const V3<T> y = {ms1[o], ms1[o + N], ms1[o + 2 * N]};
    const T s = rsqrt_t<T>(y.x * y.x + y.y * y.y + y.z * y.z);
    mi = {y.x * s, y.y * s, y.z * s};
    m[o] = mi.x; m[o + N] = mi.y; m[o + 2 * N] = mi.z;
    kv = {k7[o], k7[o + N], k7[o + 2 * N]};
    k1[o] = kv.x; k1[o + N] = kv.y; k1[o + 2 * N] = kv.z;
  } else {
    if (C.done) return;
    mi = {m[o], m[o + N], m[o + 2 * N]};
    kv = {k1[o], k1[o + N], k1[o + 2 * N]};
  }
  if (C.done) return;
  const T c = T(C.h_att * a21);
  ms0[o] = mi.x + c * kv.x;
  ms0[o + N] = mi.y + c * kv.y;
  ms0[o + 2 * N] = mi.z + c * kv.z;
}

// ---------------------------------------------------------------------------
// Device-side Dormand-Prince controller, one thread per instance (FP64).
// ---------------------------------------------------------------------------
__global__ void k_controller(DevCtl* ctl, int batch, const double* __restrict__ replay_h) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  DevCtl& C = ctl[b];
  if (C.done) {
    C.pending_finish = 0;
    C.err_bits = 0ull;
    return;
  }
  const double h = C.h_att;
  const double err = __longlong_as_double((long long)C.err_bits) / C.rtol;
  C.err_bits = 0ull;
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

// Fixed-order reduction of per-block partial sums: out[b][q] = sum_j partial[b][j][q].
__global__ void k_reduce_partials(const double* __restrict__ partial, int nb, int K,
                                  double* __restrict__ out) {
  const int b = blockIdx.x;
  for (int q = 0; q < K; ++q) {
    double v = 0;
    for (int j = threadIdx.x; j < nb; j += 64) v += partial[((size_t)b * nb + j) * K + q];
    v = wave_sum(v);
    if (threadIdx.x == 0) out[(size_t)b * K + q] = v;
  }
}

// ---------------------------------------------------------------------------
// NEB.  Pass 0 (images n = 0..n_img-2): partial sums of |m^{n+1}-m^n|^2 and,
// for inner images, of |t|^2 and H.t with the unnormalised projected tangent t.
// Pass 1 (inner images): G = H - (H.t)t + k (d+ - d-) t with normalised t,
// m' = normalize(m + h_g2 m x (m x G)) into img_out.
// ---------------------------------------------------------------------------
// Total image energy from the five per-term sums (quadratic terms carry -mu0 Ms V/2,
// Zeeman -mu0 Ms V).
__device__ __forceinline__ double neb_energy(const double* E5, int n, double cq, double cz) {
  const double* s = E5 + (size_t)n * 5;
  return cq * (s[0] + s[1] + s[2] + s[3]) + cz * s[4];
}

__device__ __forceinline__ void neb_weights(const double* E5, double cq, double cz, int n, double& wp,
                                            double& wm) {
  const double Ep = neb_energy(E5, n - 1, cq, cz), Ec = neb_energy(E5, n, cq, cz);
  const double En = neb_energy(E5, n + 1, cq, cz);
  if (En > Ec && Ec > Ep) { wp = 1; wm = 0; }
  else if (En < Ec && Ec < Ep) { wp = 0; wm = 1; }
  else {
    const double a = fabs(En - Ec), c = fabs(Ep - Ec);
    const double dmax = fmax(a, c), dmin = fmin(a, c);
    if (En > Ep) { wp = dmax; wm = dmin; } else { wp = dmin; wm = dmax; }
  }
}

template <typename T>
__global__ void __launch_bounds__(kNT) k_neb(Geo g, int n_img, const T* __restrict__ img,
                                             T* __restrict__ img_out, const T* __restrict__ H,
                                             const double* __restrict__ E5, double cq, double cz,
                                             const double* __restrict__ sums,
                                             double* __restrict__ partial, double k_spring,
                                             double h_g2, int pass) {
  __shared__ double red[3][kNT / 64];
  const long long N = g.N;
  const long long bpi = (N + kNT - 1) / kNT;
  const int n = (int)(blockIdx.x / bpi) + (pass == 0 ? 0 : 1);
  const long long i = (blockIdx.x % bpi) * kNT + threadIdx.x;
  const long long S = 3 * N;
  double s_d = 0, s_tt = 0, s_ht = 0;
  const bool inner = n >= 1 && n <= n_img - 2;
  double wp = 0, wm = 0;
  if (inner) neb_weights(E5, cq, cz, n, wp, wm);
  if (i < N) {
    const T* mc = img + (size_t)n * S;
    const V3<T> a = ld3(mc, N, i);
    const V3<T> nx = ld3(mc + S, N, i);
    const double dx = (double)nx.x - a.x, dy = (double)nx.y - a.y, dz = (double)nx.z - a.z;
    if (pass == 0) s_d = dx * dx + dy * dy + dz * dz;
    if (inner) {
      const V3<T> pv = ld3(mc - S, N, i);
      double tx = wp * dx + wm * ((double)a.x - pv.x);
      double ty = wp * dy + wm * ((double)a.y - pv.y);
      double tz = wp * dz + wm * ((double)a.z - pv.z);
      const double tm = tx * a.x + ty * a.y + tz * a.z;
      tx -= tm * a.x; ty -= tm * a.y; tz -= tm * a.z;
      const V3<T> h = ld3(H + (size_t)n * S, N, i);
      if (pass == 0) {
        s_tt = tx * tx + ty * ty + tz * tz;
        s_ht = h.x * tx + h.y * ty + h.z * tz;
      } else {
        const double tn = sqrt(sums[(size_t)n * 3 + 1]);
        const double ht = sums[(size_t)n * 3 + 2] / tn;
        const double dplus = sqrt(sums[(size_t)n * 3 + 0]);
        const double dminus = sqrt(sums[(size_t)(n - 1) * 3 + 0]);
        const double f = k_spring * (dplus - dminus) - ht;
        const T Gx = T(h.x + f * tx / tn), Gy = T(h.y + f * ty / tn), Gz = T(h.z + f * tz / tn);
        const V3<T> mxG = {a.y * Gz - a.z * Gy, a.z * Gx - a.x * Gz, a.x * Gy - a.y * Gx};
        const V3<T> mmG = {a.y * mxG.z - a.z * mxG.y, a.z * mxG.x - a.x * mxG.z,
                           a.x * mxG.y - a.y * mxG.x};
        const T c = T(h_g2);
        V3<T> y = {a.x + c * mmG.x, a.y + c * mmG.y, a.z + c * mmG.z};
        const T s = rsqrt_t<T>(y.x * y.x + y.y * y.y + y.z * y.z);
        T* o = img_out + (size_t)n * S;
        o[i] = y.x * s; o[N + i] = y.y * s; o[2 * N + i] = y.z * s;
      }
    }
  }
  if (pass == 0) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const double w0 = wave_sum(s_d), w1 = wave_sum(s_tt), w2 = wave_sum(s_ht);
    if (lane == 0) { red[0][wave] = w0; red[1][wave] = w1; red[2][wave] = w2; }
    __syncthreads();
    if (threadIdx.x < 3) {
      double v = 0;
      for (int j = 0; j < kNT / 64; ++j) v += red[threadIdx.x][j];
      partial[((size_t)n * bpi + (blockIdx.x % bpi)) * 3 + threadIdx.x] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static size_t lds_x(const Geo& g, const Tuning& tu, size_t csz) { return (size_t)tu.ty_x * col_stride(g.Lx) * csz; }

int eval_blocks_per_inst(const Geo& g, const Tuning& tu) {
  return ((g.ny + tu.ty_x - 1) / tu.ty_x) * g.nz;
}

template <typename T>
hipError_t launch_eval(const HotPlan<T>& hp, int batch, const T* m, const Epi<T>& epi, bool demag,
                       hipStream_t s, hipEvent_t* ev) {
  const Geo& g = hp.g;
  const Tuning& tu = hp.tu;
  const size_t csz = sizeof(Cx<T>);
  const int xtiles = (g.ny + tu.ty_x - 1) / tu.ty_x;
  int e = 0;
  auto mark = [&]() {
    if (ev) (void)hipEventRecord(ev[e++], s);
  };
  if (demag) {
    const int ftiles = (g.ny + tu.ty_f - 1) / tu.ty_f;
    const size_t ldsf = (size_t)tu.ty_f * col_stride(g.Lx) * csz;
    mark();
    k_fwd_x<T><<<dim3((unsigned)(batch * 3 * g.nz * ftiles)), tu.nt_f, ldsf, s>>>(hp, m, epi.ctl);
    if (g.nz == 1) {
      const int tiles = (g.Xp + tu.cb_y2 - 1) / tu.cb_y2;
      const size_t lds = (size_t)3 * tu.cb_y2 * col_stride(g.Py) * csz;
      mark();
      k_y_fused2d<T><<<dim3((unsigned)(batch * tiles)), 3 * tu.cb_y2 * tu.tpc_y2, lds, s>>>(hp, epi.ctl);
    } else {
      const long long rows = 3LL * g.nz * g.Xp;
      const long long ytiles = (rows + tu.cb_y - 1) / tu.cb_y;
      const size_t ldsy = (size_t)tu.cb_y * col_stride(g.Py) * csz;
      mark();
      k_y3d<T, false><<<dim3((unsigned)(batch * ytiles)), tu.cb_y * tu.tpc_y, ldsy, s>>>(hp, epi.ctl);
      const long long nq = (long long)g.Xp * g.Py;
      const long long ztiles = (nq + tu.qz - 1) / tu.qz;
      const size_t ldsz = (size_t)3 * tu.qz * col_stride(g.Pz) * csz;
      mark();
      if (!launch_z_reg<T>(hp, batch, epi.ctl, s))
        k_z3d<T><<<dim3((unsigned)(batch * ztiles)), 3 * tu.qz * tu.tpc_z, ldsz, s>>>(hp, epi.ctl);
      mark();
      k_y3d<T, true><<<dim3((unsigned)(batch * ytiles)), tu.cb_y * tu.tpc_y, ldsy, s>>>(hp, epi.ctl);
    }
    mark();
    k_inv_x<T, true><<<dim3((unsigned)(batch * g.nz * xtiles)), tu.nt_i, lds_x(g, tu, csz), s>>>(hp, m, epi);
  } else {
    mark();
    k_inv_x<T, false><<<dim3((unsigned)(batch * g.nz * xtiles)), tu.nt_i, 0, s>>>(hp, m, epi);
  }
  mark();
  return hipGetLastError();
}

template <typename T>
hipError_t launch_begin(const Geo& g, int batch, T* m, T* ms0, const T* ms1, T* k1, const T* k7,
                        double a21, DevCtl* ctl, hipStream_t s) {
  const long long bpi = (g.N + kNT - 1) / kNT;
  k_begin<T><<<dim3((unsigned)(batch * bpi)), kNT, 0, s>>>(g, m, ms0, ms1, k1, k7, a21, ctl);
  return hipGetLastError();
}

hipError_t launch_controller(DevCtl* ctl, int batch, const double* replay_h, hipStream_t s) {
  k_controller<<<dim3((batch + 63) / 64), 64, 0, s>>>(ctl, batch, replay_h);
  return hipGetLastError();
}

hipError_t launch_energy_reduce(const double* partial, int batch, int blocks_per_inst, double* out,
                                hipStream_t s) {
  k_reduce_partials<<<dim3(batch), 64, 0, s>>>(partial, blocks_per_inst, 5, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_neb(const Geo& g, int n_img, const T* img, T* img_out, const T* H,
                      const double* E5, double cq, double cz, double* sums, double* partial,
                      double k_spring, double h_g2, int pass, hipStream_t s) {
  const long long bpi = (g.N + kNT - 1) / kNT;
  const int nimg_launch = pass == 0 ? n_img - 1 : n_img - 2;
  k_neb<T><<<dim3((unsigned)(nimg_launch * bpi)), kNT, 0, s>>>(g, n_img, img, img_out, H, E5, cq, cz,
                                                                sums, partial, k_spring, h_g2, pass);
  if (pass == 0) k_reduce_partials<<<dim3(n_img - 1), 64, 0, s>>>(partial, (int)bpi, 3, sums);
  return hipGetLastError();
}

#define MMX_INST(T)                                                                                \
  template hipError_t launch_eval<T>(const HotPlan<T>&, int, const T*, const Epi<T>&, bool,        \
                                     hipStream_t, hipEvent_t*);                                    \
  template hipError_t launch_begin<T>(const Geo&, int, T*, T*, const T*, T*, const T*, double,     \
                                      DevCtl*, hipStream_t);                                       \
  template hipError_t launch_neb<T>(const Geo&, int, const T*, T*, const T*, const double*, double, \
                                    double, double*, double*, double, double, int, hipStream_t);
MMX_INST(float)
MMX_INST(double)

}  // namespace mmx
