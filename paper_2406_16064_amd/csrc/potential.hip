// Demag field through the magnetic scalar potential (the paper, section
// "Magnetostatic energy": with the scalar potential the three inverse Fourier
// transforms of the demag field become one).
//
// u(r) = sum_j M_j . S(r - r_j) at the cell corners (vertices), S the potential
// of a uniformly magnetised unit cuboid (setup.hip); H_d of a cell is
// -(1/(4 d_a)) times the sum over its four a-edges of u(+ end) - u(- end).  On
// P >= 2n points per axis the vertex - cell displacements ((i - 1/2) d, i in
// [-n+1, n]) fill the circular convolution exactly.
//
// Passes of one evaluation (3-D groups, nz >= 2; single group):
//   x, y forward   the Newell route's passes (M_a -> Sy[3][nz][Xp][Py])
//   z              forward z of the 3 components, u^ = -i Phi sum_a C_a M^_a
//                  (scaled by Ms / (Px Py Pz)), inverse z of u^ alone; the
//                  nz + 1 vertex planes go back to Sy, plane k at k Xp Py
//   y inverse      columns (k, kx) of u^: inverse y, the ny + 1 vertex rows to
//                  V = Sx as [nz+1][XB][ny+1][4] (kx in blocks of 4)
//   x inverse      2 (TY + 1) vertex rows (planes z, z + 1) of TY cell rows:
//                  complex-to-real along x (nx + 1 vertices), the edge
//                  differences, local fields, LL and the epilogue
#include <type_traits>

#include "hotpath.hpp"
#include "potential.hpp"

namespace mmx {

// Vertex rows of the potential after the inverse y pass, in the x-pass buffer:
// V[k][XB][ny + 1][kSxB] per instance (kx in blocks of kSxB, as the Newell
// route keeps its x spectrum), so that a y tile of whole blocks writes
// contiguous runs and an x workgroup reads kSxB (TY + 1) contiguous entries per
// block.
template <typename T>
__device__ __forceinline__ Cx<T>* vaddr(const HotPlan<T>& hp, int b, int k, int kx, int y) {
  const Geo& g = hp.g;
  return hp.Sx + (size_t)b * g.sx + (((size_t)k * g.XB + (kx >> 2)) * (g.ny + 1) + y) * kSxB + (kx & 3);
}

// ---------------------------------------------------------------------------
// z pass: QZ consecutive (kx, ky) points of one instance.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(512) k_pot_z(HotPlan<T> hp, PotTab<T> pt, int QZ, int tpc) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  const Geo& g = hp.g;
  const long long nq = (long long)g.Xp * g.Py;
  const long long tiles = (nq + QZ - 1) / QZ;
  const long long tile = (long long)blockIdx.x % tiles;
  const int b = (int)((long long)blockIdx.x / tiles);
  const long long q0 = tile * QZ;
  const int nqt = (int)((nq - q0) < QZ ? (nq - q0) : QZ);
  const int cs = col_stride(g.Pz);
  const int sh = hp.fd[2].psh;
  Cx<T>* base = hp.Sy + (size_t)b * g.sy;  // [3][nz][Xp Py] in, [nz + 1][Xp Py] out
  const size_t plane = (size_t)nq;
  for (int t = threadIdx.x; t < 3 * g.Pz * QZ; t += blockDim.x) {  // column c QZ + j, element z
    const int j = t % QZ;
    const int cz = t / QZ;
    const int c = cz / g.Pz, z = cz - c * g.Pz;
    Cx<T> v = {T(0), T(0)};
    if (z < g.nz && j < nqt) v = gld(base + ((size_t)c * g.nz + z) * plane + q0 + j);
    lds[(c * QZ + j) * cs + pidx(z, sh)] = v;
  }
  __syncthreads();
  fft_columns<T, false, false>(lds, hp.fd[2], cs, 3 * QZ, tpc, hp.fd[2].tw);
  __syncthreads();
  const T s = T(ldu(&hp.prm[b].demag_scale));  // Ms / (Px Py Pz)
  const size_t cstride = (size_t)g.Kz * g.Xp * g.Ky;
  for (int t = threadIdx.x; t < QZ * g.Pz; t += blockDim.x) {
    const int j = t % QZ, kz = t / QZ;
    if (j >= nqt) continue;
    const long long q = q0 + j;
    const int kx = (int)(q / g.Py), ky = (int)(q - (long long)kx * g.Py);
    const bool fy = ky > g.Py - ky, fz = kz > g.Pz - kz;  // folded indices: parities below
    const int kyf = fy ? g.Py - ky : ky, kzf = fz ? g.Pz - kz : kz;
    const size_t off = ((size_t)kzf * g.Xp + kx) * g.Ky + kyf;
    // parities of the folded kernel under ky -> Py - ky, kz -> Pz - kz (the
    // lattice is symmetric about the half-cell shift): C_x odd in both, C_y
    // odd in kz, C_z odd in ky
    const T cxv = gld(pt.kp + off) * ((fy != fz) ? T(-1) : T(1));
    const T cyv = gld(pt.kp + cstride + off) * (fz ? T(-1) : T(1));
    const T czv = gld(pt.kp + 2 * cstride + off) * (fy ? T(-1) : T(1));
    const int pk = pidx(kz, sh);
    const Cx<T> mx = lds[(0 * QZ + j) * cs + pk], my = lds[(1 * QZ + j) * cs + pk];
    const Cx<T> mz = lds[(2 * QZ + j) * cs + pk];
    const Cx<T> w = {cxv * mx.x + cyv * my.x + czv * mz.x, cxv * mx.y + cyv * my.y + czv * mz.y};
    // -i Phi w s, Phi = phx[kx] phy[ky] phz[kz]
    const Cx<T> ph = cmul(cmul(gld(pt.phx + kx), gld(pt.phy + ky)), gld(pt.phz + kz));
    const Cx<T> pw = cmul(ph, w);
    lds[(0 * QZ + j) * cs + pk] = Cx<T>{pw.y * s, -pw.x * s};
  }
  __syncthreads();
  fft_columns<T, true, false>(lds, hp.fd[2], cs, QZ, (int)blockDim.x / QZ, hp.fd[2].tw);
  __syncthreads();
  for (int t = threadIdx.x; t < (g.nz + 1) * QZ; t += blockDim.x) {
    const int j = t % QZ, z = t / QZ;
    if (j < nqt) gst(base + (size_t)z * plane + q0 + j, lds[j * cs + pidx(z, sh)]);
  }
}

// ---------------------------------------------------------------------------
// z pass with one (kx, ky) column per lane and the Pz-point transforms in
// registers (FP32, 3-smooth Pz up to 32): the 3 forward transforms, the
// product into the one scalar spectrum, its inverse transform.  HALF: nz =
// Pz / 2, the upper half of every input column a compile-time zero.
// ---------------------------------------------------------------------------
template <typename T, int PZ, bool HALF>
__global__ void __launch_bounds__(kNT, 2) k_pot_z_reg(HotPlan<T> hp, PotTab<T> pt) {
  const Geo& g = hp.g;
  const long long nq = (long long)g.Xp * g.Py;
  const long long qb = (nq + kNT - 1) / kNT;
  // the grid is padded to a multiple of 8: the workgroups of one kx row (whose
  // columns ky and Py - ky read the same folded kernel entries) share an XCD
  const long long bid = xcd_tile((long long)blockIdx.x, (long long)gridDim.x);
  if (bid >= (long long)hp.batch * qb) return;
  const int b = (int)(bid / qb);
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
  asm volatile("" : "+v"(base));  // stores recompute their addresses (fewer live registers)
#pragma unroll
  for (int c = 0; c < 3; ++c) RegFft<T, PZ, 1, false>::run(v[c], hp.twz);
  const int kx = (int)q / g.Py, ky = (int)q - kx * g.Py;
  const bool fy = ky > g.Py - ky;
  const int kyf = fy ? g.Py - ky : ky;
  const size_t cstride = (size_t)g.Kz * g.Xp * g.Ky;
  const T s = T(ldu(&hp.prm[b].demag_scale));
  const Cx<T> pxy = cmul(gld(pt.phx + kx), gld(pt.phy + ky));
#pragma unroll
  for (int kz = 0; kz < PZ; ++kz) {
    const bool fz = kz > PZ - kz;
    const int kzf = fz ? PZ - kz : kz;
    const size_t off = ((size_t)kzf * g.Xp + kx) * g.Ky + kyf;
    // parities of the folded kernel: C_x odd in ky and kz, C_y in kz, C_z in ky
    const T cxv = gld(pt.kp + off) * ((fy != fz) ? -s : s);
    const T cyv = gld(pt.kp + cstride + off) * (fz ? -s : s);
    const T czv = gld(pt.kp + 2 * cstride + off) * (fy ? -s : s);
    const Cx<T> a = v[0][kz], bb = v[1][kz], cc = v[2][kz];
    const Cx<T> w = {cxv * a.x + cyv * bb.x + czv * cc.x, cxv * a.y + cyv * bb.y + czv * cc.y};
    const Cx<T> pw = cmul(cmul(pxy, ldu(pt.phz + kz)), w);
    v[0][kz] = Cx<T>{pw.y, -pw.x};  // -i Phi w
  }
  RegFft<T, PZ, 1, true>::run(v[0], hp.twz);
#pragma unroll
  for (int z = 0; z < PZ; ++z)
    if (HALF ? z <= PZ / 2 : z <= g.nz) gst(base + (size_t)z * plane, v[0][z]);
}

// ---------------------------------------------------------------------------
// y inverse: CB consecutive kx of vertex plane k of one instance.
// ---------------------------------------------------------------------------
template <typename T, bool R16>
__global__ void __launch_bounds__(512) k_pot_yinv(HotPlan<T> hp, int CB, int tpc) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  const Geo& g = hp.g;
  const int tiles = (g.Xp + CB - 1) / CB;
  unsigned bid = blockIdx.x;
  const int tile = (int)(bid % (unsigned)tiles); bid /= (unsigned)tiles;
  const int k = (int)(bid % (unsigned)(g.nz + 1));
  const int b = (int)(bid / (unsigned)(g.nz + 1));
  const int kx0 = tile * CB;
  const int ncol = g.Xp - kx0 < CB ? g.Xp - kx0 : CB;
  const int cs = col_stride(g.Py);
  const int sh = hp.fd[1].psh;
  const Cx<T>* src = hp.Sy + (size_t)b * g.sy + ((size_t)k * g.Xp + kx0) * g.Py;  // ncol contiguous columns
  for (int t = threadIdx.x; t < ncol * g.Py; t += blockDim.x) {
    const int i = t / g.Py, y = t - i * g.Py;
    lds[i * cs + pidx(y, sh)] = gld(src + t);
  }
  __syncthreads();
  fft_columns<T, true, false, R16>(lds, hp.fd[1], cs, ncol, tpc, hp.fd[1].tw);
  __syncthreads();
  for (int t = threadIdx.x; t < (g.ny + 1) * ncol; t += blockDim.x) {
    const int y = t / ncol, i = t - y * ncol;
    gst(vaddr(hp, b, k, kx0 + i, y), lds[i * cs + pidx(y, sh)]);
  }
}

// y inverse with the transform compiled for Py = SL (a power of two, SL/EPT
// threads a column): columns read straight from global memory by the first
// stage and the vertex rows written by the last.
template <typename T>
struct VStore {  // column kx0 + c of the vertex plane starting at base (V[k]); rows 0..ny only
  Cx<T>* base;
  int ny, kx0;
  template <bool CHK>
  __device__ __forceinline__ void put(int c, int e, Cx<T> v) const {
    const int kx = kx0 + c;
    if (e <= ny) gst(base + ((size_t)(kx >> 2) * (ny + 1) + e) * kSxB + (kx & 3), v);
  }
};

template <typename T, int SL, int EPT>
__global__ void __launch_bounds__(512) k_pot_yinv_s(HotPlan<T> hp, int CB) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  const Geo& g = hp.g;
  const int tiles = (g.Xp + CB - 1) / CB;
  unsigned bid = blockIdx.x;
  const int tile = (int)(bid % (unsigned)tiles); bid /= (unsigned)tiles;
  const int k = (int)(bid % (unsigned)(g.nz + 1));
  const int b = (int)(bid / (unsigned)(g.nz + 1));
  const int kx0 = tile * CB;
  const int ncol = g.Xp - kx0 < CB ? g.Xp - kx0 : CB;
  constexpr int TPC = SL / EPT;
  const int c = (int)threadIdx.x / TPC;
  const int cc = c < ncol ? c : 0;
  const Cx<T>* src = hp.Sy + (size_t)b * g.sy + (size_t)k * g.Xp * g.Py;
  const ColLoad<T> ld{src, (uint32_t)((kx0 + cc) * g.Py) * (uint32_t)sizeof(Cx<T>), g.Py};
  const VStore<T> st{vaddr(hp, b, k, 0, 0), g.ny, kx0};
  fft_static<T, SL, (EPT > 8), true, true, true, false, false, false, EPT>(lds, hp.fd[1].tw, col_stride(SL), ncol,
                                                                          ld, st, NoHook{});
}

// ---------------------------------------------------------------------------
// x inverse + edge differences + local fields + epilogue: TY cell rows of
// plane z of one instance (MODE_FIELD, MODE_RHS, MODE_ENERGY, and the
// Runge-Kutta MODE_STAGE / MODE_ERROR of the integrators).  The TY + 1
// vertex rows of vertex planes z and z + 1 are loaded (kSxB (TY + 1)
// contiguous entries per kx block), transformed together, and each cell reads
// its eight corners from LDS.
// ---------------------------------------------------------------------------
template <typename T, int MODE, int CPT>
__global__ void __launch_bounds__(512) k_pot_x(HotPlan<T> hp, const Epi<T>* __restrict__ epis, int tpc, T gx, T gy,
                                              T gz) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<T>* lds = reinterpret_cast<Cx<T>*>(smem);
  __shared__ double red[5][512 / 64];
  const Geo& g = hp.g;
  const int TY = hp.tu.ty_x;
  const int tiles = (g.ny + TY - 1) / TY;
  const long long nblk = (long long)hp.batch * g.nz * tiles;
  // the grid is padded to a multiple of 8; consecutive tiles (neighbouring z
  // planes, which share a vertex plane) run on the same XCD
  const long long bidx = xcd_tile((long long)blockIdx.x, (long long)gridDim.x);
  if (bidx >= nblk) return;
  unsigned bid = (unsigned)bidx;
  const int z = (int)(bid % (unsigned)g.nz); bid /= (unsigned)g.nz;
  const int tile = (int)(bid % (unsigned)tiles);
  const int b = (int)(bid / (unsigned)tiles);
  constexpr bool RK = MODE == MODE_STAGE || MODE == MODE_ERROR;
  DevCtl* const ctl = ldu(&epis->ctl);
  if constexpr (RK) {
    if (ctl && ldu(&ctl[b].done)) return;  // the whole workgroup: b is uniform
  }
  const int y0 = tile * TY;
  const int nrow = g.ny - y0 < TY ? g.ny - y0 : TY;
  const int cs = col_stride(g.Lx);
  const int sh = hp.fd[0].psh;
  const int R1 = TY + 1;      // vertex rows per plane
  const int ncol = 2 * R1;    // column p R1 + r: vertex row y0 + r of vertex plane z + p
  Cx<T>* const twl = lds + ncol * cs;
  Cx<T>* const postl = twl + g.Lx;
  const bool add_hd = (ldu(&hp.prm[b].terms) & MM_DEMAG_POTENTIAL) != 0;
  if (add_hd) {
    TableCopy<T, 4> tab;
    tab.issue(hp.fd[0].tw, g.Lx, hp.post, g.Lx + 1);
    // per vertex plane and kx block: the kSxB (nrow + 1) entries of rows y0 ..
    // y0 + nrow, contiguous; U loads a thread in flight before their LDS stores
    const int per = kSxB * R1;
    const int tot = 2 * g.XB * per;
    constexpr int U = 4;
    for (int t0 = threadIdx.x; t0 < tot; t0 += U * blockDim.x) {
      Cx<T> v[U];
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const int t = t0 + j * blockDim.x;
        const int pb = t / per, q = t - pb * per;
        const int p = pb / g.XB, kb = pb - p * g.XB;
        const int r = q >> 2, k = kb * kSxB + (q & 3);
        v[j] = {T(0), T(0)};
        if (t < tot && r <= nrow && k < g.Xp) v[j] = gld(vaddr(hp, b, z + p, k, y0 + r));
      }
#pragma unroll
      for (int j = 0; j < U; ++j) {
        const int t = t0 + j * blockDim.x;
        const int pb = t / per, q = t - pb * per;
        const int p = pb / g.XB, kb = pb - p * g.XB;
        const int r = q >> 2, k = kb * kSxB + (q & 3);
        if (t < tot && r <= nrow && k < g.Xp) lds[(p * R1 + r) * cs + pidx(k, sh)] = v[j];
      }
    }
    tab.store(twl);
    __syncthreads();
    // complex-to-real through the half-length transform:
    // Z[k] = (X[k] + conj X[Lx-k]) + i (X[k] - conj X[Lx-k]) conj(W^k), k in [0, Lx)
    const int half = g.Lx / 2;
    for (int t = threadIdx.x; t < ncol * (half + 1); t += blockDim.x) {
      const int col = t / (half + 1), k = t - col * (half + 1);
      Cx<T>* cp = lds + col * cs;
      const int k2 = g.Lx - k;
      const Cx<T> Xa = cp[pidx(k, sh)], Xb = cp[pidx(k2, sh)];
      {
        const Cx<T> s_ = cadd(Xa, cconj(Xb));
        const Cx<T> d_ = cmul(csub(Xa, cconj(Xb)), cconj(postl[k]));
        cp[pidx(k, sh)] = Cx<T>{s_.x - d_.y, s_.y + d_.x};
      }
      if (k > 0 && k < k2) {
        const Cx<T> s_ = cadd(Xb, cconj(Xa));
        const Cx<T> d_ = cmul(csub(Xb, cconj(Xa)), cconj(postl[k2]));
        cp[pidx(k2, sh)] = Cx<T>{s_.x - d_.y, s_.y + d_.x};
      }
    }
    __syncthreads();
    // the full inverse transform (vertex nx needs the entry Lx / 2); compiled
    // for the power-of-two lengths when the workgroup has Lx / 16 threads a column
    const bool st16 = (g.Lx == 128 || g.Lx == 256 || g.Lx == 512 || g.Lx == 1024) &&
                      ncol * (g.Lx / 16) <= (int)blockDim.x;
    if (st16) {
      switch (g.Lx) {
        case 128: fft_static<T, 128, false, true, false, false, true, false, false, 16>(lds, twl, cs, ncol, NoLoad<T>{}, NoStore<T>{}, NoHook{}); break;
        case 256: fft_static<T, 256, false, true, false, false, true, false, false, 16>(lds, twl, cs, ncol, NoLoad<T>{}, NoStore<T>{}, NoHook{}); break;
        case 512: fft_static<T, 512, false, true, false, false, true, false, false, 16>(lds, twl, cs, ncol, NoLoad<T>{}, NoStore<T>{}, NoHook{}); break;
        default: fft_static<T, 1024, false, true, false, false, true, false, false, 16>(lds, twl, cs, ncol, NoLoad<T>{}, NoStore<T>{}, NoHook{}); break;
      }
    } else {
      fft_columns<T, true, true>(lds, hp.fd[0], cs, ncol, tpc, twl);
    }
    __syncthreads();
  }
  // u at vertex (x, row r, plane p) of this tile: real x of column p R1 + r
  auto u = [&](int x, int r, int p) -> T {
    const Cx<T> c = lds[(p * R1 + r) * cs + pidx(x >> 1, sh)];
    return (x & 1) ? c.y : c.x;
  };
  const Epi<T> epi = ldu(epis);
  const DevParams Pd = ldu(hp.prm + b);
  const LocalCoef<T> P = local_coef<T>(Pd);
  const T g1 = T(Pd.g1), g2 = T(Pd.g2);
  const long long N = g.N;
  const size_t ib = (size_t)b * epi.inst_stride;
  const T* mb = epi.in + ib;
  double esum[5] = {0, 0, 0, 0, 0};
  const int ncell = nrow * g.nx;
  // Runge-Kutta epilogues: h times the coefficients of the combination (the
  // last entry multiplies the slope of this stage); the error pass keeps the
  // largest error norm and |k|^2 of its cells
  T hcoef[7] = {0, 0, 0, 0, 0, 0, 0};
  T hlast = T(0);
  double emax = 0.0, kmax = 0.0;
  if constexpr (RK) {
    const double h = ldu(&ctl[b].h_att);
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      hcoef[j] = j + 1 < epi.nk ? T(h * epi.coef[j]) : T(0);
      if (j + 1 == epi.nk) hlast = T(h * epi.coef[j]);
    }
  }
  // CPT > 0: at most CPT cells a thread, unrolled, their results stored after
  // the last of them (so the loads of every cell can be in flight together)
  constexpr int NS = CPT > 0 ? CPT : 1;
  V3<T> res[NS], res2[NS];
  COff cos[NS];
  auto cell = [&](int e, int slot) {
    const int r = e / g.nx, x = e - r * g.nx;
    const int y = y0 + r;
    const COff co = coff_of<T>(N, (z * g.ny + y) * g.nx + x);
    const Nbr<T> nb = load_nbr<T>(g, P.terms, mb, co, x, y, z);
    // the step's m and earlier slopes, issued with the neighbours
    V3<T> kb[6];
    V3<T> mbv = {T(0), T(0), T(0)};
    if constexpr (RK) {
      if constexpr (MODE == MODE_STAGE) mbv = ld3o(epi.mbase + ib, co);
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        if (hcoef[j] != T(0)) kb[j] = ld3o(epi.kprev[j] + ib, co);
        else kb[j] = {T(0), T(0), T(0)};
      }
    }
    LocalTerms lt = {0, 0, 0, 0};
    V3<T> H;
    if constexpr (MODE == MODE_ENERGY) H = local_field<T, true>(g, P, nb, x, y, z, &lt);
    else H = local_field<T, false>(g, P, nb, x, y, z, nullptr);
    V3<T> hd = {T(0), T(0), T(0)};
    if (add_hd) {
      const T a000 = u(x, r, 0), a100 = u(x + 1, r, 0), a010 = u(x, r + 1, 0), a110 = u(x + 1, r + 1, 0);
      const T a001 = u(x, r, 1), a101 = u(x + 1, r, 1), a011 = u(x, r + 1, 1), a111 = u(x + 1, r + 1, 1);
      hd.x = gx * ((a100 - a000) + (a110 - a010) + (a101 - a001) + (a111 - a011));
      hd.y = gy * ((a010 - a000) + (a110 - a100) + (a011 - a001) + (a111 - a101));
      hd.z = gz * ((a001 - a000) + (a101 - a100) + (a011 - a010) + (a111 - a110));
      H.x += hd.x; H.y += hd.y; H.z += hd.z;
    }
    const V3<T> mi = nb.mi;
    V3<T> o = H;
    if constexpr (MODE == MODE_RHS || RK) o = ll_rhs(mi, H, g1, g2);
    if constexpr (MODE == MODE_STAGE) {  // next stage input m + h sum_j a_j k_j (this stage's slope last)
      const V3<T> acc = rk_combine(mbv, kb, hcoef, hlast, o, epi.project != 0);
      if constexpr (CPT > 0) res2[slot] = acc;
      else st3o(epi.msn + ib, co, acc);
    }
    if constexpr (MODE == MODE_ERROR) rk_error(kb, hcoef, hlast, o, emax, kmax);
    if constexpr (MODE == MODE_ENERGY) {
      esum[0] += lt.ex;
      if (add_hd) esum[1] += (double)mi.x * hd.x + (double)mi.y * hd.y + (double)mi.z * hd.z;
      esum[2] += lt.dmi;
      esum[3] += lt.an;
      esum[4] += lt.ze;
    } else if constexpr (CPT > 0) {
      res[slot] = o;
      cos[slot] = co;
    } else {
      st3o(epi.out + ib, co, o);
    }
  };
  if constexpr (CPT == 0) {
    for (int e = threadIdx.x; e < ncell; e += blockDim.x) cell(e, 0);
  } else {
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int e = threadIdx.x + k * blockDim.x;
      if (e < ncell) cell(e, k);
    }
    if constexpr (MODE != MODE_ENERGY) {
#pragma unroll
      for (int k = 0; k < CPT; ++k)
        if ((int)threadIdx.x + k * (int)blockDim.x < ncell) {
          st3o(epi.out + ib, cos[k], res[k]);
          if constexpr (MODE == MODE_STAGE) st3o(epi.msn + ib, cos[k], res2[k]);
        }
    }
  }
  if constexpr (MODE == MODE_ERROR) error_pass_end(emax, kmax, ctl, b, tiles * g.nz, epi.replay, red);
  if constexpr (MODE == MODE_ENERGY) energy_pass_end(esum, epi.partial, b, tiles * g.nz, (int)(bidx % (tiles * g.nz)), red);
}

// ---------------------------------------------------------------------------
// Launch shapes and the pass sequence.
// ---------------------------------------------------------------------------
template <typename T>
PotShape pot_shape(const HotPlan<T>& h) {
  PotShape p{};
  const Geo& g = h.g;
  const size_t csz = sizeof(Cx<T>);
  p.tpc_z = h.tu.tpc_z;
  p.qz = h.tu.qz;
  // y inverse: columns of Py points, at most 80 KB of LDS
  p.tpc_y = h.tu.tpc_y;
  int cb = 16;
  while (cb > 1 && ((size_t)cb * col_stride(g.Py) * csz > 80 * 1024 || cb * p.tpc_y > 512)) cb /= 2;
  p.cb_y = cb;
  p.tpc_x = h.tu.tpc_x;
  const int ncol = 2 * (h.tu.ty_x + 1);
  const bool p2 = g.Lx == 128 || g.Lx == 256 || g.Lx == 512 || g.Lx == 1024;
  const int want = p2 && ncol * (g.Lx / 16) <= 512 ? std::max(p.tpc_x, g.Lx / 16) : p.tpc_x;
  p.nt_x = std::min(512, std::max(64, (ncol * want + 63) / 64 * 64));
  // epilogue cells per thread (1, 2, 4 or 8 unrolled; 0: a loop), with as many
  // threads as that takes, up to 512
  const int ncell = h.tu.ty_x * g.nx;
  p.cpt_x = 0;
  for (int c : {1, 2, 4, 8})
    if (p.cpt_x == 0 && (ncell + c - 1) / c <= 512) p.cpt_x = c;
  if (p.cpt_x > 0) p.nt_x = std::max(p.nt_x, std::min(512, ((ncell + p.cpt_x - 1) / p.cpt_x + 63) / 64 * 64));
  p.tpc_x = p.nt_x / ncol;
  // y inverse compiled for Py (2^k from 256 to 2048): SL/16 threads a column
  p.sl_y = (g.Py == 256 || g.Py == 512 || g.Py == 1024 || g.Py == 2048) ? g.Py : 0;
  if (p.sl_y) {
    p.cb_ys = std::max(1, 512 / (p.sl_y / 16));
    while (p.cb_ys > 1 && (size_t)p.cb_ys * col_stride(p.sl_y) * csz > 80 * 1024) p.cb_ys /= 2;
  }
  p.lds_x = ((size_t)ncol * col_stride(g.Lx) + 2 * g.Lx + 1) * csz;
  return p;
}

template <typename T>
bool pot_supported(const HotPlan<T>& h, int tpc_x_min) {
  const PotShape p = pot_shape(h);
  return h.g.nz >= 2 && p.tpc_x >= tpc_x_min && p.lds_x <= 160 * 1024;
}

// The register z pass where it applies (FP32, Pz a 3-smooth length up to 32);
// false: the caller launches the LDS version.
template <typename T>
bool pot_z_reg(const HotPlan<T>& h, const PotTab<T>& pt, hipStream_t s) {
  if constexpr (sizeof(T) != 4) {
    (void)h; (void)pt; (void)s;
    return false;
  } else {
    const Geo& g = h.g;
    const dim3 grid((unsigned)(((long long)h.batch * (((long long)g.Xp * g.Py + kNT - 1) / kNT) + 7) / 8 * 8));
    const bool half = 2 * g.nz == g.Pz;
#define MMX_PZ(PZ)                                                             \
  case PZ:                                                                     \
    if (half && PZ % 2 == 0) k_pot_z_reg<T, PZ, true><<<grid, kNT, 0, s>>>(h, pt); \
    else k_pot_z_reg<T, PZ, false><<<grid, kNT, 0, s>>>(h, pt);                \
    return true;
    switch (g.Pz) {
      MMX_PZ(4)
      MMX_PZ(6)
      MMX_PZ(8)
      MMX_PZ(12)
      MMX_PZ(16)
      MMX_PZ(18)
      MMX_PZ(24)
      MMX_PZ(32)
      default: return false;
    }
#undef MMX_PZ
  }
}

template <typename T>
hipError_t launch_potential(const GroupSet<T>& gs, const Epi<T>* epis, const PotTab<T>& pt, int mode,
                            hipStream_t s, unsigned pass_mask) {
  const HotPlan<T>& h = gs.h[0];
  const Geo& g = h.g;
  const size_t csz = sizeof(Cx<T>);
  const PotShape p = pot_shape(h);
  // x and y forward: the passes of the Newell route (pass bits 0 and 1)
  if (pass_mask & 3u) {
    const hipError_t er = launch_eval<T>(gs, epis, mode, true, s, nullptr, false, false, pass_mask & 3u);
    if (er != hipSuccess) return er;
  }
  if (pass_mask & 4u) {
    if (!pot_z_reg<T>(h, pt, s)) {
      const long long blocks = (long long)h.batch * (((long long)g.Xp * g.Py + p.qz - 1) / p.qz);
      const size_t lds = (size_t)3 * p.qz * col_stride(g.Pz) * csz;
      k_pot_z<T><<<dim3((unsigned)blocks), 3 * p.qz * p.tpc_z, lds, s>>>(h, pt, p.qz, p.tpc_z);
    }
  }
  if ((pass_mask & 8u) && p.sl_y) {
    const long long blocks = (long long)h.batch * (g.nz + 1) * ((g.Xp + p.cb_ys - 1) / p.cb_ys);
    const size_t lds = (size_t)p.cb_ys * col_stride(p.sl_y) * csz;
    const dim3 grid((unsigned)blocks), blk((unsigned)(p.cb_ys * (p.sl_y / 16)));
    switch (p.sl_y) {
      case 256: k_pot_yinv_s<T, 256, 16><<<grid, blk, lds, s>>>(h, p.cb_ys); break;
      case 512: k_pot_yinv_s<T, 512, 16><<<grid, blk, lds, s>>>(h, p.cb_ys); break;
      case 1024: k_pot_yinv_s<T, 1024, 16><<<grid, blk, lds, s>>>(h, p.cb_ys); break;
      default: k_pot_yinv_s<T, 2048, 16><<<grid, blk, lds, s>>>(h, p.cb_ys); break;
    }
  } else if (pass_mask & 8u) {
    bool r16 = false;
    for (int st = 0; st < h.fd[1].nst; ++st) r16 = r16 || radix_of(h.fd[1].code, st) == 16;
    const long long blocks = (long long)h.batch * (g.nz + 1) * ((g.Xp + p.cb_y - 1) / p.cb_y);
    const size_t lds = (size_t)p.cb_y * col_stride(g.Py) * csz;
    const int nt = std::max(64, (p.cb_y * p.tpc_y + 63) / 64 * 64);
    if (r16) k_pot_yinv<T, true><<<dim3((unsigned)blocks), nt, lds, s>>>(h, p.cb_y, p.tpc_y);
    else k_pot_yinv<T, false><<<dim3((unsigned)blocks), nt, lds, s>>>(h, p.cb_y, p.tpc_y);
  }
  if (pass_mask & 16u) {
    const long long blocks = ((long long)h.batch * g.nz * ((g.ny + h.tu.ty_x - 1) / h.tu.ty_x) + 7) / 8 * 8;
    const T cx = T(pt.gdx), cy = T(pt.gdy), cz = T(pt.gdz);
    const int cpt = p.cpt_x;
    const dim3 grid((unsigned)blocks);
    auto go = [&](auto mode_c) {
      constexpr int MD = decltype(mode_c)::value;
      switch (cpt) {
        case 1: k_pot_x<T, MD, 1><<<grid, p.nt_x, p.lds_x, s>>>(h, epis, p.tpc_x, cx, cy, cz); break;
        case 2: k_pot_x<T, MD, 2><<<grid, p.nt_x, p.lds_x, s>>>(h, epis, p.tpc_x, cx, cy, cz); break;
        case 4: k_pot_x<T, MD, 4><<<grid, p.nt_x, p.lds_x, s>>>(h, epis, p.tpc_x, cx, cy, cz); break;
        case 8: k_pot_x<T, MD, 8><<<grid, p.nt_x, p.lds_x, s>>>(h, epis, p.tpc_x, cx, cy, cz); break;
        default: k_pot_x<T, MD, 0><<<grid, p.nt_x, p.lds_x, s>>>(h, epis, p.tpc_x, cx, cy, cz); break;
      }
    };
    switch (mode) {
      case MODE_FIELD: go(std::integral_constant<int, MODE_FIELD>{}); break;
      case MODE_ENERGY: go(std::integral_constant<int, MODE_ENERGY>{}); break;
      case MODE_STAGE: go(std::integral_constant<int, MODE_STAGE>{}); break;
      case MODE_ERROR: go(std::integral_constant<int, MODE_ERROR>{}); break;
      default: go(std::integral_constant<int, MODE_RHS>{});
    }
  }
  return hipGetLastError();
}

#define MMX_POT_INST(T)                                                                                      \
  template PotShape pot_shape<T>(const HotPlan<T>&);                                                         \
  template bool pot_supported<T>(const HotPlan<T>&, int);                                                    \
  template hipError_t launch_potential<T>(const GroupSet<T>&, const Epi<T>*, const PotTab<T>&, int, hipStream_t, \
                                          unsigned);
MMX_POT_INST(float)
MMX_POT_INST(double)

}  // namespace mmx
