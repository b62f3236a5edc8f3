// Launchers and the remaining kernels of the hot path (the kernels and the
// inverse-x launcher are in hotpath.hpp; the inverse-x instantiations are
// compiled in invx_*.hip, one translation unit each).
#include "hotpath.hpp"

namespace mmx {

int eval_blocks_per_inst(const Geo& g, const Tuning& tu) { return ((g.ny + tu.ty_x - 1) / tu.ty_x) * g.nz; }

extern template void inv_x_launch<float, true, false>(int, int, bool, const Launch<float>&, long long, int, size_t,
                                                       hipStream_t);
extern template void inv_x_launch<float, true, true>(int, int, bool, const Launch<float>&, long long, int, size_t,
                                                       hipStream_t);
extern template void inv_x_launch<float, false, false>(int, int, bool, const Launch<float>&, long long, int, size_t,
                                                       hipStream_t);
extern template void inv_x_launch<float, false, true>(int, int, bool, const Launch<float>&, long long, int, size_t,
                                                       hipStream_t);
extern template void inv_x_launch<double, true, false>(int, int, bool, const Launch<double>&, long long, int, size_t,
                                                       hipStream_t);
extern template void inv_x_launch<double, true, true>(int, int, bool, const Launch<double>&, long long, int, size_t,
                                                       hipStream_t);
extern template void inv_x_launch<double, false, false>(int, int, bool, const Launch<double>&, long long, int, size_t,
                                                       hipStream_t);
extern template void inv_x_launch<double, false, true>(int, int, bool, const Launch<double>&, long long, int, size_t,
                                                       hipStream_t);

// ---------------------------------------------------------------------------
// Step begin: finish the previous accepted attempt (project y5, FSAL copy),
// then form the stage-2 input m + h a21 k1.  One thread per cell.
// ---------------------------------------------------------------------------
__host__ __device__ inline long long begin_blocks(const Geo& g, int batch) {
  return (long long)batch * ((g.N + kNT - 1) / kNT);
}

template <typename T>
__global__ void __launch_bounds__(kNT) k_begin(Launch<T> L) {
  long long bid;
  const int gi = group_of(L, bid);
  const HotPlan<T> hp = hot_plan(L, gi);
  const Epi<T> ep = ldu(L.epis + gi);
  const Geo& g = hp.g;
  if (bid >= begin_blocks(g, hp.batch)) return;
  const long long N = g.N;
  const long long blocks_per = (N + kNT - 1) / kNT;
  const int b = (int)(bid / blocks_per);
  const long long i = (bid % blocks_per) * kNT + threadIdx.x;
  if (i >= N) return;
  const DevCtl C = ldu(ep.ctl + b);
  const size_t o = (size_t)b * 3 * N + i;
  V3<T> mi;
  V3<T> kv;
  if (C.pending_finish) {
    const V3<T> y = ld3(ep.bms1, N, (long long)o);
    const T s = rsqrt_t<T>(y.x * y.x + y.y * y.y + y.z * y.z);
    mi = {y.x * s, y.y * s, y.z * s};
    gst(ep.bm + o, mi.x); gst(ep.bm + o + N, mi.y); gst(ep.bm + o + 2 * N, mi.z);
    kv = ld3(ep.bk7, N, (long long)o);
    gst(ep.bk1 + o, kv.x); gst(ep.bk1 + o + N, kv.y); gst(ep.bk1 + o + 2 * N, kv.z);
  } else {
    if (C.done) return;
    mi = ld3(ep.bm, N, (long long)o);
    kv = ld3(ep.bk1, N, (long long)o);
  }
  if (C.done) return;
  const T c = T(C.h_att * ep.a21);
  gst(ep.bms0 + o, mi.x + c * kv.x);
  gst(ep.bms0 + o + N, mi.y + c * kv.y);
  gst(ep.bms0 + o + 2 * N, mi.z + c * kv.z);
}

// ---------------------------------------------------------------------------
// Steepest descent with Barzilai-Borwein steps (energy minimisation).
// ---------------------------------------------------------------------------
// g = m x (m x H) per cell (stored) and, when `stats`, per-block FP64 sums of
// s.s, s.y and y.y with s = m - m_prev, y = g - g_prev (the differences taken
// in FP64 from the stored values); when `check`, the block's largest |dm/dt|^2
// of the LL equation (g1 m x H + g2 m x (m x H), the instance's coefficients).
// part: 4 doubles per block.  Blocks of kNT threads, bpi per instance;
// instances whose controller says done are skipped.
template <typename T>
__global__ void __launch_bounds__(kNT) k_sd_stats(const T* __restrict__ m, const T* __restrict__ H,
                                                  const T* __restrict__ mp, const T* __restrict__ gp,
                                                  T* __restrict__ g, double* __restrict__ part, long long N,
                                                  int bpi, int stats, int check, const DevParams* __restrict__ prm,
                                                  const DevCtl* __restrict__ ctl) {
  __shared__ double red[4][kNT / 64];
  const int b = (int)(blockIdx.x / (unsigned)bpi);
  const int blk = (int)(blockIdx.x - (unsigned)b * (unsigned)bpi);
  if (ctl && ctl[b].done) return;
  const long long i = (long long)blk * kNT + threadIdx.x;
  double ss = 0.0, sy = 0.0, yy = 0.0, kk = 0.0;
  if (i < N) {
    const size_t o = (size_t)b * 3 * N + i;
    const V3<T> mi = ld3(m, N, (long long)o), Hi = ld3(H, N, (long long)o);
    const V3<T> f = {mi.y * Hi.z - mi.z * Hi.y, mi.z * Hi.x - mi.x * Hi.z, mi.x * Hi.y - mi.y * Hi.x};
    const V3<T> gi = {mi.y * f.z - mi.z * f.y, mi.z * f.x - mi.x * f.z, mi.x * f.y - mi.y * f.x};
    gst(g + o, gi.x); gst(g + o + N, gi.y); gst(g + o + 2 * N, gi.z);
    if (stats) {
      const V3<T> mq = ld3(mp, N, (long long)o), gq = ld3(gp, N, (long long)o);
      const double sx = (double)mi.x - (double)mq.x, sy_ = (double)mi.y - (double)mq.y;
      const double sz = (double)mi.z - (double)mq.z;
      const double yx = (double)gi.x - (double)gq.x, yy_ = (double)gi.y - (double)gq.y;
      const double yz = (double)gi.z - (double)gq.z;
      ss = sx * sx + sy_ * sy_ + sz * sz;
      sy = sx * yx + sy_ * yy_ + sz * yz;
      yy = yx * yx + yy_ * yy_ + yz * yz;
    }
    if (check) {
      const T g1 = T(prm[b].g1), g2 = T(prm[b].g2);
      const double kx = (double)(g1 * f.x + g2 * gi.x), ky = (double)(g1 * f.y + g2 * gi.y);
      const double kz = (double)(g1 * f.z + g2 * gi.z);
      kk = kx * kx + ky * ky + kz * kz;
      if (!(kk <= DBL_MAX)) kk = HUGE_VAL;
    }
  }
  if (!stats && !check) return;
  ss = wave_sum(ss); sy = wave_sum(sy); yy = wave_sum(yy); kk = wave_max(kk);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { red[0][w] = ss; red[1][w] = sy; red[2][w] = yy; red[3][w] = kk; }
  __syncthreads();
  if (threadIdx.x < 4) {
    double v = 0.0;
    for (int j = 0; j < kNT / 64; ++j) v = threadIdx.x == 3 ? fmax(v, red[3][j]) : v + red[threadIdx.x][j];
    part[((size_t)b * bpi + blk) * 4 + threadIdx.x] = v;
  }
}

// One 64-thread workgroup per instance: fixed-order sums of the block
// partials.  With `check` (a relaxation), first the stopping rule: the
// instance's largest |dm/dt| is recorded, and below its threshold (or at the
// last iteration, `last`) the instance is done after k updates.  Then the
// step rule of iteration k >= 1 (odd k: s.s / s.y, even k: s.y / y.y; a
// quotient that is not finite and positive keeps the previous step) and the
// clip to [tau_min, tau_max].
__global__ void __launch_bounds__(64) k_sd_tau(const double* __restrict__ part, int bpi, long long k,
                                               double* __restrict__ tau, double tau_min, double tau_max,
                                               int check, int last, DevCtl* __restrict__ ctl) {
  const int b = blockIdx.x;
  if (ctl && ctl[b].done) return;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < bpi; j += 64) {
    for (int q = 0; q < 3; ++q) v[q] += part[((size_t)b * bpi + j) * 4 + q];
    v[3] = fmax(v[3], part[((size_t)b * bpi + j) * 4 + 3]);
  }
  for (int q = 0; q < 3; ++q) v[q] = wave_sum(v[q]);
  v[3] = wave_max(v[3]);
  if (threadIdx.x != 0) return;
  if (check) {
    const double d = sqrt(v[3]);
    ctl[b].last_dmdt = d;
    ctl[b].n_attempt = k;
    if (d < ctl[b].stop_dmdt || last) {
      ctl[b].done = 1;
      return;
    }
  }
  if (k == 0) return;
  const double num = (k & 1) ? v[0] : v[1], den = (k & 1) ? v[1] : v[2];
  double t = num / den;
  if (!(t > 0.0) || !(t <= DBL_MAX)) t = tau[b];
  tau[b] = fmin(fmax(t, tau_min), tau_max);
}

// m_prev <- m, g_prev <- g, then the update of the energy-minimisation section:
// (1 + tau^2 |f|^2 / 4) m' = (1 - tau^2 |f|^2 / 4) m - tau g, f = m x H.
// Instances whose controller says done keep m.
template <typename T>
__global__ void __launch_bounds__(kNT) k_sd_update(T* __restrict__ m, const T* __restrict__ H,
                                                   const T* __restrict__ g, T* __restrict__ mp,
                                                   T* __restrict__ gp, const double* __restrict__ tau, long long N,
                                                   long long total, const DevCtl* __restrict__ ctl) {
  const long long t = (long long)blockIdx.x * kNT + threadIdx.x;
  if (t >= total) return;
  const long long b = t / N, i = t - b * N;
  if (ctl && ctl[b].done) return;
  const size_t o = (size_t)b * 3 * N + i;
  const V3<T> mi = ld3(m, N, (long long)o), Hi = ld3(H, N, (long long)o), gi = ld3(g, N, (long long)o);
  const V3<T> f = {mi.y * Hi.z - mi.z * Hi.y, mi.z * Hi.x - mi.x * Hi.z, mi.x * Hi.y - mi.y * Hi.x};
  const T tb = T(tau[b]);
  const T a = T(0.25) * tb * tb * (f.x * f.x + f.y * f.y + f.z * f.z);
  const T c0 = (T(1) - a) / (T(1) + a), c1 = tb / (T(1) + a);
  gst(mp + o, mi.x); gst(mp + o + N, mi.y); gst(mp + o + 2 * N, mi.z);
  gst(gp + o, gi.x); gst(gp + o + N, gi.y); gst(gp + o + 2 * N, gi.z);
  gst(m + o, c0 * mi.x - c1 * gi.x);
  gst(m + o + N, c0 * mi.y - c1 * gi.y);
  gst(m + o + 2 * N, c0 * mi.z - c1 * gi.z);
}

__global__ void k_controller(DevCtl* ctl, int n, const double* __restrict__ replay_h) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  control_step(ctl[b], replay_h);
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
// Launchers: one launch per pass over every group that takes part in it.
// ---------------------------------------------------------------------------
namespace {

template <typename T>
struct LaunchBuilder {
  Launch<T> L;
  long long total = 0;
  LaunchBuilder(const GroupSet<T>& gs, const Epi<T>* epis) {
    L.hps = gs.dh;
    L.epis = epis;
    L.ngroups = gs.n;
    L.h0 = gs.h[0];
    for (int i = 0; i <= kMaxGroups; ++i) L.off[i] = 0;
  }
  // blocks of each group (0 = the group takes no part); padded to multiples of 8
  void set(int gi, long long nb) {
    L.off[gi] = (int)total;
    total += (nb + 7) / 8 * 8;
    L.off[gi + 1] = (int)total;
  }
};

template <typename T, int PZ>
void z_reg_launch(const Launch<T>& L, long long total, bool half, hipStream_t s) {
  if constexpr (!(sizeof(T) == 8 && PZ > 16)) {  // FP64 columns beyond 16 points use lane pairs
    if constexpr (PZ % 2 == 0) {
      if (half) {
        k_z3d_reg_half<T, PZ><<<dim3((unsigned)total), kNT, 0, s>>>(L);
        return;
      }
    }
    k_z3d_reg<T, PZ><<<dim3((unsigned)total), kNT, 0, s>>>(L);
  }
}

template <typename T, int M>
void z_pair_launch(const Launch<T>& L, long long total, hipStream_t s) {
  k_z3d_pair<T, M><<<dim3((unsigned)total), kNT, 0, s>>>(L);
}

// Lane-pair register z pass: even Pz with Pz / 2 in {1,2,3,4,6,8,9,12,16}.
bool z_pair_supported(int Pz) {
  switch (Pz) {
    case 2: case 4: case 6: case 8: case 12: case 16: case 18: case 24: case 32:
      return true;
    default:
      return false;
  }
}

template <typename T>
void z_pair_dispatch(int Pz, const Launch<T>& L, long long total, hipStream_t s) {
  switch (Pz) {
    case 2: z_pair_launch<T, 1>(L, total, s); break;
    case 4: z_pair_launch<T, 2>(L, total, s); break;
    case 6: z_pair_launch<T, 3>(L, total, s); break;
    case 8: z_pair_launch<T, 4>(L, total, s); break;
    case 12: z_pair_launch<T, 6>(L, total, s); break;
    case 16: z_pair_launch<T, 8>(L, total, s); break;
    case 18: z_pair_launch<T, 9>(L, total, s); break;
    case 24: z_pair_launch<T, 12>(L, total, s); break;
    case 32: z_pair_launch<T, 16>(L, total, s); break;
    default: break;
  }
}

// One lane per column: register transforms of every 3-smooth Pz up to 32
// (FP64: up to 16; beyond that the lane-pair pass holds half the registers).
template <typename T>
bool z_reg_supported(int Pz) {
  const int lim = sizeof(T) == 4 ? 32 : 16;
  switch (Pz) {
    case 2: case 3: case 4: case 6: case 8: case 9: case 12: case 16: case 18: case 24: case 27: case 32:
      return Pz <= lim;
    default:
      return false;
  }
}

template <typename T>
void z_reg_dispatch(int Pz, const Launch<T>& L, long long total, bool half, hipStream_t s) {
  switch (Pz) {
    case 2: z_reg_launch<T, 2>(L, total, half, s); break;
    case 3: z_reg_launch<T, 3>(L, total, half, s); break;
    case 4: z_reg_launch<T, 4>(L, total, half, s); break;
    case 6: z_reg_launch<T, 6>(L, total, half, s); break;
    case 8: z_reg_launch<T, 8>(L, total, half, s); break;
    case 9: z_reg_launch<T, 9>(L, total, half, s); break;
    case 12: z_reg_launch<T, 12>(L, total, half, s); break;
    case 16: z_reg_launch<T, 16>(L, total, half, s); break;
    case 18: z_reg_launch<T, 18>(L, total, half, s); break;
    case 24: z_reg_launch<T, 24>(L, total, half, s); break;
    case 27: z_reg_launch<T, 27>(L, total, half, s); break;
    case 32: z_reg_launch<T, 32>(L, total, half, s); break;
    default: break;
  }
}

// z pass of a group: 0 lane pairs, 1 one lane per column (registers), 2 LDS
// (any Pz), 3 LDS with the transform compiled for Pz (nz = Pz/2, Pz in
// {16, 32, 64}; the instance's y buffer within 32-bit offsets).  One lane per
// column is fastest where it fits (FP32 up to 32 points); FP64 takes the
// compiled LDS kernel (a 32-point FP64 column does not fit one lane).
template <typename T>
int z_kind(const Geo& g) {
  const int Pz = g.Pz;
  const bool half = 2 * g.nz == Pz;
  const bool fits = (double)g.sy * sizeof(Cx<T>) < 4294967296.0;
  if (half && fits && (Pz == 16 || Pz == 32 || Pz == 64) && (sizeof(T) == 8 || Pz == 64)) return 3;
  if (z_reg_supported<T>(Pz)) return 1;
  if (z_pair_supported(Pz)) return 0;
  return 2;
}

// (kx,ky) columns per workgroup and transform entries per thread of k_z3d_s:
// 3 Q Pz/E threads (at most 384) and 3 Q col_stride(Pz) entries of LDS
// (at most 57 KB; 28 KB for the FP64 32-point columns, whose workgroups are
// latency-bound and gain from more of them per CU)
template <typename T> constexpr int zs_q(int Pz) {
  return Pz == 16 ? (sizeof(T) == 8 ? 32 : 64) : Pz == 32 ? 16 : (sizeof(T) == 8 ? 16 : 32);
}
constexpr int zs_e(int Pz) { return Pz == 64 ? 16 : 8; }

template <typename T>
void zs_dispatch(int Pz, const Launch<T>& L, long long total, hipStream_t s) {
  const dim3 grid((unsigned)total);
  const size_t lds = (size_t)3 * zs_q<T>(Pz) * col_stride(Pz) * sizeof(Cx<T>);
  const int nt = 3 * zs_q<T>(Pz) * (Pz / zs_e(Pz));
  switch (Pz) {
    case 16: k_z3d_s<T, 16, zs_q<T>(16), zs_e(16)><<<grid, nt, lds, s>>>(L); break;
    case 32: k_z3d_s<T, 32, zs_q<T>(32), zs_e(32)><<<grid, nt, lds, s>>>(L); break;
    default: k_z3d_s<T, 64, zs_q<T>(64), zs_e(64)><<<grid, nt, lds, s>>>(L); break;
  }
}

}  // namespace

// Cells per thread of the unrolled inverse-x epilogue for a launch with nt
// threads (0: none of 1, 2, 4, 8 fits every group).
template <typename T>
int inv_cpt(const GroupSet<T>& gs, int nt) {
  int need = 1;
  for (int i = 0; i < gs.n; ++i) {
    const int c = (gs.h[i].tu.ty_x * gs.h[i].g.nx + nt - 1) / nt;
    need = std::max(need, c);
  }
  for (int c : {1, 2, 4, 8})
    if (need <= c) return c;
  return 0;
}

template <typename T>
bool eval_fusable(const GroupSet<T>& gs) {
  int nt = 64;
  for (int i = 0; i < gs.n; ++i) nt = std::max(nt, gs.h[i].tu.nt_i);
  return inv_cpt(gs, nt) > 0;
}

// Length of the y kernels compiled for one Py (k_ypass_s / k_yinv_s), 0 for
// the general ones: every group of the pass (3-D groups only for the inverse)
// has Py = 2 ny = SL for one SL in {256, 512, 1024, 2048}, and its tile of columns
// times SL/16 threads fits a workgroup.  ept: entries per thread and stage,
// 8 (SL/8 threads a column, the plan without radix 16, p2_radix(.., false,
// ..), whose LDS padding is the y plan's for these lengths) where the
// launch shapes give a column at least SL/8 threads and the workgroup still
// fits, else 16.  nt: the threads to launch.
template <typename T>
int static_y(const GroupSet<T>& gs, bool inv, int& nt, int& ept, const bool* use = nullptr) {
  int sl = 0, cmax = 0;
  bool e8 = true;
  for (int i = 0; i < gs.n; ++i) {
    const HotPlan<T>& h = gs.h[i];
    if (inv && h.g.nz == 1) continue;
    if (use && !use[i]) continue;
    const int L = h.g.Py;
    if (L != 2 * h.g.ny || (L != 256 && L != 512 && L != 1024 && L != 2048)) return 0;
    if (sl != 0 && sl != L) return 0;
    sl = L;
    cmax = std::max(cmax, h.g.nz == 1 ? 3 * h.tu.cb_y2 : h.tu.cb_y);
    e8 = e8 && (h.g.nz == 1 ? h.tu.tpc_y2 : h.tu.tpc_y) >= L / 8;
  }
  if (sl == 0 || cmax * (sl / 16) > 512) return 0;
  ept = e8 && cmax * (sl / 8) <= 512 ? 8 : 16;
  nt = std::max(64, (cmax * (sl / ept) + 63) / 64 * 64);
  return sl;
}

// The y passes launch once per length with a compiled transform (Py = 2 ny of
// 256 to 2048) among the groups, and once for the rest (the general
// transform): key of group i, 0 for the general kernels.
template <typename T>
int y_key(const HotPlan<T>& h) {
  const int L = h.g.Py;
  return L == 2 * h.g.ny && (L == 256 || L == 512 || L == 1024 || L == 2048) ? L : 0;
}

template <typename T>
hipError_t launch_eval(const GroupSet<T>& gs, const Epi<T>* epis, int mode, bool demag, hipStream_t s,
                       hipEvent_t* ev, bool skip_fwd, bool fuse_next, unsigned pass_mask) {
  const size_t csz = sizeof(Cx<T>);
  int e = 0;
  auto mark = [&]() {
    if (ev) (void)hipEventRecord(ev[e++], s);
  };
  bool any3d = false;
  for (int i = 0; i < gs.n; ++i) any3d = any3d || gs.h[i].g.nz > 1;
  // pass numbers: 0 x forward, 1 y, 2 z (3-D), 3 y inverse (3-D), last x inverse
  auto on = [&](int p) { return ((pass_mask >> p) & 1u) != 0; };
  const int p_inv = demag ? (any3d ? 4 : 2) : 0;
  bool y16 = false;  // some group's y plan has radix-16 stages
  for (int i = 0; i < gs.n; ++i)
    for (int st = 0; st < gs.h[i].fd[1].nst; ++st) y16 = y16 || radix_of(gs.h[i].fd[1].code, st) == 16;
  if (demag) {
    if (!skip_fwd && on(0)) {  // x forward (skipped when the previous stage's inverse-x pass did it)
      // one launch per static length (every group with an even nx = Lx of
      // 128 to 1024 shares the kernel compiled for its Lx), one for the rest
      auto x_key = [&](const Geo& g) {
        return g.nx == g.Lx && (g.Lx == 128 || g.Lx == 256 || g.Lx == 512 || g.Lx == 1024) ? g.Lx : 0;
      };
      mark();
      int keys[kMaxGroups], nkeys = 0;
      for (int i = 0; i < gs.n; ++i) {
        const int k = x_key(gs.h[i].g);
        bool seen = false;
        for (int j = 0; j < nkeys; ++j) seen = seen || keys[j] == k;
        if (!seen) keys[nkeys++] = k;
      }
      for (int kk = 0; kk < nkeys; ++kk) {
        LaunchBuilder<T> lb(gs, epis);
        int nt = 64;
        size_t lds = 0;
        for (int i = 0; i < gs.n; ++i) {
          const HotPlan<T>& h = gs.h[i];
          const bool use = x_key(h.g) == keys[kk];
          lb.set(i, use ? fwd_blocks(h.g, h.tu, h.batch) : 0);
          if (!use) continue;
          nt = std::max(nt, h.tu.nt_f);
          lds = std::max(lds, ((size_t)h.tu.ty_f * col_stride(h.g.Lx) + 2 * h.g.Lx + 1) * csz);
        }
        const dim3 grid((unsigned)lb.total);
        switch (keys[kk]) {
          case 128: k_fwd_x<T, 128><<<grid, nt, lds, s>>>(lb.L); break;
          case 256: k_fwd_x<T, 256><<<grid, nt, lds, s>>>(lb.L); break;
          case 512: k_fwd_x<T, 512><<<grid, nt, lds, s>>>(lb.L); break;
          case 1024: k_fwd_x<T, 1024><<<grid, nt, lds, s>>>(lb.L); break;
          default: k_fwd_x<T, 0><<<grid, nt, lds, s>>>(lb.L);
        }
      }
    }
    if (on(1)) {  // y forward (2-D groups: fused forward / product / inverse)
      mark();
      int keys[kMaxGroups], nkeys = 0;
      for (int i = 0; i < gs.n; ++i) {
        const int k = y_key(gs.h[i]);
        bool seen = false;
        for (int j = 0; j < nkeys; ++j) seen = seen || keys[j] == k;
        if (!seen) keys[nkeys++] = k;
      }
      for (int kk = 0; kk < nkeys; ++kk) {
      bool use[kMaxGroups];
      LaunchBuilder<T> lb(gs, epis);
      int nt = 64;
      size_t lds = 0;
      for (int i = 0; i < gs.n; ++i) {
        const HotPlan<T>& h = gs.h[i];
        use[i] = y_key(h) == keys[kk];
        if (!use[i]) {
          lb.set(i, 0);
        } else if (h.g.nz == 1) {
          lb.set(i, y2d_blocks(h.g, h.tu, h.batch));
          lds = std::max(lds, ((size_t)3 * h.tu.cb_y2 * col_stride(h.g.Py) + h.g.Py) * csz +
                                  (y2d_tensor_in_lds(h.g) ? (size_t)4 * (h.tu.cb_y2 + y2d_packed(h.g)) * h.g.Ky * (csz / 2) : 0));
        } else {
          lb.set(i, y3d_blocks(h.g, h.tu, h.batch));
          lds = std::max(lds, (size_t)h.tu.cb_y * col_stride(h.g.Py) * csz);
        }
        if (use[i]) nt = std::max(nt, h.tu.nt_y);
      }
      int nts = 0, ept = 16;
      const dim3 grid((unsigned)lb.total);
      const int sly = static_y(gs, false, nts, ept, use);
      switch (sly * 100 + (sly ? ept : 0)) {
        case 25608: k_ypass_s<T, 256, 8><<<grid, nts, lds, s>>>(lb.L); break;
        case 25616: k_ypass_s<T, 256, 16><<<grid, nts, lds, s>>>(lb.L); break;
        case 51208: k_ypass_s<T, 512, 8><<<grid, nts, lds, s>>>(lb.L); break;
        case 51216: k_ypass_s<T, 512, 16><<<grid, nts, lds, s>>>(lb.L); break;
        case 102408: k_ypass_s<T, 1024, 8><<<grid, nts, lds, s>>>(lb.L); break;
        case 102416: k_ypass_s<T, 1024, 16><<<grid, nts, lds, s>>>(lb.L); break;
        case 204808: k_ypass_s<T, 2048, 8><<<grid, nts, lds, s>>>(lb.L); break;
        case 204816: k_ypass_s<T, 2048, 16><<<grid, nts, lds, s>>>(lb.L); break;
        default:
          if (y16) k_ypass<T, true><<<grid, nt, lds, s>>>(lb.L);
          else k_ypass<T, false><<<grid, nt, lds, s>>>(lb.L);
      }
      }
    }
    if (any3d) {
      // z: register transform for every supported Pz (one launch per distinct
      // Pz), LDS transform for the rest
      int done_pz[kMaxGroups];
      int ndone = 0;
      mark();
      // one launch per (Pz, nz == Pz/2) among the groups
      for (int i = 0; i < gs.n && on(2); ++i) {
        const HotPlan<T>& hi = gs.h[i];
        const int kind = z_kind<T>(hi.g);
        if (hi.g.nz == 1 || kind == 2) continue;
        const bool half = 2 * hi.g.nz == hi.g.Pz;
        const int key = (2 * hi.g.Pz + (half ? 1 : 0)) * 4 + kind;
        bool seen = false;
        for (int k = 0; k < ndone; ++k) seen = seen || done_pz[k] == key;
        if (seen) continue;
        done_pz[ndone++] = key;
        LaunchBuilder<T> lb(gs, epis);
        for (int j = 0; j < gs.n; ++j) {
          const HotPlan<T>& h = gs.h[j];
          const bool use = h.g.nz > 1 && (2 * h.g.Pz + (2 * h.g.nz == h.g.Pz ? 1 : 0)) * 4 + z_kind<T>(h.g) == key;
          const long long nb = kind == 0 ? zpair_blocks(h.g, h.batch)
                               : kind == 3 ? zs_blocks(h.g, h.batch, zs_q<T>(h.g.Pz))
                                           : zreg_blocks(h.g, h.batch);
          // a multiple of 8 (the kernels end the extra workgroups at once), so
          // that the XCD remap keeps the workgroups of one kx row -- whose
          // columns ky and Py - ky read the same folded tensor entries -- on
          // one XCD and its L2
          lb.set(j, use ? (nb + 7) / 8 * 8 : 0);
        }
        if (kind == 0) z_pair_dispatch<T>(hi.g.Pz, lb.L, lb.total, s);
        else if (kind == 3) zs_dispatch<T>(hi.g.Pz, lb.L, lb.total, s);
        else z_reg_dispatch<T>(hi.g.Pz, lb.L, lb.total, half, s);
      }
      LaunchBuilder<T> lz(gs, epis);
      int nt = 0;
      size_t lds = 0;
      for (int j = 0; j < gs.n; ++j) {
        const HotPlan<T>& h = gs.h[j];
        const bool use = h.g.nz > 1 && z_kind<T>(h.g) == 2;
        lz.set(j, use ? zlds_blocks(h.g, h.tu, h.batch) : 0);
        if (use) {
          nt = std::max(nt, 3 * h.tu.qz * h.tu.tpc_z);
          lds = std::max(lds, (size_t)3 * h.tu.qz * col_stride(h.g.Pz) * csz);
        }
      }
      if (nt > 0 && on(2)) k_z3d<T><<<dim3((unsigned)lz.total), nt, lds, s>>>(lz.L);
      // y inverse (3-D groups), one launch per key as the forward pass
      mark();
      int keys[kMaxGroups], nkeys = 0;
      for (int i = 0; i < gs.n && on(3); ++i) {
        if (gs.h[i].g.nz == 1) continue;
        const int k = y_key(gs.h[i]);
        bool seen = false;
        for (int j = 0; j < nkeys; ++j) seen = seen || keys[j] == k;
        if (!seen) keys[nkeys++] = k;
      }
      for (int kk = 0; kk < nkeys; ++kk) {
      bool usey[kMaxGroups];
      LaunchBuilder<T> ly(gs, epis);
      int nty = 64;
      size_t ldsy = 0;
      for (int j = 0; j < gs.n; ++j) {
        const HotPlan<T>& h = gs.h[j];
        usey[j] = h.g.nz > 1 && y_key(h) == keys[kk];
        ly.set(j, usey[j] ? y3d_blocks(h.g, h.tu, h.batch) : 0);
        if (usey[j]) {
          nty = std::max(nty, h.tu.nt_y);
          ldsy = std::max(ldsy, (size_t)h.tu.cb_y * col_stride(h.g.Py) * csz);
        }
      }
      int nts = 0, ept = 16;
      const dim3 gridy((unsigned)ly.total);
      const int sly = static_y(gs, true, nts, ept, usey);
      switch (sly * 100 + (sly ? ept : 0)) {
          case 25608: k_yinv_s<T, 256, 8><<<gridy, nts, ldsy, s>>>(ly.L); break;
          case 25616: k_yinv_s<T, 256, 16><<<gridy, nts, ldsy, s>>>(ly.L); break;
          case 51208: k_yinv_s<T, 512, 8><<<gridy, nts, ldsy, s>>>(ly.L); break;
          case 51216: k_yinv_s<T, 512, 16><<<gridy, nts, ldsy, s>>>(ly.L); break;
          case 102408: k_yinv_s<T, 1024, 8><<<gridy, nts, ldsy, s>>>(ly.L); break;
          case 102416: k_yinv_s<T, 1024, 16><<<gridy, nts, ldsy, s>>>(ly.L); break;
          case 204808: k_yinv_s<T, 2048, 8><<<gridy, nts, ldsy, s>>>(ly.L); break;
          case 204816: k_yinv_s<T, 2048, 16><<<gridy, nts, ldsy, s>>>(ly.L); break;
          default:
            if (y16) k_yinv<T, true><<<gridy, nty, ldsy, s>>>(ly.L);
            else k_yinv<T, false><<<gridy, nty, ldsy, s>>>(ly.L);
        }
      }
    }
  }
  if (on(p_inv)) {  // x inverse + epilogue
    LaunchBuilder<T> lb(gs, epis);
    int nt = 64;
    size_t lds = 0;
    for (int i = 0; i < gs.n; ++i) {
      const HotPlan<T>& h = gs.h[i];
      lb.set(i, inv_blocks(h.g, h.tu, h.batch));
      nt = std::max(nt, h.tu.nt_i);
      if (demag) lds = std::max(lds, ((size_t)3 * h.tu.ty_x * col_stride(h.g.Lx) + 2 * h.g.Lx + 1) * csz);
    }
    const int cpt = inv_cpt(gs, nt);
    const bool fuse = fuse_next && demag && mode == MODE_STAGE && cpt > 0;
    mark();
    // general-material form (cell arrays, interlayer coupling, spin torques): plans only
    const bool gen = gs.n == 1 && gs.h[0].gen != 0;
    if (gen) {
      if (demag) inv_x_launch<T, true, true>(mode, cpt, fuse, lb.L, lb.total, nt, lds, s);
      else inv_x_launch<T, false, true>(mode, cpt, false, lb.L, lb.total, nt, 0, s);
    } else {
      if (demag) inv_x_launch<T, true, false>(mode, cpt, fuse, lb.L, lb.total, nt, lds, s);
      else inv_x_launch<T, false, false>(mode, cpt, false, lb.L, lb.total, nt, 0, s);
    }
  }
  mark();
  return hipGetLastError();
}

template <typename T>
hipError_t launch_begin(const GroupSet<T>& gs, const Epi<T>* epis, hipStream_t s) {
  LaunchBuilder<T> lb(gs, epis);
  for (int i = 0; i < gs.n; ++i) lb.set(i, begin_blocks(gs.h[i].g, gs.h[i].batch));
  k_begin<T><<<dim3((unsigned)lb.total), kNT, 0, s>>>(lb.L);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sd_iteration(T* m, const T* H, T* g, T* mp, T* gp, double* part, double* tau, int batch,
                               long long N, long long k, double tau_min, double tau_max, const DevParams* prm,
                               DevCtl* ctl, bool last, hipStream_t s) {
  const int bpi = (int)((N + kNT - 1) / kNT);
  const int check = ctl ? 1 : 0;
  k_sd_stats<T><<<dim3((unsigned)(batch * bpi)), kNT, 0, s>>>(m, H, mp, gp, g, part, N, bpi, k > 0 ? 1 : 0, check,
                                                              prm, ctl);
  if (k > 0 || check)
    k_sd_tau<<<dim3((unsigned)batch), 64, 0, s>>>(part, bpi, k, tau, tau_min, tau_max, check, last ? 1 : 0, ctl);
  if (!last) {
    const long long total = (long long)batch * N;
    k_sd_update<T><<<dim3((unsigned)((total + kNT - 1) / kNT)), kNT, 0, s>>>(m, H, g, mp, gp, tau, N, total, ctl);
  }
  return hipGetLastError();
}

hipError_t launch_controller(DevCtl* ctl, int n, const double* replay_h, hipStream_t s) {
  k_controller<<<dim3((n + 63) / 64), 64, 0, s>>>(ctl, n, replay_h);
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

#define MMX_INST(T)                                                                               \
  template hipError_t launch_eval<T>(const GroupSet<T>&, const Epi<T>*, int, bool, hipStream_t,    \
                                     hipEvent_t*, bool, bool, unsigned);                          \
  template bool eval_fusable<T>(const GroupSet<T>&);                                              \
  template hipError_t launch_begin<T>(const GroupSet<T>&, const Epi<T>*, hipStream_t);            \
  template hipError_t launch_sd_iteration<T>(T*, const T*, T*, T*, T*, double*, double*, int, long long,   \
                                             long long, double, double, const DevParams*, DevCtl*, bool,  \
                                             hipStream_t);                                             \
  template hipError_t launch_neb<T>(const Geo&, int, const T*, T*, const T*, const double*, double, \
                                    double, double*, double*, double, double, int, hipStream_t);
MMX_INST(float)
MMX_INST(double)

}  // namespace mmx
