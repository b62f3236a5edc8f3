// Host runtime and C interface (include/mm.h): validation, plan set-up
// (padded grid, radix plans, twiddles, launch shapes, tensor spectrum),
// effective field / LL / energy calls, device-controlled Dormand-Prince runs
// with HIP-graph replay, and the NEB driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fft_core.hpp"
#include "kernels.hpp"
#include "setup.hpp"

using namespace mmx;

namespace {

thread_local std::string g_err;

mm_status fail(mm_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(call)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? MM_E_NOMEM : MM_E_HIP,                      \
                  std::string(#call) + ": " + hipGetErrorString(e_));                     \
  } while (0)

#define MMCHK(call)                  \
  do {                               \
    mm_status s_ = (call);           \
    if (s_ != MM_OK) return s_;      \
  } while (0)

bool smooth3(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

// Padded length: 2n when 3-smooth (the paper-style choice), else the smallest
// 3-smooth length >= 2n-1 (even for x).  n = 1 -> 1 (y and z only).
int pick_padded(int n, bool even) {
  if (n == 1 && !even) return 1;
  if (smooth3(2 * n)) return 2 * n;
  for (int P = 2 * n - 1;; ++P)
    if (smooth3(P) && (!even || P % 2 == 0)) return P;
}

std::vector<int> radices(int L) {
  std::vector<int> r;
  int a = 0, b = 0;
  while (L % 2 == 0) { L /= 2; ++a; }
  while (L % 3 == 0) { L /= 3; ++b; }
  int n8 = a / 3, rem = a % 3;
  if (rem == 1 && n8 > 0) { --n8; r.push_back(4); r.push_back(4); }
  else if (rem == 1) r.push_back(2);
  else if (rem == 2) r.push_back(4);
  for (int i = 0; i < n8; ++i) r.insert(r.begin(), 8);
  for (int i = 0; i < b; ++i) r.push_back(3);
  return r;
}

template <typename T>
FftPlan<T> make_fft(int L, const Cx<T>* tw) {
  FftPlan<T> p{};
  p.L = L;
  p.tw = tw;
  std::vector<int> r = L > 1 ? radices(L) : std::vector<int>{};
  p.nst = (int)r.size();
  int ns = 1;
  for (int s = 0; s < p.nst; ++s) {
    p.rad[s] = r[s];
    p.ns[s] = ns;
    ns *= r[s];
  }
  return p;
}

// Smallest threads-per-column so that each stage fits the per-thread
// butterfly budget (16/R butterflies of radix R).
template <typename T>
int min_tpc(const FftPlan<T>& p) {
  int t = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int R = p.rad[s], nb = 16 / R;
    t = std::max(t, (p.L / R + nb - 1) / nb);
  }
  return t;
}

template <typename T>
std::vector<Cx<T>> twiddles(int L) {
  std::vector<Cx<T>> w(L);
  for (int m = 0; m < L; ++m) {
    const double a = -2.0 * M_PI * (double)m / (double)L;
    w[m] = Cx<T>{(T)std::cos(a), (T)std::sin(a)};
  }
  return w;
}

// Gauss-Legendre nodes on [-1,1] by Newton iteration on P_n (FP64).
void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Tent-weighted rule on [-1,1]: n Gauss nodes on each half, weight w (1-|s|).
void tent_rules(double nodes[5][20], double wts[5][20], int nn[5]) {
  const int ns[5] = {2, 3, 4, 6, 10};
  for (int r = 0; r < 5; ++r) {
    const int n = ns[r];
    double x[10], w[10];
    gauss_legendre(n, x, w);
    nn[r] = n;
    for (int i = 0; i < n; ++i) {
      const double s = 0.5 * (1.0 + x[i]);
      const double ww = 0.5 * w[i] * (1.0 - s);
      nodes[r][i] = -s;
      wts[r][i] = ww;
      nodes[r][n + i] = s;
      wts[r][n + i] = ww;
    }
  }
}

// Dormand-Prince 5(4) coefficients (Dormand & Prince 1980).
struct Tableau {
  double a[8][7];  // a[s][j]: stage s (1-based) input uses a[s][0..s-2]
  double e[7];     // b - bhat
  Tableau() {
    std::memset(a, 0, sizeof(a));
    a[2][0] = 1.0 / 5;
    a[3][0] = 3.0 / 40; a[3][1] = 9.0 / 40;
    a[4][0] = 44.0 / 45; a[4][1] = -56.0 / 15; a[4][2] = 32.0 / 9;
    a[5][0] = 19372.0 / 6561; a[5][1] = -25360.0 / 2187; a[5][2] = 64448.0 / 6561; a[5][3] = -212.0 / 729;
    a[6][0] = 9017.0 / 3168; a[6][1] = -355.0 / 33; a[6][2] = 46732.0 / 5247; a[6][3] = 49.0 / 176;
    a[6][4] = -5103.0 / 18656;
    a[7][0] = 35.0 / 384; a[7][1] = 0.0; a[7][2] = 500.0 / 1113; a[7][3] = 125.0 / 192;
    a[7][4] = -2187.0 / 6784; a[7][5] = 11.0 / 84;
    const double bh[7] = {5179.0 / 57600, 0.0, 7571.0 / 16695, 393.0 / 640, -92097.0 / 339200,
                          187.0 / 2100, 1.0 / 40};
    for (int j = 0; j < 7; ++j) e[j] = (j < 6 ? a[7][j] : 0.0) - bh[j];
  }
};
const Tableau kDP;

bool is_fin(double v) { return std::isfinite(v); }

}  // namespace

struct mm_plan {
  mm_mesh mesh;
  mm_precision prec;
  uint32_t terms;
  int maxb;
  int ncomp;
  Geo g;
  Tuning tu;
  size_t csz, rsz;  // complex / real element sizes
  int devid;
  hipStream_t cap = nullptr;  // capture stream (default priority)
  // device buffers
  void* Sx = nullptr;
  void* Sy = nullptr;
  void* kt = nullptr;
  void* post = nullptr;
  void* twx = nullptr;
  void* twy = nullptr;
  void* twz = nullptr;
  void* fplans = nullptr;  // device FftPlan[3] (x, y, z)
  DevParams* prm = nullptr;
  DevCtl* ctl = nullptr;
  double* partial = nullptr;
  double* e5 = nullptr;
  double* replay = nullptr;
  long long replay_cap = 0;
  void* stage = nullptr;  // ms0, ms1, k1..k7 (9 x maxb x 3N)
  // NEB scratch
  void* nebH = nullptr;
  void* nebB = nullptr;
  double* nebS = nullptr;
  double* nebP = nullptr;
  // host staging (pinned)
  DevCtl* hctl = nullptr;
  double* he5 = nullptr;
  // graph cache for rk45 runs
  hipGraphExec_t gexec = nullptr;
  const void* g_m = nullptr;
  int g_batch = -1;
  int g_steps = 0;
  double imag_ratio = 0.0;  // max |Im| / max |Re| of the tensor spectrum
  bool any_demag = false;   // some instance of the last uploaded parameters enables demag
};

namespace {

mm_status check_mesh(const mm_mesh* m) {
  if (!m) return fail(MM_E_ARG, "mesh is null");
  if (m->nx < 2 || m->ny < 1 || m->nz < 1 || m->nx > 1024 || m->ny > 1024 || m->nz > 1024)
    return fail(MM_E_ARG, "mesh sizes must satisfy 2 <= nx <= 1024, 1 <= ny, nz <= 1024");
  if (!(is_fin(m->dx) && is_fin(m->dy) && is_fin(m->dz)) || m->dx <= 0 || m->dy <= 0 || m->dz <= 0)
    return fail(MM_E_ARG, "cell sizes must be finite and > 0");
  return MM_OK;
}

mm_status check_params(const mm_plan* p, const mm_params* q, int n) {
  if (!q) return fail(MM_E_ARG, "params is null");
  for (int b = 0; b < n; ++b) {
    const mm_params& r = q[b];
    const double v[] = {r.Ms, r.A, r.D, r.Ku, r.u[0], r.u[1], r.u[2], r.H[0], r.H[1], r.H[2], r.alpha, r.gamma};
    for (double x : v)
      if (!is_fin(x)) return fail(MM_E_ARG, "parameters must be finite");
    if (r.Ms <= 0) return fail(MM_E_ARG, "Ms must be > 0");
    if (r.alpha < 0) return fail(MM_E_ARG, "alpha must be >= 0");
    if (r.gamma <= 0) return fail(MM_E_ARG, "gamma must be > 0");
    if (r.A < 0) return fail(MM_E_ARG, "A must be >= 0");
    if ((r.terms & ~p->terms) != 0) return fail(MM_E_ARG, "params enable a term the plan was not built for");
    if ((r.terms & MM_ANIS_UNIAXIAL) && r.u[0] == 0 && r.u[1] == 0 && r.u[2] == 0)
      return fail(MM_E_ARG, "easy axis must be non-zero");
  }
  return MM_OK;
}

mm_status upload_params(mm_plan* p, const mm_params* q, int n, hipStream_t s) {
  std::vector<DevParams> d(n);
  const double P = (double)p->g.Px * p->g.Py * p->g.Pz;
  for (int b = 0; b < n; ++b) {
    const mm_params& r = q[b];
    DevParams& o = d[b];
    std::memset(&o, 0, sizeof(o));
    o.Ms = r.Ms;
    const double c = kMu0 * r.Ms;
    o.cex[0] = 2 * r.A / (c * p->mesh.dx * p->mesh.dx);
    o.cex[1] = 2 * r.A / (c * p->mesh.dy * p->mesh.dy);
    o.cex[2] = 2 * r.A / (c * p->mesh.dz * p->mesh.dz);
    o.cdmi[0] = r.D / (c * p->mesh.dx);
    o.cdmi[1] = r.D / (c * p->mesh.dy);
    o.can = 2 * r.Ku / c;
    const double un = std::sqrt(r.u[0] * r.u[0] + r.u[1] * r.u[1] + r.u[2] * r.u[2]);
    for (int k = 0; k < 3; ++k) {
      o.u[k] = un > 0 ? r.u[k] / un : 0.0;
      o.H[k] = r.H[k];
    }
    o.g1 = -r.gamma / (1 + r.alpha * r.alpha);
    o.g2 = -r.alpha * r.gamma / (1 + r.alpha * r.alpha);
    o.demag_scale = -r.Ms / P;
    o.terms = r.terms;
  }
  p->any_demag = false;
  for (int b = 0; b < n; ++b) p->any_demag = p->any_demag || (q[b].terms & MM_DEMAG) != 0;
  HIPCHK(hipMemcpyAsync(p->prm, d.data(), sizeof(DevParams) * n, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return MM_OK;
}

// Launch shapes.  Each workgroup keeps its LDS within 80 KiB (two per CU), the
// per-thread butterfly budget of the transforms is respected, and tiles shrink
// until a pass has about 4 workgroups per CU (small meshes) or reach their
// coalescing-friendly maximum (large meshes).
int pow2ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

mm_status choose_tuning(mm_plan* p) {
  const Geo& g = p->g;
  Tuning& t = p->tu;
  const size_t csz = p->csz;
  const size_t budget = 80 * 1024;
  const long long want = 4 * 256;  // workgroups per pass worth aiming for
  auto tpc_for = [&](int L) {
    if (p->prec == MM_F32) return min_tpc(make_fft<float>(L, nullptr));
    return min_tpc(make_fft<double>(L, nullptr));
  };
  const int tpx = tpc_for(g.Lx);
  const size_t rowb = (size_t)col_stride(g.Lx) * csz;
  // forward x: rows of one component
  {
    const long long rows = 3LL * g.nz * g.ny;
    int ty = 16;
    while (ty > 1 && ((size_t)ty * rowb > budget || ty * tpx > 512 || rows / ty < want)) ty /= 2;
    ty = std::min(ty, g.ny);
    if ((size_t)ty * rowb > 160 * 1024 || ty * tpx > 512) return fail(MM_E_ARG, "mesh too long along x");
    t.ty_f = ty;
    t.nt_f = std::min(512, std::max(64, pow2ceil(std::max(ty * tpx, ty * g.Lx / 4))));
    t.tpc_f = t.nt_f / ty;
  }
  // inverse x + epilogue: rows of all 3 components, at most 8 cells per thread
  {
    const long long rows = (long long)g.nz * g.ny;
    int ty = 16;
    while (ty > 1 && ((size_t)ty * rowb > budget || ty * tpx > 512 || ty * g.nx > 8 * 512 || rows / ty < want))
      ty /= 2;
    ty = std::min(ty, g.ny);
    if ((size_t)ty * rowb > 160 * 1024 || ty * tpx > 512 || ty * g.nx > 8 * 512)
      return fail(MM_E_ARG, "mesh too long along x");
    t.ty_x = ty;
    t.nt_i = std::min(512, std::max(64, pow2ceil(std::max(ty * tpx, ty * g.nx))));
    t.tpc_x = t.nt_i / ty;
  }
  if (g.nz == 1) {
    const int tmin = tpc_for(g.Py);
    const int tpc = std::max(tmin, std::min(2 * tmin, 64));
    const size_t colb = 3 * (size_t)col_stride(g.Py) * csz;
    int cb = 8;
    while (cb > 1 && (cb * colb > budget || 3 * cb * tpc > 512 || g.Xp / cb < want)) cb /= 2;
    if (cb * colb > 160 * 1024 || 3 * cb * tpc > 512) return fail(MM_E_ARG, "mesh too long along y");
    t.cb_y2 = cb;
    t.tpc_y2 = tpc;
  } else {
    const int tmin = tpc_for(g.Py);
    const int tpc = std::max(tmin, std::min(2 * tmin, 64));
    const size_t colb = (size_t)col_stride(g.Py) * csz;
    const long long rows = 3LL * g.nz * g.Xp;
    int cb = 16;
    while (cb > 1 && (cb * colb > budget || cb * tpc > 512 || rows / cb < want)) --cb;
    if (cb * colb > 160 * 1024 || cb * tpc > 512) return fail(MM_E_ARG, "mesh too long along y");
    t.cb_y = cb;
    t.tpc_y = tpc;
    const int tz = tpc_for(g.Pz);
    int qz = (int)(budget / (3 * col_stride(g.Pz) * csz));
    qz = std::min(qz, 512 / (3 * tz));
    qz = std::min(qz, 64);
    if (qz < 1) return fail(MM_E_ARG, "mesh too long along z for the z pass");
    t.qz = qz;
    t.tpc_z = tz;
  }
  return MM_OK;
}

template <typename T>
HotPlan<T> hot(const mm_plan* p) {
  HotPlan<T> h{};
  h.g = p->g;
  h.tu = p->tu;
  h.fp = (const FftPlan<T>*)p->fplans;
  h.twz = (const Cx<T>*)p->twz;
  h.post = (const Cx<T>*)p->post;
  h.kt = (const T*)p->kt;
  h.ncomp = p->ncomp;
  h.Sx = (Cx<T>*)p->Sx;
  h.Sy = (Cx<T>*)p->Sy;
  h.prm = p->prm;
  return h;
}

template <typename T>
mm_status upload_tables(mm_plan* p) {
  auto up = [&](void** dst, const std::vector<Cx<T>>& v) -> mm_status {
    HIPCHK(hipMalloc(dst, sizeof(Cx<T>) * std::max<size_t>(v.size(), 1)));
    HIPCHK(hipMemcpy(*dst, v.data(), sizeof(Cx<T>) * v.size(), hipMemcpyHostToDevice));
    return MM_OK;
  };
  MMCHK(up(&p->twx, twiddles<T>(p->g.Lx)));
  MMCHK(up(&p->twy, twiddles<T>(p->g.Py)));
  MMCHK(up(&p->twz, twiddles<T>(p->g.Pz)));
  std::vector<Cx<T>> post(p->g.Lx + 1);
  for (int k = 0; k <= p->g.Lx; ++k) {
    const double a = -2.0 * M_PI * k / (double)p->g.Px;
    post[k] = Cx<T>{(T)std::cos(a), (T)std::sin(a)};
  }
  MMCHK(up(&p->post, post));
  const FftPlan<T> fp[3] = {make_fft<T>(p->g.Lx, (const Cx<T>*)p->twx), make_fft<T>(p->g.Py, (const Cx<T>*)p->twy),
                            make_fft<T>(p->g.Pz, (const Cx<T>*)p->twz)};
  HIPCHK(hipMalloc(&p->fplans, sizeof(fp)));
  HIPCHK(hipMemcpy(p->fplans, fp, sizeof(fp), hipMemcpyHostToDevice));
  return MM_OK;
}

// Tensor spectrum on the device: Newell grid (FP64) -> 3-D FFT (FP64) -> fold -> cast.
template <typename T>
mm_status build_spectrum(mm_plan* p, hipStream_t s) {
  const Geo& g = p->g;
  double nodes[5][20] = {}, wts[5][20] = {};
  int nn[5];
  tent_rules(nodes, wts, nn);
  HIPCHK(setup_upload_gauss(nodes, wts, nn));
  const long long tot = (long long)g.Px * g.Py * g.Pz;
  Cx<double>* F = nullptr;
  HIPCHK(hipMalloc(&F, sizeof(Cx<double>) * tot * p->ncomp));
  std::vector<void*> tws;
  mm_status st = MM_OK;
  do {
    hipError_t e = setup_newell_grid(p->mesh, g.Px, g.Py, g.Pz, p->ncomp, F, s);
    if (e != hipSuccess) { st = fail(MM_E_HIP, std::string("newell grid: ") + hipGetErrorString(e)); break; }
    const int Ls[3] = {g.Px, g.Py, g.Pz};
    const long long inner[3] = {1, g.Px, (long long)g.Px * g.Py};
    const long long outer[3] = {(long long)g.Py * g.Pz * p->ncomp, (long long)g.Pz * p->ncomp, p->ncomp};
    for (int a = 0; a < 3 && st == MM_OK; ++a) {
      if (Ls[a] == 1) continue;
      std::vector<Cx<double>> tw = twiddles<double>(Ls[a]);
      void* d = nullptr;
      e = hipMalloc(&d, sizeof(Cx<double>) * tw.size());
      if (e != hipSuccess) { st = fail(MM_E_NOMEM, "twiddle table"); break; }
      tws.push_back(d);
      e = hipMemcpy(d, tw.data(), sizeof(Cx<double>) * tw.size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) { st = fail(MM_E_HIP, hipGetErrorString(e)); break; }
      FftPlan<double> fp = make_fft<double>(Ls[a], (const Cx<double>*)d);
      e = setup_fft_axis(F, inner[a], outer[a], fp, min_tpc(fp), s);
      if (e != hipSuccess) { st = fail(MM_E_HIP, std::string("tensor fft: ") + hipGetErrorString(e)); break; }
    }
    if (st != MM_OK) break;
    unsigned long long* stats = nullptr;
    e = hipMalloc(&stats, 2 * sizeof(unsigned long long));
    if (e != hipSuccess) { st = fail(MM_E_NOMEM, "stats"); break; }
    tws.push_back(stats);
    e = hipMemsetAsync(stats, 0, 2 * sizeof(unsigned long long), s);
    for (int c = 0; c < p->ncomp && e == hipSuccess; ++c)
      e = setup_extract<T>(F + (size_t)c * tot, g.Px, g.Py, g.Pz, c, (T*)p->kt, stats, s);
    if (e != hipSuccess) { st = fail(MM_E_HIP, std::string("extract: ") + hipGetErrorString(e)); break; }
    unsigned long long hs[2];
    e = hipMemcpyAsync(hs, stats, sizeof(hs), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { st = fail(MM_E_HIP, std::string("spectrum: ") + hipGetErrorString(e)); break; }
    double im, re;
    std::memcpy(&im, &hs[0], 8);
    std::memcpy(&re, &hs[1], 8);
    p->imag_ratio = re > 0 ? im / re : 0.0;
    if (!(p->imag_ratio < 1e-9)) st = fail(MM_E_HIP, "tensor spectrum is not real (symmetry broken)");
  } while (false);
  (void)hipStreamSynchronize(s);
  for (void* d : tws) (void)hipFree(d);
  (void)hipFree(F);
  return st;
}

void free_plan(mm_plan* p) {
  if (!p) return;
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  void* bufs[] = {p->Sx, p->Sy, p->kt, p->post, p->twx, p->twy, p->twz, p->fplans, p->prm, p->ctl, p->partial,
                  p->e5, p->replay, p->stage, p->nebH, p->nebB, p->nebS, p->nebP};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (p->hctl) (void)hipHostFree(p->hctl);
  if (p->he5) (void)hipHostFree(p->he5);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  delete p;
}

template <typename T>
mm_status eval_call(mm_plan* p, int batch, const void* m, const Epi<T>& epi, hipStream_t s,
                    hipEvent_t* ev = nullptr) {
  const bool demag = (p->terms & MM_DEMAG) != 0 && p->any_demag;
  HIPCHK(launch_eval<T>(hot<T>(p), batch, (const T*)m, epi, demag, s, ev));
  return MM_OK;
}


template <typename T>
Epi<T> epi_base(const mm_plan* p, int mode) {
  Epi<T> e{};
  e.mode = mode;
  e.inst_stride = 3 * p->g.N;
  return e;
}

mm_status common_checks(mm_plan* p, const mm_params* q, int batch) {
  if (!p) return fail(MM_E_ARG, "plan is null");
  if (batch < 1 || batch > p->maxb) return fail(MM_E_ARG, "batch must be in [1, max_batch]");
  return check_params(p, q, batch);
}

int pass_count(const mm_plan* p) {
  if (!((p->terms & MM_DEMAG) && p->any_demag)) return 1;
  return p->g.nz == 1 ? 3 : 5;
}

template <typename T>
mm_status profile_impl(mm_plan* p, int batch, const void* m, void* out, int reps, double* us, hipStream_t s) {
  const int np = pass_count(p);
  std::vector<hipEvent_t> ev((size_t)(np + 1) * reps);
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  mm_status st = MM_OK;
  Epi<T> e = epi_base<T>(p, MODE_RHS);
  e.out = (T*)out;
  for (int r = 0; r < reps && st == MM_OK; ++r) st = eval_call<T>(p, batch, m, e, s, ev.data() + (size_t)r * (np + 1));
  if (st == MM_OK) {
    hipError_t er = hipStreamSynchronize(s);
    if (er != hipSuccess) st = fail(MM_E_HIP, hipGetErrorString(er));
  }
  for (int i = 0; i < np && st == MM_OK; ++i) {
    double acc = 0.0;
    for (int r = 0; r < reps; ++r) {
      float ms = 0.f;
      hipError_t er = hipEventElapsedTime(&ms, ev[(size_t)r * (np + 1) + i], ev[(size_t)r * (np + 1) + i + 1]);
      if (er != hipSuccess) { st = fail(MM_E_HIP, hipGetErrorString(er)); break; }
      acc += ms;
    }
    us[i] = 1e3 * acc / reps;
  }
  for (auto& x : ev) (void)hipEventDestroy(x);
  return st;
}

// --- Dormand-Prince ---------------------------------------------------------
template <typename T>
T* stage_buf(mm_plan* p, int idx) {  // 0: ms0, 1: ms1, 2..8: k1..k7
  return (T*)p->stage + (size_t)idx * p->maxb * 3 * p->g.N;
}

template <typename T>
mm_status ensure_stage(mm_plan* p) {
  if (p->stage) return MM_OK;
  HIPCHK(hipMalloc(&p->stage, sizeof(T) * 9 * (size_t)p->maxb * 3 * p->g.N));
  return MM_OK;
}

template <typename T>
mm_status enqueue_attempt(mm_plan* p, int batch, T* m, hipStream_t s) {
  HIPCHK(launch_begin<T>(p->g, batch, m, stage_buf<T>(p, 0), stage_buf<T>(p, 1), stage_buf<T>(p, 2),
                         stage_buf<T>(p, 8), kDP.a[2][0], p->ctl, s));
  for (int st = 2; st <= 7; ++st) {
    const int in = (st % 2 == 0) ? 0 : 1;  // ms0 feeds even stages, ms1 odd stages
    Epi<T> e = epi_base<T>(p, st < 7 ? MODE_STAGE : MODE_ERROR);
    e.out = stage_buf<T>(p, 2 + st - 1);
    e.mbase = m;
    e.msn = stage_buf<T>(p, 1 - in);
    e.ctl = p->ctl;
    for (int j = 0; j < st - 1; ++j) e.kprev[j] = stage_buf<T>(p, 2 + j);
    e.nk = st;
    for (int j = 0; j < st; ++j) e.coef[j] = st < 7 ? kDP.a[st + 1][j] : kDP.e[j];
    MMCHK(eval_call<T>(p, batch, stage_buf<T>(p, in), e, s));
  }
  HIPCHK(launch_controller(p->ctl, batch, p->replay, s));
  return MM_OK;
}

template <typename T>
mm_status rk45_impl(mm_plan* p, const mm_params* q, int batch, void* mv, mm_rk45_state* st, double t_end,
                    long long max_steps, const double* replay_h, long long n_replay, bool single,
                    hipStream_t s) {
  MMCHK(ensure_stage<T>(p));
  MMCHK(upload_params(p, q, batch, s));
  T* m = (T*)mv;
  bool need_k1 = false;
  for (int b = 0; b < batch; ++b) {
    const mm_rk45_state& r = st[b];
    if (!(r.rtol > 0) || !is_fin(r.rtol) || !(r.h > 0) || !(r.h_min > 0) || !(r.h_max >= r.h_min) ||
        !is_fin(r.t) || !is_fin(r.h) || !is_fin(r.h_max))
      return fail(MM_E_ARG, "invalid rk45 state (rtol, h, h_min, h_max)");
    if (!r.fsal_valid) need_k1 = true;
  }
  if (replay_h) {
    if (n_replay < 1) return fail(MM_E_ARG, "n_replay must be >= 1");
    for (long long i = 0; i < n_replay; ++i)
      if (!(replay_h[i] > 0) || !is_fin(replay_h[i])) return fail(MM_E_ARG, "replay step sizes must be > 0");
    if (n_replay > p->replay_cap) {
      if (p->replay) (void)hipFree(p->replay);
      p->replay = nullptr;
      HIPCHK(hipMalloc(&p->replay, sizeof(double) * n_replay));
      p->replay_cap = n_replay;
      if (p->gexec) { (void)hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
    }
    HIPCHK(hipMemcpy(p->replay, replay_h, sizeof(double) * n_replay, hipMemcpyHostToDevice));
  }
  for (int b = 0; b < batch; ++b) {
    const mm_rk45_state& r = st[b];
    DevCtl& c = p->hctl[b];
    std::memset(&c, 0, sizeof(c));
    c.t = r.t; c.h = r.h; c.rtol = r.rtol; c.h_min = r.h_min; c.h_max = r.h_max;
    c.t_end = replay_h ? HUGE_VAL : t_end;
    c.n_accept = r.n_accept; c.n_reject = r.n_reject;
    c.max_attempt = max_steps;
    c.replay_n = replay_h ? n_replay : 0;
    if (replay_h) {
      c.h_att = replay_h[0];
    } else {
      c.h_att = std::min(std::min(r.h, r.h_max), t_end - r.t);
      if (!(t_end - r.t > r.h_min)) c.done = 1;  // arrived (a remainder below h_min counts as arrived)
      else if (c.h_att < r.h_min) return fail(MM_E_STEP_UNDERFLOW, "initial step below h_min");
    }
  }
  HIPCHK(hipMemcpyAsync(p->ctl, p->hctl, sizeof(DevCtl) * batch, hipMemcpyHostToDevice, s));
  long long extra_rhs = 0;
  if (need_k1) {
    Epi<T> e = epi_base<T>(p, MODE_RHS);
    e.out = stage_buf<T>(p, 2);
    MMCHK(eval_call<T>(p, batch, m, e, s));
    extra_rhs = 1;
  }
  const bool dbg = getenv("MMX_DEBUG_CTL") != nullptr;
  auto dump = [&](const char* tag) {
    std::vector<DevCtl> v(batch);
    (void)hipMemcpyAsync(v.data(), p->ctl, sizeof(DevCtl) * batch, hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
    fprintf(stderr, "[ctl %s] t=%g h=%g h_att=%g h_max=%g h_min=%g t_end=%g rtol=%g err=%g na=%lld nr=%lld done=%d st=%d\n",
            tag, v[0].t, v[0].h, v[0].h_att, v[0].h_max, v[0].h_min, v[0].t_end, v[0].rtol, v[0].last_err,
            v[0].n_accept, v[0].n_reject, v[0].done, v[0].status);
  };
  if (dbg) dump("upload");
  if (single) {
    MMCHK(enqueue_attempt<T>(p, batch, m, s));
    if (dbg) dump("attempt");
  } else {
    const int K = 8;  // attempts per graph launch between host polls
    if (!p->gexec || p->g_m != mv || p->g_batch != batch) {
      if (p->gexec) { (void)hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
      HIPCHK(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
      mm_status cs = MM_OK;
      for (int k = 0; k < K && cs == MM_OK; ++k) cs = enqueue_attempt<T>(p, batch, m, p->cap);
      hipGraph_t graph = nullptr;
      hipError_t ee = hipStreamEndCapture(p->cap, &graph);
      if (cs != MM_OK) { if (graph) (void)hipGraphDestroy(graph); return cs; }
      if (ee != hipSuccess) return fail(MM_E_HIP, std::string("capture: ") + hipGetErrorString(ee));
      ee = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ee != hipSuccess) { p->gexec = nullptr; return fail(MM_E_HIP, std::string("instantiate: ") + hipGetErrorString(ee)); }
      p->g_m = mv;
      p->g_batch = batch;
      p->g_steps = K;
    }
    for (;;) {
      HIPCHK(hipGraphLaunch(p->gexec, s));
      HIPCHK(hipMemcpyAsync(p->hctl, p->ctl, sizeof(DevCtl) * batch, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (dbg) dump("poll");
      bool all = true;
      for (int b = 0; b < batch; ++b) all = all && p->hctl[b].done;
      if (all) break;
    }
  }
  // finish: project the last accepted y5 and move k7 into k1
  HIPCHK(launch_begin<T>(p->g, batch, m, stage_buf<T>(p, 0), stage_buf<T>(p, 1), stage_buf<T>(p, 2),
                         stage_buf<T>(p, 8), kDP.a[2][0], p->ctl, s));
  HIPCHK(hipMemcpyAsync(p->hctl, p->ctl, sizeof(DevCtl) * batch, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  mm_status worst = MM_OK;
  for (int b = 0; b < batch; ++b) {
    const DevCtl& c = p->hctl[b];
    mm_rk45_state& r = st[b];
    r.t = c.t;
    r.h = c.h;
    const long long attempts = c.n_attempt;
    r.n_rhs += 6 * attempts + extra_rhs;
    r.n_accept = c.n_accept;
    r.n_reject = c.n_reject;
    r.last_err = c.last_err;
    r.last_accepted = c.last_accepted;
    r.fsal_valid = 1;
    if (c.status != MM_OK && worst == MM_OK) worst = (mm_status)c.status;
  }
  if (worst != MM_OK) return fail(worst, "integration stopped: " + std::string(mm_status_string(worst)));
  return MM_OK;
}

template <typename T>
mm_status energy_impl(mm_plan* p, const mm_params* q, int batch, const void* m, double* E, hipStream_t s) {
  MMCHK(upload_params(p, q, batch, s));
  Epi<T> e = epi_base<T>(p, MODE_ENERGY);
  e.partial = p->partial;
  MMCHK(eval_call<T>(p, batch, m, e, s));
  HIPCHK(launch_energy_reduce(p->partial, batch, eval_blocks_per_inst(p->g, p->tu), p->e5, s));
  HIPCHK(hipMemcpyAsync(p->he5, p->e5, sizeof(double) * 5 * batch, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int b = 0; b < batch; ++b) {
    const double c = kMu0 * q[b].Ms * p->g.dV;
    for (int k = 0; k < 5; ++k) E[5 * b + k] = -(k == 4 ? 1.0 : 0.5) * c * p->he5[5 * b + k];
  }
  return MM_OK;
}

template <typename T>
mm_status neb_impl(mm_plan* p, const mm_params* q, void* images, int n_img, double k, double h, long long n_iter,
                   double* E_out, hipStream_t s) {
  const size_t S = 3 * (size_t)p->g.N;
  if (!p->nebH) {
    HIPCHK(hipMalloc(&p->nebH, sizeof(T) * S * p->maxb));
    HIPCHK(hipMalloc(&p->nebB, sizeof(T) * S * p->maxb));
    const long long bpi = (p->g.N + 255) / 256;
    HIPCHK(hipMalloc(&p->nebS, sizeof(double) * 3 * p->maxb));
    HIPCHK(hipMalloc(&p->nebP, sizeof(double) * 3 * p->maxb * bpi));
  }
  std::vector<mm_params> qs(n_img, *q);
  MMCHK(upload_params(p, qs.data(), n_img, s));
  T* A = (T*)images;
  T* B = (T*)p->nebB;
  HIPCHK(hipMemcpyAsync(B, A, sizeof(T) * S * n_img, hipMemcpyDeviceToDevice, s));
  const double cq = -0.5 * kMu0 * q->Ms * p->g.dV, cz = -kMu0 * q->Ms * p->g.dV;
  const double hg2 = h * (-q->alpha * q->gamma / (1 + q->alpha * q->alpha));
  auto iteration = [&](T* cur, T* nxt) -> mm_status {
    Epi<T> e = epi_base<T>(p, MODE_FIELD_ENERGY);
    e.out = (T*)p->nebH;
    e.partial = p->partial;
    MMCHK(eval_call<T>(p, n_img, cur, e, s));
    HIPCHK(launch_energy_reduce(p->partial, n_img, eval_blocks_per_inst(p->g, p->tu), p->e5, s));
    HIPCHK(launch_neb<T>(p->g, n_img, cur, nxt, (const T*)p->nebH, p->e5, cq, cz, p->nebS, p->nebP, k, hg2, 0, s));
    HIPCHK(launch_neb<T>(p->g, n_img, cur, nxt, (const T*)p->nebH, p->e5, cq, cz, p->nebS, p->nebP, k, hg2, 1, s));
    return MM_OK;
  };
  // two iterations per captured graph (A -> B -> A)
  hipGraphExec_t ge = nullptr;
  if (n_iter >= 2) {
    HIPCHK(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    hipStream_t keep = s;
    s = p->cap;
    mm_status cs = iteration(A, B);
    if (cs == MM_OK) cs = iteration(B, A);
    s = keep;
    hipGraph_t graph = nullptr;
    hipError_t ee = hipStreamEndCapture(p->cap, &graph);
    if (cs != MM_OK) { if (graph) (void)hipGraphDestroy(graph); return cs; }
    if (ee != hipSuccess) return fail(MM_E_HIP, std::string("capture: ") + hipGetErrorString(ee));
    ee = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ee != hipSuccess) return fail(MM_E_HIP, std::string("instantiate: ") + hipGetErrorString(ee));
  }
  long long it = 0;
  mm_status st = MM_OK;
  for (; it + 2 <= n_iter && st == MM_OK; it += 2) {
    hipError_t ee = hipGraphLaunch(ge, s);
    if (ee != hipSuccess) st = fail(MM_E_HIP, hipGetErrorString(ee));
  }
  if (st == MM_OK && it < n_iter) {
    st = iteration(A, B);
    if (st == MM_OK) {
      hipError_t ee = hipMemcpyAsync(A, B, sizeof(T) * S * n_img, hipMemcpyDeviceToDevice, s);
      if (ee != hipSuccess) st = fail(MM_E_HIP, hipGetErrorString(ee));
    }
  }
  if (ge) (void)hipGraphExecDestroy(ge);
  if (st != MM_OK) return st;
  HIPCHK(hipMemcpyAsync(p->he5, p->e5, sizeof(double) * 5 * n_img, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (E_out)
    for (int n = 0; n < n_img; ++n) {
      const double* v = p->he5 + 5 * n;
      E_out[n] = cq * (v[0] + v[1] + v[2] + v[3]) + cz * v[4];
    }
  return MM_OK;
}

}  // namespace

extern "C" {

const char* mm_status_string(mm_status s) {
  switch (s) {
    case MM_OK: return "ok";
    case MM_E_ARG: return "invalid argument";
    case MM_E_NOMEM: return "out of device memory";
    case MM_E_HIP: return "HIP runtime error";
    case MM_E_NONFINITE: return "non-finite value in the step error";
    case MM_E_STEP_UNDERFLOW: return "step size below h_min";
    case MM_E_MAXSTEPS: return "maximum number of steps reached";
    case MM_E_STATE: return "invalid plan state";
  }
  return "unknown status";
}

const char* mm_last_error(void) { return g_err.c_str(); }

mm_status mm_plan_create(mm_plan** out, const mm_mesh* mesh, mm_precision prec, uint32_t terms, int32_t max_batch,
                         void* hip_stream) {
  if (!out) return fail(MM_E_ARG, "out is null");
  *out = nullptr;
  MMCHK(check_mesh(mesh));
  if (prec != MM_F32 && prec != MM_F64) return fail(MM_E_ARG, "precision must be MM_F32 or MM_F64");
  if (terms & ~MM_ALL_TERMS) return fail(MM_E_ARG, "unknown term bits");
  if (max_batch < 1) return fail(MM_E_ARG, "max_batch must be >= 1");
  hipStream_t s = (hipStream_t)hip_stream;
  mm_plan* p = new mm_plan();
  p->mesh = *mesh;
  p->prec = prec;
  p->terms = terms;
  p->maxb = max_batch;
  p->ncomp = mesh->nz == 1 ? 4 : 6;
  p->csz = prec == MM_F32 ? sizeof(Cx<float>) : sizeof(Cx<double>);
  p->rsz = prec == MM_F32 ? sizeof(float) : sizeof(double);
  Geo& g = p->g;
  g.nx = mesh->nx; g.ny = mesh->ny; g.nz = mesh->nz;
  g.Px = pick_padded(g.nx, true);
  g.Py = pick_padded(g.ny, false);
  g.Pz = pick_padded(g.nz, false);
  g.Lx = g.Px / 2;
  g.Xp = g.Lx + 1;
  g.Ky = g.Py / 2 + 1;
  g.Kz = g.Pz / 2 + 1;
  g.N = (long long)g.nx * g.ny * g.nz;
  g.sx = 3LL * g.nz * g.Xp * g.ny;
  g.sy = 3LL * g.nz * g.Xp * g.Py;
  g.dV = mesh->dx * mesh->dy * mesh->dz;
  mm_status st = choose_tuning(p);
  if (st != MM_OK) { free_plan(p); return st; }
  auto alloc = [&](void** d, size_t bytes) -> mm_status {
    hipError_t e = hipMalloc(d, std::max<size_t>(bytes, 16));
    if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? MM_E_NOMEM : MM_E_HIP, hipGetErrorString(e));
    return MM_OK;
  };
  do {
    hipError_t e = hipGetDevice(&p->devid);
    if (e != hipSuccess) { st = fail(MM_E_HIP, std::string("no HIP device: ") + hipGetErrorString(e)); break; }
    e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e != hipSuccess) { st = fail(MM_E_HIP, hipGetErrorString(e)); break; }
    const int bpi = eval_blocks_per_inst(g, p->tu);
    if ((st = alloc((void**)&p->prm, sizeof(DevParams) * max_batch)) != MM_OK) break;
    if ((st = alloc((void**)&p->ctl, sizeof(DevCtl) * max_batch)) != MM_OK) break;
    if ((st = alloc((void**)&p->partial, sizeof(double) * 5 * (size_t)bpi * max_batch)) != MM_OK) break;
    if ((st = alloc((void**)&p->e5, sizeof(double) * 5 * max_batch)) != MM_OK) break;
    e = hipHostMalloc((void**)&p->hctl, sizeof(DevCtl) * max_batch);
    if (e != hipSuccess) { st = fail(MM_E_NOMEM, "pinned host buffer"); break; }
    e = hipHostMalloc((void**)&p->he5, sizeof(double) * 5 * max_batch);
    if (e != hipSuccess) { st = fail(MM_E_NOMEM, "pinned host buffer"); break; }
    std::memset(p->hctl, 0, sizeof(DevCtl) * max_batch);
    if (terms & MM_DEMAG) {
      if ((st = alloc(&p->Sx, p->csz * g.sx * max_batch)) != MM_OK) break;
      if (g.nz > 1 && (st = alloc(&p->Sy, p->csz * g.sy * max_batch)) != MM_OK) break;
      if ((st = alloc(&p->kt, p->rsz * p->ncomp * (size_t)g.Kz * g.Xp * g.Ky)) != MM_OK) break;
      st = prec == MM_F32 ? upload_tables<float>(p) : upload_tables<double>(p);
      if (st != MM_OK) break;
      st = prec == MM_F32 ? build_spectrum<float>(p, s) : build_spectrum<double>(p, s);
      if (st != MM_OK) break;
    }
  } while (false);
  if (st != MM_OK) { free_plan(p); return st; }
  *out = p;
  return MM_OK;
}

mm_status mm_plan_destroy(mm_plan* plan) {
  if (!plan) return fail(MM_E_ARG, "plan is null");
  (void)hipDeviceSynchronize();
  free_plan(plan);
  return MM_OK;
}

mm_status mm_plan_padded(const mm_plan* p, int32_t* Px, int32_t* Py, int32_t* Pz) {
  if (!p || !Px || !Py || !Pz) return fail(MM_E_ARG, "null argument");
  *Px = p->g.Px; *Py = p->g.Py; *Pz = p->g.Pz;
  return MM_OK;
}

mm_status mm_demag_tensor(const mm_mesh* mesh, const int32_t* disp, int64_t n, double* out, void* hip_stream) {
  MMCHK(check_mesh(mesh));
  if (n < 0) return fail(MM_E_ARG, "n must be >= 0");
  if (n > 0 && (!disp || !out)) return fail(MM_E_ARG, "null pointer");
  double nodes[5][20] = {}, wts[5][20] = {};
  int nn[5];
  tent_rules(nodes, wts, nn);
  HIPCHK(setup_upload_gauss(nodes, wts, nn));
  hipStream_t s = (hipStream_t)hip_stream;
  HIPCHK(setup_newell_list(*mesh, disp, n, out, s));
  HIPCHK(hipStreamSynchronize(s));
  return MM_OK;
}

mm_status mm_effective_field(mm_plan* p, const mm_params* q, int32_t batch, const void* m, void* H,
                             void* hip_stream) {
  MMCHK(common_checks(p, q, batch));
  if (!m || !H) return fail(MM_E_ARG, "null array");
  hipStream_t s = (hipStream_t)hip_stream;
  MMCHK(upload_params(p, q, batch, s));
  if (p->prec == MM_F32) {
    Epi<float> e = epi_base<float>(p, MODE_FIELD);
    e.out = (float*)H;
    return eval_call<float>(p, batch, m, e, s);
  }
  Epi<double> e = epi_base<double>(p, MODE_FIELD);
  e.out = (double*)H;
  return eval_call<double>(p, batch, m, e, s);
}

mm_status mm_llg_rhs(mm_plan* p, const mm_params* q, int32_t batch, const void* m, void* dmdt, void* hip_stream) {
  MMCHK(common_checks(p, q, batch));
  if (!m || !dmdt) return fail(MM_E_ARG, "null array");
  hipStream_t s = (hipStream_t)hip_stream;
  MMCHK(upload_params(p, q, batch, s));
  if (p->prec == MM_F32) {
    Epi<float> e = epi_base<float>(p, MODE_RHS);
    e.out = (float*)dmdt;
    return eval_call<float>(p, batch, m, e, s);
  }
  Epi<double> e = epi_base<double>(p, MODE_RHS);
  e.out = (double*)dmdt;
  return eval_call<double>(p, batch, m, e, s);
}

mm_status mm_energy(mm_plan* p, const mm_params* q, int32_t batch, const void* m, double* E_out, void* hip_stream) {
  MMCHK(common_checks(p, q, batch));
  if (!m || !E_out) return fail(MM_E_ARG, "null array");
  hipStream_t s = (hipStream_t)hip_stream;
  return p->prec == MM_F32 ? energy_impl<float>(p, q, batch, m, E_out, s)
                           : energy_impl<double>(p, q, batch, m, E_out, s);
}

mm_status mm_rk45_step(mm_plan* p, const mm_params* q, int32_t batch, void* m, mm_rk45_state* st,
                       void* hip_stream) {
  MMCHK(common_checks(p, q, batch));
  if (!m || !st) return fail(MM_E_ARG, "null array");
  hipStream_t s = (hipStream_t)hip_stream;
  const long long cap = 1;
  return p->prec == MM_F32 ? rk45_impl<float>(p, q, batch, m, st, HUGE_VAL, cap + 1, nullptr, 0, true, s)
                           : rk45_impl<double>(p, q, batch, m, st, HUGE_VAL, cap + 1, nullptr, 0, true, s);
}

mm_status mm_rk45_run(mm_plan* p, const mm_params* q, int32_t batch, void* m, mm_rk45_state* st, double t_end,
                      int64_t max_steps, const double* replay_h, int64_t n_replay, void* hip_stream) {
  MMCHK(common_checks(p, q, batch));
  if (!m || !st) return fail(MM_E_ARG, "null array");
  if (max_steps < 1) return fail(MM_E_ARG, "max_steps must be >= 1");
  if (!replay_h && !is_fin(t_end)) return fail(MM_E_ARG, "t_end must be finite");
  hipStream_t s = (hipStream_t)hip_stream;
  return p->prec == MM_F32
             ? rk45_impl<float>(p, q, batch, m, st, t_end, max_steps, replay_h, n_replay, false, s)
             : rk45_impl<double>(p, q, batch, m, st, t_end, max_steps, replay_h, n_replay, false, s);
}

mm_status mm_profile_passes(mm_plan* p, const mm_params* q, int32_t batch, const void* m, void* work, int32_t reps,
                            double* us_out, int32_t* n_pass, void* hip_stream) {
  MMCHK(common_checks(p, q, batch));
  if (!m || !work || !us_out || !n_pass) return fail(MM_E_ARG, "null argument");
  if (reps < 1) return fail(MM_E_ARG, "reps must be >= 1");
  hipStream_t s = (hipStream_t)hip_stream;
  MMCHK(upload_params(p, q, batch, s));
  *n_pass = pass_count(p);
  return p->prec == MM_F32 ? profile_impl<float>(p, batch, m, work, reps, us_out, s)
                           : profile_impl<double>(p, batch, m, work, reps, us_out, s);
}

mm_status mm_neb_run(mm_plan* p, const mm_params* q, void* images, int32_t n_img, double k_spring, double h,
                     int64_t n_iter, double* E_out, void* hip_stream) {
  if (!p) return fail(MM_E_ARG, "plan is null");
  if (n_img < 3 || n_img > p->maxb) return fail(MM_E_ARG, "n_img must be in [3, max_batch]");
  MMCHK(check_params(p, q, 1));
  if (!images) return fail(MM_E_ARG, "images is null");
  if (!is_fin(k_spring) || !is_fin(h) || h <= 0 || n_iter < 1) return fail(MM_E_ARG, "invalid k_spring, h or n_iter");
  hipStream_t s = (hipStream_t)hip_stream;
  return p->prec == MM_F32 ? neb_impl<float>(p, q, images, n_img, k_spring, h, n_iter, E_out, s)
                           : neb_impl<double>(p, q, images, n_img, k_spring, h, n_iter, E_out, s);
}

}  // extern "C"
