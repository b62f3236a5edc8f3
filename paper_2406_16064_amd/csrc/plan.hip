// Host runtime and C interface (include/mm.h).
//
// An engine owns one or more geometry groups (instances that share a mesh:
// padded grid, radix plans, twiddles, launch shapes, tensor spectrum, spectral
// work buffers) plus the per-instance parameter and controller arrays.  A plan
// is an engine with one group; a batch has one group per distinct mesh, and
// every pass of an evaluation is a single launch over all groups.  On top:
// validation, effective field / LL / energy calls, device-controlled
// Dormand-Prince runs with HIP-graph replay, and the NEB driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fft_core.hpp"
#include "kernels.hpp"
#include "potential.hpp"
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

// Padded length of the scalar-potential route: the smallest 3-smooth P >= 2n
// (even along x), 1 for n = 1 off x (the 2n vertex - cell displacements must
// all fit).
int pick_padded_pot(int n, bool even) {
  if (n == 1 && !even) return 1;
  for (int P = 2 * n;; ++P)
    if (smooth3(P) && (!even || P % 2 == 0)) return P;
}

// Radices of a 3-smooth length: the power of two as 8s (a remainder as 4, 4+4
// or 2), the 3s placed after the first stage.  Where that takes more than three stages of powers of
// two, 16s replace the 8s when allow16 (the y passes, whose kernels carry the
// radix-16 code): one LDS round trip less (measured: the 1024-point y
// transforms gain, while at 512 and below the larger butterfly's registers
// cost more than the stage it saves).
std::vector<int> radices(int L, bool allow16) {
  std::vector<int> r;
  int a = 0, b = 0;
  while (L % 2 == 0) { L /= 2; ++a; }
  while (L % 3 == 0) { L /= 3; ++b; }
  for (int s = 0; s < p2_nst(a, allow16); ++s) r.push_back(p2_radix(a, allow16, s));
  // radix-3 stages right after the first stage: spans stay multiples of the
  // first radix and both ends keep an even radix where L allows
  r.insert(r.empty() ? r.end() : r.begin() + 1, b, 3);
  return r;
}

template <typename T>
FftPlan<T> make_fft(int L, const Cx<T>* tw, bool allow16 = false) {
  FftPlan<T> p{};
  p.L = L;
  p.tw = tw;
  std::vector<int> r = L > 1 ? radices(L, allow16) : std::vector<int>{};
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


mm_status check_mesh(const mm_mesh* m) {
  if (!m) return fail(MM_E_ARG, "mesh is null");
  if (m->nx < 2 || m->ny < 1 || m->nz < 1 || m->nx > 1024 || m->ny > 1024 || m->nz > 1024)
    return fail(MM_E_ARG, "mesh sizes must satisfy 2 <= nx <= 1024, 1 <= ny, nz <= 1024");
  if (!(is_fin(m->dx) && is_fin(m->dy) && is_fin(m->dz)) || m->dx <= 0 || m->dy <= 0 || m->dz <= 0)
    return fail(MM_E_ARG, "cell sizes must be finite and > 0");
  return MM_OK;
}

// The hot-path kernels address one instance's [3][N] arrays with 32-bit byte
// offsets.
mm_status check_cells(const mm_mesh* m, mm_precision prec) {
  const double bytes = 3.0 * m->nx * m->ny * m->nz * (prec == MM_F64 ? 8.0 : 4.0);
  if (bytes >= 4294967296.0) return fail(MM_E_ARG, "mesh too large: 3 nx ny nz element bytes must stay below 4 GiB");
  return MM_OK;
}

int pow2ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

constexpr int kEpiSlots = 9;  // 0: single call, 1: first slope, 2..7: stages, 8: step begin

// One geometry: mesh, padded grid, launch shapes, tables, spectrum and the
// spectral / integrator work buffers of up to `cap` instances.
struct Group {
  mm_mesh mesh;
  Geo g;
  Tuning tu;
  int ncomp = 4;
  int cap = 0;        // instances the work buffers hold
  int stage_cap = 0;  // instances the Runge-Kutta buffers hold
  int mbuf_cap = 0;
  void* Sx = nullptr;
  void* Sy = nullptr;
  void* kt = nullptr;
  void* post = nullptr;
  void* twx = nullptr;
  void* twy = nullptr;
  void* twz = nullptr;
  void* kpot = nullptr;   // scalar-potential route: folded kernel spectrum [3][Kz][Xp][Ky]
  void* phx = nullptr;    // half-cell phase tables exp(-i pi k / P) along x, y, z
  void* phy = nullptr;
  void* phz = nullptr;
  void* cells = nullptr;  // cell-based material [cells_cap][3][N] (Ms, A, D), plan precision
  std::vector<char> cells_set;  // slot i holds data
  void* stage = nullptr;  // ms0, ms1, k1..k7: 9 x stage_cap x 3N
  void* mbuf = nullptr;   // contiguous m of the group's instances (batch runs)
  long long tuned_for = 0;  // batch and NEB runs: the launch rows the launch shapes were chosen for
  bool user_shapes = false;  // shapes set by mm_plan_set_shapes or the autotuner: kept as they are
  double imag_ratio = 0.0;
};

}  // namespace

struct Engine {
  mm_precision prec;
  uint32_t terms;
  size_t csz, rsz;
  std::vector<Group> groups;
  int inst_cap = 0;  // instances the parameter / controller arrays hold
  int part_cap = 0;  // doubles the energy partial buffer holds
  hipStream_t cap = nullptr;  // capture stream (default priority)
  DevParams* prm = nullptr;
  DevCtl* ctl = nullptr;
  double* partial = nullptr;
  double* e5 = nullptr;
  double* replay = nullptr;
  long long replay_cap = 0;
  void* dhot = nullptr;  // device HotPlan<T>[kMaxGroups]
  void* depi = nullptr;  // device Epi<T>[kEpiSlots][kMaxGroups]
  DevCtl* hctl = nullptr;
  DevCtl* hctl2 = nullptr;      // second host copy of the controllers (graph launches overlap host polls)
  hipEvent_t poll_ev[2] = {nullptr, nullptr};
  double* he5 = nullptr;
  bool any_demag = false;
  bool any_pot = false;     // some instance of the current call uses the scalar-potential demag
  bool use_general = false;  // the current call runs the general-material form (kGeneralTerms)
  // graph cache of the Dormand-Prince attempt sequence
  hipGraphExec_t gexec = nullptr;
  std::vector<const void*> g_key;
  // The first slopes k1 held in the stage buffers belong to the state arrays of
  // the last adaptive run (its m pointers and instance counts).  Heun, steepest
  // descent, the autotuner and a reallocation of the stage buffers overwrite
  // them and clear k1_ok; a run on other arrays or without k1_ok recomputes k1
  // whatever the caller's fsal_valid says.
  std::vector<const void*> k1_key;
  bool k1_ok = false;
  std::vector<const void*> batch_who;  // batches: instance arrays of the last run
  // NEB scratch (group 0)
  void* nebH = nullptr;
  void* nebB = nullptr;
  double* nebS = nullptr;
  double* nebP = nullptr;
  int neb_cap = 0;
};

struct mm_plan {
  Engine e;
  int maxb;
};

struct mm_batch {
  Engine e;
};

namespace {

mm_status check_params(const Engine& E, const mm_params* q, int n) {
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
    if ((r.terms & ~E.terms) != 0) return fail(MM_E_ARG, "params enable a term the plan was not built for");
    if ((r.terms & MM_ANIS_UNIAXIAL) && r.u[0] == 0 && r.u[1] == 0 && r.u[2] == 0)
      return fail(MM_E_ARG, "easy axis must be non-zero");
    if (r.terms & MM_INTERLAYER) {
      const double v2[] = {r.J_rkky, r.D_int[0], r.D_int[1], r.D_int[2]};
      for (double x : v2)
        if (!is_fin(x)) return fail(MM_E_ARG, "interlayer parameters must be finite");
    }
    if (r.terms & MM_STT_SOT) {
      const double v2[] = {r.a_J, r.b_J, r.p[0], r.p[1], r.p[2]};
      for (double x : v2)
        if (!is_fin(x)) return fail(MM_E_ARG, "spin-orbit torque parameters must be finite");
      if (r.p[0] == 0 && r.p[1] == 0 && r.p[2] == 0) return fail(MM_E_ARG, "polarisation p must be non-zero");
    }
    if (r.terms & MM_STT_ZL) {
      const double v2[] = {r.u_zl[0], r.u_zl[1], r.u_zl[2], r.beta};
      for (double x : v2)
        if (!is_fin(x)) return fail(MM_E_ARG, "Zhang-Li parameters must be finite");
    }
  }
  return MM_OK;
}

// Terms that run in the general-material form of the inverse-x epilogue.
constexpr uint32_t kGeneralTerms = MM_CELLS | MM_INTERLAYER | MM_STT_SOT | MM_STT_ZL;

// general: the instance runs in the general-material form (unit coefficients;
// each cell applies its Ms, A_ij, D_ij, and the extra terms' coefficients)
DevParams dev_params(const mm_params& r, const Group& G, bool general) {
  DevParams o;
  std::memset(&o, 0, sizeof(o));
  const double P = (double)G.g.Px * G.g.Py * G.g.Pz;
  o.Ms = r.Ms;
  const double c = kMu0 * r.Ms;
  o.cex[0] = 2 * r.A / (c * G.mesh.dx * G.mesh.dx);
  o.cex[1] = 2 * r.A / (c * G.mesh.dy * G.mesh.dy);
  o.cex[2] = 2 * r.A / (c * G.mesh.dz * G.mesh.dz);
  o.cdmi[0] = r.D / (c * G.mesh.dx);
  o.cdmi[1] = r.D / (c * G.mesh.dy);
  o.cdmi[2] = r.D / (c * G.mesh.dz);
  o.can = 2 * r.Ku / c;
  const double un = std::sqrt(r.u[0] * r.u[0] + r.u[1] * r.u[1] + r.u[2] * r.u[2]);
  for (int k = 0; k < 3; ++k) {
    o.u[k] = un > 0 ? r.u[k] / un : 0.0;
    o.H[k] = r.H[k];
  }
  if (general) {  // unit coefficients: the kernels apply each cell's Ms, A_ij, D_ij
    for (int a = 0; a < 3; ++a) {
      const double d = a == 0 ? G.mesh.dx : a == 1 ? G.mesh.dy : G.mesh.dz;
      o.cex[a] = 2.0 / (kMu0 * d * d);
      o.cdmi[a] = 1.0 / (kMu0 * d);
      o.zu[a] = (r.terms & MM_STT_ZL) ? r.u_zl[a] / (r.gamma * d) : 0.0;
    }
    o.can = 2 * r.Ku / kMu0;
    o.Mu = r.Ms;
    o.Au = r.A;
    o.Du = r.D;
    if (r.terms & MM_INTERLAYER) {
      o.k_lo = r.k_lo;
      o.k_hi = r.k_hi;
      o.crk = r.J_rkky / (kMu0 * G.mesh.dz);
      for (int a = 0; a < 3; ++a) o.cdi[a] = r.D_int[a] / (kMu0 * G.mesh.dz);
    } else {
      o.k_lo = o.k_hi = -1;
    }
    if (r.terms & MM_STT_SOT) {
      const double pn = std::sqrt(r.p[0] * r.p[0] + r.p[1] * r.p[1] + r.p[2] * r.p[2]);
      o.sa = r.a_J / r.gamma;
      o.sb = r.b_J / r.gamma;
      for (int a = 0; a < 3; ++a) o.sp[a] = r.p[a] / pn;
    }
    o.zbeta = r.beta;
  }
  o.g1 = -r.gamma / (1 + r.alpha * r.alpha);
  o.g2 = -r.alpha * r.gamma / (1 + r.alpha * r.alpha);
  o.demag_scale = (r.terms & MM_CELLS) ? -1.0 / P : -r.Ms / P;  // cells: Ms is inside M
  if (r.terms & MM_DEMAG_POTENTIAL) o.demag_scale = r.Ms / P;   // potential route: u = S * (Ms m)
  o.terms = r.terms;
  return o;
}

// Launch shapes of one group.  Each workgroup keeps its LDS within 80 KiB (two
// per CU), the per-thread butterfly budget of the transforms is respected, and
// tiles shrink until a pass has about 4 workgroups per CU (small meshes) or
// reach their coalescing-friendly maximum (large meshes).
// launch_rows: rows (nz ny per instance) of every group of a batch launch, 0
// for one instance of this group alone: the workgroup count aimed at counts
// the whole launch, so that the meshes of a large batch take rows per
// workgroup up to the LDS and thread limits.
mm_status choose_tuning(Group& G, mm_precision prec, size_t csz, long long launch_rows = 0) {
  const Geo& g = G.g;
  Tuning& t = G.tu;
  const size_t budget = 80 * 1024;
  const long long want = 4 * 256;  // workgroups per pass worth aiming for
  auto tpc_for = [&](int L, bool allow16 = false) {
    if (prec == MM_F32) return min_tpc(make_fft<float>(L, nullptr, allow16));
    return min_tpc(make_fft<double>(L, nullptr, allow16));
  };
  const int tpx = tpc_for(g.Lx);
  const size_t rowb = (size_t)col_stride(g.Lx) * csz;
  const size_t xtab = (size_t)(2 * g.Lx + 1) * csz;  // twiddle + post tables in LDS
  const size_t ytab = (size_t)g.Py * csz;
  const size_t ktab2 = y2d_tensor_in_lds(g) ? (size_t)4 * g.Ky * (csz / 2) : 0;  // per kx column of the fused 2-D y pass
  {  // forward x: rows of one component
    const long long rows = 3LL * (launch_rows > 0 ? launch_rows : (long long)g.nz * g.ny);
    int ty = 16;
    while (ty > 1 && ((size_t)ty * rowb + xtab > budget || ty * tpx > 512 || rows / ty < want)) ty /= 2;
    while (ty > g.ny) ty /= 2;  // a power of two (the kernels split rows by shifts)
    if ((size_t)ty * rowb + xtab > 160 * 1024 || ty * tpx > 512) return fail(MM_E_ARG, "mesh too long along x");
    t.ty_f = ty;
    t.nt_f = std::min(512, std::max(64, pow2ceil(std::max(ty * tpx, ty * g.Lx / 4))));
    t.tpc_f = t.nt_f / ty;
  }
  {  // inverse x + epilogue: rows of all 3 components (3 columns per row)
    const long long rows = launch_rows > 0 ? launch_rows : (long long)g.nz * g.ny;
    int ty = 16;
    while (ty > 1 && ((size_t)3 * ty * rowb + xtab > budget || 3 * ty * tpx > 512 || rows / ty < want)) ty /= 2;
    while (ty > g.ny) ty /= 2;  // a power of two (the kernels split rows by shifts)
    if ((size_t)3 * ty * rowb + xtab > 160 * 1024 || 3 * ty * tpx > 512)
      return fail(MM_E_ARG, "mesh too long along x");
    t.ty_x = ty;
    t.nt_i = std::min(512, std::max(64, pow2ceil(std::max(3 * ty * tpx, ty * g.nx))));
    t.tpc_x = t.nt_i / (3 * ty);
  }
  const int tmin = tpc_for(g.Py, true);
  if (g.nz == 1) {
    const int tpc = std::max(tmin, std::min(2 * tmin, 64));
    const size_t colb = 3 * (size_t)col_stride(g.Py) * csz;
    int cb = 8;
    // packed: the tile of slot 0 also holds the tensor rows of kx = Lx
    const int pk = y2d_packed(g);
    while (cb > 1 && (cb * colb + (cb + pk) * ktab2 + ytab > budget || 3 * cb * tpc > 512 || g.Xp / cb < want)) cb /= 2;
    if (cb * colb + (cb + pk) * ktab2 + ytab > 160 * 1024 || 3 * cb * tpc > 512)
      return fail(MM_E_ARG, "mesh too long along y");
    t.cb_y2 = cb;
    t.tpc_y2 = tpc;
    t.nt_y = 3 * cb * tpc;
  } else {
    const int tpc = std::max(tmin, std::min(2 * tmin, 64));
    const size_t colb = (size_t)col_stride(g.Py) * csz;
    const long long rows = 3LL * g.nz * g.Xp;
    int cb = 16;  // whole kx blocks of the x-pass buffer
    while (cb > kSxB && (cb * colb > budget || cb * tpc > 512 || rows / cb < want)) cb -= kSxB;
    if (cb * colb > 160 * 1024 || cb * tpc > 512) return fail(MM_E_ARG, "mesh too long along y");
    t.cb_y = cb;
    t.tpc_y = tpc;
    t.nt_y = cb * tpc;
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
mm_status upload_tables(Group& G) {
  auto up = [&](void** dst, const std::vector<Cx<T>>& v) -> mm_status {
    HIPCHK(hipMalloc(dst, sizeof(Cx<T>) * std::max<size_t>(v.size(), 1)));
    HIPCHK(hipMemcpy(*dst, v.data(), sizeof(Cx<T>) * v.size(), hipMemcpyHostToDevice));
    return MM_OK;
  };
  MMCHK(up(&G.twx, twiddles<T>(G.g.Lx)));
  MMCHK(up(&G.twy, twiddles<T>(G.g.Py)));
  MMCHK(up(&G.twz, twiddles<T>(G.g.Pz)));
  std::vector<Cx<T>> post(G.g.Lx + 1);
  for (int k = 0; k <= G.g.Lx; ++k) {
    const double a = -2.0 * M_PI * k / (double)G.g.Px;
    post[k] = Cx<T>{(T)std::cos(a), (T)std::sin(a)};
  }
  MMCHK(up(&G.post, post));
  return MM_OK;
}

mm_status dev_alloc(void** d, size_t bytes);

// The launch shapes of the scalar-potential route fit the group's tuning.
template <typename T>
bool pot_fits(const Group& G) {
  HotPlan<T> h;
  std::memset(&h, 0, sizeof(h));
  h.g = G.g;
  h.tu = G.tu;
  return pot_supported<T>(h, min_tpc(make_fft<T>(G.g.Lx, nullptr)));
}

// Tensor spectrum on the device: Newell grid (FP64) -> 3-D FFT (FP64) -> fold -> cast.
template <typename T>
mm_status build_spectrum(Group& G, hipStream_t s) {
  const Geo& g = G.g;
  double nodes[5][20] = {}, wts[5][20] = {};
  int nn[5];
  tent_rules(nodes, wts, nn);
  HIPCHK(setup_upload_gauss(nodes, wts, nn));
  const long long tot = (long long)g.Px * g.Py * g.Pz;
  Cx<double>* F = nullptr;
  HIPCHK(hipMalloc(&F, sizeof(Cx<double>) * tot * G.ncomp));
  std::vector<void*> tws;
  mm_status st = MM_OK;
  do {
    hipError_t e = setup_newell_grid(G.mesh, g.Px, g.Py, g.Pz, G.ncomp, F, s);
    if (e != hipSuccess) { st = fail(MM_E_HIP, std::string("newell grid: ") + hipGetErrorString(e)); break; }
    const int Ls[3] = {g.Px, g.Py, g.Pz};
    const long long inner[3] = {1, g.Px, (long long)g.Px * g.Py};
    const long long outer[3] = {(long long)g.Py * g.Pz * G.ncomp, (long long)g.Pz * G.ncomp, G.ncomp};
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
      e = setup_fft_axis(F, inner[a], outer[a], describe(fp), min_tpc(fp), s);
      if (e != hipSuccess) { st = fail(MM_E_HIP, std::string("tensor fft: ") + hipGetErrorString(e)); break; }
    }
    if (st != MM_OK) break;
    unsigned long long* stats = nullptr;
    e = hipMalloc(&stats, 2 * sizeof(unsigned long long));
    if (e != hipSuccess) { st = fail(MM_E_NOMEM, "stats"); break; }
    tws.push_back(stats);
    e = hipMemsetAsync(stats, 0, 2 * sizeof(unsigned long long), s);
    for (int c = 0; c < G.ncomp && e == hipSuccess; ++c)
      e = setup_extract<T>(F + (size_t)c * tot, g.Px, g.Py, g.Pz, c, (T*)G.kt, stats, s);
    if (e != hipSuccess) { st = fail(MM_E_HIP, std::string("extract: ") + hipGetErrorString(e)); break; }
    unsigned long long hs[2];
    e = hipMemcpyAsync(hs, stats, sizeof(hs), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { st = fail(MM_E_HIP, std::string("spectrum: ") + hipGetErrorString(e)); break; }
    double im, re;
    std::memcpy(&im, &hs[0], 8);
    std::memcpy(&re, &hs[1], 8);
    G.imag_ratio = re > 0 ? im / re : 0.0;
    if (!(G.imag_ratio < 1e-9)) st = fail(MM_E_HIP, "tensor spectrum is not real (symmetry broken)");
  } while (false);
  (void)hipStreamSynchronize(s);
  for (void* d : tws) (void)hipFree(d);
  (void)hipFree(F);
  return st;
}

// Kernel spectrum of the scalar-potential route on the device: the cuboid
// potential on the vertex - cell lattice (FP64) -> 3-D FFT (FP64) -> the real
// factor C_a of S^_a = -i Phi C_a, folded and cast; phase tables on the host.
template <typename T>
mm_status build_potential(Group& G, hipStream_t s) {
  const Geo& g = G.g;
  double nodes[5][16] = {}, wts[5][16] = {};
  const int nn[5] = {14, 9, 6, 4, 3};
  for (int r = 0; r < 5; ++r) gauss_legendre(nn[r], nodes[r], wts[r]);
  HIPCHK(setup_upload_pot_gauss(nodes, wts, nn));
  const long long tot = (long long)g.Px * g.Py * g.Pz;
  Cx<double>* F = nullptr;
  HIPCHK(hipMalloc(&F, sizeof(Cx<double>) * tot * 3));
  std::vector<void*> tws;
  mm_status st = MM_OK;
  do {
    hipError_t e = setup_potential_grid(G.mesh, g.Px, g.Py, g.Pz, F, s);
    if (e != hipSuccess) { st = fail(MM_E_HIP, std::string("potential grid: ") + hipGetErrorString(e)); break; }
    const int Ls[3] = {g.Px, g.Py, g.Pz};
    const long long inner[3] = {1, g.Px, (long long)g.Px * g.Py};
    const long long outer[3] = {(long long)g.Py * g.Pz * 3, (long long)g.Pz * 3, 3};
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
      e = setup_fft_axis(F, inner[a], outer[a], describe(fp), min_tpc(fp), s);
      if (e != hipSuccess) { st = fail(MM_E_HIP, std::string("potential fft: ") + hipGetErrorString(e)); break; }
    }
    if (st != MM_OK) break;
    unsigned long long* stats = nullptr;
    e = hipMalloc(&stats, 2 * sizeof(unsigned long long));
    if (e != hipSuccess) { st = fail(MM_E_NOMEM, "stats"); break; }
    tws.push_back(stats);
    e = hipMemsetAsync(stats, 0, 2 * sizeof(unsigned long long), s);
    for (int c = 0; c < 3 && e == hipSuccess; ++c)
      e = setup_extract_pot<T>(F + (size_t)c * tot, g.Px, g.Py, g.Pz, c, (T*)G.kpot, stats, s);
    if (e != hipSuccess) { st = fail(MM_E_HIP, std::string("extract: ") + hipGetErrorString(e)); break; }
    unsigned long long hs[2];
    e = hipMemcpyAsync(hs, stats, sizeof(hs), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { st = fail(MM_E_HIP, std::string("spectrum: ") + hipGetErrorString(e)); break; }
    double im, re;
    std::memcpy(&im, &hs[0], 8);
    std::memcpy(&re, &hs[1], 8);
    G.imag_ratio = re > 0 ? im / re : 0.0;
    if (!(G.imag_ratio < 1e-9)) st = fail(MM_E_HIP, "potential spectrum is not of the half-cell form");
  } while (false);
  (void)hipStreamSynchronize(s);
  for (void* d : tws) (void)hipFree(d);
  (void)hipFree(F);
  if (st != MM_OK) return st;
  auto phase = [&](void** dst, int n, int P) -> mm_status {
    std::vector<Cx<T>> v(n);
    for (int k = 0; k < n; ++k) {
      const double a = -M_PI * (double)k / (double)P;
      v[k] = Cx<T>{(T)std::cos(a), (T)std::sin(a)};
    }
    MMCHK(dev_alloc(dst, sizeof(Cx<T>) * n));
    HIPCHK(hipMemcpy(*dst, v.data(), sizeof(Cx<T>) * n, hipMemcpyHostToDevice));
    return MM_OK;
  };
  MMCHK(phase(&G.phx, g.Xp, g.Px));
  MMCHK(phase(&G.phy, g.Py, g.Py));
  MMCHK(phase(&G.phz, g.Pz, g.Pz));
  return MM_OK;
}

mm_status dev_alloc(void** d, size_t bytes) {
  hipError_t e = hipMalloc(d, std::max<size_t>(bytes, 16));
  if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? MM_E_NOMEM : MM_E_HIP, hipGetErrorString(e));
  return MM_OK;
}

void free_group(Group& G) {
  void* bufs[] = {G.Sx, G.Sy, G.kt, G.post, G.twx, G.twy, G.twz, G.stage, G.mbuf, G.cells, G.kpot, G.phx,
                  G.phy, G.phz};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  G = Group();
}

void free_engine(Engine& E) {
  if (E.gexec) (void)hipGraphExecDestroy(E.gexec);
  E.gexec = nullptr;
  for (Group& G : E.groups) free_group(G);
  void* bufs[] = {E.prm, E.ctl, E.partial, E.e5, E.replay, E.dhot, E.depi, E.nebH, E.nebB, E.nebS, E.nebP};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (E.hctl) (void)hipHostFree(E.hctl);
  if (E.hctl2) (void)hipHostFree(E.hctl2);
  for (hipEvent_t& ev : E.poll_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (E.he5) (void)hipHostFree(E.he5);
  if (E.cap) (void)hipStreamDestroy(E.cap);
}

// Geometry of the padded grid (Px, Py, Pz), default launch shapes, the
// transform tables and the demag spectrum (Newell tensor or scalar-potential
// kernel) of G's mesh.  The grid's buffers (G.Sx, G.Sy) follow in engine_reserve.
mm_status build_padded(Engine& E, Group& G, int Px, int Py, int Pz, hipStream_t s) {
  Geo& g = G.g;
  const bool pot = (E.terms & MM_DEMAG_POTENTIAL) != 0;
  g.Px = Px;
  g.Py = Py;
  g.Pz = Pz;
  g.Lx = g.Px / 2;
  g.Xp = g.Lx + 1;
  g.Ky = g.Py / 2 + 1;
  g.Kz = g.Pz / 2 + 1;
  g.N = (long long)g.nx * g.ny * g.nz;
  g.XB = (g.Xp + kSxB - 1) / kSxB;
  g.sx = g.nz == 1 ? 3LL * g.Xp * g.ny : 3LL * g.nz * g.XB * kSxB * g.ny;
  g.sy = 3LL * g.nz * g.Xp * g.Py;
  g.dV = G.mesh.dx * G.mesh.dy * G.mesh.dz;
  MMCHK(choose_tuning(G, E.prec, E.csz));
  if (E.terms & MM_DEMAG) {
    MMCHK(dev_alloc(&G.kt, E.rsz * G.ncomp * (size_t)g.Kz * g.Xp * g.Ky));
    MMCHK(E.prec == MM_F32 ? upload_tables<float>(G) : upload_tables<double>(G));
    MMCHK(E.prec == MM_F32 ? build_spectrum<float>(G, s) : build_spectrum<double>(G, s));
  }
  if (pot) {
    const bool fits = E.prec == MM_F32 ? pot_fits<float>(G) : pot_fits<double>(G);
    if (!fits) return fail(MM_E_ARG, "mesh too long along x for the scalar-potential route's x pass");
    MMCHK(dev_alloc(&G.kpot, E.rsz * 3 * (size_t)g.Kz * g.Xp * g.Ky));
    MMCHK(E.prec == MM_F32 ? upload_tables<float>(G) : upload_tables<double>(G));
    MMCHK(E.prec == MM_F32 ? build_potential<float>(G, s) : build_potential<double>(G, s));
  }
  return MM_OK;
}

// Shortest padded lengths per axis: 2n - 1 (every displacement of the
// cell-averaged tensor fits), 2n for the scalar-potential route.
int min_padded(int n, bool pot) { return pot ? 2 * n : 2 * n - 1; }

// Geometry, tuning, tables and (with demag) the tensor spectrum of one mesh.
mm_status make_group(Engine& E, const mm_mesh& mesh, hipStream_t s, Group& G) {
  G.mesh = mesh;
  G.ncomp = mesh.nz == 1 ? 4 : 6;
  Geo& g = G.g;
  g.nx = mesh.nx; g.ny = mesh.ny; g.nz = mesh.nz;
  const bool pot = (E.terms & MM_DEMAG_POTENTIAL) != 0;
  const int Px = pot ? pick_padded_pot(g.nx, true) : pick_padded(g.nx, true);
  const int Py = pot ? pick_padded_pot(g.ny, false) : pick_padded(g.ny, false);
  const int Pz = pot ? pick_padded_pot(g.nz, false) : pick_padded(g.nz, false);
  return build_padded(E, G, Px, Py, Pz, s);
}

// Drop the buffers and tables that depend on the padded grid (the stage,
// batch and cell arrays stay).
void free_padded(Engine& E, Group& G) {
  void* bufs[] = {G.Sx, G.Sy, G.kt, G.post, G.twx, G.twy, G.twz, G.kpot, G.phx, G.phy, G.phz};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  G.Sx = G.Sy = G.kt = G.post = G.twx = G.twy = G.twz = G.kpot = G.phx = G.phy = G.phz = nullptr;
  G.cap = 0;
  G.user_shapes = false;  // the new grid starts from the default launch shapes
  G.tuned_for = 0;
  E.k1_ok = false;
  if (E.gexec) { (void)hipGraphExecDestroy(E.gexec); E.gexec = nullptr; }
}

mm_status engine_init(Engine& E, mm_precision prec, uint32_t terms) {
  E.prec = prec;
  E.terms = terms;
  E.csz = prec == MM_F32 ? sizeof(Cx<float>) : sizeof(Cx<double>);
  E.rsz = prec == MM_F32 ? sizeof(float) : sizeof(double);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(MM_E_HIP, std::string("no HIP device: ") + hipGetErrorString(e));
  e = hipStreamCreateWithFlags(&E.cap, hipStreamNonBlocking);
  if (e != hipSuccess) return fail(MM_E_HIP, hipGetErrorString(e));
  const size_t hsz = E.prec == MM_F32 ? sizeof(HotPlan<float>) : sizeof(HotPlan<double>);
  const size_t esz = E.prec == MM_F32 ? sizeof(Epi<float>) : sizeof(Epi<double>);
  MMCHK(dev_alloc(&E.dhot, hsz * kMaxGroups));
  MMCHK(dev_alloc(&E.depi, esz * kMaxGroups * kEpiSlots));
  return MM_OK;
}

// Capacity of the per-instance arrays and of each group's spectral buffers.
mm_status engine_reserve(Engine& E, const std::vector<int>& per_group) {
  int total = 0, parts = 0;
  for (size_t i = 0; i < per_group.size(); ++i) {
    Group& G = E.groups[i];
    const int n = per_group[i];
    total += n;
    parts = std::max(parts, 5 * n * eval_blocks_per_inst(G.g, G.tu));
    if (n > G.cap && (E.terms & (MM_DEMAG | MM_DEMAG_POTENTIAL))) {
      if (G.Sx) (void)hipFree(G.Sx);
      if (G.Sy) (void)hipFree(G.Sy);
      G.Sx = G.Sy = nullptr;
      MMCHK(dev_alloc(&G.Sx, E.csz * G.g.sx * n));
      if (G.g.nz > 1) MMCHK(dev_alloc(&G.Sy, E.csz * G.g.sy * n));
      G.cap = n;
      if (E.gexec) { (void)hipGraphExecDestroy(E.gexec); E.gexec = nullptr; }
    } else if (n > G.cap) {
      G.cap = n;
    }
  }
  if (total > E.inst_cap) {
    if (E.prm) (void)hipFree(E.prm);
    if (E.ctl) (void)hipFree(E.ctl);
    if (E.e5) (void)hipFree(E.e5);
    if (E.hctl) (void)hipHostFree(E.hctl);
    if (E.hctl2) (void)hipHostFree(E.hctl2);
    if (E.he5) (void)hipHostFree(E.he5);
    E.prm = nullptr; E.ctl = nullptr; E.e5 = nullptr; E.hctl = nullptr; E.hctl2 = nullptr; E.he5 = nullptr;
    MMCHK(dev_alloc((void**)&E.prm, sizeof(DevParams) * total));
    MMCHK(dev_alloc((void**)&E.ctl, sizeof(DevCtl) * total));
    MMCHK(dev_alloc((void**)&E.e5, sizeof(double) * 5 * total));
    HIPCHK(hipHostMalloc((void**)&E.hctl, sizeof(DevCtl) * total));
    HIPCHK(hipHostMalloc((void**)&E.hctl2, sizeof(DevCtl) * total));
    HIPCHK(hipHostMalloc((void**)&E.he5, sizeof(double) * 5 * total));
    std::memset(E.hctl, 0, sizeof(DevCtl) * total);
    E.inst_cap = total;
    if (E.gexec) { (void)hipGraphExecDestroy(E.gexec); E.gexec = nullptr; }
  }
  if (parts > E.part_cap) {
    if (E.partial) (void)hipFree(E.partial);
    E.partial = nullptr;
    MMCHK(dev_alloc((void**)&E.partial, sizeof(double) * parts));
    E.part_cap = parts;
  }
  return MM_OK;
}

// Upload parameters (in group order) and remember whether demag is on.
mm_status upload_params(Engine& E, const std::vector<const mm_params*>& q, const std::vector<int>& grp,
                        hipStream_t s) {
  std::vector<DevParams> d(q.size());
  E.any_demag = false;
  E.any_pot = false;
  E.use_general = false;
  for (size_t b = 0; b < q.size(); ++b) E.use_general = E.use_general || (q[b]->terms & kGeneralTerms) != 0;
  for (size_t b = 0; b < q.size(); ++b) {
    d[b] = dev_params(*q[b], E.groups[grp[b]], E.use_general);
    E.any_demag = E.any_demag || (q[b]->terms & MM_DEMAG) != 0;
    E.any_pot = E.any_pot || (q[b]->terms & MM_DEMAG_POTENTIAL) != 0;
  }
  HIPCHK(hipMemcpyAsync(E.prm, d.data(), sizeof(DevParams) * d.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return MM_OK;
}

// Host and device views of the groups for the given per-group instance counts
// (instances of group i start at inst0[i] in the parameter / controller arrays).
template <typename T>
mm_status make_set(Engine& E, const std::vector<int>& nb, GroupSet<T>& gs, std::vector<int>& inst0,
                   hipStream_t s) {
  gs.n = (int)E.groups.size();
  inst0.assign(gs.n, 0);
  int acc = 0;
  for (int i = 0; i < gs.n; ++i) {
    Group& G = E.groups[i];
    HotPlan<T>& h = gs.h[i];
    std::memset(&h, 0, sizeof(h));
    h.g = G.g;
    h.tu = G.tu;
    h.fd[0] = describe(make_fft<T>(G.g.Lx, (const Cx<T>*)G.twx));
    h.fd[1] = describe(make_fft<T>(G.g.Py, (const Cx<T>*)G.twy, true));
    h.fd[2] = describe(make_fft<T>(G.g.Pz, (const Cx<T>*)G.twz));
    h.twz = (const Cx<T>*)G.twz;
    h.post = (const Cx<T>*)G.post;
    h.kt = (const T*)G.kt;
    h.ncomp = G.ncomp;
    h.batch = nb[i];
    h.Sx = (Cx<T>*)G.Sx;
    h.Sy = (Cx<T>*)G.Sy;
    h.prm = E.prm + acc;
    h.cells = E.use_general ? (const T*)G.cells : nullptr;
    h.gen = E.use_general ? 1 : 0;
    inst0[i] = acc;
    acc += nb[i];
  }
  gs.dh = (const HotPlan<T>*)E.dhot;
  HIPCHK(hipMemcpyAsync(E.dhot, gs.h, sizeof(HotPlan<T>) * gs.n, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return MM_OK;
}

template <typename T>
Epi<T>* epi_slot(Engine& E, int slot) {
  return (Epi<T>*)E.depi + (size_t)slot * kMaxGroups;
}

template <typename T>
mm_status upload_epis(Engine& E, int slot, const std::vector<Epi<T>>& ep, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(epi_slot<T>(E, slot), ep.data(), sizeof(Epi<T>) * ep.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return MM_OK;
}

template <typename T>
Epi<T> epi_base(const Group& G, int mode) {
  Epi<T> e;
  std::memset(&e, 0, sizeof(e));
  e.mode = mode;
  e.inst_stride = 3 * G.g.N;
  return e;
}

bool demag_on(const Engine& E) { return (E.terms & MM_DEMAG) != 0 && E.any_demag; }

template <typename T>
PotTab<T> pot_tab(const Group& G) {
  PotTab<T> t;
  t.kp = (const T*)G.kpot;
  t.phx = (const Cx<T>*)G.phx;
  t.phy = (const Cx<T>*)G.phy;
  t.phz = (const Cx<T>*)G.phz;
  t.gdx = -0.25 / G.mesh.dx;
  t.gdy = -0.25 / G.mesh.dy;
  t.gdz = -0.25 / G.mesh.dz;
  return t;
}

// Back-to-back timing of the five passes of the scalar-potential route
// (after one full evaluation that fills the intermediate buffers).
template <typename T>
mm_status time_pot_passes(Engine& E, const GroupSet<T>& gs, const Epi<T>* epis, int reps, double* us,
                          hipStream_t s, double* seq = nullptr) {
  const PotTab<T> pt = pot_tab<T>(E.groups[0]);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  hipError_t er = hipEventCreate(&e1);
  if (er != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(MM_E_HIP, hipGetErrorString(er));
  }
  er = launch_potential<T>(gs, epis, pt, MODE_RHS, s);
  if (seq) {  // in evaluation order
    hipEvent_t ev[6] = {};
    for (auto& e : ev)
      if (er == hipSuccess) er = hipEventCreate(&e);
    for (int i = 0; i < 5; ++i) seq[i] = 0.0;
    for (int r = 0; r < reps && er == hipSuccess; ++r) {
      for (int i = 0; i < 5 && er == hipSuccess; ++i) {
        er = hipEventRecord(ev[i], s);
        if (er == hipSuccess) er = launch_potential<T>(gs, epis, pt, MODE_RHS, s, 1u << i);
      }
      if (er == hipSuccess) er = hipEventRecord(ev[5], s);
      if (er == hipSuccess) er = hipEventSynchronize(ev[5]);
      for (int i = 0; i < 5 && er == hipSuccess; ++i) {
        float ms = 0.f;
        er = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
        seq[i] += 1e3 * ms / reps;
      }
    }
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  for (int i = 0; i < 5 && er == hipSuccess; ++i) {
    er = hipEventRecord(e0, s);
    for (int r = 0; r < reps && er == hipSuccess; ++r) er = launch_potential<T>(gs, epis, pt, MODE_RHS, s, 1u << i);
    if (er == hipSuccess) er = hipEventRecord(e1, s);
    if (er == hipSuccess) er = hipEventSynchronize(e1);
    float ms = 0.f;
    if (er == hipSuccess) er = hipEventElapsedTime(&ms, e0, e1);
    us[i] = 1e3 * ms / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (er != hipSuccess) return fail(MM_E_HIP, hipGetErrorString(er));
  return MM_OK;
}

// --- single-group calls (plans) ----------------------------------------------

template <typename T>
mm_status single_eval(mm_plan* p, int batch, const mm_params* q, const void* m, void* out, int mode,
                      double* partial, hipStream_t s, hipEvent_t* ev = nullptr) {
  Engine& E = p->e;
  std::vector<const mm_params*> qv(batch);
  std::vector<int> grp(batch, 0);
  for (int b = 0; b < batch; ++b) qv[b] = &q[b];
  MMCHK(upload_params(E, qv, grp, s));
  GroupSet<T> gs;
  std::vector<int> inst0;
  MMCHK(make_set<T>(E, std::vector<int>{batch}, gs, inst0, s));
  std::vector<Epi<T>> ep(1, epi_base<T>(E.groups[0], mode));
  ep[0].in = (const T*)m;
  ep[0].out = (T*)out;
  ep[0].partial = partial;
  MMCHK(upload_epis<T>(E, 0, ep, s));
  if (E.any_pot) HIPCHK(launch_potential<T>(gs, epi_slot<T>(E, 0), pot_tab<T>(E.groups[0]), mode, s));
  else HIPCHK(launch_eval<T>(gs, epi_slot<T>(E, 0), mode, demag_on(E), s, ev));
  return MM_OK;
}

int pass_count(const Engine& E) {
  if (E.any_pot) return 5;
  if (!demag_on(E)) return 1;
  return E.groups[0].g.nz == 1 ? 3 : 5;
}

// Back-to-back timing: `reps` launches of one pass between two events on the
// launch stream, for each pass in turn (after one full evaluation that fills
// every intermediate buffer).  us[p] = mean duration of pass p.
template <typename T>
mm_status time_each_pass(Engine& E, const GroupSet<T>& gs, const Epi<T>* epis, int mode, int reps, int np,
                         double* us, hipStream_t s, double* seq = nullptr) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  hipError_t er = hipEventCreate(&e1);
  if (er != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(MM_E_HIP, hipGetErrorString(er));
  }
  mm_status st = MM_OK;
  er = launch_eval<T>(gs, epis, mode, demag_on(E), s);
  if (seq) {  // in evaluation order: each pass after the one whose output it reads
    std::vector<hipEvent_t> ev(np + 1, nullptr);
    for (auto& e : ev)
      if (er == hipSuccess) er = hipEventCreate(&e);
    for (int i = 0; i < np; ++i) seq[i] = 0.0;
    for (int r = 0; r < reps && er == hipSuccess; ++r) {
      for (int i = 0; i < np && er == hipSuccess; ++i) {
        er = hipEventRecord(ev[i], s);
        if (er == hipSuccess) er = launch_eval<T>(gs, epis, mode, demag_on(E), s, nullptr, false, false, 1u << i);
      }
      if (er == hipSuccess) er = hipEventRecord(ev[np], s);
      if (er == hipSuccess) er = hipEventSynchronize(ev[np]);
      for (int i = 0; i < np && er == hipSuccess; ++i) {
        float ms = 0.f;
        er = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
        seq[i] += 1e3 * ms / reps;
      }
    }
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  for (int i = 0; i < np && er == hipSuccess; ++i) {
    const unsigned bit = (unsigned)i;  // pass i in launch order has bit i (see launch_eval)
    er = hipEventRecord(e0, s);
    for (int r = 0; r < reps && er == hipSuccess; ++r)
      er = launch_eval<T>(gs, epis, mode, demag_on(E), s, nullptr, false, false, 1u << bit);
    if (er == hipSuccess) er = hipEventRecord(e1, s);
    if (er == hipSuccess) er = hipEventSynchronize(e1);
    float ms = 0.f;
    if (er == hipSuccess) er = hipEventElapsedTime(&ms, e0, e1);
    us[i] = 1e3 * ms / reps;
  }
  if (er != hipSuccess) st = fail(MM_E_HIP, hipGetErrorString(er));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

template <typename T>
mm_status profile_impl(mm_plan* p, const mm_params* q, int batch, const void* m, void* out, int reps, double* us,
                       hipStream_t s, double* seq) {
  Engine& E = p->e;
  MMCHK(single_eval<T>(p, batch, q, m, out, MODE_RHS, nullptr, s));
  GroupSet<T> gs;
  std::vector<int> inst0;
  MMCHK(make_set<T>(E, std::vector<int>{batch}, gs, inst0, s));
  if (E.any_pot) return time_pot_passes<T>(E, gs, epi_slot<T>(E, 0), reps, us, s, seq);
  return time_each_pass<T>(E, gs, epi_slot<T>(E, 0), MODE_RHS, reps, pass_count(E), us, s, seq);
}

// Energies from the partial sums `partial` (device, [batch][blocks][5]) of one
// MODE_ENERGY evaluation: reduce into e5 (device, [batch][5]), copy to the
// plan's pinned host buffer, scale to joules.
mm_status energy_finish(Engine& E, const mm_params* q, int batch, const double* partial, double* e5,
                        double* E_out, hipStream_t s) {
  const Group& G = E.groups[0];
  HIPCHK(launch_energy_reduce(partial, batch, eval_blocks_per_inst(G.g, G.tu), e5, s));
  HIPCHK(hipMemcpyAsync(E.he5, e5, sizeof(double) * 5 * batch, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int b = 0; b < batch; ++b) {
    const double c = kMu0 * (E.use_general ? 1.0 : q[b].Ms) * G.g.dV;  // general form: Ms in the sums
    for (int k = 0; k < 5; ++k) E_out[5 * b + k] = -(k == 4 ? 1.0 : 0.5) * c * E.he5[5 * b + k];
  }
  return MM_OK;
}

template <typename T>
mm_status energy_impl(mm_plan* p, const mm_params* q, int batch, const void* m, double* E_out, hipStream_t s) {
  Engine& E = p->e;
  MMCHK(single_eval<T>(p, batch, q, m, nullptr, MODE_ENERGY, E.partial, s));
  return energy_finish(E, q, batch, E.partial, E.e5, E_out, s);
}

// --- Dormand-Prince over every group -----------------------------------------

template <typename T>
T* stage_buf(const Group& G, int idx) {  // 0: ms0, 1: ms1, 2..8: k1..k7
  return (T*)G.stage + (size_t)idx * G.stage_cap * 3 * G.g.N;
}

template <typename T>
mm_status ensure_stage(Engine& E, Group& G, int n) {
  if (G.stage && G.stage_cap >= n) return MM_OK;
  if (G.stage) (void)hipFree(G.stage);
  G.stage = nullptr;
  E.k1_ok = false;
  MMCHK(dev_alloc(&G.stage, sizeof(T) * 9 * (size_t)n * 3 * G.g.N));
  G.stage_cap = n;
  if (E.gexec) { (void)hipGraphExecDestroy(E.gexec); E.gexec = nullptr; }
  return MM_OK;
}

// Epilogue tables of every slot for the groups' state arrays m[i] (device).
template <typename T>
mm_status upload_step_epis(Engine& E, const std::vector<T*>& m, const std::vector<int>& inst0, hipStream_t s) {
  const int ng = (int)E.groups.size();
  for (int slot = 1; slot < kEpiSlots; ++slot) {
    std::vector<Epi<T>> ep;
    for (int i = 0; i < ng; ++i) {
      const Group& G = E.groups[i];
      Epi<T> e = epi_base<T>(G, MODE_RHS);
      e.ctl = E.ctl + inst0[i];
      if (slot == 1) {  // first slope k1 = f(m)
        e.mode = MODE_RHS;
        e.in = m[i];
        e.out = stage_buf<T>(G, 2);
        e.ctl = nullptr;
      } else if (slot < 8) {  // stage st evaluates its input and forms the next one
        const int st = slot;
        const int in = (st % 2 == 0) ? 0 : 1;  // ms0 feeds even stages, ms1 odd stages
        e.mode = st < 7 ? MODE_STAGE : MODE_ERROR;
        e.in = stage_buf<T>(G, in);
        e.out = stage_buf<T>(G, 2 + st - 1);
        e.mbase = m[i];
        e.msn = stage_buf<T>(G, 1 - in);
        for (int j = 0; j < st - 1; ++j) e.kprev[j] = stage_buf<T>(G, 2 + j);
        e.nk = st;
        e.replay = E.replay;
        for (int j = 0; j < st; ++j) e.coef[j] = st < 7 ? kDP.a[st + 1][j] : kDP.e[j];
      } else {  // step begin
        e.bm = m[i];
        e.bms0 = stage_buf<T>(G, 0);
        e.bms1 = stage_buf<T>(G, 1);
        e.bk1 = stage_buf<T>(G, 2);
        e.bk7 = stage_buf<T>(G, 8);
        e.a21 = kDP.a[2][0];
      }
      ep.push_back(e);
    }
    MMCHK(upload_epis<T>(E, slot, ep, s));
  }
  return MM_OK;
}

// One evaluation of epilogue slot `slot` in `mode`, through the plan's demag
// route: the scalar-potential passes (no fused forward pass), else the Newell
// passes, which skip the forward x pass (skip_x) when the previous stage's
// inverse-x pass has done it and fuse it into this one (fuse).
template <typename T>
hipError_t eval_slot(Engine& E, const GroupSet<T>& gs, int slot, int mode, hipStream_t s, bool skip_x = false,
                     bool fuse = false) {
  if (E.any_pot) return launch_potential<T>(gs, epi_slot<T>(E, slot), pot_tab<T>(E.groups[0]), mode, s);
  return launch_eval<T>(gs, epi_slot<T>(E, slot), mode, demag_on(E), s, nullptr, skip_x, fuse);
}

// The inverse-x passes of the Runge-Kutta stages can transform the next stage
// input forward along x (Newell route, launch shape permitting).
template <typename T>
bool stage_fusable(const Engine& E, const GroupSet<T>& gs) {
  return !E.any_pot && demag_on(E) && eval_fusable<T>(gs);
}

template <typename T>
mm_status enqueue_attempt(Engine& E, const GroupSet<T>& gs, int n_total, hipStream_t s) {
  HIPCHK(launch_begin<T>(gs, epi_slot<T>(E, 8), s));
  // stages 2..6 transform the next stage input forward along x in their
  // inverse-x pass when the launch shape allows it; stages 3..7 then skip it
  const bool fz = stage_fusable<T>(E, gs);
  for (int st = 2; st <= 7; ++st)
    HIPCHK(eval_slot<T>(E, gs, st, st < 7 ? MODE_STAGE : MODE_ERROR, s, fz && st > 2, fz && st < 7));
  // the step decision runs in the last workgroup of each instance in the error
  // pass; instances already done keep their pending projection, which the next
  // step-begin repeats idempotently
  (void)n_total;
  return MM_OK;
}

// Fixed-step Heun (explicit trapezoid) with projection, n_steps of size h:
// k1 = f(m), m1 = m + h k1 (stage epilogue, slot 2); k2 = f(m1),
// m <- (m + h (k1 + k2) / 2) / |...| per cell (stage epilogue, slot 3, in
// place: each cell's m is read by its own thread only, before its store).
// The stage epilogues take h from the controllers (h_att, nothing done).
// Where the launch shape allows, each stage's inverse-x pass also transforms
// the next stage input along x (stage 2: the next step's m), so that only the
// first stage of a call runs the forward x pass.  Buffers: stage 0 = m1,
// 2 = k1, 3 = k2 (the Dormand-Prince slopes of a later adaptive call are
// recomputed: its state must say fsal_valid = 0).
template <typename T>
mm_status heun_impl(mm_plan* p, const mm_params* q, int batch, T* m, double h, long long n_steps, hipStream_t s) {
  Engine& E = p->e;
  Group& G = E.groups[0];
  std::vector<const mm_params*> qv(batch);
  std::vector<int> grp(batch, 0);
  for (int b = 0; b < batch; ++b) qv[b] = &q[b];
  MMCHK(ensure_stage<T>(E, G, batch));
  E.k1_ok = false;  // the steps below overwrite the first-slope buffer
  MMCHK(upload_params(E, qv, grp, s));
  GroupSet<T> gs;
  std::vector<int> inst0;
  MMCHK(make_set<T>(E, std::vector<int>{batch}, gs, inst0, s));
  for (int b = 0; b < batch; ++b) {
    std::memset(&E.hctl[b], 0, sizeof(DevCtl));
    E.hctl[b].h_att = h;
  }
  HIPCHK(hipMemcpyAsync(E.ctl + inst0[0], E.hctl, sizeof(DevCtl) * batch, hipMemcpyHostToDevice, s));
  Epi<T> e1 = epi_base<T>(G, MODE_STAGE);
  e1.ctl = E.ctl + inst0[0];
  Epi<T> e2 = e1;
  e1.in = m;
  e1.out = stage_buf<T>(G, 2);
  e1.mbase = m;
  e1.msn = stage_buf<T>(G, 0);
  e1.nk = 1;
  e1.coef[0] = 1.0;
  e2.in = stage_buf<T>(G, 0);
  e2.out = stage_buf<T>(G, 3);
  e2.mbase = m;
  e2.msn = m;
  e2.project = 1;
  e2.kprev[0] = stage_buf<T>(G, 2);
  e2.nk = 2;
  e2.coef[0] = 0.5;
  e2.coef[1] = 0.5;
  MMCHK(upload_epis<T>(E, 2, std::vector<Epi<T>>{e1}, s));
  MMCHK(upload_epis<T>(E, 3, std::vector<Epi<T>>{e2}, s));
  const bool fz = stage_fusable<T>(E, gs);
  for (long long i = 0; i < n_steps; ++i) {
    HIPCHK(eval_slot<T>(E, gs, 2, MODE_STAGE, s, fz && i > 0, fz));
    HIPCHK(eval_slot<T>(E, gs, 3, MODE_STAGE, s, fz, fz));
  }
  return MM_OK;
}

// Steepest descent with Barzilai-Borwein steps, n_iter iterations: H_eff(m)
// by a field evaluation (epilogue slot 4), then launch_sd_iteration.  Buffers:
// stage 4 = H, 5 = g, 6 = m_prev, 7 = g_prev.  tau_out (host, nullable): the
// last step size of each instance.  stop > 0 (rad/s): a relaxation -- each
// iteration first checks the largest |dm/dt| of its m, instances below stop
// are done (their later launches return at once), and one last check follows
// the n_iter-th update; the host polls the controllers every kPollSd
// iterations and ends early once every instance is done.  iters_out /
// dmdt_out (host, nullable): updates made and the last largest |dm/dt|
// (rad/s).  Synchronises.
constexpr long long kPollSd = 16;

// Bytes of per-call scratch of sd_impl for `batch` instances of G: the block
// partial sums (4 doubles per block), padded to 256 bytes, then the step sizes.
size_t sd_part_bytes(const Group& G, int batch) {
  const size_t bpi = (size_t)((G.g.N + 255) / 256);
  return (sizeof(double) * 4 * bpi * batch + 255) / 256 * 256;
}
size_t sd_scratch_bytes(const Group& G, int batch) { return sd_part_bytes(G, batch) + sizeof(double) * batch; }

// ext (device, nullable): caller-provided scratch of sd_scratch_bytes(G, batch)
// bytes; then nothing is allocated or freed, and the stage buffers must already
// hold `batch` instances (MM_E_STATE otherwise).
template <typename T>
mm_status sd_impl(mm_plan* p, const mm_params* q, int batch, T* m, long long n_iter, double tau0, double tau_min,
                  double tau_max, double* tau_out, double stop, long long* iters_out, double* dmdt_out,
                  hipStream_t s, unsigned char* ext = nullptr) {
  Engine& E = p->e;
  Group& G = E.groups[0];
  const bool relax = stop > 0.0;
  if (ext && !(G.stage && G.stage_cap >= batch))
    return fail(MM_E_STATE, "the plan's stage buffers do not hold this batch yet: one mm_sd_run, mm_heun_run or "
                            "mm_rk45_* call with at least as many instances allocates them");
  std::vector<const mm_params*> qv(batch);
  std::vector<int> grp(batch, 0);
  for (int b = 0; b < batch; ++b) qv[b] = &q[b];
  MMCHK(ensure_stage<T>(E, G, batch));
  E.k1_ok = false;  // stage buffers 4..7 hold the iteration's vectors (k3..k6 of an adaptive run)
  MMCHK(upload_params(E, qv, grp, s));
  GroupSet<T> gs;
  std::vector<int> inst0;
  MMCHK(make_set<T>(E, std::vector<int>{batch}, gs, inst0, s));
  DevCtl* const ctl = relax ? E.ctl + inst0[0] : nullptr;
  if (relax) {
    for (int b = 0; b < batch; ++b) {
      std::memset(&E.hctl[b], 0, sizeof(DevCtl));
      E.hctl[b].stop_dmdt = stop;
    }
    HIPCHK(hipMemcpyAsync(ctl, E.hctl, sizeof(DevCtl) * batch, hipMemcpyHostToDevice, s));
  }
  T* const H = stage_buf<T>(G, 4);
  Epi<T> e = epi_base<T>(G, MODE_FIELD);
  e.in = m;
  e.out = H;
  e.ctl = ctl;
  MMCHK(upload_epis<T>(E, 4, std::vector<Epi<T>>{e}, s));
  const long long N = G.g.N;
  const size_t bpi = (size_t)((N + 255) / 256);
  double* part = nullptr;
  double* tau = nullptr;
  mm_status st = MM_OK;
  if (ext) {
    part = (double*)ext;
    tau = (double*)(ext + sd_part_bytes(G, batch));
  } else {
    MMCHK(dev_alloc((void**)&part, sizeof(double) * 4 * bpi * batch));
    st = dev_alloc((void**)&tau, sizeof(double) * batch);
  }
  std::vector<double> t0(batch, tau0);
  hipError_t er = st == MM_OK ? hipMemcpyAsync(tau, t0.data(), sizeof(double) * batch, hipMemcpyHostToDevice, s)
                              : hipSuccess;
  const long long n_launch = relax ? n_iter + 1 : n_iter;
  for (long long k = 0; st == MM_OK && er == hipSuccess && k < n_launch; ++k) {
    er = eval_slot<T>(E, gs, 4, MODE_FIELD, s);
    if (er == hipSuccess)
      er = launch_sd_iteration<T>(m, H, stage_buf<T>(G, 5), stage_buf<T>(G, 6), stage_buf<T>(G, 7), part, tau,
                                  batch, N, k, tau_min, tau_max, E.prm + inst0[0], ctl, relax && k == n_iter, s);
    if (relax && er == hipSuccess && (k + 1) % kPollSd == 0 && k + 1 < n_launch) {
      er = hipMemcpyAsync(E.hctl, ctl, sizeof(DevCtl) * batch, hipMemcpyDeviceToHost, s);
      if (er == hipSuccess) er = hipStreamSynchronize(s);
      bool all = er == hipSuccess;
      for (int b = 0; b < batch && all; ++b) all = E.hctl[b].done != 0;
      if (all) break;
    }
  }
  {  // the buffers are freed below: nothing may still use them
    const hipError_t es = hipStreamSynchronize(s);
    if (er == hipSuccess) er = es;
  }
  if (st == MM_OK && er == hipSuccess && tau_out) er = hipMemcpy(tau_out, tau, sizeof(double) * batch,
                                                                 hipMemcpyDeviceToHost);
  if (st == MM_OK && er == hipSuccess && relax) er = hipMemcpy(E.hctl, ctl, sizeof(DevCtl) * batch,
                                                               hipMemcpyDeviceToHost);
  if (st == MM_OK && er != hipSuccess) st = fail(MM_E_HIP, hipGetErrorString(er));
  if (!ext) {
    (void)hipFree(part);
    if (tau) (void)hipFree(tau);
  }
  if (st != MM_OK || !relax) return st;
  bool all_stopped = true;
  for (int b = 0; b < batch; ++b) {
    if (iters_out) iters_out[b] = E.hctl[b].n_attempt;
    if (dmdt_out) dmdt_out[b] = E.hctl[b].last_dmdt;
    all_stopped = all_stopped && E.hctl[b].last_dmdt < stop;
  }
  if (!all_stopped) return fail(MM_E_MAXSTEPS, "relaxation: the largest |dm/dt| stayed above the threshold");
  return MM_OK;
}

// Timing of the kernels of one adaptive attempt (measurement aid): us[0] the
// step-begin kernel, us[1 .. np] the passes of a stage evaluation with its
// inverse-x pass in the form the captured attempt uses (stage epilogue, fused
// forward x when fused), us[np + 1] the inverse-x pass with the error
// epilogue.  Stage-epilogue and the forward-x figures average stages 2..6.
// attempt limit of the timing runs (the error pass decides steps as it is
// timed; the limit must not stop the instance)
constexpr long long kNoLimit = 1LL << 60;

struct StepProfile {
  int reps = 0;
  double us[16] = {};
  double seq[16] = {};  // the same kernels timed in attempt order (each after the kernel it depends on)
  bool want_seq = false;
  int n = 0;
  int fused = 0;
};

template <typename T>
mm_status profile_step(Engine& E, const GroupSet<T>& gs, StepProfile& pr, hipStream_t s) {
  const int np = pass_count(E);
  const bool fz = demag_on(E) && eval_fusable<T>(gs);
  pr.fused = fz ? 1 : 0;
  pr.n = np + 2;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  hipError_t er = hipEventCreate(&e1);
  if (er != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(MM_E_HIP, hipGetErrorString(er));
  }
  auto timed = [&](auto&& launch) -> double {
    float ms = 0.f;
    if (er == hipSuccess) er = hipEventRecord(e0, s);
    for (int r = 0; r < pr.reps && er == hipSuccess; ++r) er = launch();
    if (er == hipSuccess) er = hipEventRecord(e1, s);
    if (er == hipSuccess) er = hipEventSynchronize(e1);
    if (er == hipSuccess) er = hipEventElapsedTime(&ms, e0, e1);
    return 1e3 * ms / pr.reps;
  };
  // the step-begin kernel (stage-2 input from m and k1), then one full stage
  // so that every intermediate buffer holds data
  pr.us[0] = timed([&]() { return launch_begin<T>(gs, epi_slot<T>(E, 8), s); });
  if (er == hipSuccess) er = launch_eval<T>(gs, epi_slot<T>(E, 2), MODE_STAGE, demag_on(E), s);
  for (int i = 0; i < np && er == hipSuccess; ++i) {
    const unsigned bit = 1u << i;
    double acc = 0.0;
    if (i + 1 < np) {  // transform passes: the same kernels in every stage
      acc = timed([&]() { return launch_eval<T>(gs, epi_slot<T>(E, 2), MODE_STAGE, demag_on(E), s, nullptr, false,
                                                false, bit); });
    } else {  // inverse x with the stage epilogue: mean over stages 2..6
      for (int stg = 2; stg <= 6 && er == hipSuccess; ++stg)
        acc += timed([&]() { return launch_eval<T>(gs, epi_slot<T>(E, stg), MODE_STAGE, demag_on(E), s, nullptr,
                                                   false, fz, bit); });
      acc /= 5.0;
    }
    pr.us[1 + i] = acc;
  }
  const unsigned last = 1u << (np - 1);
  pr.us[np + 1] = timed([&]() { return launch_eval<T>(gs, epi_slot<T>(E, 7), MODE_ERROR, demag_on(E), s, nullptr,
                                                      false, false, last); });
  // In attempt order: whole attempts as the captured graph runs them (step
  // begin, then stages 2..7 pass by pass, the fused forward x transforms
  // included), an event before every kernel; seq[k] = mean duration of kernel
  // kind k over every launch of that kind (the caller's m is a copy here).
  if (pr.want_seq) {
    const int nslot = 2 + 6 * np;  // begin, x forward of stage 2, then np passes per stage
    std::vector<hipEvent_t> ev(nslot + 1, nullptr);
    for (auto& e : ev)
      if (er == hipSuccess) er = hipEventCreate(&e);
    std::vector<double> acc(16, 0.0);
    std::vector<int> cnt(16, 0);
    for (int r = 0; r < pr.reps && er == hipSuccess; ++r) {
      int k = 0;
      std::vector<int> kind;
      er = hipEventRecord(ev[k++], s);
      if (er == hipSuccess) er = launch_begin<T>(gs, epi_slot<T>(E, 8), s);
      kind.push_back(0);
      for (int stg = 2; stg <= 7 && er == hipSuccess; ++stg) {
        const int mode = stg < 7 ? MODE_STAGE : MODE_ERROR;
        for (int i = 0; i < np && er == hipSuccess; ++i) {
          if (i == 0 && demag_on(E) && fz && stg > 2) continue;  // done by the previous stage's fused pass
          er = hipEventRecord(ev[k++], s);
          if (er == hipSuccess)
            er = launch_eval<T>(gs, epi_slot<T>(E, stg), mode, demag_on(E), s, nullptr, fz && stg > 2,
                                fz && stg < 7, 1u << i);
          kind.push_back(i + 1 == np ? (stg < 7 ? np : np + 1) : 1 + i);
        }
      }
      if (er == hipSuccess) er = hipEventRecord(ev[k], s);
      if (er == hipSuccess) er = hipEventSynchronize(ev[k]);
      for (int j = 0; j < k && er == hipSuccess; ++j) {
        float ms = 0.f;
        er = hipEventElapsedTime(&ms, ev[j], ev[j + 1]);
        acc[kind[j]] += 1e3 * ms;
        cnt[kind[j]] += 1;
      }
    }
    for (int i = 0; i < np + 2; ++i) pr.seq[i] = cnt[i] > 0 ? acc[i] / cnt[i] : 0.0;
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  mm_status st = er == hipSuccess ? MM_OK : fail(MM_E_HIP, hipGetErrorString(er));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

// Integrate the instances of every group.  m[i]: contiguous state of group i's
// nb[i] instances; q / st / t_end: per instance, in group order.  With prof
// set, only times the attempt's kernels after the set-up (no state advance).
template <typename T>
mm_status run_core(Engine& E, const std::vector<T*>& m, const std::vector<int>& nb,
                   const std::vector<const mm_params*>& q, std::vector<mm_rk45_state*>& st,
                   const std::vector<double>& t_end, long long max_steps, const double* replay_h,
                   long long n_replay, bool single, std::vector<int>& status, hipStream_t s,
                   StepProfile* prof = nullptr, double stop = 0.0) {
  const int ng = (int)E.groups.size();
  const int n_total = (int)q.size();
  std::vector<int> grp;
  for (int i = 0; i < ng; ++i) grp.insert(grp.end(), nb[i], i);
  for (int i = 0; i < ng; ++i) MMCHK(ensure_stage<T>(E, E.groups[i], std::max(nb[i], 1)));
  MMCHK(upload_params(E, q, grp, s));
  GroupSet<T> gs;
  std::vector<int> inst0;
  MMCHK(make_set<T>(E, nb, gs, inst0, s));
  std::vector<const void*> k1_key;
  for (int i = 0; i < ng; ++i) {
    k1_key.push_back(m[i]);
    k1_key.push_back((const void*)(intptr_t)nb[i]);
  }
  bool need_k1 = !E.k1_ok || E.k1_key != k1_key;
  for (int b = 0; b < n_total; ++b) {
    const mm_rk45_state& r = *st[b];
    if (!(r.rtol > 0) || !is_fin(r.rtol) || !(r.h > 0) || !(r.h_min > 0) || !(r.h_max >= r.h_min) ||
        !is_fin(r.t) || !is_fin(r.h) || !is_fin(r.h_max))
      return fail(MM_E_ARG, "invalid rk45 state (rtol, h, h_min, h_max)");
    if (!r.fsal_valid) need_k1 = true;
  }
  if (replay_h) {
    if (n_replay < 1) return fail(MM_E_ARG, "n_replay must be >= 1");
    for (long long i = 0; i < n_replay; ++i)
      if (!(replay_h[i] > 0) || !is_fin(replay_h[i])) return fail(MM_E_ARG, "replay step sizes must be > 0");
    if (n_replay > E.replay_cap) {
      if (E.replay) (void)hipFree(E.replay);
      E.replay = nullptr;
      MMCHK(dev_alloc((void**)&E.replay, sizeof(double) * n_replay));
      E.replay_cap = n_replay;
      if (E.gexec) { (void)hipGraphExecDestroy(E.gexec); E.gexec = nullptr; }
    }
    HIPCHK(hipMemcpy(E.replay, replay_h, sizeof(double) * n_replay, hipMemcpyHostToDevice));
  }
  for (int b = 0; b < n_total; ++b) {
    const mm_rk45_state& r = *st[b];
    DevCtl& c = E.hctl[b];
    std::memset(&c, 0, sizeof(c));
    c.t = r.t; c.h = r.h; c.rtol = r.rtol; c.h_min = r.h_min; c.h_max = r.h_max;
    c.t_end = replay_h ? HUGE_VAL : t_end[b];
    c.n_accept = r.n_accept; c.n_reject = r.n_reject;
    c.max_attempt = max_steps;
    c.stop_dmdt = stop;
    c.replay_n = replay_h ? n_replay : 0;
    if (replay_h) {
      c.h_att = replay_h[0];
    } else {
      c.h_att = std::min(std::min(r.h, r.h_max), t_end[b] - r.t);
      if (!(t_end[b] - r.t > r.h_min)) c.done = 1;  // arrived (a remainder below h_min counts as arrived)
      else if (c.h_att < r.h_min) return fail(MM_E_STEP_UNDERFLOW, "initial step below h_min");
    }
  }
  HIPCHK(hipMemcpyAsync(E.ctl, E.hctl, sizeof(DevCtl) * n_total, hipMemcpyHostToDevice, s));
  MMCHK(upload_step_epis<T>(E, m, inst0, s));
  long long extra_rhs = 0;
  if (need_k1) {
    E.k1_ok = false;
    HIPCHK(eval_slot<T>(E, gs, 1, MODE_RHS, s));
    extra_rhs = 1;
  }
  E.k1_ok = true;  // k1 of these arrays from here on (the finishing step keeps it so)
  E.k1_key = k1_key;
  if (prof) return profile_step<T>(E, gs, *prof, s);
  if (single) {
    MMCHK(enqueue_attempt<T>(E, gs, n_total, s));
  } else {
    const int K = 8;  // attempts per graph launch between host polls
    std::vector<const void*> key;
    for (int i = 0; i < ng; ++i) {
      key.push_back(m[i]);
      key.push_back((const void*)(intptr_t)nb[i]);
    }
    key.push_back((const void*)(intptr_t)(demag_on(E) ? 1 : 0));
    if (!E.gexec || E.g_key != key) {
      if (E.gexec) { (void)hipGraphExecDestroy(E.gexec); E.gexec = nullptr; }
      HIPCHK(hipStreamBeginCapture(E.cap, hipStreamCaptureModeThreadLocal));
      mm_status cs = MM_OK;
      for (int k = 0; k < K && cs == MM_OK; ++k) cs = enqueue_attempt<T>(E, gs, n_total, E.cap);
      hipGraph_t graph = nullptr;
      hipError_t ee = hipStreamEndCapture(E.cap, &graph);
      if (cs != MM_OK) { if (graph) (void)hipGraphDestroy(graph); return cs; }
      if (ee != hipSuccess) return fail(MM_E_HIP, std::string("capture: ") + hipGetErrorString(ee));
      ee = hipGraphInstantiate(&E.gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ee != hipSuccess) { E.gexec = nullptr; return fail(MM_E_HIP, std::string("instantiate: ") + hipGetErrorString(ee)); }
      E.g_key = key;
    }
    // Up to two graph launches in flight, each followed by a copy of the
    // controllers into its own host buffer: the host reads one while the next
    // graph runs.  A further launch is queued only while some instance may
    // still have attempts left after the ones in flight (bounded by its
    // attempt limit as last seen), so a run bounded by max_steps launches no
    // graph that has nothing to do; one that ends at t_end may queue one
    // (every kernel of it returns at once for finished instances).
    for (hipEvent_t& ev : E.poll_ev)
      if (!ev) HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    DevCtl* const hb[2] = {E.hctl, E.hctl2};
    auto remaining = [&](const DevCtl* h, bool& all) {
      long long r = 0;
      all = true;
      for (int b = 0; b < n_total; ++b) {
        if (h[b].done) continue;
        all = false;
        r = std::max(r, h[b].max_attempt - h[b].n_attempt);
      }
      return r;
    };
    bool all = false;
    long long rem = remaining(E.hctl, all);  // the state just uploaded
    int head = 0, inflight = 0;
    auto launch = [&]() -> mm_status {
      const int slot = (head + inflight) & 1;
      HIPCHK(hipGraphLaunch(E.gexec, s));
      HIPCHK(hipMemcpyAsync(hb[slot], E.ctl, sizeof(DevCtl) * n_total, hipMemcpyDeviceToHost, s));
      HIPCHK(hipEventRecord(E.poll_ev[slot], s));
      ++inflight;
      return MM_OK;
    };
    if (!all) {
      MMCHK(launch());
      for (;;) {
        if (inflight < 2 && rem > (long long)K * inflight) MMCHK(launch());
        HIPCHK(hipEventSynchronize(E.poll_ev[head]));
        rem = remaining(hb[head], all);
        head ^= 1;
        --inflight;
        if (all) break;
        if (inflight == 0) MMCHK(launch());
      }
    }
    HIPCHK(hipStreamSynchronize(s));
  }
  // finish: project the last accepted y5 and move k7 into k1
  HIPCHK(launch_begin<T>(gs, epi_slot<T>(E, 8), s));
  HIPCHK(hipMemcpyAsync(E.hctl, E.ctl, sizeof(DevCtl) * n_total, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  status.assign(n_total, MM_OK);
  mm_status worst = MM_OK;
  for (int b = 0; b < n_total; ++b) {
    const DevCtl& c = E.hctl[b];
    mm_rk45_state& r = *st[b];
    r.t = c.t;
    r.h = c.h;
    r.n_rhs += 6 * c.n_attempt + extra_rhs;
    r.n_accept = c.n_accept;
    r.n_reject = c.n_reject;
    r.last_err = c.last_err;
    r.last_accepted = c.last_accepted;
    r.fsal_valid = 1;
    status[b] = c.status;
    if (c.status != MM_OK && worst == MM_OK) worst = (mm_status)c.status;
  }
  if (worst != MM_OK) return fail(worst, "integration stopped: " + std::string(mm_status_string(worst)));
  return MM_OK;
}

template <typename T>
mm_status plan_rk45(mm_plan* p, const mm_params* q, int batch, void* mv, mm_rk45_state* st, double t_end,
                    long long max_steps, const double* replay_h, long long n_replay, bool single, hipStream_t s,
                    StepProfile* prof = nullptr, double stop = 0.0) {
  std::vector<const mm_params*> qv(batch);
  std::vector<mm_rk45_state*> sv(batch);
  for (int b = 0; b < batch; ++b) {
    qv[b] = &q[b];
    sv[b] = &st[b];
  }
  std::vector<int> status;
  return run_core<T>(p->e, std::vector<T*>{(T*)mv}, std::vector<int>{batch}, qv, sv,
                     std::vector<double>(batch, t_end), max_steps, replay_h, n_replay, single, status, s, prof,
                     stop);
}

template <typename T>
mm_status batch_run(mm_batch* bt, mm_instance* inst, int n, long long max_steps, hipStream_t s) {
  Engine& E = bt->e;
  const int ng = (int)E.groups.size();
  std::vector<int> nb(ng, 0);
  std::vector<std::vector<int>> members(ng);
  for (int i = 0; i < n; ++i) members[inst[i].mesh_id].push_back(i);
  for (int g = 0; g < ng; ++g) nb[g] = (int)members[g].size();
  // launch shapes for the whole launch: one launch per pass covers every
  // instance of every group, so each mesh takes rows per workgroup up to the
  // LDS and thread limits when the launch has workgroups enough
  long long launch_rows = 0;
  for (int g = 0; g < ng; ++g) launch_rows += (long long)E.groups[g].g.nz * E.groups[g].g.ny * nb[g];
  for (int g = 0; g < ng; ++g) {
    Group& G = E.groups[g];
    if (nb[g] == 0 || launch_rows == G.tuned_for) continue;
    MMCHK(choose_tuning(G, E.prec, E.csz, launch_rows));
    G.tuned_for = launch_rows;
    if (E.gexec) { (void)hipGraphExecDestroy(E.gexec); E.gexec = nullptr; }
    E.k1_ok = false;
  }
  MMCHK(engine_reserve(E, nb));
  // gather every group's instances into its contiguous state buffer
  std::vector<T*> m(ng, nullptr);
  for (int g = 0; g < ng; ++g) {
    Group& G = E.groups[g];
    const size_t S = 3 * (size_t)G.g.N;
    if (nb[g] > G.mbuf_cap) {
      if (G.mbuf) (void)hipFree(G.mbuf);
      G.mbuf = nullptr;
      MMCHK(dev_alloc(&G.mbuf, sizeof(T) * S * nb[g]));
      G.mbuf_cap = nb[g];
      if (E.gexec) { (void)hipGraphExecDestroy(E.gexec); E.gexec = nullptr; }
    }
    m[g] = (T*)G.mbuf;
    for (int k = 0; k < nb[g]; ++k)
      HIPCHK(hipMemcpyAsync(m[g] + k * S, inst[members[g][k]].m, sizeof(T) * S, hipMemcpyDeviceToDevice, s));
  }
  std::vector<const mm_params*> q;
  std::vector<mm_rk45_state*> st;
  std::vector<double> t_end;
  std::vector<int> order;
  std::vector<const void*> who;  // the instances' own arrays, in group order
  for (int g = 0; g < ng; ++g)
    for (int i : members[g]) {
      q.push_back(&inst[i].p);
      st.push_back(&inst[i].st);
      t_end.push_back(inst[i].t_end);
      order.push_back(i);
      who.push_back(inst[i].m);
    }
  // the group buffers are the same for every run: the first slopes they hold
  // belong to the instances of the last run only
  if (who != E.batch_who) E.k1_ok = false;
  E.batch_who = who;
  std::vector<int> status;
  mm_status r = run_core<T>(E, m, nb, q, st, t_end, max_steps, nullptr, 0, false, status, s);
  // scatter back (also after an integration error: m holds the last accepted state)
  for (int g = 0; g < ng; ++g) {
    const size_t S = 3 * (size_t)E.groups[g].g.N;
    for (int k = 0; k < nb[g]; ++k)
      HIPCHK(hipMemcpyAsync(inst[members[g][k]].m, m[g] + k * S, sizeof(T) * S, hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  for (size_t j = 0; j < order.size(); ++j) inst[order[j]].status = j < status.size() ? status[j] : (int)r;
  return r;
}

template <typename T>
mm_status neb_impl(mm_plan* p, const mm_params* q, void* images, int n_img, double k, double h, long long n_iter,
                   double* E_out, hipStream_t s) {
  Engine& E = p->e;
  {  // launch shapes for all the images (one launch per pass), unless set by the caller
    Group& Gm = E.groups[0];
    const long long rows = (long long)Gm.g.nz * Gm.g.ny * n_img;
    if (!Gm.user_shapes && rows != Gm.tuned_for) {
      MMCHK(choose_tuning(Gm, E.prec, E.csz, rows));
      Gm.tuned_for = rows;
      MMCHK(engine_reserve(E, std::vector<int>{p->maxb}));
      if (E.gexec) { (void)hipGraphExecDestroy(E.gexec); E.gexec = nullptr; }
      E.k1_ok = false;
    }
  }
  const Group& G = E.groups[0];
  const size_t S = 3 * (size_t)G.g.N;
  if (E.neb_cap < n_img) {
    void* bufs[] = {E.nebH, E.nebB, E.nebS, E.nebP};
    for (void* b : bufs)
      if (b) (void)hipFree(b);
    const long long bpi = (G.g.N + 255) / 256;
    MMCHK(dev_alloc(&E.nebH, sizeof(T) * S * n_img));
    MMCHK(dev_alloc(&E.nebB, sizeof(T) * S * n_img));
    MMCHK(dev_alloc((void**)&E.nebS, sizeof(double) * 3 * n_img));
    MMCHK(dev_alloc((void**)&E.nebP, sizeof(double) * 3 * n_img * bpi));
    E.neb_cap = n_img;
  }
  std::vector<const mm_params*> qv(n_img, q);
  MMCHK(upload_params(E, qv, std::vector<int>(n_img, 0), s));
  GroupSet<T> gs;
  std::vector<int> inst0;
  MMCHK(make_set<T>(E, std::vector<int>{n_img}, gs, inst0, s));
  T* A = (T*)images;
  T* B = (T*)E.nebB;
  // slot 2 evaluates A, slot 3 evaluates B (fields and energy partials)
  for (int slot = 2; slot <= 3; ++slot) {
    std::vector<Epi<T>> ep(1, epi_base<T>(G, MODE_FIELD_ENERGY));
    ep[0].in = slot == 2 ? A : B;
    ep[0].out = (T*)E.nebH;
    ep[0].partial = E.partial;
    MMCHK(upload_epis<T>(E, slot, ep, s));
  }
  HIPCHK(hipMemcpyAsync(B, A, sizeof(T) * S * n_img, hipMemcpyDeviceToDevice, s));
  const double cq = -0.5 * kMu0 * q->Ms * G.g.dV, cz = -kMu0 * q->Ms * G.g.dV;
  const double hg2 = h * (-q->alpha * q->gamma / (1 + q->alpha * q->alpha));
  const int bpi = eval_blocks_per_inst(G.g, G.tu);
  auto iteration = [&](T* cur, T* nxt, hipStream_t ss) -> mm_status {
    HIPCHK(launch_eval<T>(gs, epi_slot<T>(E, cur == A ? 2 : 3), MODE_FIELD_ENERGY, demag_on(E), ss));
    HIPCHK(launch_energy_reduce(E.partial, n_img, bpi, E.e5, ss));
    HIPCHK(launch_neb<T>(G.g, n_img, cur, nxt, (const T*)E.nebH, E.e5, cq, cz, E.nebS, E.nebP, k, hg2, 0, ss));
    HIPCHK(launch_neb<T>(G.g, n_img, cur, nxt, (const T*)E.nebH, E.e5, cq, cz, E.nebS, E.nebP, k, hg2, 1, ss));
    return MM_OK;
  };
  // two iterations per captured graph (A -> B -> A)
  hipGraphExec_t ge = nullptr;
  if (n_iter >= 2) {
    HIPCHK(hipStreamBeginCapture(E.cap, hipStreamCaptureModeThreadLocal));
    mm_status cs = iteration(A, B, E.cap);
    if (cs == MM_OK) cs = iteration(B, A, E.cap);
    hipGraph_t graph = nullptr;
    hipError_t ee = hipStreamEndCapture(E.cap, &graph);
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
    st = iteration(A, B, s);
    if (st == MM_OK) {
      hipError_t ee = hipMemcpyAsync(A, B, sizeof(T) * S * n_img, hipMemcpyDeviceToDevice, s);
      if (ee != hipSuccess) st = fail(MM_E_HIP, hipGetErrorString(ee));
    }
  }
  if (ge) (void)hipGraphExecDestroy(ge);
  if (st != MM_OK) return st;
  if (n_iter == 0) {  // no iteration: the energies of the images as given
    HIPCHK(launch_eval<T>(gs, epi_slot<T>(E, 2), MODE_FIELD_ENERGY, demag_on(E), s));
    HIPCHK(launch_energy_reduce(E.partial, n_img, bpi, E.e5, s));
  }
  HIPCHK(hipMemcpyAsync(E.he5, E.e5, sizeof(double) * 5 * n_img, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (E_out)
    for (int n = 0; n < n_img; ++n) {
      const double* v = E.he5 + 5 * n;
      E_out[n] = cq * (v[0] + v[1] + v[2] + v[3]) + cz * v[4];
    }
  return MM_OK;
}

// Whether a launch shape is valid for a group (LDS, butterfly budget, cells
// per thread, workgroup size).
bool tuning_ok(const Group& G, const Tuning& t, mm_precision prec, size_t csz) {
  const Geo& g = G.g;
  auto tmin = [&](int L, bool allow16 = false) {
    return prec == MM_F32 ? min_tpc(make_fft<float>(L, nullptr, allow16))
                          : min_tpc(make_fft<double>(L, nullptr, allow16));
  };
  const size_t lim = 160 * 1024;
  const size_t rowb = (size_t)col_stride(g.Lx) * csz;
  const size_t xtab = (size_t)(2 * g.Lx + 1) * csz;
  const size_t ytab = (size_t)g.Py * csz;
  auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
  if (!pow2(t.ty_f) || !pow2(t.ty_x)) return false;
  if (t.ty_f < 1 || t.ty_f > g.ny || t.nt_f > 512 || t.nt_f < 64 || t.tpc_f * t.ty_f > t.nt_f) return false;
  if (t.tpc_f < tmin(g.Lx) || (size_t)t.ty_f * rowb + xtab > lim) return false;
  if (t.ty_x < 1 || t.ty_x > g.ny || t.nt_i > 512 || t.nt_i < 64 || 3 * t.tpc_x * t.ty_x > t.nt_i) return false;
  if (t.tpc_x < tmin(g.Lx) || (size_t)3 * t.ty_x * rowb + xtab > lim) return false;
  const size_t colb = (size_t)col_stride(g.Py) * csz;
  if (g.nz == 1) {
    if (t.cb_y2 < 1 || t.nt_y > 512 || t.tpc_y2 < tmin(g.Py, true) || 3 * t.cb_y2 * t.tpc_y2 > t.nt_y) return false;
    if (3 * t.cb_y2 * colb + ytab + (y2d_tensor_in_lds(g) ? (size_t)4 * (t.cb_y2 + y2d_packed(g)) * g.Ky * (csz / 2) : 0) > lim)
      return false;
  } else {
    if (t.cb_y < 1 || (t.cb_y % kSxB != 0 && kSxB % t.cb_y != 0) || t.nt_y > 512 || t.tpc_y < tmin(g.Py, true) || t.cb_y * t.tpc_y > t.nt_y)
      return false;
    if (t.cb_y * colb > lim) return false;
  }
  return true;
}

// Per-pass timing with the group's current shapes: each pass launched `reps`
// times back to back between two events (as mm_profile_passes does).
template <typename T>
mm_status time_passes(Engine& E, int batch, int reps, std::vector<double>& us, hipStream_t s) {
  GroupSet<T> gs;
  std::vector<int> inst0;
  MMCHK(make_set<T>(E, std::vector<int>{batch}, gs, inst0, s));
  const int np = pass_count(E);
  us.assign(np, 0.0);
  return time_each_pass<T>(E, gs, epi_slot<T>(E, 0), MODE_RHS, reps, np, us.data(), s);
}

// The first candidate (in the fixed order they were timed) whose time is
// within the run-to-run timing noise (3%) of the fastest: near-ties resolve
// the same way on every run.  `none` when nothing was timed.
inline Tuning first_near_best(const std::vector<std::pair<double, Tuning>>& timed, const Tuning& none) {
  double tmin = 1e300;
  for (const auto& c : timed) tmin = std::min(tmin, c.first);
  for (const auto& c : timed)
    if (c.first <= tmin * 1.03) return c.second;
  return none;
}

// Measure candidate launch shapes of each pass on the device and keep the
// fastest per pass (the passes' shapes are independent of each other).
template <typename T>
mm_status autotune_impl(mm_plan* p, const mm_params* q, int batch, const void* m, void* work, int reps,
                        hipStream_t s) {
  Engine& E = p->e;
  Group& G = E.groups[0];
  MMCHK(single_eval<T>(p, batch, q, m, work, MODE_RHS, nullptr, s));
  const Tuning base = G.tu;
  const int np = pass_count(E);
  const int last = np - 1;  // the inverse-x pass
  auto try_all = [&](const std::vector<Tuning>& cands, std::vector<int> passes, Tuning& best) -> mm_status {
    std::vector<std::pair<double, Tuning>> timed;
    for (const Tuning& c : cands) {
      if (!tuning_ok(G, c, E.prec, E.csz)) continue;
      G.tu = c;
      MMCHK(engine_reserve(E, std::vector<int>{p->maxb}));
      std::vector<double> us;
      MMCHK(time_passes<T>(E, batch, reps, us, s));
      double t = 0.0;
      for (int k : passes) t += us[k];
      timed.emplace_back(t, c);
    }
    best = first_near_best(timed, best);
    G.tu = best;
    return MM_OK;
  };
  Tuning best = base;
  if (demag_on(E)) {
    std::vector<Tuning> c;
    for (int ty : {1, 2, 4, 8, 16})
      for (int nt : {64, 128, 256, 512}) {
        Tuning t = best;
        t.ty_f = ty; t.nt_f = nt; t.tpc_f = nt / ty;
        c.push_back(t);
      }
    MMCHK(try_all(c, {0}, best));
    c.clear();
    const std::vector<int> cbs = G.g.nz == 1 ? std::vector<int>{1, 2, 3, 4, 6, 8} : std::vector<int>{1, 2, 4, 8, 12, 16};
    for (int cb : cbs)
      for (int tf : {1, 2, 4}) {
        Tuning t = best;
        const int tmin = E.prec == MM_F32 ? min_tpc(make_fft<float>(G.g.Py, nullptr, true))
                                          : min_tpc(make_fft<double>(G.g.Py, nullptr, true));
        if (G.g.nz == 1) {
          t.cb_y2 = cb; t.tpc_y2 = tmin * tf; t.nt_y = 3 * cb * t.tpc_y2;
        } else {
          t.cb_y = cb; t.tpc_y = tmin * tf; t.nt_y = cb * t.tpc_y;
        }
        c.push_back(t);
      }
    MMCHK(try_all(c, G.g.nz > 1 ? std::vector<int>{1, 3} : std::vector<int>{1}, best));
  }
  {
    // inverse-x shapes are chosen for the adaptive step, where the pass runs
    // with the stage epilogues (and, where the shape allows, the next stage's
    // forward x transform): cost = the inverse-x and forward-x launches of
    // one attempt, timed back to back from a temporary state
    std::vector<mm_rk45_state> tmp(batch);
    for (auto& r : tmp) {
      std::memset(&r, 0, sizeof(r));
      r.h = 1e-13; r.rtol = 1e-6; r.h_min = 1e-20; r.h_max = 1e-10;
    }
    std::vector<const mm_params*> qv(batch);
    std::vector<mm_rk45_state*> sv(batch);
    for (int b = 0; b < batch; ++b) { qv[b] = &q[b]; sv[b] = &tmp[b]; }
    std::vector<std::pair<double, Tuning>> timed;
    for (int ty : {1, 2, 4, 8, 16})
      for (int nt : {128, 256, 512}) {
        Tuning t = best;
        t.ty_x = ty; t.nt_i = nt; t.tpc_x = nt / (3 * ty);
        if (!tuning_ok(G, t, E.prec, E.csz)) continue;
        G.tu = t;
        MMCHK(engine_reserve(E, std::vector<int>{p->maxb}));
        StepProfile pr;
        pr.reps = reps;
        std::vector<int> status;
        MMCHK(run_core<T>(E, std::vector<T*>{(T*)const_cast<void*>(m)}, std::vector<int>{batch}, qv, sv,
                          std::vector<double>(batch, 1.0), kNoLimit, nullptr, 0, true, status, s, &pr));
        const int n = pr.n;  // begin, passes..., error
        double cost = 5.0 * pr.us[n - 2] + pr.us[n - 1];
        if (demag_on(E)) cost += (pr.fused ? 1.0 : 6.0) * pr.us[1];
        timed.emplace_back(cost, t);
      }
    best = first_near_best(timed, best);
    (void)last;
  }
  G.tu = best;
  G.user_shapes = true;
  E.k1_ok = false;  // the timing runs' stages used the stage buffers for its own state
  MMCHK(engine_reserve(E, std::vector<int>{p->maxb}));
  if (E.gexec) { (void)hipGraphExecDestroy(E.gexec); E.gexec = nullptr; }
  return MM_OK;
}

// Candidate padded lengths of one axis, the plan's default first: the default
// rule, the smallest 3-smooth length >= the minimum and the smallest power of
// two >= the minimum (x even; an axis of one cell off x keeps 1).
std::vector<int> padded_candidates(int n, bool even, bool pot) {
  std::vector<int> c{pot ? pick_padded_pot(n, even) : pick_padded(n, even)};
  if (n == 1 && !even) return c;
  const int lo = min_padded(n, pot);
  int s3 = lo;
  while (!(smooth3(s3) && (!even || s3 % 2 == 0))) ++s3;
  int p2 = 2;
  while (p2 < lo) p2 *= 2;
  for (int v : {s3, p2})
    if (std::find(c.begin(), c.end(), v) == c.end()) c.push_back(v);
  return c;
}

// Measure one dm/dt evaluation on every combination of the axes' candidate
// padded lengths (each built with its spectrum and default launch shapes) and
// keep the first within 3% of the fastest, in candidate order.
template <typename T>
mm_status tune_padding_impl(mm_plan* p, const mm_params* q, int batch, const void* m, void* work, int reps,
                            hipStream_t s) {
  Engine& E = p->e;
  Group& G = E.groups[0];
  const bool pot = (E.terms & MM_DEMAG_POTENTIAL) != 0;
  if (!(E.terms & (MM_DEMAG | MM_DEMAG_POTENTIAL))) return MM_OK;  // no transforms to size
  const std::vector<int> cx = padded_candidates(G.g.nx, true, pot);
  const std::vector<int> cy = padded_candidates(G.g.ny, false, pot);
  const std::vector<int> cz = padded_candidates(G.g.nz, false, pot);
  const int P0[3] = {G.g.Px, G.g.Py, G.g.Pz};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(MM_E_HIP, "hipEventCreate failed");
  }
  auto rebuild = [&](int Px, int Py, int Pz) -> mm_status {
    free_padded(E, G);
    MMCHK(build_padded(E, G, Px, Py, Pz, s));
    return engine_reserve(E, std::vector<int>{p->maxb});
  };
  std::vector<std::pair<double, std::array<int, 3>>> timed;
  mm_status st = MM_OK;
  for (int Px : cx)
    for (int Py : cy)
      for (int Pz : cz) {
        if (st != MM_OK) break;
        const double sy = (double)E.csz * 3.0 * G.g.nz * (Px / 2 + 1) * (double)Py;
        if (sy >= 4294967296.0) continue;  // one instance's spectrum must stay below 4 GiB
        st = rebuild(Px, Py, Pz);
        if (st == MM_E_ARG) {  // the grid does not fit the kernels' limits: not a candidate
          st = MM_OK;
          continue;
        }
        if (st == MM_OK) st = single_eval<T>(p, batch, q, m, work, MODE_RHS, nullptr, s);
        if (st != MM_OK) break;
        GroupSet<T> gs;
        std::vector<int> inst0;
        st = make_set<T>(E, std::vector<int>{batch}, gs, inst0, s);
        if (st != MM_OK) break;
        const Epi<T>* ep = epi_slot<T>(E, 0);
        hipError_t er = hipEventRecord(e0, s);
        for (int r = 0; r < reps && er == hipSuccess; ++r)
          er = E.any_pot ? launch_potential<T>(gs, ep, pot_tab<T>(G), MODE_RHS, s)
                         : launch_eval<T>(gs, ep, MODE_RHS, demag_on(E), s);
        if (er == hipSuccess) er = hipEventRecord(e1, s);
        if (er == hipSuccess) er = hipEventSynchronize(e1);
        float ms = 0.f;
        if (er == hipSuccess) er = hipEventElapsedTime(&ms, e0, e1);
        if (er != hipSuccess) st = fail(MM_E_HIP, hipGetErrorString(er));
        timed.push_back({(double)ms / reps, {Px, Py, Pz}});
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::array<int, 3> best = {P0[0], P0[1], P0[2]};
  if (st == MM_OK && !timed.empty()) {
    double tmin = 1e300;
    for (const auto& c : timed) tmin = std::min(tmin, c.first);
    for (const auto& c : timed)
      if (c.first <= tmin * 1.03) {
        best = c.second;
        break;
      }
  }
  // keep the choice (or, after a failure, go back to the default grid)
  const mm_status rs = rebuild(best[0], best[1], best[2]);
  return st != MM_OK ? st : rs;
}

// Calls a plan of the scalar-potential route serves: evaluations and the
// integrators (adaptive, Heun, steepest descent and their relaxations); not
// the attempt profiler or the autotuner, which time the Newell passes.
enum CallKind { kCallOther, kCallEval, kCallIntegrator };

mm_status plan_checks(mm_plan* p, const mm_params* q, int batch, CallKind kind = kCallOther) {
  if (!p) return fail(MM_E_ARG, "plan is null");
  if (batch < 1 || batch > p->maxb) return fail(MM_E_ARG, "batch must be in [1, max_batch]");
  MMCHK(check_params(p->e, q, batch));
  if (p->e.terms & MM_DEMAG_POTENTIAL) {
    if (kind == kCallOther)
      return fail(MM_E_ARG, "plans of the scalar-potential demag route serve evaluations and the integrators; "
                            "the attempt profiler and the autotuner time the Newell passes");
    for (int b = 0; b < batch; ++b)
      if (q[b].terms & kGeneralTerms)
        return fail(MM_E_ARG, "the scalar-potential demag route takes uniform material without interlayer or "
                              "torque terms");
  }
  const Group& G = p->e.groups[0];
  for (int b = 0; b < batch; ++b) {
    if ((q[b].terms & MM_CELLS) && (b >= (int)G.cells_set.size() || !G.cells_set[b]))
      return fail(MM_E_STATE, "instance " + std::to_string(b) + " uses MM_CELLS but mm_plan_set_cells was "
                              "not called for its slot");
    if ((q[b].terms & MM_INTERLAYER) && !(q[b].k_lo >= 0 && q[b].k_lo < q[b].k_hi && q[b].k_hi < G.g.nz))
      return fail(MM_E_ARG, "interlayer layers need 0 <= k_lo < k_hi < nz");
  }
  return MM_OK;
}

template <typename T>
mm_status set_cells_impl(mm_plan* p, int inst, const double* Ms, const double* A, const double* D, hipStream_t s) {
  Group& G = p->e.groups[0];
  const size_t N = (size_t)G.g.N;
  if (!G.cells) {
    MMCHK(dev_alloc(&G.cells, sizeof(T) * 3 * N * p->maxb));
    G.cells_set.assign(p->maxb, 0);
  }
  std::vector<T> h(3 * N);
  for (size_t i = 0; i < N; ++i) {
    h[i] = T(Ms[i]);
    h[N + i] = T(A[i]);
    h[2 * N + i] = T(D[i]);
  }
  HIPCHK(hipMemcpyAsync((T*)G.cells + (size_t)inst * 3 * N, h.data(), sizeof(T) * 3 * N, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  G.cells_set[inst] = 1;
  return MM_OK;
}

}  // namespace

// --- allocation-free steepest descent ---------------------------------------
// mm_sd_run allocates its per-block partial sums and step sizes on every call;
// mm_sd_run_noalloc takes them from `scratch`, a fixed array in device memory
// of kScratchBytes.  Each GPU the library runs on holds its own copy until the
// process ends.  In host code the array's name is not a device address: the
// address comes from hipGetSymbolAddress, once per device, with that device
// current, and only that address is passed to kernels and copies.
constexpr size_t kScratchBytes = size_t(16) << 20;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
namespace {
std::mutex g_scratch_mu;
unsigned char* g_scratch_at[kScratchDevices] = {};

mm_status scratch_address(unsigned char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices) return fail(MM_E_HIP, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(MM_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_at[dev] = (unsigned char*)ptr;
  }
  *out = g_scratch_at[dev];
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
  MMCHK(check_cells(mesh, prec));
  if (terms & ~MM_TERM_MASK) return fail(MM_E_ARG, "unknown term bits");
  if (max_batch < 1) return fail(MM_E_ARG, "max_batch must be >= 1");
  if (terms & MM_DEMAG_POTENTIAL) {
    if (terms & MM_DEMAG) return fail(MM_E_ARG, "MM_DEMAG_POTENTIAL replaces MM_DEMAG: not both");
    if (mesh->nz < 2) return fail(MM_E_ARG, "the scalar-potential demag route needs nz >= 2");
    if (terms & kGeneralTerms)
      return fail(MM_E_ARG, "the scalar-potential demag route takes uniform material without interlayer or "
                            "torque terms");
  }
  hipStream_t s = (hipStream_t)hip_stream;
  mm_plan* p = new mm_plan();
  p->maxb = max_batch;
  mm_status st = engine_init(p->e, prec, terms);
  if (st == MM_OK) {
    p->e.groups.emplace_back();
    st = make_group(p->e, *mesh, s, p->e.groups[0]);
  }
  if (st == MM_OK) st = engine_reserve(p->e, std::vector<int>{max_batch});
  if (st != MM_OK) {
    free_engine(p->e);
    delete p;
    return st;
  }
  *out = p;
  return MM_OK;
}

mm_status mm_plan_destroy(mm_plan* plan) {
  if (!plan) return fail(MM_E_ARG, "plan is null");
  (void)hipDeviceSynchronize();
  free_engine(plan->e);
  delete plan;
  return MM_OK;
}

mm_status mm_plan_set_cells(mm_plan* p, int32_t instance, const double* Ms, const double* A, const double* D,
                            void* hip_stream) {
  if (!p) return fail(MM_E_ARG, "plan is null");
  if (!(p->e.terms & MM_CELLS)) return fail(MM_E_ARG, "the plan was created without MM_CELLS");
  if (instance < 0 || instance >= p->maxb) return fail(MM_E_ARG, "instance must be in [0, max_batch)");
  if (!Ms || !A || !D) return fail(MM_E_ARG, "Ms, A and D must all be given");
  const long long N = p->e.groups[0].g.N;
  for (long long i = 0; i < N; ++i) {
    if (!is_fin(Ms[i]) || Ms[i] < 0) return fail(MM_E_ARG, "cell Ms must be finite and >= 0");
    if (!is_fin(A[i]) || A[i] < 0) return fail(MM_E_ARG, "cell A must be finite and >= 0");
    if (!is_fin(D[i])) return fail(MM_E_ARG, "cell D must be finite");
  }
  hipStream_t s = (hipStream_t)hip_stream;
  return p->e.prec == MM_F32 ? set_cells_impl<float>(p, instance, Ms, A, D, s)
                             : set_cells_impl<double>(p, instance, Ms, A, D, s);
}

mm_status mm_scalar_potential_kernel(const mm_mesh* mesh, const int32_t* disp, int64_t n, double* out,
                                     void* hip_stream) {
  MMCHK(check_mesh(mesh));
  if (n < 0) return fail(MM_E_ARG, "n must be >= 0");
  if (n > 0 && (!disp || !out)) return fail(MM_E_ARG, "null pointer");
  double nodes[5][16] = {}, wts[5][16] = {};
  const int nn[5] = {14, 9, 6, 4, 3};
  for (int r = 0; r < 5; ++r) gauss_legendre(nn[r], nodes[r], wts[r]);
  HIPCHK(setup_upload_pot_gauss(nodes, wts, nn));
  hipStream_t s = (hipStream_t)hip_stream;
  HIPCHK(setup_potential_list(*mesh, disp, n, out, s));
  HIPCHK(hipStreamSynchronize(s));
  return MM_OK;
}

mm_status mm_plan_padded(const mm_plan* p, int32_t* Px, int32_t* Py, int32_t* Pz) {
  if (!p || !Px || !Py || !Pz) return fail(MM_E_ARG, "null argument");
  const Geo& g = p->e.groups[0].g;
  *Px = g.Px; *Py = g.Py; *Pz = g.Pz;
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
  MMCHK(plan_checks(p, q, batch, kCallEval));
  if (!m || !H) return fail(MM_E_ARG, "null array");
  hipStream_t s = (hipStream_t)hip_stream;
  return p->e.prec == MM_F32 ? single_eval<float>(p, batch, q, m, H, MODE_FIELD, nullptr, s)
                             : single_eval<double>(p, batch, q, m, H, MODE_FIELD, nullptr, s);
}

mm_status mm_llg_rhs(mm_plan* p, const mm_params* q, int32_t batch, const void* m, void* dmdt, void* hip_stream) {
  MMCHK(plan_checks(p, q, batch, kCallEval));
  if (!m || !dmdt) return fail(MM_E_ARG, "null array");
  hipStream_t s = (hipStream_t)hip_stream;
  return p->e.prec == MM_F32 ? single_eval<float>(p, batch, q, m, dmdt, MODE_RHS, nullptr, s)
                             : single_eval<double>(p, batch, q, m, dmdt, MODE_RHS, nullptr, s);
}

mm_status mm_energy(mm_plan* p, const mm_params* q, int32_t batch, const void* m, double* E_out, void* hip_stream) {
  MMCHK(plan_checks(p, q, batch, kCallEval));
  if (!m || !E_out) return fail(MM_E_ARG, "null array");
  hipStream_t s = (hipStream_t)hip_stream;
  return p->e.prec == MM_F32 ? energy_impl<float>(p, q, batch, m, E_out, s)
                             : energy_impl<double>(p, q, batch, m, E_out, s);
}

mm_status mm_rk45_step(mm_plan* p, const mm_params* q, int32_t batch, void* m, mm_rk45_state* st,
                       void* hip_stream) {
  MMCHK(plan_checks(p, q, batch, kCallIntegrator));
  if (!m || !st) return fail(MM_E_ARG, "null array");
  hipStream_t s = (hipStream_t)hip_stream;
  return p->e.prec == MM_F32 ? plan_rk45<float>(p, q, batch, m, st, HUGE_VAL, 2, nullptr, 0, true, s)
                             : plan_rk45<double>(p, q, batch, m, st, HUGE_VAL, 2, nullptr, 0, true, s);
}

mm_status mm_rk45_run(mm_plan* p, const mm_params* q, int32_t batch, void* m, mm_rk45_state* st, double t_end,
                      int64_t max_steps, const double* replay_h, int64_t n_replay, void* hip_stream) {
  MMCHK(plan_checks(p, q, batch, kCallIntegrator));
  if (!m || !st) return fail(MM_E_ARG, "null array");
  if (max_steps < 1) return fail(MM_E_ARG, "max_steps must be >= 1");
  if (!replay_h && !is_fin(t_end)) return fail(MM_E_ARG, "t_end must be finite");
  hipStream_t s = (hipStream_t)hip_stream;
  return p->e.prec == MM_F32
             ? plan_rk45<float>(p, q, batch, m, st, t_end, max_steps, replay_h, n_replay, false, s)
             : plan_rk45<double>(p, q, batch, m, st, t_end, max_steps, replay_h, n_replay, false, s);
}

mm_status mm_sd_run(mm_plan* p, const mm_params* q, int32_t batch, void* m, int64_t n_iter, double tau0,
                    double tau_min, double tau_max, double* tau_out, void* hip_stream) {
  MMCHK(plan_checks(p, q, batch, kCallIntegrator));
  if (!m) return fail(MM_E_ARG, "null array");
  if (n_iter < 0) return fail(MM_E_ARG, "n_iter must be >= 0");
  if (!(tau_min > 0) || !is_fin(tau_max) || !(tau_min <= tau0) || !(tau0 <= tau_max))
    return fail(MM_E_ARG, "need 0 < tau_min <= tau0 <= tau_max (finite)");
  hipStream_t s = (hipStream_t)hip_stream;
  return p->e.prec == MM_F32
             ? sd_impl<float>(p, q, batch, (float*)m, n_iter, tau0, tau_min, tau_max, tau_out, 0.0, nullptr, nullptr, s)
             : sd_impl<double>(p, q, batch, (double*)m, n_iter, tau0, tau_min, tau_max, tau_out, 0.0, nullptr, nullptr,
                               s);
}

mm_status mm_sd_run_noalloc(mm_plan* p, const mm_params* q, int32_t batch, void* m, int64_t n_iter, double tau0,
                            double tau_min, double tau_max, double* tau_out, void* hip_stream) {
  MMCHK(plan_checks(p, q, batch, kCallIntegrator));
  if (!m) return fail(MM_E_ARG, "null array");
  if (n_iter < 0) return fail(MM_E_ARG, "n_iter must be >= 0");
  if (!(tau_min > 0) || !is_fin(tau_max) || !(tau_min <= tau0) || !(tau0 <= tau_max))
    return fail(MM_E_ARG, "need 0 < tau_min <= tau0 <= tau_max (finite)");
  const size_t need = sd_scratch_bytes(p->e.groups[0], batch);
  if (need > kScratchBytes)
    return fail(MM_E_ARG, "mm_sd_run_noalloc needs " + std::to_string(need) + " bytes of scratch for this batch; "
                          "the fixed scratch holds " + std::to_string(kScratchBytes));
  unsigned char* ptr = nullptr;
  MMCHK(scratch_address(&ptr));
  hipStream_t s = (hipStream_t)hip_stream;
  return p->e.prec == MM_F32
             ? sd_impl<float>(p, q, batch, (float*)m, n_iter, tau0, tau_min, tau_max, tau_out, 0.0, nullptr, nullptr, s,
                              ptr)
             : sd_impl<double>(p, q, batch, (double*)m, n_iter, tau0, tau_min, tau_max, tau_out, 0.0, nullptr, nullptr,
                               s, ptr);
}

// stopping_dmdt in degrees per nanosecond -> rad/s
static double dmdt_rad_s(double deg_ns) { return deg_ns * (M_PI / 180.0) * 1e9; }

mm_status mm_sd_relax(mm_plan* p, const mm_params* q, int32_t batch, void* m, double stopping_dmdt, int64_t max_iter,
                      double tau0, double tau_min, double tau_max, int64_t* iters_out, double* dmdt_out,
                      double* tau_out, void* hip_stream) {
  MMCHK(plan_checks(p, q, batch, kCallIntegrator));
  if (!m) return fail(MM_E_ARG, "null array");
  if (!(stopping_dmdt > 0) || !is_fin(stopping_dmdt)) return fail(MM_E_ARG, "stopping_dmdt must be finite and > 0");
  if (max_iter < 0) return fail(MM_E_ARG, "max_iter must be >= 0");
  if (!(tau_min > 0) || !is_fin(tau_max) || !(tau_min <= tau0) || !(tau0 <= tau_max))
    return fail(MM_E_ARG, "need 0 < tau_min <= tau0 <= tau_max (finite)");
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<long long> it(batch, 0);
  std::vector<double> dm(batch, 0.0);
  const double stop = dmdt_rad_s(stopping_dmdt);
  mm_status r = p->e.prec == MM_F32
                    ? sd_impl<float>(p, q, batch, (float*)m, max_iter, tau0, tau_min, tau_max, tau_out, stop, it.data(),
                                     dm.data(), s)
                    : sd_impl<double>(p, q, batch, (double*)m, max_iter, tau0, tau_min, tau_max, tau_out, stop,
                                      it.data(), dm.data(), s);
  if (r == MM_OK || r == MM_E_MAXSTEPS)
    for (int b = 0; b < batch; ++b) {
      if (iters_out) iters_out[b] = it[b];
      if (dmdt_out) dmdt_out[b] = dm[b] / dmdt_rad_s(1.0);
    }
  return r;
}

mm_status mm_rk45_relax(mm_plan* p, const mm_params* q, int32_t batch, void* m, mm_rk45_state* st,
                        double stopping_dmdt, int64_t max_steps, double* dmdt_out, void* hip_stream) {
  MMCHK(plan_checks(p, q, batch, kCallIntegrator));
  if (!m || !st) return fail(MM_E_ARG, "null array");
  if (!(stopping_dmdt > 0) || !is_fin(stopping_dmdt)) return fail(MM_E_ARG, "stopping_dmdt must be finite and > 0");
  if (max_steps < 1) return fail(MM_E_ARG, "max_steps must be >= 1");
  hipStream_t s = (hipStream_t)hip_stream;
  const double stop = dmdt_rad_s(stopping_dmdt);
  mm_status r = p->e.prec == MM_F32
                    ? plan_rk45<float>(p, q, batch, m, st, HUGE_VAL, max_steps, nullptr, 0, false, s, nullptr, stop)
                    : plan_rk45<double>(p, q, batch, m, st, HUGE_VAL, max_steps, nullptr, 0, false, s, nullptr, stop);
  if (dmdt_out && (r == MM_OK || r == MM_E_MAXSTEPS))
    for (int b = 0; b < batch; ++b) dmdt_out[b] = p->e.hctl[b].last_dmdt / dmdt_rad_s(1.0);
  return r;
}

mm_status mm_heun_run(mm_plan* p, const mm_params* q, int32_t batch, void* m, double h, int64_t n_steps,
                      void* hip_stream) {
  MMCHK(plan_checks(p, q, batch, kCallIntegrator));
  if (!m) return fail(MM_E_ARG, "null array");
  if (!(h > 0) || !is_fin(h)) return fail(MM_E_ARG, "h must be finite and > 0");
  if (n_steps < 0) return fail(MM_E_ARG, "n_steps must be >= 0");
  hipStream_t s = (hipStream_t)hip_stream;
  return p->e.prec == MM_F32 ? heun_impl<float>(p, q, batch, (float*)m, h, n_steps, s)
                             : heun_impl<double>(p, q, batch, (double*)m, h, n_steps, s);
}

mm_status mm_profile_step(mm_plan* p, const mm_params* q, int32_t batch, void* m, const mm_rk45_state* st,
                          int32_t reps, double* us_out, int32_t* n_out, int32_t* fused_out, double* seq_out,
                          void* hip_stream) {
  MMCHK(plan_checks(p, q, batch));
  if (!m || !st || !us_out || !n_out || !fused_out) return fail(MM_E_ARG, "null argument");
  if (reps < 1) return fail(MM_E_ARG, "reps must be >= 1");
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<mm_rk45_state> copy(st, st + batch);  // the caller's states are not advanced
  // ... nor its m: the attempts timed in order run on a copy
  const size_t bytes = p->e.rsz * 3 * (size_t)p->e.groups[0].g.N * batch;
  void* mc = nullptr;
  MMCHK(dev_alloc(&mc, bytes));
  hipError_t e = hipMemcpyAsync(mc, m, bytes, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) {
    (void)hipFree(mc);
    return fail(MM_E_HIP, hipGetErrorString(e));
  }
  StepProfile pr;
  pr.reps = reps;
  pr.want_seq = seq_out != nullptr;
  const double t_end = copy[0].t + 1.0;  // any end beyond one step
  mm_status r = p->e.prec == MM_F32
                    ? plan_rk45<float>(p, q, batch, mc, copy.data(), t_end, kNoLimit, nullptr, 0, true, s, &pr)
                    : plan_rk45<double>(p, q, batch, mc, copy.data(), t_end, kNoLimit, nullptr, 0, true, s, &pr);
  e = hipStreamSynchronize(s);
  (void)hipFree(mc);
  p->e.k1_ok = false;  // the first slopes belong to the copy
  if (r != MM_OK) return r;
  if (e != hipSuccess) return fail(MM_E_HIP, hipGetErrorString(e));
  for (int i = 0; i < pr.n; ++i) us_out[i] = pr.us[i];
  if (seq_out)
    for (int i = 0; i < pr.n; ++i) seq_out[i] = pr.seq[i];
  *n_out = pr.n;
  *fused_out = pr.fused;
  return MM_OK;
}

mm_status mm_profile_passes(mm_plan* p, const mm_params* q, int32_t batch, const void* m, void* work, int32_t reps,
                            double* us_out, int32_t* n_pass, double* seq_out, void* hip_stream) {
  MMCHK(plan_checks(p, q, batch, kCallEval));
  if (!m || !work || !us_out || !n_pass) return fail(MM_E_ARG, "null argument");
  if (reps < 1) return fail(MM_E_ARG, "reps must be >= 1");
  hipStream_t s = (hipStream_t)hip_stream;
  mm_status st = p->e.prec == MM_F32 ? profile_impl<float>(p, q, batch, m, work, reps, us_out, s, seq_out)
                                     : profile_impl<double>(p, q, batch, m, work, reps, us_out, s, seq_out);
  *n_pass = pass_count(p->e);
  return st;
}

// Launch shapes in the layout mm_plan_autotune reports.
static void shapes_of(const mm_plan* p, int32_t* out) {
  const Tuning& t = p->e.groups[0].tu;
  const bool d2 = p->e.groups[0].g.nz == 1;
  const int v[8] = {t.ty_f, t.nt_f, d2 ? t.cb_y2 : t.cb_y, d2 ? t.tpc_y2 : t.tpc_y, t.nt_y, t.ty_x, t.nt_i, 0};
  for (int i = 0; i < 8; ++i) out[i] = v[i];
}

mm_status mm_plan_autotune(mm_plan* p, const mm_params* q, int32_t batch, const void* m, void* work, int32_t reps,
                           int32_t* shape_out, void* hip_stream) {
  MMCHK(plan_checks(p, q, batch));
  if (!m || !work) return fail(MM_E_ARG, "null array");
  if (reps < 1) return fail(MM_E_ARG, "reps must be >= 1");
  hipStream_t s = (hipStream_t)hip_stream;
  MMCHK(p->e.prec == MM_F32 ? autotune_impl<float>(p, q, batch, m, work, reps, s)
                            : autotune_impl<double>(p, q, batch, m, work, reps, s));
  if (shape_out) shapes_of(p, shape_out);
  return MM_OK;
}

mm_status mm_plan_tune_padding(mm_plan* p, const mm_params* q, int32_t batch, const void* m, void* work,
                               int32_t reps, int32_t* padded_out, void* hip_stream) {
  MMCHK(plan_checks(p, q, batch, kCallEval));
  if (!m || !work) return fail(MM_E_ARG, "null pointer");
  if (reps < 1) return fail(MM_E_ARG, "reps must be >= 1");
  hipStream_t s = (hipStream_t)hip_stream;
  MMCHK(p->e.prec == MM_F32 ? tune_padding_impl<float>(p, q, batch, m, work, reps, s)
                            : tune_padding_impl<double>(p, q, batch, m, work, reps, s));
  if (padded_out) {
    padded_out[0] = p->e.groups[0].g.Px;
    padded_out[1] = p->e.groups[0].g.Py;
    padded_out[2] = p->e.groups[0].g.Pz;
  }
  return MM_OK;
}

mm_status mm_plan_shapes(const mm_plan* p, int32_t* shape_out) {
  if (!p || !shape_out) return fail(MM_E_ARG, "null pointer");
  shapes_of(p, shape_out);
  return MM_OK;
}

mm_status mm_plan_set_shapes(mm_plan* p, const int32_t* shape) {
  if (!p || !shape) return fail(MM_E_ARG, "null pointer");
  Group& G = p->e.groups[0];
  Tuning t = G.tu;
  t.ty_f = shape[0];
  t.nt_f = shape[1];
  t.tpc_f = t.ty_f > 0 ? t.nt_f / t.ty_f : 0;
  if (G.g.nz == 1) {
    t.cb_y2 = shape[2];
    t.tpc_y2 = shape[3];
  } else {
    t.cb_y = shape[2];
    t.tpc_y = shape[3];
  }
  t.nt_y = shape[4];
  t.ty_x = shape[5];
  t.nt_i = shape[6];
  t.tpc_x = t.ty_x > 0 ? t.nt_i / (3 * t.ty_x) : 0;
  if (!tuning_ok(G, t, p->e.prec, p->e.csz)) return fail(MM_E_ARG, "launch shapes not valid for this plan");
  if (p->e.terms & MM_DEMAG_POTENTIAL) {  // the scalar-potential passes derive their shapes from these
    const Tuning keep = G.tu;
    G.tu = t;
    const bool fits = p->e.prec == MM_F32 ? pot_fits<float>(G) : pot_fits<double>(G);
    G.tu = keep;
    if (!fits) return fail(MM_E_ARG, "launch shapes do not fit the scalar-potential route's passes");
  }
  G.tu = t;
  G.user_shapes = true;
  MMCHK(engine_reserve(p->e, std::vector<int>{p->maxb}));
  if (p->e.gexec) {
    (void)hipGraphExecDestroy(p->e.gexec);
    p->e.gexec = nullptr;
  }
  return MM_OK;
}

mm_status mm_neb_run(mm_plan* p, const mm_params* q, void* images, int32_t n_img, double k_spring, double h,
                     int64_t n_iter, double* E_out, void* hip_stream) {
  if (!p) return fail(MM_E_ARG, "plan is null");
  if (n_img < 3 || n_img > p->maxb) return fail(MM_E_ARG, "n_img must be in [3, max_batch]");
  MMCHK(check_params(p->e, q, 1));
  if ((q->terms & kGeneralTerms) || (p->e.terms & MM_DEMAG_POTENTIAL))
    return fail(MM_E_ARG, "NEB chains take uniform material, the Newell demag and no interlayer or torque terms");
  if (!images) return fail(MM_E_ARG, "images is null");
  if (!is_fin(k_spring) || !is_fin(h) || h <= 0 || n_iter < 0) return fail(MM_E_ARG, "invalid k_spring, h or n_iter");
  hipStream_t s = (hipStream_t)hip_stream;
  return p->e.prec == MM_F32 ? neb_impl<float>(p, q, images, n_img, k_spring, h, n_iter, E_out, s)
                             : neb_impl<double>(p, q, images, n_img, k_spring, h, n_iter, E_out, s);
}

mm_status mm_batch_create(mm_batch** out, const mm_mesh* meshes, int32_t n_meshes, mm_precision prec,
                          uint32_t terms, void* hip_stream) {
  if (!out) return fail(MM_E_ARG, "out is null");
  *out = nullptr;
  if (!meshes || n_meshes < 1 || n_meshes > kMaxGroups)
    return fail(MM_E_ARG, "need 1 to 16 meshes");
  for (int i = 0; i < n_meshes; ++i) MMCHK(check_mesh(&meshes[i]));
  if (prec != MM_F32 && prec != MM_F64) return fail(MM_E_ARG, "precision must be MM_F32 or MM_F64");
  for (int i = 0; i < n_meshes; ++i) MMCHK(check_cells(&meshes[i], prec));
  if (terms & ~MM_TERM_MASK) return fail(MM_E_ARG, "unknown term bits");
  if (terms & (kGeneralTerms | MM_DEMAG_POTENTIAL))
    return fail(MM_E_ARG, "batches take uniform material, the Newell demag and no interlayer or torque terms");
  hipStream_t s = (hipStream_t)hip_stream;
  mm_batch* b = new mm_batch();
  mm_status st = engine_init(b->e, prec, terms);
  b->e.groups.resize(n_meshes);
  for (int i = 0; i < n_meshes && st == MM_OK; ++i) st = make_group(b->e, meshes[i], s, b->e.groups[i]);
  if (st != MM_OK) {
    free_engine(b->e);
    delete b;
    return st;
  }
  *out = b;
  return MM_OK;
}

mm_status mm_batch_run(mm_batch* bt, mm_instance* inst, int32_t n_inst, int64_t max_steps, void* hip_stream) {
  if (!bt || !inst) return fail(MM_E_ARG, "null argument");
  if (n_inst < 1) return fail(MM_E_ARG, "n_inst must be >= 1");
  if (max_steps < 1) return fail(MM_E_ARG, "max_steps must be >= 1");
  const int ng = (int)bt->e.groups.size();
  for (int i = 0; i < n_inst; ++i) {
    if (inst[i].mesh_id < 0 || inst[i].mesh_id >= ng) return fail(MM_E_ARG, "mesh_id out of range");
    if (!inst[i].m) return fail(MM_E_ARG, "instance m is null");
    if (!is_fin(inst[i].t_end)) return fail(MM_E_ARG, "t_end must be finite");
    MMCHK(check_params(bt->e, &inst[i].p, 1));
  }
  hipStream_t s = (hipStream_t)hip_stream;
  return bt->e.prec == MM_F32 ? batch_run<float>(bt, inst, n_inst, max_steps, s)
                              : batch_run<double>(bt, inst, n_inst, max_steps, s);
}

mm_status mm_batch_destroy(mm_batch* bt) {
  if (!bt) return fail(MM_E_ARG, "batch is null");
  (void)hipDeviceSynchronize();
  free_engine(bt->e);
  delete bt;
  return MM_OK;
}

}  // extern "C"
