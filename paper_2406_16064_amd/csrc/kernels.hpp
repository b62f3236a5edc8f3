// Launch-side view of the hot-path kernels (geometry, stage arguments, launchers).
#pragma once

#include "mm_internal.hpp"

namespace mmx {

// x-pass buffer Sx, per instance and component:
//   2-D groups (nz = 1): [Xp][ny] -- columns of the fused y pass contiguous;
//   3-D groups: [nz][XB][ny][kSxB] -- kx in blocks of kSxB, so that the x passes
//     (TY rows: kSxB TY contiguous entries per block) and the y passes (a tile
//     of kSxB columns: one contiguous block) both move whole cache lines.
constexpr int kSxB = 4;

// Mesh and padded-grid geometry shared by every pass.
struct Geo {
  int nx, ny, nz;
  int Px, Py, Pz;
  int Lx;          // Px / 2: length of the packed complex x transform
  int Xp;          // Lx + 1: number of kx kept after the real-to-complex transform
  int Ky, Kz;      // Py/2 + 1, Pz/2 + 1: folded extents of the tensor spectrum
  int XB;          // 3-D groups: kx blocks of kSxB in the x-pass buffer, ceil(Xp / kSxB)
  int pad_;
  long long N;     // cells per instance
  long long sx;    // complex elements of the x-pass buffer per instance (layouts below)
  long long sy;    // complex elements of the y-pass buffer per instance: 3*nz*Xp*Py
  double dV;       // cell volume
};

enum Mode : int {
  MODE_FIELD = 0,        // write H_eff
  MODE_RHS = 1,          // write dm/dt
  MODE_STAGE = 2,        // write k_s and the next Runge-Kutta stage input
  MODE_ERROR = 3,        // write k_7 and reduce the embedded error norm
  MODE_ENERGY = 4,       // per-term energy partial sums
  MODE_FIELD_ENERGY = 5  // write H_eff and energy partial sums (NEB)
};

// What one launch does for one group of instances (a group = instances that
// share a mesh): the evaluated input, the fused epilogue after H_eff is known
// at a cell, and the arguments of the step-begin kernel.
template <typename T> struct Epi {
  int mode;
  const T* in;            // magnetisation evaluated by this pass sequence
  T* out;                 // H (FIELD*), dm/dt (RHS), k_s (STAGE/ERROR)
  const T* mbase;         // m at the start of the step (STAGE)
  T* msn;                 // next stage input (STAGE)
  const T* kprev[7];      // k_1..k_7 (entries used by coef)
  double coef[7];         // stage: a_{s+1,j}; error: b_j - bhat_j; multiplied by h_att
  int nk;                 // number of k entries combined (including the current one)
  int project;            // STAGE: store the next stage input projected onto |m| = 1
  double* partial;        // energy partials [batch][blocks_per_inst][5]
  DevCtl* ctl;            // per-instance controller (skip done instances; h_att; err)
  const double* replay;   // MODE_ERROR: replayed step sizes (controller in the last workgroup)
  long long inst_stride;  // elements per instance of m-like arrays (3N)
  // step begin
  T* bm;
  T* bms0;
  const T* bms1;
  T* bk1;
  const T* bk7;
  double a21;
};

// The fused 2-D y pass stages the tensor rows of its kx columns in LDS up to
// Py = 1024; longer columns read them from global memory in the product loop,
// which keeps two workgroups per CU (three 2048-point columns and the twiddle
// table take 71 KB of LDS).  Host and kernel size the LDS by this predicate.
__host__ __device__ inline bool y2d_tensor_in_lds(const Geo& g) { return g.Py <= 1024; }

// From Py = 1024 on, the fused 2-D y pass carries the kx = 0 and kx = Lx
// columns (both real in y) as one complex column, Lx workgroup slots instead
// of Lx + 1: the extra workgroup of a kx = Lx column unbalances the CUs once
// each column takes long (Py = 1024, 2048: 7% a pass); at Py = 512 the longer
// packed workgroup costs more than the balance gains.
__host__ __device__ inline bool y2d_packed(const Geo& g) { return g.Py >= 1024; }

struct Tuning {
  int ty_f;     // rows per workgroup of the forward x pass
  int tpc_f;    // threads per row of its transform
  int nt_f;     // threads per workgroup
  int ty_x;     // rows per workgroup of the inverse x pass + epilogue
  int tpc_x;    // threads per column there (3 * ty_x columns)
  int nt_i;
  int cb_y;     // columns per workgroup of the 3-D y passes
  int tpc_y;
  int cb_y2;    // kx columns per workgroup of the fused 2-D y pass (x3 components)
  int tpc_y2;
  int nt_y;     // threads per workgroup of the y passes
  int qz;       // (kx,ky) columns per workgroup of the LDS z pass (x3 components)
  int tpc_z;
};

// Static description of one group (device resident, one entry per group).
template <typename T> struct HotPlan {
  Geo g;
  Tuning tu;
  FftDesc<T> fd[3];        // x (length Px/2), y (Py), z (Pz) radix plans
  const Cx<T>* twz;        // z twiddles (register z pass)
  const Cx<T>* post;       // exp(-2 pi i k / Px), k = 0..Lx
  const T* kt;             // tensor spectrum [ncomp][Kz][Xp][Ky]
  int ncomp;               // 4 (nz = 1) or 6
  int batch;               // instances in the group
  Cx<T>* Sx;               // [batch][sx] (layout above)
  Cx<T>* Sy;               // [batch][3][nz][Xp][Py] (3-D only)
  const DevParams* prm;    // [batch]
  const T* cells;          // cell-based material [batch][3][N] (Ms, A, D per cell) or null
  int gen;                 // launch the general-material form of the inverse-x epilogue
  int pad_;
};

constexpr int kMaxGroups = 16;

// Kernel argument of every hot-path launch: the groups it covers and where
// each group's workgroups start (multiples of 8, so the XCD of a workgroup
// follows its index inside the group).
template <typename T> struct Launch {
  const HotPlan<T>* hps;     // device [ngroups]
  const Epi<T>* epis;        // device [ngroups]
  int ngroups;
  int off[kMaxGroups + 1];   // off[ngroups] = grid size
  HotPlan<T> h0;             // copy of hps[0]: group 0 reads its plan with the kernel
                             // arguments (one scalar memory round trip less)
};

// Host-side view of a set of groups for launching.
template <typename T> struct GroupSet {
  int n;
  HotPlan<T> h[kMaxGroups];  // host copies (block counts, launch shapes)
  const HotPlan<T>* dh;      // device copies
};

// One effective-field evaluation with the fused epilogue for every group
// (epis: device array [n], all with epilogue `mode`).  With ev != nullptr an
// event is recorded before each pass and after the last one (pass timing;
// single group only).
// skip_fwd: the forward x pass was already done by the previous launch's
// inverse-x pass (fuse_next there).  fuse_next (MODE_STAGE): the inverse-x
// pass also transforms the next stage input forward along x; ignored where
// the launch shape does not allow it -- eval_fusable() tells in advance.
// pass_mask: bit p launches pass p (0 x forward, 1 y, 2 z, 3 y inverse, then
// x inverse: bit 4 in 3-D, bit 2 in 2-D, bit 0 without demag) -- for timing
// single passes.
template <typename T>
hipError_t launch_eval(const GroupSet<T>& gs, const Epi<T>* epis, int mode, bool demag, hipStream_t s,
                       hipEvent_t* ev = nullptr, bool skip_fwd = false, bool fuse_next = false,
                       unsigned pass_mask = ~0u);

template <typename T>
bool eval_fusable(const GroupSet<T>& gs);

template <typename T>
hipError_t launch_begin(const GroupSet<T>& gs, const Epi<T>* epis, hipStream_t s);

hipError_t launch_controller(DevCtl* ctl, int n, const double* replay_h, hipStream_t s);
// One steepest-descent iteration k of `batch` instances after H = H_eff(m):
// g = m x (m x H), for k >= 1 the Barzilai-Borwein step from the block sums
// (part: batch x ceil(N / 256) x 4 doubles) into tau[b], then m_prev, g_prev
// and the update of m.  Arrays [batch][3][N].  With ctl (a relaxation; prm
// gives the LL coefficients): first the stopping rule on the largest |dm/dt|
// of m (ctl[b].stop_dmdt, rad/s), done instances skipped from then on; `last`
// only checks (no update) and marks every instance done.
template <typename T>
hipError_t launch_sd_iteration(T* m, const T* H, T* g, T* mp, T* gp, double* part, double* tau, int batch,
                               long long N, long long k, double tau_min, double tau_max, const DevParams* prm,
                               DevCtl* ctl, bool last, hipStream_t s);

hipError_t launch_energy_reduce(const double* partial, int batch, int blocks_per_inst, double* out,
                                hipStream_t s);

int eval_blocks_per_inst(const Geo& g, const Tuning& tu);

// NEB: tangent/projection sums (pass 0) and the relaxation update (pass 1) of one chain.
template <typename T>
hipError_t launch_neb(const Geo& g, int n_img, const T* img, T* img_out, const T* H,
                      const double* E5, double cq, double cz, double* sums, double* partial,
                      double k_spring, double h_g2, int pass, hipStream_t s);

}  // namespace mmx
