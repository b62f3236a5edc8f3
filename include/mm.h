/*
 * mm.h -- C interface of the MI355X finite-difference micromagnetics hot path.
 *
 * The library evaluates the effective field of a regular cell mesh (demag by a
 * zero-padded FFT convolution with the cell-averaged Newell tensor, six-neighbour
 * exchange, interfacial DMI, uniaxial anisotropy, Zeeman), the Landau-Lifshitz
 * right-hand side, and advances it with adaptive Dormand-Prince 5(4) plus
 * projection onto the unit sphere.  Paper: MicroMagnetic.jl (arXiv 2406.16064),
 * sections "Micromagnetics" (effective field, exchange, magnetostatic energy
 * eq_demag_energy2 / eq_hd1, DMI), "Atomistic Spin Model / Anisotropy" and
 * "Zeeman energy" (the field forms written per cell), "LLG equation" (eq_llg2,
 * the adaptive Dormand-Prince method and projection), "Miscellaneous" (NEB).
 *
 * Conventions shared by every call
 * --------------------------------
 * - SI units: lengths in m, fields in A/m, Ms in A/m, A in J/m, D in J/m^2,
 *   Ku in J/m^3, gamma in m/(A s), time in s, energies in J.
 * - Magnetisation / field arrays are DEVICE pointers, structure of arrays
 *   [batch][3][nz][ny][nx], x fastest, element type = the plan's precision
 *   (float for MM_F32, double for MM_F64).  The caller owns them.
 * - Compute calls are ordered on the given HIP stream (hipStream_t passed as
 *   void*; NULL = the default stream) and return before the work finishes,
 *   except where a call says it synchronises.
 * - Every call returns an mm_status.  Arguments are validated before any HIP
 *   call; on MM_E_ARG nothing is launched.  mm_last_error() gives a
 *   thread-local message for the last failure.  On an integration error the
 *   magnetisation holds the last accepted state.
 * - Plans are not thread safe; use one plan per host thread.
 */
#ifndef MM_H
#define MM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MM_OK = 0,
  MM_E_ARG = -1,            /* invalid argument (sizes, parameters, null pointers)   */
  MM_E_NOMEM = -2,          /* device allocation failed                              */
  MM_E_HIP = -3,            /* a HIP runtime call failed (message in mm_last_error)  */
  MM_E_NONFINITE = -4,      /* NaN/Inf met in the error norm of a step               */
  MM_E_STEP_UNDERFLOW = -5, /* adaptive step fell below h_min                        */
  MM_E_MAXSTEPS = -6,       /* attempted-step limit reached before t_end             */
  MM_E_STATE = -7           /* call not valid in the current plan state              */
} mm_status;

typedef enum { MM_F32 = 0, MM_F64 = 1 } mm_precision;

/* effective-field terms (bit set) */
enum {
  MM_EXCHANGE = 1u,         /* six-neighbour exchange, open boundaries              */
  MM_DEMAG = 2u,            /* Newell-tensor convolution, zero padded               */
  MM_DMI_INTERFACIAL = 4u,  /* interfacial (C_nv) DMI, e_ij = e_z x r_ij            */
  MM_ANIS_UNIAXIAL = 8u,    /* uniaxial anisotropy, easy axis u                     */
  MM_ZEEMAN = 16u,          /* uniform static applied field                         */
  MM_DMI_BULK = 32u,        /* bulk (classes T, O) DMI, e_ij = r_ij                 */
  MM_DMI_D2D = 64u,         /* class D2d DMI, e_ij = {e_x, -e_x, -e_y, e_y, 0, 0}   */
  MM_CELLS = 128u,          /* cell-based Ms, A, D of the instance (mm_plan_set_cells) */
  MM_INTERLAYER = 256u,     /* RKKY and interlayer DMI between layers k_lo and k_hi   */
  MM_STT_SOT = 512u,        /* Slonczewski / spin-orbit torque (a_J, b_J, p)          */
  MM_STT_ZL = 1024u,        /* Zhang-Li spin-transfer torque (u_zl, beta)             */
  MM_DEMAG_POTENTIAL = 2048u /* demag through the magnetic scalar potential            */
};
/* the five terms of the standard path; MM_TERM_MASK: every known bit.  The
 * three DMI classes share the constant D; each enabled one adds its field
 * (section "Dzyaloshinskii-Moriya Energy", the unified neighbour form) and
 * its energy to the DMI entry. */
#define MM_ALL_TERMS 31u
#define MM_TERM_MASK 4095u

/* Regular mesh of nx*ny*nz cuboid cells of size dx*dy*dz (paper: FDMesh).
 * Limits: 1 <= n <= 1024 per axis, nx >= 2; d > 0 and finite. */
typedef struct { int32_t nx, ny, nz; double dx, dy, dz; } mm_mesh;

/* Uniform material and field parameters of one instance.
 * u: easy axis (normalised by the library); H: applied field (A/m).
 * alpha >= 0, gamma > 0 (2.21e5 is the paper's value), Ms > 0.
 * terms: subset of the plan's terms that is switched on.
 * The fields after `terms` are read only when their term is on:
 * MM_INTERLAYER (section "Interlayer Exchange Interaction"): layers
 *   z = k_lo and z = k_hi (0 <= k_lo < k_hi < nz) couple cell by cell (x, y)
 *   with the energy per area -J_rkky m_lo . m_hi + D_int . (m_lo x m_hi)
 *   (J/m^2); the field at k_lo is (J_rkky m_hi + D_int x m_hi)/(mu0 Ms dz), at
 *   k_hi (J_rkky m_lo - D_int x m_lo)/(mu0 Ms dz); only magnetic pairs couple.
 *   Its energies add to the exchange (RKKY) and DMI (interlayer DMI) entries.
 * MM_STT_SOT (section "Spin transfer torques", eq_llg_stt2): the torque
 *   -a_J m x (m x p) - b_J m x p (a_J, b_J in 1/s; p normalised by the
 *   library), folded into H_eff as (b_J p + a_J m x p)/gamma.
 * MM_STT_ZL (eq_llg_stt, Zhang-Li): -(u . grad) m + beta m x (u . grad) m with
 *   the drift velocity u_zl (m/s), folded into H_eff as -(m x v + beta v)/gamma,
 *   v = (u . grad) m by central differences (one-sided next to a missing or
 *   empty neighbour, zero with neither).
 * Torques carry no energy.  These three terms and MM_CELLS run in the
 * general-material form of the inverse-x epilogue (plans only; batches and
 * NEB chains refuse them). */
typedef struct {
  double Ms, A, D, Ku;
  double u[3];
  double H[3];
  double alpha, gamma;
  uint32_t terms;
  int32_t k_lo, k_hi;
  double J_rkky;
  double D_int[3];
  double a_J, b_J;
  double p[3];
  double u_zl[3];
  double beta;
} mm_params;

/* Adaptive Dormand-Prince state of one instance (caller owned, plain data so it
 * can be saved next to m for checkpoint/resume).
 * Inputs:  t, h (next step to try), rtol (> 0; also the absolute tolerance,
 *          since |m| = 1), h_min, h_max, fsal_valid (set 0 whenever m was
 *          changed outside the library, which forces a fresh first slope).
 *          The library also recomputes the first slope by itself when the
 *          run is on other arrays than the plan's last adaptive run, or when
 *          a Heun, steepest-descent or autotune call (or a larger batch) has
 *          reused the plan's stage buffers since.
 * Outputs: t, h, counters, last_err (error norm / rtol of the last attempt),
 *          last_accepted, fsal_valid. */
typedef struct {
  double t, h, rtol, h_min, h_max;
  int64_t n_accept, n_reject, n_rhs;
  double last_err;
  int32_t last_accepted;
  int32_t fsal_valid;
} mm_rk45_state;

typedef struct mm_plan mm_plan;

/* Create a plan for `max_batch` instances that share one mesh (the tensor
 * spectrum is shared; parameters are per instance).  Builds the Newell tensor
 * (FP64) and its spectrum on the device, then casts it to the plan precision.
 * `terms` is the set of terms any later call may enable.  Synchronises.
 * MM_E_ARG also when one instance's [3][nx ny nz] array would take 4 GiB or
 * more (the kernels address it with 32-bit offsets).
 * Paper: section "Magnetostatic energy" (Newell tensor, FFT acceleration). */
mm_status mm_plan_create(mm_plan** out, const mm_mesh* mesh, mm_precision prec,
                         uint32_t terms, int32_t max_batch, void* hip_stream);
mm_status mm_plan_destroy(mm_plan* plan);

/* Cell-based material of instance slot `instance` (0 <= instance < max_batch)
 * of a plan created with MM_CELLS among its terms: per-cell saturation
 * magnetisation Ms (A/m, >= 0), exchange constant A (J/m, >= 0) and DMI
 * constant D (J/m^2), host FP64 arrays [nz][ny][nx] (x fastest), copied (in
 * the plan precision) before the call returns.  Instances whose params.terms
 * include MM_CELLS use them in place of params.Ms, A and D (which are then
 * ignored; Ku, u, H, alpha, gamma stay uniform).  Paper: section "Design"
 * (set_Ms with a function of position: cells with Ms = 0 lie outside the
 * sample), section "Exchange energy" (cell-based A_i, pair coefficient
 * A_ij = 2 A_i A_j / (A_i + A_j)) and the last sentence of section
 * "Dzyaloshinskii-Moriya Energy" (D_ij = 2 D_i D_j / (D_i + D_j)).  Readings:
 * an empty cell (Ms = 0) has H = 0 and dm/dt = 0 and is nobody's neighbour;
 * D_ij = 0 unless D_i D_j > 0; A_ij = 0 when A_i + A_j = 0; the demag input is
 * M = Ms_i m_i; energies weight each cell by its Ms_i.  m must hold unit
 * vectors in every cell, empty ones included (they are carried unchanged).
 * Instances of one call may mix cell-based and uniform material;
 * MM_E_STATE when a call's instance uses MM_CELLS before its slot was set.
 * Batches (mm_batch_*) and NEB chains take uniform material only.
 * Allocates the plan's cell arrays on first use; synchronises. */
mm_status mm_plan_set_cells(mm_plan* plan, int32_t instance, const double* Ms, const double* A, const double* D,
                            void* hip_stream);

/* MM_DEMAG_POTENTIAL: the demag field through the magnetic scalar potential,
 * the route of section "Magnetostatic energy" that replaces the three inverse
 * transforms of the demag field by one.  Reading (the paper prints no
 * formulas): u(r) = sum_j Ms m_j . S(r - r_j), S the potential of a uniformly
 * magnetised unit cuboid (the closed form of its two charged faces near the
 * cell, quadrature of the defining integral far from it), evaluated at the
 * cell corners; the field of a cell is -(1/(4 d_a)) times the sum over its
 * four a-edges of u(+ end) - u(- end), which tends to the Newell field as the
 * mesh is refined.  A plan takes MM_DEMAG_POTENTIAL in place of MM_DEMAG (not
 * both); it needs nz >= 2 (on one-cell films the two vertex planes would
 * still take two inverse transforms), pads to P >= 2n per axis, and serves
 * mm_effective_field, mm_llg_rhs, mm_energy, mm_profile_passes,
 * mm_plan_set_shapes and the integrators (mm_rk45_*, mm_heun_run, mm_sd_*:
 * every stage runs the five potential passes, none fused into the previous
 * one); mm_profile_step, mm_plan_autotune, NEB and batches refuse such plans
 * with MM_E_ARG.  Uniform material only.  Instances switch the term on with
 * the same bit. */

/* The cuboid potential S at the vertex - cell displacements
 * ((I - 1/2) dx, (J - 1/2) dy, (K - 1/2) dz), disp[k] = (I, J, K) (device int32
 * [n][3]); out: device double [n][3] (S_x, S_y, S_z, in m).  FP64. */
mm_status mm_scalar_potential_kernel(const mm_mesh* mesh, const int32_t* disp, int64_t n, double* out,
                                     void* hip_stream);

/* Padded FFT grid chosen for the plan (each P >= 2n-1; x even). */
mm_status mm_plan_padded(const mm_plan* plan, int32_t* Px, int32_t* Py, int32_t* Pz);

/* Newell tensor entries at integer displacements disp[k] = (I,J,K) (device
 * int32 array [n][3]); out is a device double array [n][6] ordered
 * xx, yy, zz, xy, xz, yz.  FP64; synchronous w.r.t. the stream on return of
 * data only after a stream sync.  Paper: eq_demag_energy2 / eq_hd1. */
mm_status mm_demag_tensor(const mm_mesh* mesh, const int32_t* disp, int64_t n,
                          double* out, void* hip_stream);

/* H_eff of `batch` instances: m, H are [batch][3][nz][ny][nx] device arrays;
 * params is a host array of `batch` entries.  Paper: H_eff = -(1/mu0 Ms) dE/dm
 * and the per-term formulas of section "Micromagnetics". */
mm_status mm_effective_field(mm_plan* plan, const mm_params* params, int32_t batch,
                             const void* m, void* H, void* hip_stream);

/* dm/dt of the LL form (eq_llg2) for `batch` instances; same layout as above. */
mm_status mm_llg_rhs(mm_plan* plan, const mm_params* params, int32_t batch,
                     const void* m, void* dmdt, void* hip_stream);

/* Energies in J of `batch` instances, E_out[batch][5] host array ordered
 * exchange, demag, dmi, anisotropy, zeeman (disabled terms give 0).  FP64
 * accumulation.  Synchronises.  Paper: w_i (exchange), eq_demag_energy. */
mm_status mm_energy(mm_plan* plan, const mm_params* params, int32_t batch,
                    const void* m, double* E_out, void* hip_stream);

/* One attempted adaptive Dormand-Prince step per instance (accepted or
 * rejected, recorded in st[b]); m is projected onto |m| = 1 after an accepted
 * step.  st is a host array of `batch` states.  Synchronises.
 * Paper: section "LLG equation". */
mm_status mm_rk45_step(mm_plan* plan, const mm_params* params, int32_t batch,
                       void* m, mm_rk45_state* st, void* hip_stream);

/* Integrate every instance to t_end (or, with replay_h, take exactly the
 * n_replay accepted steps replay_h[0..n_replay) of host memory, shared by all
 * instances).  max_steps bounds the attempts per instance.  Steps run under a
 * device-side controller and a captured HIP graph; the host only polls.
 * Synchronises.  Returns the first non-OK instance status. */
mm_status mm_rk45_run(mm_plan* plan, const mm_params* params, int32_t batch,
                      void* m, mm_rk45_state* st, double t_end, int64_t max_steps,
                      const double* replay_h, int64_t n_replay, void* hip_stream);

/* Fixed-step Heun integration (explicit trapezoid: k1 = f(m), k2 = f(m + h k1),
 * m <- m + h (k1 + k2) / 2) of `batch` instances in place, each step followed
 * by the projection m <- m / |m| per cell; n_steps steps of size h (seconds,
 * finite, > 0; n_steps >= 0).  No error control.  Paper: the integrator of
 * the section "Performance" (N x N x 1 films, demagnetisation + exchange +
 * Zeeman); the projection as in section "LLG equation".  Uses the plan's
 * stage buffers: a later mm_rk45_* call on the plan recomputes its first
 * slope, whatever fsal_valid says.  Asynchronous on hip_stream apart from the
 * upload of the step tables. */
mm_status mm_heun_run(mm_plan* plan, const mm_params* params, int32_t batch, void* m, double h,
                      int64_t n_steps, void* hip_stream);

/* Energy minimisation by steepest descent with Barzilai-Borwein step sizes
 * (section "Steepest descent energy minimization", eq_update): n_iter
 * iterations on `batch` instances in place.  Per cell, f = m x H_eff and
 * g = m x f; (1 + tau^2 |f|^2 / 4) m' = (1 - tau^2 |f|^2 / 4) m - tau g (|m|
 * kept).  tau (m/A, one per instance): tau0 at iteration 0; at iteration k
 * the first rule s.s / s.y for odd k, the second s.y / y.y for even k, over
 * all cells of the instance (s = m_k - m_{k-1}, y = g_k - g_{k-1}, FP64
 * sums); a quotient that is not finite and positive keeps the previous tau;
 * clipped to [tau_min, tau_max].  Needs 0 < tau_min <= tau0 <= tau_max.
 * tau_out (host, batch doubles, nullable): the last tau.  Uses the plan's
 * stage buffers (a later mm_rk45_* call recomputes its first slope).
 * Synchronises. */
mm_status mm_sd_run(mm_plan* plan, const mm_params* params, int32_t batch, void* m, int64_t n_iter,
                    double tau0, double tau_min, double tau_max, double* tau_out, void* hip_stream);

/* mm_sd_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same iteration, kernels and results, but the per-call scratch that mm_sd_run
 * allocates and frees (FP64 partial sums, 4 per 256 cells per instance, and
 * the step sizes) comes from a fixed 16 MiB array in device memory that every
 * GPU the library runs on holds until the process ends.  This call allocates
 * nothing: MM_E_ARG when the batch needs more scratch than that
 * (32 * ceil(nx ny nz / 256) * batch bytes, rounded up to 256, plus 8 * batch;
 * e.g. 16 instances of 512 x 512 x 16 cells), MM_E_STATE when the plan's stage
 * buffers do not yet hold `batch` instances (one earlier mm_sd_run,
 * mm_heun_run or mm_rk45_* call on the plan with at least `batch` instances
 * allocates them).  Every call on one GPU shares that GPU's scratch: calls that
 * overlap on one GPU (other streams or host threads) race.  Synchronises. */
mm_status mm_sd_run_noalloc(mm_plan* plan, const mm_params* params, int32_t batch, void* m, int64_t n_iter,
                            double tau0, double tau_min, double tau_max, double* tau_out, void* hip_stream);

/* Relaxation by steepest descent (the iteration of mm_sd_run) that stops on
 * the largest |dm/dt| (section "Design": the relax task's stopping_dmdt).
 * Iteration k evaluates H_eff(m_k); its measure is the largest |dm/dt| over
 * the cells of the LL right-hand side (eq_llg2, the instance's alpha and
 * gamma) of m_k, in degrees per nanosecond.  An instance whose measure is
 * below stopping_dmdt (> 0, deg/ns) stops before that iteration's update, with
 * m = m_k and k updates made; at most max_iter updates (>= 0), followed by one
 * last check.  iters_out (host, batch int64, nullable): updates made;
 * dmdt_out (host, batch doubles, nullable): the last measure (deg/ns);
 * tau_out as for mm_sd_run.  MM_E_MAXSTEPS when some instance ended above the
 * threshold (iters_out = max_iter; its m is the last iterate).  Uses the
 * plan's stage buffers.  Synchronises (the host polls every 16 iterations and
 * returns once every instance has stopped). */
mm_status mm_sd_relax(mm_plan* plan, const mm_params* params, int32_t batch, void* m, double stopping_dmdt,
                      int64_t max_iter, double tau0, double tau_min, double tau_max, int64_t* iters_out,
                      double* dmdt_out, double* tau_out, void* hip_stream);

/* Relaxation by the adaptive Dormand-Prince integration of mm_rk45_run (no
 * end time) that stops on the largest |dm/dt| (section "Design": the relax
 * task's stopping_dmdt).  After every accepted step the slope of the new
 * state (the first-same-as-last slope f(y5), y5 before the projection) gives
 * the measure, the largest |dm/dt| over the cells in degrees per nanosecond;
 * an instance stops after the first accepted step whose measure is below
 * stopping_dmdt (> 0, deg/ns).  At most max_steps attempts per instance
 * (MM_E_MAXSTEPS otherwise).  st in/out as for mm_rk45_run (t advances);
 * dmdt_out (host, batch doubles, nullable): the last measure (deg/ns).
 * Synchronises. */
mm_status mm_rk45_relax(mm_plan* plan, const mm_params* params, int32_t batch, void* m, mm_rk45_state* st,
                        double stopping_dmdt, int64_t max_steps, double* dmdt_out, void* hip_stream);

/* Nudged elastic band on a chain of n_img images (n_img <= max_batch, >= 3)
 * stored as images[n_img][3][nz][ny][nx]: n_iter iterations of the
 * precession-free relaxation with time step h and spring constant k_spring
 * (A/m); end images stay fixed.  E_out (host, n_img) receives the image
 * energies before the last iteration (n_iter = 0: of the images as given,
 * which stay unchanged).  Synchronises.  Paper: "Miscellaneous"
 * (NEB); tangent, spring and distance follow the project's stated reading. */
mm_status mm_neb_run(mm_plan* plan, const mm_params* params, void* images, int32_t n_img,
                     double k_spring, double h, int64_t n_iter, double* E_out,
                     void* hip_stream);

/* Batched integration of instances of different meshes (parameter sweeps).
 * A batch is created for up to 16 distinct meshes; each run takes any number
 * of instances, each naming its mesh, and advances all of them together:
 * every kernel pass is one launch over all meshes' instances, each instance
 * has its own parameters, adaptive step size, controller and t_end, and the
 * step sequence is a captured HIP graph (finished instances idle).  This is
 * the paper's parameter sweep (section "Design", sim_with with _s suffixes,
 * run there one instance after the other) batched on one GPU. */
typedef struct mm_batch mm_batch;
typedef struct {
  int32_t mesh_id;     /* index into the meshes of mm_batch_create            */
  mm_params p;         /* parameters of this instance                        */
  void* m;             /* device array [3][nz][ny][nx] (plan precision), in/out */
  mm_rk45_state st;    /* in/out, as for mm_rk45_run                         */
  double t_end;        /* integrate to this time                             */
  int32_t status;      /* out: mm_status of this instance                    */
} mm_instance;

/* Builds the geometry (padded grid, tables, Newell spectrum) of every mesh.
 * Synchronises. */
mm_status mm_batch_create(mm_batch** out, const mm_mesh* meshes, int32_t n_meshes,
                          mm_precision prec, uint32_t terms, void* hip_stream);
/* Runs every instance to its t_end (at most max_steps attempts each).
 * Synchronises; returns the first non-OK instance status (details per
 * instance in inst[i].status). */
mm_status mm_batch_run(mm_batch* batch, mm_instance* inst, int32_t n_inst, int64_t max_steps,
                       void* hip_stream);
mm_status mm_batch_destroy(mm_batch* batch);

/* Autotuner: times candidate launch shapes of every kernel pass (rows or
 * columns per workgroup, threads per transform, workgroup size) on `reps`
 * dm/dt evaluations of m (output scratch in `work`, same layout) and keeps, per
 * pass, the first candidate in its fixed order whose time is within 3% of the
 * fastest (near-ties resolve alike from run to run).  shape_out (nullable, 8 ints) receives the chosen shapes:
 * x-forward rows, x-forward threads, y columns, y threads per column, y
 * threads, x-inverse rows, x-inverse threads, 0.  Synchronises. */
mm_status mm_plan_autotune(mm_plan* plan, const mm_params* params, int32_t batch, const void* m,
                           void* work, int32_t reps, int32_t* shape_out, void* hip_stream);

/* Choice of the padded FFT grid by measurement.  Per axis the candidates are
 * the plan's default (2n when 3-smooth, else the smallest 3-smooth length
 * >= 2n - 1), the smallest 3-smooth length >= 2n - 1 and the smallest power of
 * two >= 2n - 1 (x even; 2n in place of 2n - 1 for the scalar-potential
 * route); every combination whose spectrum per instance stays below 4 GiB is
 * built (its demag spectrum included) and `reps` dm/dt evaluations of the
 * `batch` instances m (device, as mm_llg_rhs; work: device output buffer of
 * the same size) are timed back to back.  The plan keeps the first grid, in
 * the order above, within 3% of the fastest, with default launch shapes (run
 * mm_plan_autotune after).  Any padded length >= 2n - 1 gives the same fields
 * up to rounding (section "Magnetostatic energy": the zero-padded FFT
 * convolution).  padded_out (host int32[3], nullable): Px, Py, Pz kept.
 * Drops the plan's first slopes (the next adaptive call recomputes them) and
 * its captured graph.  Allocates; synchronises. */
mm_status mm_plan_tune_padding(mm_plan* plan, const mm_params* params, int32_t batch, const void* m, void* work,
                               int32_t reps, int32_t* padded_out, void* hip_stream);

/* The plan's current launch shapes (8 ints, the layout above).  Host only. */
mm_status mm_plan_shapes(const mm_plan* plan, int32_t* shape_out);

/* Set the launch shapes (8 ints as above; the last is ignored), e.g. ones an
 * earlier autotune reported for this mesh, precision and device.  Every shape
 * is checked against the plan (LDS per workgroup, threads per transform and
 * per workgroup, rows per workgroup a power of two no larger than ny, y
 * columns whole kx blocks or a divisor of one in 3-D); MM_E_ARG and nothing
 * changed otherwise.  Results do not depend on the shapes beyond FP rounding.
 * Host only (may reallocate the plan's scratch; not while its work is in
 * flight). */
mm_status mm_plan_set_shapes(mm_plan* plan, const int32_t* shape);

/* Measurement aid: after one dm/dt evaluation of `batch` instances (output
 * written to `work`, same layout as m), launches each kernel pass `reps`
 * times back to back between two HIP events on hip_stream and returns in
 * us_out[0..*n_pass) the mean duration of one launch of each pass in
 * microseconds, in launch order: x forward, y (2-D: fused forward/product/
 * inverse; 3-D: forward, z with product, inverse), x inverse with the fused
 * local fields and LL (dm/dt epilogue).  Without demag there is one pass.
 * us_out must hold at least 5 entries.  seq_out (nullable, 5 entries): the
 * same passes timed in evaluation order -- `reps` whole evaluations, each
 * pass after the one whose output it reads, an event before every pass.
 * Synchronises. */
mm_status mm_profile_passes(mm_plan* plan, const mm_params* params, int32_t batch, const void* m,
                            void* work, int32_t reps, double* us_out, int32_t* n_pass,
                            double* seq_out, void* hip_stream);

/* Measurement aid for the adaptive step: sets up one Dormand-Prince attempt of
 * `batch` instances from m and the states st (as mm_rk45_run would; neither m
 * nor st is advanced; the stage buffers and the first slope are computed),
 * then times each kernel of the attempt `reps` times back to back between two
 * HIP events on hip_stream.  us_out[0]: the step-begin kernel; us_out[1 .. n-2]:
 * the passes of one stage evaluation in launch order, the last of them the
 * inverse-x pass with the stage epilogue (mean over stages 2..6, in the form
 * the captured attempt runs: with the next stage's forward x transform when
 * *fused_out is 1); us_out[n-1]: the inverse-x pass with the error epilogue.
 * *n_out = passes + 2 (at most 7); us_out must hold 8 entries.  seq_out
 * (nullable, 8 entries, same layout): the same kernels timed in attempt order
 * -- `reps` whole attempts as the captured graph runs them, each kernel after
 * the one whose output it reads (so caches hold what they hold in a real
 * run), an event before every kernel; the mean over every launch of a kind.
 * These attempts run on a copy of m.  Synchronises. */
mm_status mm_profile_step(mm_plan* plan, const mm_params* params, int32_t batch, void* m,
                          const mm_rk45_state* st, int32_t reps, double* us_out, int32_t* n_out,
                          int32_t* fused_out, double* seq_out, void* hip_stream);

const char* mm_status_string(mm_status s);
const char* mm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MM_H */
