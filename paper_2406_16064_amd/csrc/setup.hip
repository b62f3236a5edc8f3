// One-off setup on the device, in FP64: the cell-averaged demag tensor on the
// padded grid and its spectrum.
//
// The tensor (paper, section "Magnetostatic energy": H_d,i = -sum_j N_{i-j} M_j,
// Newell et al. 1993) is the average over the target cell of the field of a
// uniformly magnetised source cell,
//     N(R) = - int_{[-d,d]^3} D(R+u) prod_a (1 - |u_a|/d_a) du,
//     D(r) = (3 r r^T - r^2 I) / (4 pi r^5).
// Near the origin (|R| < 3 max d) it is evaluated with Newell's closed forms
// f and g and the 27-point second-difference stencil; further out with
// Gauss-Legendre quadrature of the integral (n nodes on each half interval:
// 10, 6, 4, 3, 2 from |R|/max d = 3, 6, 16, 40, 300), which avoids the
// catastrophic cancellation of the closed forms at large distance.
//
// The padded kernel K[i] holds N at the wrapped displacement of index i (zero
// at the unused Nyquist index and beyond the mesh extent); its forward FFT is
// real (each component is even or odd in each axis), is folded to
// (Px/2+1, Py/2+1, Pz/2+1) and cast to the plan precision.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fft_core.hpp"
#include "setup.hpp"

namespace mmx {

__constant__ double c_gl_nodes[5][20];
__constant__ double c_gl_wts[5][20];
__constant__ int c_gl_n[5];

__device__ __forceinline__ double nf(double x, double y, double z) {
  x = fabs(x); y = fabs(y); z = fabs(z);
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  double s = (2.0 * x2 - y2 - z2) * R * (1.0 / 6.0);
  if (y > 0 && x2 + z2 > 0) s += 0.5 * y * (z2 - x2) * asinh(y / sqrt(x2 + z2));
  if (z > 0 && x2 + y2 > 0) s += 0.5 * z * (y2 - x2) * asinh(z / sqrt(x2 + y2));
  if (x > 0 && y > 0 && z > 0) s -= x * y * z * atan(y * z / (x * R));
  return s;
}

__device__ __forceinline__ double ng(double x, double y, double z) {
  const double sg = (x > 0 ? 1.0 : (x < 0 ? -1.0 : 0.0)) * (y > 0 ? 1.0 : (y < 0 ? -1.0 : 0.0));
  if (sg == 0.0) return 0.0;
  x = fabs(x); y = fabs(y); z = fabs(z);
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  double s = -x * y * R * (1.0 / 3.0);
  if (z > 0) s += x * y * z * asinh(z / sqrt(x2 + y2));
  s += y * (1.0 / 6.0) * (3.0 * z2 - y2) * asinh(x / sqrt(y2 + z2));
  s += x * (1.0 / 6.0) * (3.0 * z2 - x2) * asinh(y / sqrt(x2 + z2));
  if (z > 0) {
    s -= z2 * z * (1.0 / 6.0) * atan(x * y / (z * R));
    s -= 0.5 * z * y2 * atan(x * z / (y * R));
    s -= 0.5 * z * x2 * atan(y * z / (x * R));
  }
  return sg * s;
}

// sum_{a,b,c} w_a w_b w_c F(p + a dp, q + b dq, r + c dr), w = (-1, 2, -1)
template <bool G>
__device__ double stencil27(double p, double q, double r, double dp, double dq, double dr) {
  double s = 0.0;
  for (int a = -1; a <= 1; ++a) {
    const double wa = a == 0 ? 2.0 : -1.0;
    for (int b = -1; b <= 1; ++b) {
      const double wb = b == 0 ? 2.0 : -1.0;
      for (int c = -1; c <= 1; ++c) {
        const double wc = c == 0 ? 2.0 : -1.0;
        const double v = G ? ng(p + a * dp, q + b * dq, r + c * dr) : nf(p + a * dp, q + b * dq, r + c * dr);
        s += wa * wb * wc * v;
      }
    }
  }
  return s;
}

// out: xx, yy, zz, xy, xz, yz
__device__ void tensor_at(double X, double Y, double Z, double dx, double dy, double dz, double out[6]) {
  const double dmax = fmax(dx, fmax(dy, dz));
  const double rho = sqrt(X * X + Y * Y + Z * Z) / dmax;
  if (rho < 3.0) {
    const double c = 1.0 / (4.0 * M_PI * dx * dy * dz);
    out[0] = c * stencil27<false>(X, Y, Z, dx, dy, dz);
    out[1] = c * stencil27<false>(Y, X, Z, dy, dx, dz);
    out[2] = c * stencil27<false>(Z, Y, X, dz, dy, dx);
    out[3] = c * stencil27<true>(X, Y, Z, dx, dy, dz);
    out[4] = c * stencil27<true>(X, Z, Y, dx, dz, dy);
    out[5] = c * stencil27<true>(Y, Z, X, dy, dz, dx);
    return;
  }
  const int rule = rho >= 300.0 ? 0 : rho >= 40.0 ? 1 : rho >= 16.0 ? 2 : rho >= 6.0 ? 3 : 4;
  const int n2 = 2 * c_gl_n[rule];
  double sxx = 0, syy = 0, szz = 0, sxy = 0, sxz = 0, syz = 0;
  for (int i = 0; i < n2; ++i) {
    const double rx = X + c_gl_nodes[rule][i] * dx;
    const double wx = c_gl_wts[rule][i] * dx;
    for (int j = 0; j < n2; ++j) {
      const double ry = Y + c_gl_nodes[rule][j] * dy;
      const double wxy = wx * c_gl_wts[rule][j] * dy;
      for (int k = 0; k < n2; ++k) {
        const double rz = Z + c_gl_nodes[rule][k] * dz;
        const double w = wxy * c_gl_wts[rule][k] * dz;
        const double r2 = rx * rx + ry * ry + rz * rz;
        const double ir = 1.0 / sqrt(r2);
        const double ir2 = ir * ir;
        const double f = w * ir * ir2 * ir2;  // w / r^5
        const double t = 3.0 * f;
        sxx += t * rx * rx - f * r2;
        syy += t * ry * ry - f * r2;
        szz += t * rz * rz - f * r2;
        sxy += t * rx * ry;
        sxz += t * rx * rz;
        syz += t * ry * rz;
      }
    }
  }
  const double c = -1.0 / (4.0 * M_PI);
  out[0] = c * sxx; out[1] = c * syy; out[2] = c * szz;
  out[3] = c * sxy; out[4] = c * sxz; out[5] = c * syz;
}

// Wrapped displacement of padded index i (P points, n cells); ok = false where
// the entry must be zero (Nyquist index of an even P, or |I| >= n).
__device__ __forceinline__ int wrap_disp(int i, int P, int n, bool& ok) {
  int I = i;
  if (2 * i > P) I = i - P;
  ok = !(2 * i == P) && (I < n) && (-I < n);
  return I;
}

__global__ void k_newell_grid(mm_mesh mesh, int Px, int Py, int Pz, int ncomp, Cx<double>* __restrict__ out) {
  const long long tot = (long long)Px * Py * Pz;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const int ix = (int)(idx % Px);
  const int iy = (int)((idx / Px) % Py);
  const int iz = (int)(idx / ((long long)Px * Py));
  bool okx, oky, okz;
  const int I = wrap_disp(ix, Px, mesh.nx, okx);
  const int J = wrap_disp(iy, Py, mesh.ny, oky);
  const int K = wrap_disp(iz, Pz, mesh.nz, okz);
  double t[6] = {0, 0, 0, 0, 0, 0};
  if (okx && oky && okz) tensor_at(I * mesh.dx, J * mesh.dy, K * mesh.dz, mesh.dx, mesh.dy, mesh.dz, t);
  for (int c = 0; c < ncomp; ++c) out[(size_t)c * tot + idx] = Cx<double>{t[c], 0.0};
}

__global__ void k_newell_list(mm_mesh mesh, const int32_t* __restrict__ disp, long long n, double* __restrict__ out) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double t[6];
  tensor_at(disp[3 * k] * mesh.dx, disp[3 * k + 1] * mesh.dy, disp[3 * k + 2] * mesh.dz, mesh.dx, mesh.dy,
            mesh.dz, t);
  for (int c = 0; c < 6; ++c) out[6 * k + c] = t[c];
}

// Forward C2C FFT along one axis of data laid out [outer][L][inner] (FP64).
// Workgroup: cb columns; columns are consecutive outer rows when inner == 1,
// else consecutive inner positions of one outer row.
__global__ void __launch_bounds__(512) k_fft_axis(Cx<double>* __restrict__ data, long long inner,
                                                 long long outer, int cb, int tpc, FftDesc<double> p) {
  extern __shared__ __align__(16) unsigned char smem[];
  Cx<double>* lds = reinterpret_cast<Cx<double>*>(smem);
  const int L = p.L;
  const int cs = col_stride(L);
  const long long ncols = inner * outer;
  const long long c0 = (long long)blockIdx.x * cb;
  const int ncol = (int)((ncols - c0) < cb ? (ncols - c0) : cb);
  auto addr = [&](long long col, int e) -> size_t {
    const long long o = col / inner, ii = col - o * inner;
    return ((size_t)o * L + e) * inner + ii;
  };
  for (int t = threadIdx.x; t < cb * L; t += blockDim.x) {
    int cl, e;
    if (inner == 1) { cl = t / L; e = t - cl * L; } else { cl = t % cb; e = t / cb; }
    if (cl < ncol) lds[cl * cs + pidx(e, p.psh)] = data[addr(c0 + cl, e)];
  }
  __syncthreads();
  fft_columns<double, false, false>(lds, p, cs, ncol, tpc, p.tw);
  for (int t = threadIdx.x; t < cb * L; t += blockDim.x) {
    int cl, e;
    if (inner == 1) { cl = t / L; e = t - cl * L; } else { cl = t % cb; e = t / cb; }
    if (cl < ncol) data[addr(c0 + cl, e)] = lds[cl * cs + pidx(e, p.psh)];
  }
}

// Fold the real spectrum: kt[c][kz][kx][ky] = Re F[c][kz][ky][kx] for
// kx <= Px/2, ky <= Py/2, kz <= Pz/2; also track the largest |Im| / max|Re|.
template <typename T>
__global__ void k_extract(const Cx<double>* __restrict__ F, int Px, int Py, int Pz, int c, T* __restrict__ kt,
                          unsigned long long* __restrict__ stats) {
  const int Xp = Px / 2 + 1, Ky = Py / 2 + 1, Kz = Pz / 2 + 1;
  const long long tot = (long long)Kz * Xp * Ky;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const int ky = (int)(idx % Ky);
  const int kx = (int)((idx / Ky) % Xp);
  const int kz = (int)(idx / ((long long)Ky * Xp));
  const Cx<double> v = F[((size_t)kz * Py + ky) * Px + kx];
  kt[(size_t)c * tot + idx] = T(v.x);
  atomicMax(&stats[0], (unsigned long long)__double_as_longlong(fabs(v.y)));
  atomicMax(&stats[1], (unsigned long long)__double_as_longlong(fabs(v.x)));
}

// ---------------------------------------------------------------------------
// Scalar-potential route.  S(R) = (1/4 pi) int_cell (R - r') / |R - r'|^3 dr' is
// the potential at R of a uniformly magnetised unit cuboid of size d centred at
// 0 (component a for M = e_a).  Integrated along a it is the potential of the
// two charged a-faces, (1/4 pi) [I(R_a - d_a/2) - I(R_a + d_a/2)], where I(w)
// integrates 1/sqrt(x^2 + y^2 + w^2) over the face rectangle (in coordinates
// relative to R), with the antiderivative
//   G(x, y, z) = x asinh(y / sqrt(x^2 + z^2)) + y asinh(x / sqrt(y^2 + z^2)) - z atan(x y / (z r)).
// Near the cell (|R| < 3 max d) the closed form, beyond it Gauss-Legendre
// quadrature of the volume integral (n nodes per axis over the cell: 14, 9,
// 6, 4, 3 from |R| / max d = 3, 6, 16, 40, 300), where the face differences of
// the closed form would cancel.  The grid holds S at the vertex - cell
// displacements ((i - 1/2) dx, ...), i in [-n+1, n], index i mod P.
// ---------------------------------------------------------------------------
__constant__ double c_pq_nodes[5][16];
__constant__ double c_pq_wts[5][16];
__constant__ int c_pq_n[5];

__device__ __forceinline__ double face_g(double x, double y, double z) {
  const double r = sqrt(x * x + y * y + z * z);
  double s = 0.0;
  const double ax = sqrt(x * x + z * z), ay = sqrt(y * y + z * z);
  if (x != 0.0 && ax > 0.0) s += x * asinh(y / ax);
  if (y != 0.0 && ay > 0.0) s += y * asinh(x / ay);
  if (z != 0.0 && r > 0.0) s -= z * atan(x * y / (z * r));
  return s;
}

__device__ __forceinline__ double face_i(double x1, double x2, double y1, double y2, double w) {
  return face_g(x2, y2, w) - face_g(x1, y2, w) - face_g(x2, y1, w) + face_g(x1, y1, w);
}

__device__ void potential_at(double X, double Y, double Z, double dx, double dy, double dz, double out[3]) {
  const double R[3] = {X, Y, Z}, d[3] = {dx, dy, dz};
  const double dmax = fmax(dx, fmax(dy, dz));
  const double rho = sqrt(X * X + Y * Y + Z * Z) / dmax;
  if (rho < 3.0) {
    for (int a = 0; a < 3; ++a) {
      const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
      const double x1 = -0.5 * d[b] - R[b], x2 = 0.5 * d[b] - R[b];
      const double y1 = -0.5 * d[c] - R[c], y2 = 0.5 * d[c] - R[c];
      out[a] = (face_i(x1, x2, y1, y2, R[a] - 0.5 * d[a]) - face_i(x1, x2, y1, y2, R[a] + 0.5 * d[a])) /
               (4.0 * M_PI);
    }
    return;
  }
  const int rule = rho >= 300.0 ? 4 : rho >= 40.0 ? 3 : rho >= 16.0 ? 2 : rho >= 6.0 ? 1 : 0;
  const int n = c_pq_n[rule];
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int i = 0; i < n; ++i) {
    const double vx = X - 0.5 * dx * c_pq_nodes[rule][i];
    const double wi = c_pq_wts[rule][i];
    for (int j = 0; j < n; ++j) {
      const double vy = Y - 0.5 * dy * c_pq_nodes[rule][j];
      const double wij = wi * c_pq_wts[rule][j];
      for (int k = 0; k < n; ++k) {
        const double vz = Z - 0.5 * dz * c_pq_nodes[rule][k];
        const double r2 = vx * vx + vy * vy + vz * vz;
        const double ir = 1.0 / sqrt(r2);
        const double f = wij * c_pq_wts[rule][k] * ir * ir * ir;
        sx += f * vx;
        sy += f * vy;
        sz += f * vz;
      }
    }
  }
  const double c = dx * dy * dz / (8.0 * 4.0 * M_PI);
  out[0] = c * sx; out[1] = c * sy; out[2] = c * sz;
}

// Lattice index of padded index i (P points, n cells): i for i <= n, i - P
// when that is >= -n + 1; ok = false otherwise (the entry stays zero).
__device__ __forceinline__ int vertex_disp(int i, int P, int n, bool& ok) {
  const int I = i <= n ? i : i - P;
  ok = I >= -n + 1 && I <= n;
  return I;
}

__global__ void k_potential_grid(mm_mesh mesh, int Px, int Py, int Pz, Cx<double>* __restrict__ out) {
  const long long tot = (long long)Px * Py * Pz;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const int ix = (int)(idx % Px);
  const int iy = (int)((idx / Px) % Py);
  const int iz = (int)(idx / ((long long)Px * Py));
  bool okx, oky, okz;
  const int I = vertex_disp(ix, Px, mesh.nx, okx);
  const int J = vertex_disp(iy, Py, mesh.ny, oky);
  const int K = vertex_disp(iz, Pz, mesh.nz, okz);
  double t[3] = {0.0, 0.0, 0.0};
  if (okx && oky && okz)
    potential_at((I - 0.5) * mesh.dx, (J - 0.5) * mesh.dy, (K - 0.5) * mesh.dz, mesh.dx, mesh.dy, mesh.dz, t);
  for (int c = 0; c < 3; ++c) out[(size_t)c * tot + idx] = Cx<double>{t[c], 0.0};
}

__global__ void k_potential_list(mm_mesh mesh, const int32_t* __restrict__ disp, long long n,
                                 double* __restrict__ out) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double t[3];
  potential_at((disp[3 * k] - 0.5) * mesh.dx, (disp[3 * k + 1] - 0.5) * mesh.dy, (disp[3 * k + 2] - 0.5) * mesh.dz,
               mesh.dx, mesh.dy, mesh.dz, t);
  for (int c = 0; c < 3; ++c) out[3 * k + c] = t[c];
}

// The spectrum of component c, S^_c(k) = -i Phi(k) C_c(k) with the half-cell
// phase Phi(k) = exp(-i pi (kx/Px + ky/Py + kz/Pz)) and C_c real (the lattice
// is symmetric about the half-cell shift): kp[c][kz][kx][ky] = C_c for
// kx <= Px/2, ky <= Py/2, kz <= Pz/2 (the rest follows by parity); tracks the
// largest |Im| / max |Re| of S^ i conj(Phi).
template <typename T>
__global__ void k_extract_pot(const Cx<double>* __restrict__ F, int Px, int Py, int Pz, int c, T* __restrict__ kp,
                              unsigned long long* __restrict__ stats) {
  const int Xp = Px / 2 + 1, Ky = Py / 2 + 1, Kz = Pz / 2 + 1;
  const long long tot = (long long)Kz * Xp * Ky;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const int ky = (int)(idx % Ky);
  const int kx = (int)((idx / Ky) % Xp);
  const int kz = (int)(idx / ((long long)Ky * Xp));
  const Cx<double> v = F[((size_t)kz * Py + ky) * Px + kx];
  double sn, cn;
  sincospi((double)kx / Px + (double)ky / Py + (double)kz / Pz, &sn, &cn);
  // v * i * conj(Phi) = v * i * (cn + i sn) = v * (-sn + i cn)
  const double re = -v.x * sn - v.y * cn, im = v.x * cn - v.y * sn;
  kp[(size_t)c * tot + idx] = T(re);
  atomicMax(&stats[0], (unsigned long long)__double_as_longlong(fabs(im)));
  atomicMax(&stats[1], (unsigned long long)__double_as_longlong(fabs(re)));
}

// ---------------------------------------------------------------------------
hipError_t setup_upload_pot_gauss(const double nodes[5][16], const double wts[5][16], const int n[5]) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_pq_nodes), nodes, sizeof(double) * 80);
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_pq_wts), wts, sizeof(double) * 80);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_pq_n), n, sizeof(int) * 5);
}

hipError_t setup_potential_grid(const mm_mesh& mesh, int Px, int Py, int Pz, Cx<double>* out, hipStream_t s) {
  const long long tot = (long long)Px * Py * Pz;
  k_potential_grid<<<dim3((unsigned)((tot + 255) / 256)), 256, 0, s>>>(mesh, Px, Py, Pz, out);
  return hipGetLastError();
}

hipError_t setup_potential_list(const mm_mesh& mesh, const int32_t* disp, long long n, double* out,
                                hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_potential_list<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(mesh, disp, n, out);
  return hipGetLastError();
}

template <typename T>
hipError_t setup_extract_pot(const Cx<double>* F, int Px, int Py, int Pz, int c, T* kp, unsigned long long* stats,
                             hipStream_t s) {
  const long long tot = (long long)(Pz / 2 + 1) * (Px / 2 + 1) * (Py / 2 + 1);
  k_extract_pot<T><<<dim3((unsigned)((tot + 255) / 256)), 256, 0, s>>>(F, Px, Py, Pz, c, kp, stats);
  return hipGetLastError();
}

template hipError_t setup_extract_pot<float>(const Cx<double>*, int, int, int, int, float*, unsigned long long*,
                                             hipStream_t);
template hipError_t setup_extract_pot<double>(const Cx<double>*, int, int, int, int, double*, unsigned long long*,
                                              hipStream_t);

// ---------------------------------------------------------------------------
hipError_t setup_upload_gauss(const double nodes[5][20], const double wts[5][20], const int n[5]) {
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_gl_nodes), nodes, sizeof(double) * 100);
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_gl_wts), wts, sizeof(double) * 100);
  if (e != hipSuccess) return e;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_gl_n), n, sizeof(int) * 5);
}

hipError_t setup_newell_grid(const mm_mesh& mesh, int Px, int Py, int Pz, int ncomp, Cx<double>* out,
                             hipStream_t s) {
  const long long tot = (long long)Px * Py * Pz;
  k_newell_grid<<<dim3((unsigned)((tot + 255) / 256)), 256, 0, s>>>(mesh, Px, Py, Pz, ncomp, out);
  return hipGetLastError();
}

hipError_t setup_newell_list(const mm_mesh& mesh, const int32_t* disp, long long n, double* out,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_newell_list<<<dim3((unsigned)((n + 255) / 256)), 256, 0, s>>>(mesh, disp, n, out);
  return hipGetLastError();
}

hipError_t setup_fft_axis(Cx<double>* data, long long inner, long long outer, const FftDesc<double>& p,
                          int tpc, hipStream_t s) {
  if (p.L == 1) return hipSuccess;
  const size_t colb = (size_t)col_stride(p.L) * sizeof(Cx<double>);
  int cb = (int)(65536 / colb);
  if (cb < 1) cb = 1;
  if (cb * tpc > 512) cb = 512 / tpc;
  if (cb > 64) cb = 64;
  const long long ncols = inner * outer;
  const long long nblk = (ncols + cb - 1) / cb;
  k_fft_axis<<<dim3((unsigned)nblk), cb * tpc, cb * colb, s>>>(data, inner, outer, cb, tpc, p);
  return hipGetLastError();
}

template <typename T>
hipError_t setup_extract(const Cx<double>* F, int Px, int Py, int Pz, int c, T* kt, unsigned long long* stats,
                         hipStream_t s) {
  const long long tot = (long long)(Pz / 2 + 1) * (Px / 2 + 1) * (Py / 2 + 1);
  k_extract<T><<<dim3((unsigned)((tot + 255) / 256)), 256, 0, s>>>(F, Px, Py, Pz, c, kt, stats);
  return hipGetLastError();
}

template hipError_t setup_extract<float>(const Cx<double>*, int, int, int, int, float*, unsigned long long*,
                                         hipStream_t);
template hipError_t setup_extract<double>(const Cx<double>*, int, int, int, int, double*, unsigned long long*,
                                          hipStream_t);

}  // namespace mmx
