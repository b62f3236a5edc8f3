// Device setup of the demag tensor spectrum (FP64).
#pragma once

#include "mm_internal.hpp"

namespace mmx {

hipError_t setup_upload_gauss(const double nodes[5][20], const double wts[5][20], const int n[5]);
hipError_t setup_newell_grid(const mm_mesh& mesh, int Px, int Py, int Pz, int ncomp, Cx<double>* out,
                             hipStream_t s);
hipError_t setup_newell_list(const mm_mesh& mesh, const int32_t* disp, long long n, double* out,
                             hipStream_t s);
hipError_t setup_upload_pot_gauss(const double nodes[5][16], const double wts[5][16], const int n[5]);
hipError_t setup_potential_grid(const mm_mesh& mesh, int Px, int Py, int Pz, Cx<double>* out, hipStream_t s);
hipError_t setup_potential_list(const mm_mesh& mesh, const int32_t* disp, long long n, double* out,
                                hipStream_t s);
template <typename T>
hipError_t setup_extract_pot(const Cx<double>* F, int Px, int Py, int Pz, int c, T* kp, unsigned long long* stats,
                             hipStream_t s);
hipError_t setup_fft_axis(Cx<double>* data, long long inner, long long outer, const FftDesc<double>& p,
                          int tpc, hipStream_t s);
template <typename T>
hipError_t setup_extract(const Cx<double>* F, int Px, int Py, int Pz, int c, T* kt, unsigned long long* stats,
                         hipStream_t s);

}  // namespace mmx
