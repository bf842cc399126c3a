// Kernel argument blocks and launch entry points (host side of the kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bbdg {

// Arguments of the fused stage kernel.  In stage mode the kernel reads qin
// (and res unless read_res == 0), writes res and qout; in right-hand-side
// modes it reads qin and writes the right-hand side to qout.
template <typename T>
struct StageArgs {
  const T* qin;
  T* qout;
  T* res;
  const double* geo;      // K x kGeoStride
  const int32_t* etoe;    // K x 4, -1 on the boundary
  const uint8_t* etofo;   // K x 4: neighbour face | orientation << 2
  const uint16_t* tab;    // index tables of the order
  int64_t K;
  T rk_a, rk_b, dt;
  int read_res;
  int bc;
  // Batched multi-stage launches (mode kBatched): S shots stored shot-major
  // (S, 4, K, Np); stage s reads buffer s % 2 of {qout, qalt} and writes the
  // other; a Ricker point source per shot is added to the pressure equation;
  // receivers sample the pressure after every fifth stage.
  int64_t shots;
  T* qalt;
  int64_t nstages;
  double t0, dtd;           // start time and step of the wavelet clock
  const int32_t* src_elem;  // S: source element of each shot (-1: none)
  const T* src_coef;        // S x Np: kappa (M^k)^{-1} B(lambda_s)
  double f0, tshift;        // Ricker peak frequency and delay
  int R;                    // receivers per shot
  const int32_t* rec_elem;  // R
  const T* rec_coef;        // R x Np: B_alpha(lambda_r)
  T* traces;                // steps x S x R
};

template <typename T>
hipError_t launch_stage(int N, int mode, const StageArgs<T>& a, hipStream_t stream);

// Persistent cooperative launch of a whole batched run; wpb = waves per
// workgroup (1, 2 or 4).  Fails (no launch) when the grid cannot be co-resident.
template <typename T>
hipError_t launch_batched(int N, int wpb, const StageArgs<T>& a, hipStream_t stream);

// Arguments of the dense nodal comparator stage kernel: the same fields,
// geometry and connectivity plus the dense operators
//   dr   [3][NpP][Kv]  Dr_i = V (D^i - D^0) V^{-1}, zero padded
//   lift [NpP][Kl]     the four face lifts side by side, zero padded
template <typename T>
struct NodalArgs {
  const T* qin;
  T* qout;
  T* res;
  const double* geo;
  const int32_t* etoe;
  const uint8_t* etofo;
  const uint16_t* tab;
  const T* dr;
  const T* lift;
  int64_t K;
  T rk_a, rk_b, dt;
  int read_res;
  int bc;
};

template <typename T>
hipError_t launch_nodal_stage(int N, int mode, const NodalArgs<T>& a, hipStream_t stream);

hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, hipStream_t stream);

}  // namespace bbdg
