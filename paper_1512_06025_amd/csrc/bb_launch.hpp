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
  const T* tgeo;          // K x kTGeoStride derived geometry (FP64 groups of several elements derive it from geo)
  const int32_t* etoe;    // K x 4, -1 on the boundary
  const uint8_t* etofo;   // K x 4: neighbour face | orientation << 2
  const uint16_t* tab;    // index tables of the order
  int64_t K;
  T rk_a, rk_b, dt;
  int read_res;
  int bc;
  int nt_store;  // 1: FP64 stage outputs with non-temporal stores (single-stage launches)
  // Batched multi-stage launches (mode kBatched): S shots stored shot-major
  // (S, K, 4, Np); stage s reads buffer s % 2 of {qout, qalt} and writes the
  // other; a Ricker point source per shot is added to the pressure equation;
  // receivers sample the pressure after every fifth stage.
  int64_t shots;
  T* qalt;
  int64_t nstages;
  double dtd;               // time step
  const int32_t* src_elem;  // S: source element of each shot (-1: none)
  const T* src_coef;        // S x Np: kappa (M^k)^{-1} B(lambda_s)
  const double* amp;        // nstages: wavelet value at each stage time
  int R;                    // receivers per shot
  const int32_t* rec_elem;  // R
  const T* rec_coef;        // R x Np: B_alpha(lambda_r)
  T* traces;                // steps x S x R
  // Optional record of every stage for the adjoint (batched mode): the
  // pressure right-hand side incl. source, (stages, S, K, Np), and per face
  // (stored once, by the element with the lower index, or the only one) the
  // jumps [[p]] and g_f.[[u]] / |g_f| on that element's face nodes,
  // (stages, S, F, 2, Nfp); rec_face (K x 4) numbers the F faces.
  T* rec_p;
  T* rec_j;
  const int32_t* rec_face;
  int64_t nfaces;
  // Grid-barrier words of batched launches (kSyncBytes): arrival counters,
  // zeroed before every launch, and a sticky timeout flag.
  uint32_t* sync;
  uint64_t barrier_timeout;  // longest wait at a grid barrier, wall-clock ticks
};

constexpr size_t kSyncBytes = 2048;
constexpr int kSyncFlagWord = 288;  // index of the timeout flag in sync

template <typename T>
hipError_t launch_stage(int N, int mode, const StageArgs<T>& a, hipStream_t stream);

// Persistent cooperative launch of a whole batched run; wpb = waves per
// workgroup (2, 4 or 8).  Fails (no launch) when the grid cannot be co-resident.
template <typename T>
hipError_t launch_batched(int N, int wpb, const StageArgs<T>& a, hipStream_t stream);

// Co-residency of the batched kernel of order N with wpb waves per workgroup
// (record != 0: the instantiation that records stages for the adjoint) on
// the current device: out = {workgroups per CU by the occupancy query, the
// bound derived from the kernel's VGPRs, LDS and scratch (what cooperative
// launches use), VGPRs, static LDS bytes, scratch bytes per lane, CUs}.
template <typename T>
hipError_t batched_residency(int N, int wpb, int record, int out[6]);

// Zeroes the arrival counters of the grid barrier (one tiny kernel).
hipError_t launch_barrier_reset(uint32_t* sync, hipStream_t stream);

// Fills a[0..n) with NaN when the timeout flag of sync is set.
template <typename T>
hipError_t launch_poison(const uint32_t* sync, T* a, int64_t n, hipStream_t stream);

// amp[i] = Ricker wavelet (peak frequency f0, delay ts) at the time of stage
// i of the LSRK4 steps step0, step0 + 1, ... of a run from t0 with step dt:
// t0 + (step0 + i / 5) dt + c_(i % 5) dt.
hipError_t launch_wavelet(double* amp, int64_t nstages, double t0, int64_t step0, double dt, double f0, double ts,
                          hipStream_t stream);

// One reverse stage of the discrete adjoint of the batched LSRK4 run.
//   u = rb + b_s qb (qb completed with the neighbour terms of the previous
//   reverse stage, z_in), qb <- qb + dt A^T u (own-element part), rb <- a_s u,
//   z_out = the face adjoint each neighbour needs, and the gradient terms
//   of this stage are added to gk (S, K) and gt (S, K, 4) in FP64.
template <typename T>
struct AdjointArgs {
  T* rb;             // (S, K, 4, Np) in/out
  T* qb;             // (S, K, 4, Np) in/out, own-element part
  const T* z_in;     // (S, K, 4, 2, Nfp) of the previous reverse stage (pull != 0)
  T* z_out;          // (S, K, 4, 2, Nfp)
  const T* rec_p;    // (S, K, Np) record of this forward stage
  const T* rec_j;    // (S, F, 2, Nfp): [[p]] and g.[[u]] / |g| as seen by the face's owner
  const int32_t* rec_face;  // K x 4: face number of (element, face)
  int64_t nfaces;           // F
  double* gk;        // (S, K)
  double* gt;        // (S, K, 4)
  const double* geo;
  const T* ageo;     // FP32: K x kAGeoStride derived geometry (the FP64 kernel derives it from geo)
  const int32_t* etoe;
  const uint8_t* etofo;
  const uint16_t* tab;
  int64_t K, shots;
  T a_s, b_s, dt;
  int pull;
  int bc;
};

template <typename T>
hipError_t launch_adjoint_stage(int N, const AdjointArgs<T>& a, hipStream_t stream);

// qb[s][rec_elem[r]][0] += (traces[s][r] - obs[s][r]) rec_coef[r] for one step
// (qb element-major (S, K, 4, Np); traces, obs: (S, R) slices); the receivers
// of one element are summed in receiver order (deterministic).
template <typename T>
hipError_t launch_inject_receivers(int Np, int64_t K, int64_t shots, int R, const int32_t* rec_elem,
                                   const T* rec_coef, const T* traces, const T* obs, T* qb, hipStream_t stream);

// J = 1/2 sum (traces - obs)^2 over n values, accumulated in FP64 by one workgroup.
template <typename T>
hipError_t launch_misfit(int64_t n, const T* traces, const T* obs, double* J, hipStream_t stream);

// grad[k] = sum_s gk[s][k] + (1/(2 c_k)) (sum_f w_f gt[s][k][f] + sum_f gt[s][nb][nf]),
// w_f = 2 on boundary faces (c+ = c there) else 1, second sum over interior faces.
hipError_t launch_gradient_finalize(int64_t K, int64_t shots, const double* geo, const int32_t* etoe,
                                    const uint8_t* etofo, const double* gk, const double* gt, double* grad,
                                    hipStream_t stream);

// Arguments of the dense nodal comparator stage kernels: the same fields,
// geometry and connectivity plus the dense operators; for the MFMA kernel
//   dr   [3][NpP][Kv]  Dr_i = V (D^i - D^0) V^{-1}, zero padded
//   lift [NpP][Kl]     the four face lifts side by side, zero padded
// (the element-per-thread kernel takes them in its own layout, below).
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
  T* flux;  // element-per-thread comparator: its face-node flux buffer (4, K, 4 Nfp)
  int64_t K;
  T rk_a, rk_b, dt;
  int read_res;
  int bc;
  int nt_store;  // 1: FP64 stage outputs with non-temporal stores (single-stage launches)
};

template <typename T>
hipError_t launch_nodal_stage(int N, int mode, const NodalArgs<T>& a, hipStream_t stream);

// Element-per-thread nodal comparator: rows per register block (the operator
// layouts of its NodalArgs are built for it on the host, see nodal_ept.hip):
// dr = opv [Np][NB B][4], lift = opl [4 Nfp][NB B], NB = ceil(Np / B); it
// launches a flux kernel (writing flux) and the element-per-thread kernel.
constexpr int ept_block_rows(int N, bool f64) {
  return (N + 1) * (N + 2) * (N + 3) / 6 < (f64 ? 16 : 32) ? (N + 1) * (N + 2) * (N + 3) / 6 : (f64 ? 16 : 32);
}

template <typename T>
hipError_t launch_nodal_ept(int N, int mode, const NodalArgs<T>& a, hipStream_t stream);

hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, hipStream_t stream);

}  // namespace bbdg
