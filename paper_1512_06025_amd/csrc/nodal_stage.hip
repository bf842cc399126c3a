// Dense nodal DG comparator stage kernel (gfx950, MFMA).
//
// The same DG scheme as the Bernstein-Bezier path (Section 2 flux, strong form
// of Section 3) in the Lagrange basis of the equispaced lattice: the unknowns
// are point values at the control-point positions, so face nodes of
// neighbouring elements match through the same tables.  Dense operators
// (built on the host):
//   Dr_i = V (D^i - D^0) V^{-1}, i = 1..3  -> grad f = sum_i grad(lambda_i) Dr_i f
//   LIFT = [V E_L^f L_0 Vf^{-1}]_f         -> lifted flux of the four faces
// with V (Vf) the Bernstein-Vandermonde matrix of the volume (face) lattice.
//
// Each wave owns blocks of 4 elements = 16 columns (element-major, field
// fastest); waves of a workgroup are independent after loading the tables.  The volume term is three MFMA GEMMs (NpP x Kv) x (Kv x 16), the
// surface term one MFMA GEMM (NpP x Kl) x (Kl x 16) on the face-node fluxes
// (the p flux and the velocity flux scaled by the three components of g_f),
// followed by the fused LSRK4 update.  MFMA tiles are 16 x 16 x 4
// (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32); lane l holds A[l%16][l/16]
// and B[l/16][l%16]; accumulator register r of lane l is D[row][l%16] with
// row = l/16 + 4r for the FP64 instruction and 4(l/16) + r for the FP32 one.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bb_common.hpp"
#include "bb_launch.hpp"

namespace bbdg {

namespace {

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef f64x4 acc;
  static __device__ __forceinline__ acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int r) { return kq + 4 * r; }
};
template <>
struct Mfma<float> {
  typedef f32x4 acc;
  static __device__ __forceinline__ acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
  static __device__ __forceinline__ acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int r) { return 4 * kq + r; }
};

}  // namespace

// Waves per workgroup: bounded by the two per-wave LDS buffers.
template <int N, typename T>
struct NodalWaves {
  static constexpr int value = sizeof(T) == 8 ? (N <= 5 ? 4 : (N <= 7 ? 2 : 1)) : (N <= 7 ? 4 : 2);
};

template <int N, typename T, int MODE>
__global__ __launch_bounds__((64 * NodalWaves<N, T>::value)) void nodal_stage_kernel(NodalArgs<T> A) {
  constexpr int Np = np_of(N), Nfp = nfp_of(N);
  constexpr NodalDims D = nodal_dims(N);
  constexpr int NpP = D.NpP, Kv = D.Kv, Kl = D.Kl;
  constexpr int EB = 4, NC = 16;  // elements per block, columns per block
  constexpr int WPB = NodalWaves<N, T>::value;
  // bx: volume B operand X[col][k] (also read for own face traces), later the
  //     lift output [row][col]; by: volume outputs [row][col], later the flux
  //     block F[k][col] (the B operand of the lift)
  constexpr int SZX = (NC * Kv > NpP * NC) ? NC * Kv : NpP * NC;
  constexpr int SZY = (NpP > Kl ? NpP : Kl) * NC;
  constexpr int NIT = (EB * Np + 63) / 64;  // (node, element) items per lane
  constexpr int NFI = (EB * 4 * Nfp + 63) / 64;
  constexpr bool kVol = (MODE != kRhsSurface);
  constexpr bool kSurf = (MODE != kRhsVolume);
  using M = Mfma<T>;
  typedef typename M::acc acc_t;

  __shared__ uint16_t t_nbr[24 * Nfp];
  __shared__ uint16_t t_fnode[4 * Nfp];
  __shared__ __attribute__((aligned(16))) T bx[WPB][SZX];
  __shared__ __attribute__((aligned(16))) T by[WPB][SZY];
  __shared__ double shg[WPB][EB * kGeoStride];
  __shared__ int32_t she[WPB][EB * 4];
  __shared__ uint8_t shf[WPB][EB * 4];

  const int tid = threadIdx.x;
  const TabLayout L = tab_layout(N);
  for (int i = tid; i < 24 * Nfp; i += 64 * WPB) t_nbr[i] = A.tab[L.nbrnode + i];
  for (int i = tid; i < 4 * Nfp; i += 64 * WPB) t_fnode[i] = A.tab[L.fnode + i];
  __syncthreads();
  T* const xs = bx[tid >> 6];  // X[col][k] = xs[col * Kv + k]; lift output [row][col] = xs[row * NC + col]
  T* const ys = by[tid >> 6];  // Y[row][col] = ys[row * NC + col]; F[k][col] = ys[k * NC + col]

  const int lane0 = tid & 63, w = tid >> 6;
  const int64_t K = A.K, KNp = K * Np;
  const int64_t G = (K + EB - 1) / EB;
  const int xcd = blockIdx.x & 7;
  const int64_t g_lo = G * xcd / 8, g_hi = G * (xcd + 1) / 8;
  const int64_t wstride = (int64_t)(gridDim.x >> 3) * WPB;

  for (int64_t g = g_lo + (int64_t)(blockIdx.x >> 3) * WPB + w; g < g_hi; g += wstride) {
    int lane = lane0;
    asm volatile("" : "+v"(lane));
    const int64_t e0 = g * EB;
    const int ri = lane & 15;  // MFMA row / column index within a tile
    const int kq = lane >> 4;  // MFMA k index (0..3) / accumulator row block

    // ---- header, own coefficients -------------------------------------------
    wave_sync_lds();
    for (int v = lane; v < EB * kGeoStride; v += 64) {
      const int64_t idx = e0 * kGeoStride + v;
      shg[w][v] = idx < K * kGeoStride ? A.geo[idx] : 0.0;
    }
    if (lane < EB * 4) {
      const int64_t idx = e0 * 4 + lane;
      she[w][lane] = idx < K * 4 ? A.etoe[idx] : -1;
      shf[w][lane] = idx < K * 4 ? A.etofo[idx] : 0;
    }
    T qv[NIT][4];
#pragma unroll
    for (int r = 0; r < NIT; ++r) {
      const int v = lane + 64 * r;
      const int el = v / Np, n = v - el * Np;
      const bool ok = v < EB * Np && e0 + el < K;
      const int64_t off = ok ? (e0 + el) * Np + n : 0;
#pragma unroll
      for (int f = 0; f < 4; ++f) qv[r][f] = ok ? A.qin[f * KNp + off] : (T)0;
    }
    // volume B operand: xs[col][k], col = 4 el + field, zero padding for k >= Np
    for (int v = lane; v < NC * Kv; v += 64) xs[v] = 0;
    wave_sync_lds();
#pragma unroll
    for (int r = 0; r < NIT; ++r) {
      const int v = lane + 64 * r;
      if (v < EB * Np) {
        const int el = v / Np, n = v - el * Np;
#pragma unroll
        for (int f = 0; f < 4; ++f) xs[(4 * el + f) * Kv + n] = qv[r][f];
      }
    }
    wave_sync_lds();

    T rhs[NIT][4];
#pragma unroll
    for (int r = 0; r < NIT; ++r)
#pragma unroll
      for (int f = 0; f < 4; ++f) rhs[r][f] = 0;

    // ---- volume: Y_i = Dr_i X, combined with grad(lambda_i) per element ------
    if constexpr (kVol) {
      for (int i = 0; i < 3; ++i) {
        const T* Di = A.dr + (size_t)i * NpP * Kv;
        for (int mt = 0; mt < NpP / 16; ++mt) {
          acc_t c = M::zero();
#pragma unroll 4
          for (int k0 = 0; k0 < Kv; k0 += 4) {
            const T a = Di[(mt * 16 + ri) * Kv + k0 + kq];
            const T b = xs[ri * Kv + k0 + kq];
            c = M::mac(a, b, c);
          }
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) ys[(mt * 16 + M::row(kq, rr)) * NC + ri] = c[rr];
        }
        wave_sync_lds();
#pragma unroll
        for (int r = 0; r < NIT; ++r) {
          const int v = lane + 64 * r;
          if (v >= EB * Np) continue;
          const int el = v / Np, n = v - el * Np;
          const double* ge = shg[w] + el * kGeoStride;
          const T gx = (T)ge[3 * i], gy = (T)ge[3 * i + 1], gz = (T)ge[3 * i + 2];
          const T kap = (T)ge[9];
          const T* y = ys + n * NC + 4 * el;
          rhs[r][0] -= kap * (gx * y[1] + gy * y[2] + gz * y[3]);
          rhs[r][1] -= gx * y[0];
          rhs[r][2] -= gy * y[0];
          rhs[r][3] -= gz * y[0];
        }
        wave_sync_lds();
      }
    }

    // ---- surface: flux on face nodes, then R = LIFT F ---------------------------
    if constexpr (kSurf) {
      for (int v = lane; v < Kl * NC; v += 64) ys[v] = 0;
      wave_sync_lds();
#pragma unroll
      for (int r = 0; r < NFI; ++r) {
        const int v = lane + 64 * r;
        const int el = v / (4 * Nfp);
        const int rem = v - el * 4 * Nfp;
        const int f = rem / Nfp, gg = rem - f * Nfp;
        if (v >= EB * 4 * Nfp || e0 + el >= K) continue;
        const int n = t_fnode[f * Nfp + gg];
        const T pm = xs[(4 * el) * Kv + n], um = xs[(4 * el + 1) * Kv + n], vm = xs[(4 * el + 2) * Kv + n],
                wm = xs[(4 * el + 3) * Kv + n];
        const double* ge = shg[w] + el * kGeoStride;
        double lx, ly, lz;  // grad lambda_f
        if (f == 0) {
          lx = -(ge[0] + ge[3] + ge[6]);
          ly = -(ge[1] + ge[4] + ge[7]);
          lz = -(ge[2] + ge[5] + ge[8]);
        } else {
          lx = ge[3 * (f - 1)];
          ly = ge[3 * (f - 1) + 1];
          lz = ge[3 * (f - 1) + 2];
        }
        const T gx = (T)(-2.0 * lx), gy = (T)(-2.0 * ly), gz = (T)(-2.0 * lz);
        const int nb = she[w][el * 4 + f];
        T jp, jgu;
        if (nb >= 0) {
          const int info = shf[w][el * 4 + f];
          const int64_t off = (int64_t)nb * Np + t_nbr[((info & 3) * 6 + (info >> 2)) * Nfp + gg];
          jp = A.qin[off] - pm;
          jgu = gx * (A.qin[KNp + off] - um) + gy * (A.qin[2 * KNp + off] - vm) + gz * (A.qin[3 * KNp + off] - wm);
        } else if (A.bc == 0) {
          jp = 0;
          jgu = (T)(-2) * (gx * um + gy * vm + gz * wm);
        } else {
          jp = (T)(-2) * pm;
          jgu = 0;
        }
        const T sp = (T)ge[10 + f] * jp - (T)(0.5 * ge[9]) * jgu;
        const T su = (T)ge[14 + f] * jgu - (T)0.5 * jp;
        T* col = ys + (f * Nfp + gg) * NC + 4 * el;
        col[0] = sp;
        col[1] = gx * su;
        col[2] = gy * su;
        col[3] = gz * su;
      }
      wave_sync_lds();
      for (int mt = 0; mt < NpP / 16; ++mt) {
        acc_t c = M::zero();
#pragma unroll 4
        for (int k0 = 0; k0 < Kl; k0 += 4) {
          const T a = A.lift[(mt * 16 + ri) * Kl + k0 + kq];
          const T b = ys[(k0 + kq) * NC + ri];
          c = M::mac(a, b, c);
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) xs[(mt * 16 + M::row(kq, rr)) * NC + ri] = c[rr];
      }
      wave_sync_lds();
#pragma unroll
      for (int r = 0; r < NIT; ++r) {
        const int v = lane + 64 * r;
        if (v >= EB * Np) continue;
        const int el = v / Np, n = v - el * Np;
#pragma unroll
        for (int f = 0; f < 4; ++f) rhs[r][f] += xs[n * NC + 4 * el + f];
      }
    }

    // ---- update / store ------------------------------------------------------------
#pragma unroll
    for (int r = 0; r < NIT; ++r) {
      const int v = lane + 64 * r;
      const int el = v / Np, n = v - el * Np;
      if (v >= EB * Np || e0 + el >= K) continue;
      const int64_t off = (e0 + el) * Np + n;
      if constexpr (MODE == kStage) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const T rs = A.dt * rhs[r][f] + (A.read_res ? A.rk_a * A.res[f * KNp + off] : (T)0);
          A.res[f * KNp + off] = rs;
          A.qout[f * KNp + off] = qv[r][f] + A.rk_b * rs;
        }
      } else {
#pragma unroll
        for (int f = 0; f < 4; ++f) A.qout[f * KNp + off] = rhs[r][f];
      }
    }
  }
}

template <int N, typename T, int MODE>
static hipError_t nodal_launch_one(const NodalArgs<T>& a, hipStream_t stream) {
  constexpr int WPB = NodalWaves<N, T>::value;
  const int64_t groups = (a.K + 3) / 4;
  if (groups <= 0) return hipSuccess;
  static int resident = 0, cus = 0;
  if (resident == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return hipErrorInvalidDevice;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, nodal_stage_kernel<N, T, MODE>, 64 * WPB, 0) != hipSuccess)
      return hipErrorInvalidValue;
    resident = occ > 0 ? occ : 1;
  }
  const int64_t needed = (groups + WPB - 1) / WPB;
  int64_t grid = (int64_t)resident * cus;
  if (grid > ((needed + 7) / 8) * 8) grid = ((needed + 7) / 8) * 8;
  grid = ((grid + 7) / 8) * 8;
  if (grid < 8) grid = 8;
  (void)hipGetLastError();  // drop errors left by earlier, unrelated calls
  hipLaunchKernelGGL((nodal_stage_kernel<N, T, MODE>), dim3((unsigned)grid), dim3(64 * WPB), 0, stream, a);
  return hipGetLastError();
}

template <typename T, int MODE>
static hipError_t nodal_launch_mode(int N, const NodalArgs<T>& a, hipStream_t s) {
  switch (N) {
    case 1: return nodal_launch_one<1, T, MODE>(a, s);
    case 2: return nodal_launch_one<2, T, MODE>(a, s);
    case 3: return nodal_launch_one<3, T, MODE>(a, s);
    case 4: return nodal_launch_one<4, T, MODE>(a, s);
    case 5: return nodal_launch_one<5, T, MODE>(a, s);
    case 6: return nodal_launch_one<6, T, MODE>(a, s);
    case 7: return nodal_launch_one<7, T, MODE>(a, s);
    case 8: return nodal_launch_one<8, T, MODE>(a, s);
    case 9: return nodal_launch_one<9, T, MODE>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_nodal_stage(int N, int mode, const NodalArgs<T>& a, hipStream_t s) {
  switch (mode) {
    case kStage: return nodal_launch_mode<T, kStage>(N, a, s);
    case kRhsFull: return nodal_launch_mode<T, kRhsFull>(N, a, s);
    case kRhsVolume: return nodal_launch_mode<T, kRhsVolume>(N, a, s);
    case kRhsSurface: return nodal_launch_mode<T, kRhsSurface>(N, a, s);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_nodal_stage<double>(int, int, const NodalArgs<double>&, hipStream_t);
template hipError_t launch_nodal_stage<float>(int, int, const NodalArgs<float>&, hipStream_t);

}  // namespace bbdg
