// Element-per-thread dense nodal DG comparator (gfx950, vector FMA).
//
// The paper's second nodal baseline (Section 4.2, "element-per-thread"): every
// thread owns one element and applies the dense derivative and lift matrices
// to it in row blocks, the operator entries of a block being shared by all
// threads, so that each entry fetched is reused by a whole wavefront of
// elements.  Here the entries are wave-uniform scalar loads (SGPR operands of
// v_fma, through the scalar cache) instead of blocks staged in shared memory,
// and the 64 lanes of a wave are 64 elements.  The scheme is the same as the
// Bernstein-Bezier path and the MFMA comparator (Section 2 upwind flux, strong
// form of Section 3) in the Lagrange basis of the equispaced lattice:
//   grad p = sum_{d=1..3} grad(lambda_d) (Dr_d p),
//   div u  = sum_{d=1..3} Dr_d h_d,  h_d = grad(lambda_d) . u  (per node),
//   rhs    = (-kappa div u, -grad p) + LIFT (sp, g_f su) on the 4 Nfp face nodes,
// with Dr_d = V (D^d - D^0) V^{-1} and LIFT = [V E_L^f L_0 Vf^{-1}]_f.  Per row
// block of B output nodes a thread keeps 4 B accumulators in registers; the
// input values (own nodes, own and neighbour face traces and the upwind flux)
// are re-read and recomputed for every block (the price of the blocking that
// the paper notes), through L1/L2.  Volume, flux, lift and the LSRK4 update
// run in one kernel (the paper used separate flux and lift kernels).
//
// Operator layouts (built on the host, rows padded with zeros to NB B):
//   opv [Np][NB B][4]:  (Dr_1, Dr_2, Dr_3, 0) of row i for input node j
//   opl [4 Nfp][NB B]:  LIFT row i for face node m = f Nfp + g
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bb_common.hpp"
#include "bb_launch.hpp"

namespace bbdg {

template <int N, typename T, int MODE>
__global__ __launch_bounds__(256) void nodal_ept_kernel(NodalArgs<T> A, const T* __restrict__ opv,
                                                        const T* __restrict__ opl, int64_t blocks) {
  constexpr int Np = np_of(N), Nfp = nfp_of(N);
  constexpr int B = ept_block_rows(N, sizeof(T) == 8);
  constexpr int NB = (Np + B - 1) / B, NpB = NB * B;
  constexpr bool kVol = (MODE != kRhsSurface);
  constexpr bool kSurf = (MODE != kRhsVolume);
  constexpr TabLayout L = tab_layout(N);

  __shared__ uint16_t t_nbr[24 * Nfp];
  __shared__ uint16_t t_fnode[4 * Nfp];
  for (int i = threadIdx.x; i < 24 * Nfp; i += 256) t_nbr[i] = A.tab[L.nbrnode + i];
  for (int i = threadIdx.x; i < 4 * Nfp; i += 256) t_fnode[i] = A.tab[L.fnode + i];
  __syncthreads();

  // XCD-aware: workgroup b runs on XCD b % 8; each XCD takes a contiguous
  // eighth of the element range, so neighbour traces stay in its L2
  const int64_t per_xcd = (blocks + 7) / 8;
  const int64_t lb = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (lb >= blocks) return;
  const int64_t K = A.K;
  const int64_t e = lb * 256 + threadIdx.x;
  if (e >= K) return;
  const uint32_t KNp = (uint32_t)(K * Np);
  const uint32_t base = (uint32_t)e * Np;

  // per-element geometry and flux weights (see kGeoStride)
  const double* ge = A.geo + e * kGeoStride;
  T gl[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) gl[i] = (T)ge[i];
  const T kap = (T)ge[9];
  T ap[4], bu[4];
  int32_t nb[4];
  uint32_t info[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    ap[f] = (T)ge[10 + f];
    bu[f] = (T)ge[14 + f];
    nb[f] = A.etoe[e * 4 + f];
    info[f] = A.etofo[e * 4 + f];
  }
  const T* q0 = A.qin;
  const T* q1 = A.qin + KNp;
  const T* q2 = A.qin + 2 * (size_t)KNp;
  const T* q3 = A.qin + 3 * (size_t)KNp;

  for (int blk = 0; blk < NB; ++blk) {
    const int i0 = blk * B;
    T r[4][B];
#pragma unroll
    for (int b = 0; b < B; ++b) r[0][b] = r[1][b] = r[2][b] = r[3][b] = 0;

    if constexpr (kVol) {
      // acc: Dr_1 p, Dr_2 p, Dr_3 p, sum_d Dr_d h_d
#pragma unroll 1
      for (int j = 0; j < Np; ++j) {
        const T p = q0[base + j], u = q1[base + j], v = q2[base + j], w = q3[base + j];
        const T h1 = gl[0] * u + gl[1] * v + gl[2] * w;
        const T h2 = gl[3] * u + gl[4] * v + gl[5] * w;
        const T h3 = gl[6] * u + gl[7] * v + gl[8] * w;
        const T* o = opv + ((size_t)j * NpB + i0) * 4;
#pragma unroll
        for (int b = 0; b < B; ++b) {
          const T d1 = o[4 * b], d2 = o[4 * b + 1], d3 = o[4 * b + 2];
          r[0][b] += d1 * p;
          r[1][b] += d2 * p;
          r[2][b] += d3 * p;
          r[3][b] += d1 * h1 + d2 * h2 + d3 * h3;
        }
      }
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const T a1 = r[0][b], a2 = r[1][b], a3 = r[2][b];
        r[0][b] = -kap * r[3][b];
        r[1][b] = -(gl[0] * a1 + gl[3] * a2 + gl[6] * a3);
        r[2][b] = -(gl[1] * a1 + gl[4] * a2 + gl[7] * a3);
        r[3][b] = -(gl[2] * a1 + gl[5] * a2 + gl[8] * a3);
      }
    }

    if constexpr (kSurf) {
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        // g_f = -2 grad(lambda_f), grad(lambda_0) = -(sum of the others)
        T gx, gy, gz;
        if (f == 0) {
          gx = (T)2 * (gl[0] + gl[3] + gl[6]);
          gy = (T)2 * (gl[1] + gl[4] + gl[7]);
          gz = (T)2 * (gl[2] + gl[5] + gl[8]);
        } else {
          gx = (T)(-2) * gl[3 * (f - 1)];
          gy = (T)(-2) * gl[3 * (f - 1) + 1];
          gz = (T)(-2) * gl[3 * (f - 1) + 2];
        }
        const int nbf = nb[f];
        const uint16_t* perm = t_nbr + ((info[f] & 3) * 6 + (info[f] >> 2)) * Nfp;
        const uint32_t nbase = nbf >= 0 ? (uint32_t)nbf * Np : 0u;
#pragma unroll 1
        for (int g = 0; g < Nfp; ++g) {
          const int n = t_fnode[f * Nfp + g];
          const T pm = q0[base + n], um = q1[base + n], vm = q2[base + n], wm = q3[base + n];
          const T gum = gx * um + gy * vm + gz * wm;
          T jp, jgu;
          if (nbf >= 0) {
            const uint32_t o = nbase + perm[g];
            jp = q0[o] - pm;
            jgu = gx * q1[o] + gy * q2[o] + gz * q3[o] - gum;
          } else if (A.bc == 0) {  // rigid wall mirror
            jp = 0;
            jgu = (T)(-2) * gum;
          } else {  // pressure-release mirror
            jp = (T)(-2) * pm;
            jgu = 0;
          }
          const T sp = ap[f] * jp - (T)0.5 * kap * jgu;
          const T su = bu[f] * jgu - (T)0.5 * jp;
          const T sx = gx * su, sy = gy * su, sz = gz * su;
          const T* o = opl + (size_t)(f * Nfp + g) * NpB + i0;
#pragma unroll
          for (int b = 0; b < B; ++b) {
            const T l = o[b];
            r[0][b] += l * sp;
            r[1][b] += l * sx;
            r[2][b] += l * sy;
            r[3][b] += l * sz;
          }
        }
      }
    }

    // update / store the rows of this block
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int i = i0 + b;
      if (i >= Np) break;
      const uint32_t off = base + i;
      if constexpr (MODE == kStage) {
#pragma unroll
        for (int fl = 0; fl < 4; ++fl) {
          const uint32_t o = fl * KNp + off;
          const T rs = A.dt * r[fl][b] + (A.read_res ? A.rk_a * A.res[o] : (T)0);
          A.res[o] = rs;
          A.qout[o] = A.qin[o] + A.rk_b * rs;
        }
      } else {
#pragma unroll
        for (int fl = 0; fl < 4; ++fl) A.qout[fl * KNp + off] = r[fl][b];
      }
    }
  }
}

template <int N, typename T, int MODE>
static hipError_t ept_launch_one(const NodalArgs<T>& a, hipStream_t stream) {
  const int64_t blocks = (a.K + 255) / 256;
  if (blocks <= 0) return hipSuccess;
  const int64_t grid = (blocks + 7) / 8 * 8;
  (void)hipGetLastError();  // drop errors left by earlier, unrelated calls
  hipLaunchKernelGGL((nodal_ept_kernel<N, T, MODE>), dim3((unsigned)grid), dim3(256), 0, stream, a, a.dr, a.lift,
                     blocks);
  return hipGetLastError();
}

template <typename T, int MODE>
static hipError_t ept_launch_mode(int N, const NodalArgs<T>& a, hipStream_t s) {
  switch (N) {
    case 1: return ept_launch_one<1, T, MODE>(a, s);
    case 2: return ept_launch_one<2, T, MODE>(a, s);
    case 3: return ept_launch_one<3, T, MODE>(a, s);
    case 4: return ept_launch_one<4, T, MODE>(a, s);
    case 5: return ept_launch_one<5, T, MODE>(a, s);
    case 6: return ept_launch_one<6, T, MODE>(a, s);
    case 7: return ept_launch_one<7, T, MODE>(a, s);
    case 8: return ept_launch_one<8, T, MODE>(a, s);
    case 9: return ept_launch_one<9, T, MODE>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_nodal_ept(int N, int mode, const NodalArgs<T>& a, hipStream_t s) {
  switch (mode) {
    case kStage: return ept_launch_mode<T, kStage>(N, a, s);
    case kRhsFull: return ept_launch_mode<T, kRhsFull>(N, a, s);
    case kRhsVolume: return ept_launch_mode<T, kRhsVolume>(N, a, s);
    case kRhsSurface: return ept_launch_mode<T, kRhsSurface>(N, a, s);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_nodal_ept<double>(int, int, const NodalArgs<double>&, hipStream_t);
template hipError_t launch_nodal_ept<float>(int, int, const NodalArgs<float>&, hipStream_t);

}  // namespace bbdg
