// Element-per-thread dense nodal DG comparator (gfx950, vector FMA).
//
// The paper's second nodal baseline (Section 4.2, "element-per-thread"): every
// thread owns one element and applies the dense derivative and lift matrices
// to it in blocks of output rows, the operator entries of a block being
// shared by all threads, so that each entry fetched is reused by a whole
// workgroup of elements: here 256 consecutive elements (four waves of 64), the
// operator tile of the current row block and input chunk staged in LDS and
// read with wave-uniform (broadcast) addresses.
// As in the paper the surface work is split: a flux kernel writes the upwind
// flux of every face node to a buffer, and the element-per-thread kernel
// applies the derivative matrices, the lift and the LSRK4 update.  The scheme
// is the one of the Bernstein-Bezier path and of the MFMA comparator (Section
// 2 upwind flux, strong form of Section 3) in the Lagrange basis of the
// equispaced lattice:
//   grad p = sum_{d=1..3} grad(lambda_d) (Dr_d p),
//   div u  = sum_{d=1..3} Dr_d h_d,  h_d = grad(lambda_d) . u  (per node),
//   rhs    = (-kappa div u, -grad p) + LIFT (sp, g_f su) on the 4 Nfp face nodes,
// with Dr_d = V (D^d - D^0) V^{-1} and LIFT = [V E_L^f L_0 Vf^{-1}]_f.
//
// Data movement of the element-per-thread kernel: the inputs of an element
// (its 4 Np coefficients, then its 4 x 4 Nfp flux values) are read in chunks
// of J nodes for the wave's 64 elements with coalesced loads (each element's
// J values are contiguous) into a per-wave LDS buffer laid out node-major,
// [field][node][element], from which every lane reads its own element with
// conflict-free accesses.  Each block of B output rows keeps 4 B accumulators
// in registers and re-reads the chunks (the redundant loads of the blocking
// the paper notes, here from L2).  The block's right-hand side goes back
// through the same LDS buffer so that the LSRK4 update reads and writes the
// fields with coalesced accesses.
//
// Operator layouts (built on the host, rows padded with zeros to NB B):
//   opv [Np][NB B][4]:  (Dr_1, Dr_2, Dr_3, 0) of row i for input node j
//   opl [4 Nfp][NB B]:  LIFT row i for face node m = f Nfp + g
// Flux buffer (library-owned): F (4, K, 4 Nfp) of the element type, the
// components (sp, g_x su, g_y su, g_z su) of face node m of element k at
// F[c][k 4 Nfp + m].
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bb_common.hpp"
#include "bb_launch.hpp"

namespace bbdg {

namespace {

__device__ __forceinline__ void ept_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

}  // namespace

// Upwind flux on every face node (one thread per element face node): own
// trace, the neighbour's through the orientation tables or the boundary
// mirror, then sp = a_p [[p]] - kappa/2 g.[[u]] and su = b_u g.[[u]] - [[p]]/2
// (the weights of kGeoStride), stored as (sp, g su).
template <int N, typename T>
__global__ __launch_bounds__(256) void ept_flux_kernel(NodalArgs<T> A, T* __restrict__ F) {
  constexpr int Np = np_of(N), Nfp = nfp_of(N), NL = 4 * Nfp;
  constexpr TabLayout L = tab_layout(N);
  __shared__ uint16_t t_nbr[24 * Nfp];
  __shared__ uint16_t t_fnode[4 * Nfp];
  for (int i = threadIdx.x; i < 24 * Nfp; i += 256) t_nbr[i] = A.tab[L.nbrnode + i];
  for (int i = threadIdx.x; i < 4 * Nfp; i += 256) t_fnode[i] = A.tab[L.fnode + i];
  __syncthreads();
  const int64_t K = A.K;
  const int64_t items = K * NL;
  const size_t KL = (size_t)K * NL;
  for (int64_t it = (int64_t)blockIdx.x * 256 + threadIdx.x; it < items; it += (int64_t)gridDim.x * 256) {
    const int64_t e = it / NL;
    const int m = (int)(it - e * NL);
    const int f = m / Nfp, g = m - f * Nfp;
    const double* ge = A.geo + e * kGeoStride;
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
    const uint32_t own = (uint32_t)e * (4 * Np) + t_fnode[m];  // element-major fields
    const T pm = A.qin[own], um = A.qin[Np + own], vm = A.qin[2 * Np + own], wm = A.qin[3 * Np + own];
    const T gum = gx * um + gy * vm + gz * wm;
    const int32_t nb = A.etoe[e * 4 + f];
    T jp, jgu;
    if (nb >= 0) {
      const uint32_t info = A.etofo[e * 4 + f];
      const uint32_t o = (uint32_t)nb * (4 * Np) + t_nbr[((info & 3) * 6 + (info >> 2)) * Nfp + g];
      jp = A.qin[o] - pm;
      jgu = gx * A.qin[Np + o] + gy * A.qin[2 * Np + o] + gz * A.qin[3 * Np + o] - gum;
    } else if (A.bc == 0) {  // rigid wall mirror
      jp = 0;
      jgu = (T)(-2) * gum;
    } else {  // pressure-release mirror
      jp = (T)(-2) * pm;
      jgu = 0;
    }
    const T sp = (T)ge[10 + f] * jp - (T)(0.5 * ge[9]) * jgu;
    const T su = (T)ge[14 + f] * jgu - (T)0.5 * jp;
    F[it] = sp;
    F[KL + it] = gx * su;
    F[2 * KL + it] = gy * su;
    F[3 * KL + it] = gz * su;
  }
}

// Chunk of J nodes per staging round and LDS row padding: rows of 64 + PAD
// values, so that the staging writes (J consecutive nodes of one element per
// J lanes) spread over the banks.
template <typename T>
struct EptStage {
  static constexpr int J = sizeof(T) == 8 ? 8 : 16;
  static constexpr int PAD = sizeof(T) == 8 ? 8 : 4;
  static constexpr int ROW = 64 + PAD;
};

// Stages values [n0, n0 + J) of the 4 arrays src + c * cstride (element k's
// len values at k * estride) for the wave's elements e0 .. e0 + 63 into
// s[c][jj][lane]; out-of-range entries read as zero.
template <typename T>
__device__ __forceinline__ void ept_stage(T* s, const T* src, size_t cstride, size_t estride, int len, int n0,
                                          int64_t e0, int64_t K, int lane) {
  constexpr int J = EptStage<T>::J, ROW = EptStage<T>::ROW;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int it = 0; it < J; ++it) {
      const int idx = it * 64 + lane;
      const int el = idx / J, jj = idx % J;
      const int n = n0 + jj;
      T v = 0;
      if (n < len && e0 + el < K) v = src[c * cstride + (size_t)(e0 + el) * estride + n];
      s[(c * J + jj) * ROW + el] = v;
    }
  }
}

template <int N, typename T, int MODE>
__global__ __launch_bounds__(256) void nodal_ept_kernel(NodalArgs<T> A, const T* __restrict__ opv,
                                                        const T* __restrict__ opl, const T* __restrict__ F,
                                                        int64_t blocks) {
  constexpr int Np = np_of(N), Nfp = nfp_of(N), NL = 4 * Nfp;
  constexpr int B = ept_block_rows(N, sizeof(T) == 8);
  constexpr int NB = (Np + B - 1) / B, NpB = NB * B;
  constexpr int J = EptStage<T>::J, ROW = EptStage<T>::ROW;
  constexpr bool kVol = (MODE != kRhsSurface);
  constexpr bool kSurf = (MODE != kRhsVolume);
  static_assert(64 * (B + 1) <= 4 * J * ROW, "the output rows fit in the staging buffer");

  __shared__ __attribute__((aligned(16))) T stage_buf[4][4 * J * ROW];
  // operator tile of the current row block and chunk, shared by the four
  // waves: (Dr_1, Dr_2, Dr_3, 0) of B rows for J inputs, or LIFT of B rows
  // for J face nodes
  __shared__ __attribute__((aligned(16))) T op_tile[J * B * 4];

  // XCD-aware: workgroup b runs on XCD b % 8; each XCD takes a contiguous
  // eighth of the workgroups, so neighbouring elements share an L2
  const int64_t per_xcd = (blocks + 7) / 8;
  const int64_t lb = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (lb >= blocks) return;  // whole workgroup: no barrier follows
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  const int lane = tid & 63;
  const int64_t K = A.K;
  const int64_t e0 = (lb * 4 + w) * 64;  // the wave's first element (may lie past K: the wave
                                         // still takes part in the workgroup's barriers)
  T* s = stage_buf[w];
  const int64_t e = e0 + lane;
  const bool live = e < K;

  // per-element geometry (see kGeoStride)
  T gl[9];
  T kap = 0;
  {
    const double* ge = A.geo + (live ? e : 0) * kGeoStride;
#pragma unroll
    for (int i = 0; i < 9; ++i) gl[i] = (T)ge[i];
    kap = (T)ge[9];
  }

  for (int blk = 0; blk < NB; ++blk) {
    const int i0 = blk * B;
    T r[4][B];
#pragma unroll
    for (int b = 0; b < B; ++b) r[0][b] = r[1][b] = r[2][b] = r[3][b] = 0;

    if constexpr (kVol) {
      // acc: Dr_1 p, Dr_2 p, Dr_3 p, sum_d Dr_d h_d
      for (int j0 = 0; j0 < Np; j0 += J) {
        const int jn = Np - j0 < J ? Np - j0 : J;
        __syncthreads();  // the previous chunk's tile and buffers are consumed
        ept_stage<T>(s, A.qin, Np, 4 * Np, Np, j0, e0, K, lane);  // element-major fields
        for (int t = tid; t < jn * B * 4; t += 256) {
          const int jj = t / (B * 4), rest = t - jj * (B * 4);
          op_tile[t] = opv[((size_t)(j0 + jj) * NpB + i0) * 4 + rest];
        }
        __syncthreads();
#pragma unroll 1
        for (int jj = 0; jj < jn; ++jj) {
          const T p = s[(0 * J + jj) * ROW + lane], u = s[(1 * J + jj) * ROW + lane];
          const T v = s[(2 * J + jj) * ROW + lane], ww = s[(3 * J + jj) * ROW + lane];
          const T h1 = gl[0] * u + gl[1] * v + gl[2] * ww;
          const T h2 = gl[3] * u + gl[4] * v + gl[5] * ww;
          const T h3 = gl[6] * u + gl[7] * v + gl[8] * ww;
          const T* o = op_tile + jj * B * 4;
#pragma unroll
          for (int b = 0; b < B; ++b) {
            const T d1 = o[4 * b], d2 = o[4 * b + 1], d3 = o[4 * b + 2];
            r[0][b] += d1 * p;
            r[1][b] += d2 * p;
            r[2][b] += d3 * p;
            r[3][b] += d1 * h1 + d2 * h2 + d3 * h3;
          }
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
      for (int m0 = 0; m0 < NL; m0 += J) {
        const int mn = NL - m0 < J ? NL - m0 : J;
        __syncthreads();
        ept_stage<T>(s, F, (size_t)K * NL, NL, NL, m0, e0, K, lane);
        for (int t = tid; t < mn * B; t += 256) {
          const int jj = t / B, b = t - jj * B;
          op_tile[t] = opl[(size_t)(m0 + jj) * NpB + i0 + b];
        }
        __syncthreads();
#pragma unroll 1
        for (int jj = 0; jj < mn; ++jj) {
          const T sp = s[(0 * J + jj) * ROW + lane], sx = s[(1 * J + jj) * ROW + lane];
          const T sy = s[(2 * J + jj) * ROW + lane], sz = s[(3 * J + jj) * ROW + lane];
          const T* o = op_tile + jj * B;
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

    // update / store the rows of this block: each field's B x 64 block goes
    // through LDS ([element][row], rows of B + 1) so that the global accesses
    // are coalesced (B consecutive values of one element per B lanes)
    const int bn = Np - i0 < B ? Np - i0 : B;
#pragma unroll
    for (int fl = 0; fl < 4; ++fl) {
      ept_wave_sync();  // the wave's own buffer: no workgroup barrier needed
#pragma unroll
      for (int b = 0; b < B; ++b) s[lane * (B + 1) + b] = r[fl][b];
      ept_wave_sync();
      for (int idx = lane; idx < 64 * B; idx += 64) {
        const int el = idx / B, b = idx % B;
        if (b >= bn || e0 + el >= K) continue;
        const uint32_t o = (uint32_t)(e0 + el) * (4 * Np) + fl * Np + i0 + b;
        const T rhs = s[el * (B + 1) + b];
        if constexpr (MODE == kStage) {
          const T rs = A.dt * rhs + (A.read_res ? A.rk_a * A.res[o] : (T)0);
          A.res[o] = rs;
          A.qout[o] = A.qin[o] + A.rk_b * rs;
        } else {
          A.qout[o] = rhs;
        }
      }
    }
  }
}

template <int N, typename T, int MODE>
static hipError_t ept_launch_one(const NodalArgs<T>& a, hipStream_t stream) {
  if (a.K <= 0) return hipSuccess;
  if (!a.flux) return hipErrorInvalidValue;
  constexpr int NL = 4 * nfp_of(N);
  (void)hipGetLastError();  // drop errors left by earlier, unrelated calls
  if (MODE != kRhsVolume) {
    const int64_t items = a.K * NL;
    int64_t fgrid = (items + 255) / 256;
    if (fgrid > 65536) fgrid = 65536;
    hipLaunchKernelGGL((ept_flux_kernel<N, T>), dim3((unsigned)fgrid), dim3(256), 0, stream, a, a.flux);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t blocks = (a.K + 255) / 256;  // four waves of 64 elements
  const int64_t grid = (blocks + 7) / 8 * 8;
  hipLaunchKernelGGL((nodal_ept_kernel<N, T, MODE>), dim3((unsigned)grid), dim3(256), 0, stream, a, a.dr, a.lift,
                     (const T*)a.flux, blocks);
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
