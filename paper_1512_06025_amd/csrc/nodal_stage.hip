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
// A workgroup of four waves takes a block of EB elements, NC = 4 EB columns
// (element-major, field fastest), and computes the block's right-hand side
// as MFMA GEMMs whose B operands sit in LDS, laid out k-major ([k][column],
// rows padded to NC + 16 so that the 16 x 4 operand reads are free of bank
// conflicts), and whose A operands (the operators, shared by every block)
// come from L1/L2; every A tile a wave loads feeds the MFMAs of its column
// tiles, and in FP64 (and FP32 at N = 9) the A values of the next chunk of
// k-steps are loaded into registers while the current chunk's MFMAs run.  The waves split the 16-row tiles of the output (and, where there
// are fewer row tiles than waves, the column tiles).
//   1. Stage the block's nodal values X (Kv x NC) in LDS.
//   2. Volume: for i = 1..3, Y_i = Dr_i X by MFMA, then the geometric
//      combination in registers: the four columns of an element are four
//      neighbouring lanes of the accumulator, so rhs_p = -kappa sum_i
//      grad(lambda_i).(Y_i u, Y_i v, Y_i w) and rhs_u = -sum_i grad(lambda_i)
//      Y_i p are quad reductions and broadcasts (DPP).
//   3. The upwind flux of every face node (own traces from X, the
//      neighbour's from global memory) goes to registers; once every wave is
//      done with X the fluxes (sp, g su) replace it in LDS as the B operand
//      of the lift (Kl x NC), and rhs += LIFT F is accumulated on the same
//      registers.
//   4. The fused LSRK4 update reads and writes the fields from the
//      accumulator layout.
// MFMA tiles are 16 x 16 x 4 (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32);
// lane l holds A[l%16][l/16] and B[l/16][l%16]; accumulator register r of
// lane l is D[row][l%16] with row = l/16 + 4r for the FP64 instruction and
// 4(l/16) + r for the FP32 one.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bb_common.hpp"
#include "bb_launch.hpp"

namespace bbdg {

namespace {

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

// Lane permutations within groups of four lanes (DPP quad_perm).
template <int CTRL>
__device__ __forceinline__ float quad_perm(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double quad_perm(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(v & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kQuadBcast0 = 0x00;  // every lane of the quad reads lane 0
constexpr int kQuadSwap1 = 0xB1;   // (1, 0, 3, 2)
constexpr int kQuadSwap2 = 0x4E;   // (2, 3, 0, 1)

// Applies NOPS operators, each a 16-row slice of a dense matrix in global
// memory (K columns, operator o at a_ptr + o op_stride; this lane's row and
// k offset already in a_ptr), to the block's B operand in LDS (b already at
// this lane's k row, b[k0 ncp + 16 ct + bcol] the column tiles): y = A_o B
// on CTW column tiles, then done(o, y).  The A values of a chunk of up to 8
// (FP64) or 16 (FP32) k-steps sit in registers, and the next chunk's loads (the next operator's
// first chunk included) are issued before the current chunk's MFMAs, so the
// L2 latency of the operator reads overlaps the matrix work.
template <int NOPS, int K, int CTW, typename M, typename T, typename Done>
__device__ __forceinline__ void mfma_ops(const T* __restrict__ a_ptr, size_t op_stride, const T* b, int ncp,
                                         int bcol, Done&& done) {
  typedef typename M::acc acc_t;
  constexpr int KCM = sizeof(T) == 8 ? 8 : 16;  // k-steps per chunk (registers: 2 KCM values)
  constexpr int KS = K / 4, KC = KS < KCM ? KS : KCM, NCH = (KS + KC - 1) / KC, NQ = NOPS * NCH;
  T a0[KC], a1[KC];
  auto load = [&](T (&dst)[KC], int q) {
    const int o = q / NCH, ch = q % NCH;
    const T* p = a_ptr + (size_t)o * op_stride + ch * KC * 4;
#pragma unroll
    for (int kk = 0; kk < KC; ++kk)
      if (ch * KC + kk < KS) dst[kk] = p[kk * 4];
  };
  load(a0, 0);
  acc_t y[CTW];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int o = q / NCH, ch = q % NCH;
    if (ch == 0) {
#pragma unroll
      for (int ct = 0; ct < CTW; ++ct) y[ct] = M::zero();
    }
    if (q + 1 < NQ) {
      if (q & 1) {
        load(a0, q + 1);
      } else {
        load(a1, q + 1);
      }
    }
    const T(&cur)[KC] = (q & 1) ? a1 : a0;
#pragma unroll
    for (int kk = 0; kk < KC; ++kk) {
      const int ks = ch * KC + kk;
      if (ks >= KS) break;
#pragma unroll
      for (int ct = 0; ct < CTW; ++ct) y[ct] = M::mac(cur[kk], b[ks * 4 * ncp + ct * 16 + bcol], y[ct]);
    }
    if (ch == NCH - 1) {
      done(o, y);
      // keep the next operator's LDS reads from being hoisted above this
      // point (registers); its first A chunk is already in flight
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

}  // namespace

#ifndef BBDG_NODAL_EB_F64
#define BBDG_NODAL_EB_F64(N) ((N) <= 4 ? 16 : ((N) == 5 ? 12 : ((N) <= 7 ? 8 : 4)))
#endif
#ifndef BBDG_NODAL_EB_F32
#define BBDG_NODAL_EB_F32(N) ((N) <= 6 ? 16 : 8)
#endif

// Block shape of order N: EB elements per workgroup (NC = 4 EB columns, CT
// column tiles of 16), LDS rows of NCP values, MT row tiles.  The four waves
// form WR groups along the rows and WC = 4 / WR along the columns (fewer row
// tiles than waves at low order): a wave takes at most RPW row tiles and CTW
// column tiles.  NIT face-node items per thread for the flux.
template <int N, typename T>
struct NodalCfg {
  static constexpr int Np = np_of(N), Nfp = nfp_of(N), NL = 4 * nfp_of(N);
  static constexpr NodalDims D = nodal_dims(N);
  static constexpr int NpP = D.NpP, Kv = D.Kv, Kl = D.Kl;
  static constexpr int KMAX = Kv > Kl ? Kv : Kl;
  static constexpr int EB = sizeof(T) == 8 ? BBDG_NODAL_EB_F64(N) : BBDG_NODAL_EB_F32(N);
  static constexpr int NC = 4 * EB, CT = NC / 16, NCP = NC + 16;
  static constexpr int MT = NpP / 16;
  static constexpr int WR = MT >= 4 ? 4 : (MT >= 2 ? 2 : 1), WC = 4 / WR;
  static constexpr int RPW = (MT + WR - 1) / WR, CTW = CT / WC > 0 ? CT / WC : 1;
  static constexpr int NIT = (EB * NL + 255) / 256;
  static_assert(CT % WC == 0 || CT < WC, "column tiles split evenly over the column groups");
};

template <int N, typename T, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void nodal_stage_kernel(NodalArgs<T> A,
                                                                                            int64_t blocks) {
  using C = NodalCfg<N, T>;
  using M = Mfma<T>;
  typedef typename M::acc acc_t;
  constexpr int Np = C::Np, Nfp = C::Nfp, NL = C::NL, Kv = C::Kv, Kl = C::Kl, NpP = C::NpP;
  constexpr int EB = C::EB, NC = C::NC, CT = C::CT, NCP = C::NCP, MT = C::MT, RPW = C::RPW, NIT = C::NIT;
  constexpr int WR = C::WR, CTW = C::CTW;
  constexpr bool kVol = (MODE != kRhsSurface);
  constexpr bool kSurf = (MODE != kRhsVolume);
  constexpr TabLayout L = tab_layout(N);

  __shared__ __attribute__((aligned(16))) T buf[C::KMAX * NCP];
  __shared__ double shg[EB * kGeoStride];
  __shared__ int32_t she[EB * 4];
  __shared__ uint8_t shf[EB * 4];
  __shared__ uint16_t t_nbr[24 * Nfp];
  __shared__ uint16_t t_fnode[4 * Nfp];

  // XCD-aware: workgroup b runs on XCD b % 8, which takes a contiguous
  // eighth of the element blocks (neighbour traces then share its L2)
  const int64_t per_xcd = (blocks + 7) / 8;
  const int64_t lb = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (lb >= blocks) return;  // the whole workgroup
  const int tid = threadIdx.x;
  const int64_t K = A.K;
  const int64_t e0 = lb * EB;

  for (int i = tid; i < 24 * Nfp; i += 256) t_nbr[i] = A.tab[L.nbrnode + i];
  for (int i = tid; i < 4 * Nfp; i += 256) t_fnode[i] = A.tab[L.fnode + i];
  for (int v = tid; v < EB * kGeoStride; v += 256) {
    const int64_t idx = e0 * kGeoStride + v;
    shg[v] = idx < K * kGeoStride ? A.geo[idx] : 0.0;
  }
  if (tid < EB * 4) {
    const int64_t idx = e0 * 4 + tid;
    she[tid] = idx < K * 4 ? A.etoe[idx] : -1;
    shf[tid] = idx < K * 4 ? A.etofo[idx] : 0;
  }
  // X: buf[k][col] = field (col % 4) of element e0 + col / 4 at node k
  for (int idx = tid; idx < Kv * NC; idx += 256) {
    const int k = idx / NC, col = idx - k * NC;
    const int el = col >> 2, fl = col & 3;
    T v = 0;
    if (k < Np && e0 + el < K) v = A.qin[(uint32_t)(e0 + el) * (4 * Np) + fl * Np + k];
    buf[k * NCP + col] = v;
  }
  __syncthreads();

  const int w = tid >> 6, lane = tid & 63;
  const int ri = lane & 15;  // MFMA row / column index within a tile
  const int kq = lane >> 4;  // MFMA k index (0..3) / accumulator row block
  const int fl = ri & 3;     // field of this lane's columns
  const int wr = w % WR;     // this wave's row group: row tiles wr, wr + WR, ...
  const int c0 = (w / WR) * CTW;  // and its first column tile
  const bool cols = c0 < CT;      // (no columns for this wave when CT < WC)

  acc_t rhs[RPW][CTW];
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int ct = 0; ct < CTW; ++ct) rhs[r][ct] = M::zero();

  // ---- volume: Y_i = Dr_i X, combined with grad(lambda_i) per element ---------------
  // (FP64 and FP32 at N = 9: operator reads software-pipelined through
  // registers, mfma_ops; FP32 below: one operator at a time, A read per
  // k-step, which keeps the register count and the occupancy up.  Measured on
  // 196,608 tets: the pipeline is 2-10 % faster in FP64 at N = 3..7 and 4 %
  // in FP32 at N = 9, but 2-6 % slower in FP32 at N = 3..7.)
  constexpr bool kPipe = sizeof(T) == 8 || N >= 9;
  auto combine = [&](int r, int i, acc_t(&y)[CTW]) {
#pragma unroll
    for (int ct = 0; ct < CTW; ++ct) {
      const int el = (c0 + ct) * 4 + (ri >> 2);
      // d(lambda_{i+1})/d(x_{fl-1}) on velocity lanes, 0 on pressure lanes
      const T gc = fl ? (T)shg[el * kGeoStride + 3 * i + fl - 1] : (T)0;
      const T kap = (T)shg[el * kGeoStride + 9];
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const T yv = y[ct][rr];
        const T p = quad_perm<kQuadBcast0>(yv);
        T s = gc * yv;
        s += quad_perm<kQuadSwap1>(s);
        s += quad_perm<kQuadSwap2>(s);
        rhs[r][ct][rr] -= fl ? gc * p : kap * s;
      }
    }
  };
  if constexpr (kVol) {
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int rt = wr + WR * r;
      if (rt >= MT || !cols) break;
      if constexpr (kPipe) {
        mfma_ops<3, Kv, CTW, M>(A.dr + (size_t)(rt * 16 + ri) * Kv + kq, (size_t)NpP * Kv, buf + kq * NCP, NCP,
                                c0 * 16 + ri, [&](int i, acc_t(&y)[CTW]) { combine(r, i, y); });
      } else {
#pragma unroll 1
        for (int i = 0; i < 3; ++i) {
          acc_t y[CTW];
#pragma unroll
          for (int ct = 0; ct < CTW; ++ct) y[ct] = M::zero();
          const T* Ai = A.dr + (size_t)i * NpP * Kv + (size_t)(rt * 16 + ri) * Kv + kq;
#pragma unroll 4
          for (int k0 = 0; k0 < Kv; k0 += 4) {
            const T a = Ai[k0];
#pragma unroll
            for (int ct = 0; ct < CTW; ++ct)
              y[ct] = M::mac(a, buf[(k0 + kq) * NCP + (c0 + ct) * 16 + ri], y[ct]);
          }
          combine(r, i, y);
        }
      }
    }
  }

  // ---- upwind flux of every face node of the block, into registers ----------------
  T fv[kSurf ? NIT : 1][4];
  if constexpr (kSurf) {
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
      const int it = tid + 256 * j;
      const int el = it / NL, m = it - el * NL;
      fv[j][0] = fv[j][1] = fv[j][2] = fv[j][3] = 0;
      if (it >= EB * NL || e0 + el >= K) continue;
      const int f = m / Nfp, g = m - f * Nfp;
      const int n = t_fnode[m];
      const T pm = buf[n * NCP + 4 * el], um = buf[n * NCP + 4 * el + 1], vm = buf[n * NCP + 4 * el + 2],
              wm = buf[n * NCP + 4 * el + 3];
      const double* ge = shg + el * kGeoStride;
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
      const T gum = gx * um + gy * vm + gz * wm;
      const int nb = she[el * 4 + f];
      T jp, jgu;
      if (nb >= 0) {
        const int info = shf[el * 4 + f];
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
      fv[j][0] = sp;
      fv[j][1] = gx * su;
      fv[j][2] = gy * su;
      fv[j][3] = gz * su;
    }
  }

  // ---- surface: the fluxes replace X in LDS, rhs += LIFT F ---------------------------
  if constexpr (kSurf) {
    __syncthreads();  // every wave is done with X
#pragma unroll
    for (int j = 0; j < NIT; ++j) {
      const int it = tid + 256 * j;
      if (it >= EB * NL) continue;
      const int el = it / NL, m = it - el * NL;
#pragma unroll
      for (int c = 0; c < 4; ++c) buf[m * NCP + 4 * el + c] = fv[j][c];
    }
    for (int idx = tid; idx < (Kl - NL) * NC; idx += 256) buf[(NL + idx / NC) * NCP + idx % NC] = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int rt = wr + WR * r;
      if (rt >= MT || !cols) break;
      if constexpr (kPipe) {
        mfma_ops<1, Kl, CTW, M>(A.lift + (size_t)(rt * 16 + ri) * Kl + kq, 0, buf + kq * NCP, NCP, c0 * 16 + ri,
                                [&](int, acc_t(&y)[CTW]) {
#pragma unroll
          for (int ct = 0; ct < CTW; ++ct) rhs[r][ct] += y[ct];
        });
      } else {
        const T* Lr = A.lift + (size_t)(rt * 16 + ri) * Kl + kq;
#pragma unroll 4
        for (int k0 = 0; k0 < Kl; k0 += 4) {
          const T a = Lr[k0];
#pragma unroll
          for (int ct = 0; ct < CTW; ++ct)
            rhs[r][ct] = M::mac(a, buf[(k0 + kq) * NCP + (c0 + ct) * 16 + ri], rhs[r][ct]);
        }
      }
    }
  }

  // ---- update / store from the accumulator layout -----------------------------------------
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const int rt = wr + WR * r;
    if (rt >= MT || !cols) break;
#pragma unroll
    for (int ct = 0; ct < CTW; ++ct) {
      const int64_t e = e0 + (c0 + ct) * 4 + (ri >> 2);
      if (e >= K) continue;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int row = rt * 16 + M::row(kq, rr);
        if (row >= Np) continue;
        const uint32_t o = (uint32_t)e * (4 * Np) + fl * Np + row;
        if constexpr (MODE == kStage) {
          const T rs = A.dt * rhs[r][ct][rr] + (A.read_res ? A.rk_a * A.res[o] : (T)0);
          A.res[o] = rs;
          A.qout[o] = A.qin[o] + A.rk_b * rs;
        } else {
          A.qout[o] = rhs[r][ct][rr];
        }
      }
    }
  }
}

template <int N, typename T, int MODE>
static hipError_t nodal_launch_one(const NodalArgs<T>& a, hipStream_t stream) {
  using C = NodalCfg<N, T>;
  const int64_t blocks = (a.K + C::EB - 1) / C::EB;
  if (blocks <= 0) return hipSuccess;
  const int64_t grid = (blocks + 7) / 8 * 8;
  (void)hipGetLastError();  // drop errors left by earlier, unrelated calls
  hipLaunchKernelGGL((nodal_stage_kernel<N, T, MODE>), dim3((unsigned)grid), dim3(256), 0, stream, a, blocks);
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
