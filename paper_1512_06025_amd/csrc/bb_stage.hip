// Fused Bernstein-Bezier DG stage kernel for gfx950 (wave64).
//
// One 64-lane workgroup owns EPW consecutive elements (EPW = 64/Np for
// Np <= 32, otherwise 1) and computes, for each of them:
//   1. the element's coefficients of (p,u,v,w) staged in LDS ([node][field]);
//   2. surface part 1: on every face node the exterior trace (neighbour's
//      coinciding control point through the orientation table, or the mirror
//      state), and the upwind flux (Section 2) pre-scaled so that
//        rhs_p   += sum_f E_L^f L_0 sp^f,   sp = kappa/2 (tau_p |g| [[p]] - g.[[u]])
//        rhs_u_i += sum_f g_i E_L^f L_0 su^f, su = 1/2 (tau_u g.[[u]]/|g| - [[p]])
//      with g = Fscale_f n_f = -2 grad(lambda_f) (only two face vectors per
//      face need lifting, because the velocity flux is a scalar times n);
//   3. surface part 2: w_0 = L_0 s on the 8 face vectors (at most 7 nonzeros
//      per row; L_0[b,b] = 1/2 sum_k (b_k+1)^2, L_0[b, b+e_k-e_m] = 1/2 (b_k+1) b_m,
//      the entries of ((N+1)^2/2)(E^{N+1}_N)^T E^{N+1}_N, Section 3.1.2);
//   4. surface part 3: E_L^f applied as N one-degree reductions
//      w_j = (E^{N-j+1}_{N-j})^T w_{j-1},  [E^T w](b) = sum_k (b_k+1)/(m+1) w(b+e_k)
//      (the slice-by-slice order of Algorithm 1), all levels kept in LDS; the
//      volume node alpha then gathers ell_{alpha_f} w_{alpha_f}(alpha without f)
//      from every face, ell_j = (-1)^j C(N,j)/(1+j);
//   5. volume part (Algorithm 2 with the row form of Lemma 1, Appendix A.1):
//      (D^i f)(alpha) = sum_j alpha_j f[alpha + e_i - e_j]; the physical
//      gradient is sum_{i=1..3} grad(lambda_i) (D^i - D^0) f;
//   6. the low-storage RK4 update res = a res + dt rhs, q_out = q + b res
//      (fused; stage mode), or a plain store of the right-hand side.
// The workgroup is a single wavefront, so its barriers are cheap and no
// other wave waits on it.  Fields ping-pong between q_in and q_out, so a
// stage never overwrites a trace that another workgroup still reads.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bb_common.hpp"
#include "bb_launch.hpp"

namespace bbdg {

template <int N>
struct Ell {
  // ell_j = (-1)^j C(N,j)/(1+j), j = 0..N (Section 3.1.2)
  static constexpr double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
  }
  static constexpr double value(int j) { return ((j & 1) ? -1.0 : 1.0) * binom(N, j) / (1.0 + j); }
};

template <int N>
__device__ __forceinline__ double ell_of(int j) {
  double r = 0.0;
#pragma unroll
  for (int i = 0; i <= N; ++i) r = (j == i) ? Ell<N>::value(i) : r;
  return r;
}

template <int N, typename T, int MODE>
__global__ __launch_bounds__(64) void bb_stage_kernel(StageArgs<T> A) {
  constexpr int Np = np_of(N);
  constexpr int Nfp = nfp_of(N);
  constexpr int EPW = (Np <= 32) ? (64 / Np) : 1;
  constexpr int NPL = (EPW * Np + 63) / 64;
  constexpr bool kVol = (MODE != kRhsSurface);
  constexpr bool kSurf = (MODE != kRhsVolume);
  constexpr TabLayout L = tab_layout(N);

  __shared__ T sq[EPW][Np][4];
  __shared__ T sflux[EPW][8][Nfp];
  __shared__ T slev[EPW][8][Np];

  const int lane = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * EPW;
  const int64_t K = A.K;
  const int64_t KNp = K * Np;
  const uint16_t* __restrict__ tab = A.tab;

  // ---- 1. own coefficients -> registers and LDS ----------------------------
  T qv[NPL][4];
#pragma unroll
  for (int r = 0; r < NPL; ++r) {
    const int v = lane + 64 * r;
    if (v < EPW * Np) {
      const int el = v / Np;
      const int n = v - el * Np;
      const int64_t e = e0 + el;
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        T x = 0;
        if (e < K) x = A.qin[f * KNp + e * Np + n];
        qv[r][f] = x;
        sq[el][n][f] = x;
      }
    }
  }
  __syncthreads();

  if constexpr (kSurf) {
    // ---- 2. traces and upwind flux ----------------------------------------
    for (int v = lane; v < EPW * 4 * Nfp; v += 64) {
      const int el = v / (4 * Nfp);
      const int rem = v - el * 4 * Nfp;
      const int f = rem / Nfp;
      const int g = rem - f * Nfp;
      const int64_t e = e0 + el;
      T sp = 0, su = 0;
      if (e < K) {
        const int n = tab[L.fnode + f * Nfp + g];
        const T pm = sq[el][n][0], um = sq[el][n][1], vm = sq[el][n][2], wm = sq[el][n][3];
        const double* ge = A.geo + e * kGeoStride;
        double gx, gy, gz;
        if (f == 0) {
          gx = 2.0 * (ge[0] + ge[3] + ge[6]);
          gy = 2.0 * (ge[1] + ge[4] + ge[7]);
          gz = 2.0 * (ge[2] + ge[5] + ge[8]);
        } else {
          gx = -2.0 * ge[3 * (f - 1) + 0];
          gy = -2.0 * ge[3 * (f - 1) + 1];
          gz = -2.0 * ge[3 * (f - 1) + 2];
        }
        const double gn = sqrt(gx * gx + gy * gy + gz * gz);
        const double ce = ge[9];
        const int32_t nb = A.etoe[e * 4 + f];
        double cp = ce;
        T jp, jgu;
        const T tgx = (T)gx, tgy = (T)gy, tgz = (T)gz;
        if (nb >= 0) {
          const int info = A.etofo[e * 4 + f];
          const int f2 = info & 3;
          const int o = info >> 2;
          const int n2 = tab[L.nbrnode + (f2 * 6 + o) * Nfp + g];
          const int64_t off = (int64_t)nb * Np + n2;
          const T pp = A.qin[off], up = A.qin[KNp + off], vp = A.qin[2 * KNp + off],
                  wp = A.qin[3 * KNp + off];
          cp = A.geo[(int64_t)nb * kGeoStride + 9];
          jp = pp - pm;
          jgu = tgx * (up - um) + tgy * (vp - vm) + tgz * (wp - wm);
        } else if (A.bc == 0) {  // rigid wall mirror
          jp = 0;
          jgu = (T)(-2) * (tgx * um + tgy * vm + tgz * wm);
        } else {  // pressure-release mirror
          jp = (T)(-2) * pm;
          jgu = 0;
        }
        const T tau_p = (T)(2.0 / (ce + cp));
        const T tau_u = (T)(0.5 * (ce + cp));
        const T kap = (T)(ce * ce);
        sp = (T)0.5 * kap * (tau_p * (T)gn * jp - jgu);
        su = (T)0.5 * (tau_u * jgu / (T)gn - jp);
      }
      sflux[el][f][g] = sp;
      sflux[el][4 + f][g] = su;
    }
    __syncthreads();

    // ---- 3. w_0 = L_0 s (level 0 of every face vector) ---------------------
    for (int v = lane; v < EPW * 8 * Nfp; v += 64) {
      const int el = v / (8 * Nfp);
      const int rem = v - el * 8 * Nfp;
      const int vec = rem / Nfp;
      const int g = rem - vec * Nfp;
      // face-local (b0,b1,b2) of position g = (a0,a1,a2) of volume node g (a3 = 0)
      const int b0 = tab[L.alpha + 4 * g + 0];
      const int b1 = tab[L.alpha + 4 * g + 1];
      const int b2 = tab[L.alpha + 4 * g + 2];
      const T* s = sflux[el][vec];
      T acc = (T)(0.5 * ((b0 + 1) * (b0 + 1) + (b1 + 1) * (b1 + 1) + (b2 + 1) * (b2 + 1))) * s[g];
      const int row = tri_row(b2, N);
      if (b1 >= 1) {
        acc += (T)(0.5 * (b0 + 1) * b1) * s[row + b1 - 1];                        // +e0 -e1
        acc += (T)(0.5 * (b2 + 1) * b1) * s[tri_row(b2 + 1, N) + b1 - 1];         // +e2 -e1
      }
      if (b2 >= 1) {
        acc += (T)(0.5 * (b0 + 1) * b2) * s[tri_row(b2 - 1, N) + b1];             // +e0 -e2
        acc += (T)(0.5 * (b1 + 1) * b2) * s[tri_row(b2 - 1, N) + b1 + 1];         // +e1 -e2
      }
      if (b0 >= 1) {
        acc += (T)(0.5 * (b1 + 1) * b0) * s[row + b1 + 1];                        // +e1 -e0
        acc += (T)(0.5 * (b2 + 1) * b0) * s[tri_row(b2 + 1, N) + b1];            // +e2 -e0
      }
      slev[el][vec][g] = acc;
    }
    __syncthreads();

    // ---- 4. one-degree reductions, level j = 1..N ---------------------------
#pragma unroll
    for (int j = 1; j <= N; ++j) {
      const int m = N - j;
      const int out0 = level_off(j, N);
      const int in0 = level_off(j - 1, N);
      const int Tm = tri_of(m);
      const T inv = (T)(1.0 / (m + 1));
      for (int v = lane; v < EPW * 8 * Tm; v += 64) {
        const int el = v / (8 * Tm);
        const int rem = v - el * 8 * Tm;
        const int vec = rem / Tm;
        const int s = rem - vec * Tm;
        // position out0 + s of the face-layered vector = volume node out0 + s seen from face 3
        const int nn = out0 + s;
        const int b0 = tab[L.alpha + 4 * nn + 0];
        const int b1 = tab[L.alpha + 4 * nn + 1];
        const int b2 = tab[L.alpha + 4 * nn + 2];
        const T* w = slev[el][vec];
        const int i0 = in0 + tri_row(b2, m + 1) + b1;       // b + e0
        const int i2 = in0 + tri_row(b2 + 1, m + 1) + b1;   // b + e2
        const T acc = (T)(b0 + 1) * w[i0] + (T)(b1 + 1) * w[i0 + 1] + (T)(b2 + 1) * w[i2];
        slev[el][vec][nn] = acc * inv;
      }
      __syncthreads();
    }
  }

  // ---- 5./6. per node: volume term, lift gather, update --------------------
#pragma unroll
  for (int r = 0; r < NPL; ++r) {
    const int v = lane + 64 * r;
    if (v >= EPW * Np) continue;
    const int el = v / Np;
    const int n = v - el * Np;
    const int64_t e = e0 + el;
    if (e >= K) continue;
    const double* ge = A.geo + e * kGeoStride;
    T gl[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int d = 0; d < 3; ++d) gl[i][d] = (T)ge[3 * i + d];
    const T kap = (T)(ge[9] * ge[9]);
    int a[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = tab[L.alpha + 4 * n + i];

    T rhs[4] = {0, 0, 0, 0};
    if constexpr (kVol) {
      int nb[12];
#pragma unroll
      for (int p = 0; p < 12; ++p) nb[p] = tab[L.vnbr + 12 * n + p];
      // pair index of (a, b): 3a + (b < a ? b : b - 1)
      auto P = [&](int ai, int bi) { return nb[3 * ai + (bi < ai ? bi : bi - 1)]; };
      T grad[4][3];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const T fc = sq[el][n][f];
        T dl[3];
#pragma unroll
        for (int i = 1; i <= 3; ++i) {
          T d = (T)a[0] * (sq[el][P(i, 0)][f] - fc) + (T)a[i] * (fc - sq[el][P(0, i)][f]);
#pragma unroll
          for (int m = 1; m <= 3; ++m) {
            if (m == i) continue;
            d += (T)a[m] * (sq[el][P(i, m)][f] - sq[el][P(0, m)][f]);
          }
          dl[i - 1] = d;
        }
#pragma unroll
        for (int dd = 0; dd < 3; ++dd) grad[f][dd] = gl[0][dd] * dl[0] + gl[1][dd] * dl[1] + gl[2][dd] * dl[2];
      }
      rhs[0] = -kap * (grad[1][0] + grad[2][1] + grad[3][2]);
      rhs[1] = -grad[0][0];
      rhs[2] = -grad[0][1];
      rhs[3] = -grad[0][2];
    }
    if constexpr (kSurf) {
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        T gx, gy, gz;
        if (f == 0) {
          gx = (T)2 * (gl[0][0] + gl[1][0] + gl[2][0]);
          gy = (T)2 * (gl[0][1] + gl[1][1] + gl[2][1]);
          gz = (T)2 * (gl[0][2] + gl[1][2] + gl[2][2]);
        } else {
          gx = (T)(-2) * gl[f - 1][0];
          gy = (T)(-2) * gl[f - 1][1];
          gz = (T)(-2) * gl[f - 1][2];
        }
        const int pos = tab[L.proj + 4 * n + f];
        const T ell = (T)ell_of<N>(a[f]);
        const T lp = ell * slev[el][f][pos];
        const T lu = ell * slev[el][4 + f][pos];
        rhs[0] += lp;
        rhs[1] += gx * lu;
        rhs[2] += gy * lu;
        rhs[3] += gz * lu;
      }
    }

    const int64_t off = e * Np + n;
    if constexpr (MODE == kStage) {
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        T rs = A.dt * rhs[f];
        if (A.read_res) rs += A.rk_a * A.res[f * KNp + off];
        A.res[f * KNp + off] = rs;
        A.qout[f * KNp + off] = qv[r][f] + A.rk_b * rs;
      }
    } else {
#pragma unroll
      for (int f = 0; f < 4; ++f) A.qout[f * KNp + off] = rhs[f];
    }
  }
}

template <int N, typename T, int MODE>
static hipError_t launch_one(const StageArgs<T>& a, hipStream_t stream) {
  constexpr int Np = np_of(N);
  constexpr int EPW = (Np <= 32) ? (64 / Np) : 1;
  const int64_t groups = (a.K + EPW - 1) / EPW;
  if (groups <= 0) return hipSuccess;
  if (groups > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((bb_stage_kernel<N, T, MODE>), dim3((unsigned)groups), dim3(64), 0, stream, a);
  return hipGetLastError();
}

template <typename T, int MODE>
static hipError_t launch_mode(int N, const StageArgs<T>& a, hipStream_t stream) {
  switch (N) {
    case 1: return launch_one<1, T, MODE>(a, stream);
    case 2: return launch_one<2, T, MODE>(a, stream);
    case 3: return launch_one<3, T, MODE>(a, stream);
    case 4: return launch_one<4, T, MODE>(a, stream);
    case 5: return launch_one<5, T, MODE>(a, stream);
    case 6: return launch_one<6, T, MODE>(a, stream);
    case 7: return launch_one<7, T, MODE>(a, stream);
    case 8: return launch_one<8, T, MODE>(a, stream);
    case 9: return launch_one<9, T, MODE>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_stage(int N, int mode, const StageArgs<T>& a, hipStream_t stream) {
  switch (mode) {
    case kStage: return launch_mode<T, kStage>(N, a, stream);
    case kRhsFull: return launch_mode<T, kRhsFull>(N, a, stream);
    case kRhsVolume: return launch_mode<T, kRhsVolume>(N, a, stream);
    case kRhsSurface: return launch_mode<T, kRhsSurface>(N, a, stream);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_stage<double>(int, int, const StageArgs<double>&, hipStream_t);
template hipError_t launch_stage<float>(int, int, const StageArgs<float>&, hipStream_t);

}  // namespace bbdg
