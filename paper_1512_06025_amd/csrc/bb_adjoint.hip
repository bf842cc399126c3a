// Discrete adjoint of the Bernstein-Bezier DG stage (gfx950, wave64).
//
// The forward stage is res <- a_s res + dt (A(m) q + f), q <- q + b_s res.
// Its reverse, with qb and rb the adjoints of q and res, is
//   u = rb + b_s qb,  qb <- qb + dt A^T u,  rb <- a_s u,
//   grad_m += dt u^T d(A q + f)/dm        (q, f: the forward stage's input).
// A^T is applied with the transposes of the kernels of the forward stage:
//   volume: (D^{iT} x)(beta) = beta_i x(beta) + sum_{j != i} (beta_j+1) x(beta - e_i + e_j)
//           (the transpose of the row form of Lemma 1 / Appendix A.1; the
//           term is absent when beta_i = 0), with the chain rule transposed;
//   surface: L^{fT} = L_0 (E_L^f)^T (Section 3.1.2; L_0 is symmetric).  The
//           transpose of the one-degree reductions is degree raising,
//           (E y)(b) = sum_k b_k/m y(b - e_k), so (E_L^f)^T x is evaluated by
//           Horner's rule over the layers x_j = ell_j x|_{alpha_f = j}:
//           y = x_N, y <- x_j + E y for j = N-1..0.  The result on the face
//           nodes goes through the transposed upwind flux of Section 2 to the
//           own traces and, through z_out, to the neighbours' traces, which
//           each element pulls from z_in at the start of the next reverse
//           stage (a face's two sides are updated by their own waves, with
//           no atomics).
// Gradient with respect to m_k = kappa_k = c_k^2: the pressure equation of
// element k (with the source) is proportional to kappa_k at fixed taus, so
// that part is u_p . P / kappa_k with P the recorded pressure right-hand
// side; tau_p and tau_u of a face depend on s = c_k + c_+, and
// d/ds of the face flux, contracted with the face adjoint, goes to gt and is
// split between the two elements of the face by launch_gradient_finalize.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "bb_common.hpp"
#include "bb_launch.hpp"

namespace bbdg {

namespace {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A double moved between lanes by a DPP lane pattern (two 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(v & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over each row of 16 lanes, left in every lane of the row: pairs and
// quads (quad_perm [1,0,3,2], [2,3,0,1]), then half rows (row_half_mirror)
// and rows (row_mirror).  Vector instructions only, no LDS round trip.
__device__ __forceinline__ double row_sum16(double t) {
  t += dpp_f64<0xB1>(t);
  t += dpp_f64<0x4E>(t);
  t += dpp_f64<0x141>(t);
  t += dpp_f64<0x140>(t);
  return t;
}

__device__ __forceinline__ double lane_f64(double x, int l) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// position stride of the lift items: the next power of two when that costs
// no extra pass over the 64 lanes (decoding then needs shifts only)
__host__ __device__ constexpr int a_pow2ceil(int x) {
  int p = 1;
  while (p < x) p *= 2;
  return p;
}
__host__ __device__ constexpr int a_item_stride(int cnt, int groups) {
  return (groups * a_pow2ceil(cnt) + 63) / 64 == (groups * cnt + 63) / 64 ? a_pow2ceil(cnt) : cnt;
}

template <int N, typename T>
struct AShape {
  static constexpr int Np = np_of(N);
  static constexpr int Nfp = nfp_of(N);
  static constexpr int E = (Np <= 32) ? (64 / Np) : 1;
  static constexpr int NPL = (E * Np + 63) / 64;
  // face items (element, face, position) over the 64 lanes, positions strided
  // by SF (a power of two where that costs no extra pass)
  static constexpr int SF = a_item_stride(Nfp, E * 4);
  static constexpr int NFI = (E * 4 * SF + 63) / 64;
  static constexpr int FB = sizeof(T) == 8 ? (N >= 8 ? 1 : (N >= 6 ? 2 : 4)) : (N >= 8 ? 2 : 4);

  static constexpr int WPB = (N >= 8) ? 2 : 4;
  static constexpr int NHE = (E * 4 + 63) / 64;
  // per element geometry (T): grad lambda_0..3 (12), kappa; per face f at
  // 16 + FS f: g (3), a_p, a_u, b_u, |g|, 1/|g|, -a_p/s (the reciprocals
  // are taken once per face, not per face node)
  static constexpr int FS = 12;
  static constexpr int GEO = 16 + 4 * FS;
};

template <typename T>
struct alignas(2 * sizeof(T)) APair {
  T p, u;
};

// occupancy target (waves per SIMD) bounding the register allocation
template <int N, typename T>
struct AOcc {
  static constexpr int f64[10] = {0, 2, 3, 3, 4, 4, 3, 3, 2, 2};
  static constexpr int f32[10] = {0, 3, 3, 4, 6, 6, 4, 4, 3, 3};
  static constexpr int value = sizeof(T) == 8 ? f64[N] : f32[N];
};

template <int N>
struct AEll {
  static constexpr double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
  }
  static constexpr double value(int j) { return ((j & 1) ? -1.0 : 1.0) * binom(N, j) / (1.0 + j); }
};

// One group's header (per-element geometry, connectivity) held across the
// previous group's work: lane v keeps header word v.
// FP32 groups carry the derived geometry (float, computed once on the host);
// FP64 groups the double header, from which the kernel derives it.
template <int N, typename T>
struct AHeader {
  static constexpr bool kTG = sizeof(T) == 4;
  static constexpr int GS = kTG ? kAGeoStride : kGeoStride;  // header words per element
  static constexpr int NG = (AShape<N, T>::E * GS + 63) / 64;
  typename std::conditional<kTG, T, double>::type geo[NG];
  int32_t etoe[AShape<N, T>::NHE];
  uint32_t fo[AShape<N, T>::NHE];
  int32_t rf[AShape<N, T>::NHE];  // face numbers of the stage records
};

template <int N, typename T>
__device__ __forceinline__ void load_aheader(AHeader<N, T>& h, const AdjointArgs<T>& A, int64_t e0, int lane) {
  using S = AShape<N, T>;
  using H = AHeader<N, T>;
#pragma unroll
  for (int r = 0; r < H::NG; ++r) {
    const int v = lane + 64 * r;
    int64_t idx = e0 * H::GS + v;
    if (v >= S::E * H::GS || idx >= A.K * H::GS) idx = 0;
    if constexpr (H::kTG) {
      h.geo[r] = A.ageo[idx];
    } else {
      h.geo[r] = A.geo[idx];
    }
  }
#pragma unroll
  for (int r = 0; r < S::NHE; ++r) {
    const int v = lane + 64 * r;
    int64_t idx = e0 * 4 + v;
    if (v >= S::E * 4 || idx >= A.K * 4) idx = 0;
    h.etoe[r] = A.etoe[idx];
    h.fo[r] = A.etofo[idx];
    h.rf[r] = A.rec_face[idx];
  }
}

}  // namespace

template <int N, typename T>
__global__ __launch_bounds__((64 * AShape<N, T>::WPB)) __attribute__((amdgpu_waves_per_eu(AOcc<N, T>::value)))
void bb_adjoint_kernel(AdjointArgs<T> A) {
  using S = AShape<N, T>;
  constexpr int Np = S::Np, Nfp = S::Nfp, E = S::E, NPL = S::NPL, NFI = S::NFI;
  constexpr int FB = S::FB, WPB = S::WPB, GEO = S::GEO, FS = S::FS;
  constexpr TabLayout L = tab_layout(N);
  // Per-element gradient sums (FP64) with one element per wave: row sums by
  // DPP lane permutes, vector instructions only (measured faster in FP32
  // than one lane adding the values serially, and in FP64 than butterflies
  // through LDS permutes); several elements per wave add serially.
  constexpr bool kShuffleSums = E == 1;

  __shared__ uint16_t t_fnode[4 * Nfp];
  __shared__ uint16_t t_fperm[6 * Nfp];
  __shared__ uint32_t t_alpha[Np];
  __shared__ uint16_t t_vnbr[Np][12];
  __shared__ uint16_t t_proj[Np][4];
  __shared__ T t_ell[N + 1];
  __shared__ uint8_t t_l0p[Nfp][8];
  __shared__ T t_l0c[7][Nfp];
  // degree raising into layer position nn (layers of the face-3 view):
  // sources in the next layer and weights b_k / m
  __shared__ uint16_t t_rsp[Np][3];
  __shared__ T t_rsc[3][Np];

  __shared__ T su[WPB][E][1][Np];       // u_p of u = rb + b_s qb (the velocity enters through sh)
  __shared__ T sh[WPB][E][4][Np];       // h_i = grad(lambda_i) . u_vel
  __shared__ APair<T> slev[WPB][E][FB][Np];  // layered face vectors (p, velocity) pairs
  __shared__ APair<T> sfl[WPB][E][FB][Nfp];  // L^{fT} results on the face nodes
  __shared__ T sface[WPB][E][4][3][Nfp];  // per-face node contributions (p, u, tau term)
  __shared__ double sred[WPB][E][5];    // gradient partial sums
  __shared__ T sgeo[WPB][E][GEO];
  using H = AHeader<N, T>;
  static_assert(!H::kTG || GEO == kAGeoStride, "sgeo holds the derived geometry layout");
  __shared__ double shg[H::kTG ? 1 : WPB][H::kTG ? 1 : E * kGeoStride];  // FP64 header staging
  __shared__ int32_t she[WPB][E * 4];
  __shared__ uint8_t shf[WPB][E * 4];
  __shared__ int32_t shr[WPB][E * 4];

  const int tid = threadIdx.x;
  for (int i = tid; i < 4 * Nfp; i += 64 * WPB) t_fnode[i] = A.tab[L.fnode + i];
  for (int i = tid; i < 6 * Nfp; i += 64 * WPB) t_fperm[i] = A.tab[L.fperm + i];
  for (int i = tid; i < Np; i += 64 * WPB) {
    const uint16_t* a = A.tab + L.alpha + 4 * i;
    t_alpha[i] = (uint32_t)a[0] | ((uint32_t)a[1] << 8) | ((uint32_t)a[2] << 16) | ((uint32_t)a[3] << 24);
    for (int p = 0; p < 12; ++p) t_vnbr[i][p] = A.tab[L.vnbr + 12 * i + p];
    for (int f = 0; f < 4; ++f) t_proj[i][f] = A.tab[L.proj + 4 * i + f];
  }
  if (tid <= N) {
    double e = 0.0;
    for (int j = 0; j <= N; ++j) e = (tid == j) ? AEll<N>::value(j) : e;
    t_ell[tid] = (T)e;
  }
  __syncthreads();
  for (int gg = tid; gg < Nfp; gg += 64 * WPB) {
    const uint32_t ap = t_alpha[gg];
    const int b0 = ap & 255, b1 = (ap >> 8) & 255, b2 = (ap >> 16) & 255;
    const int row = tri_row(b2, N);
    const int rdn = b2 >= 1 ? tri_row(b2 - 1, N) : 0;
    const int rup = tri_row(b2 + 1, N);
    const int pos[6] = {row + b1 - 1, rup + b1 - 1, rdn + b1, rdn + b1 + 1, row + b1 + 1, rup + b1};
    const int cw[6] = {(b0 + 1) * b1, (b2 + 1) * b1, (b0 + 1) * b2, (b1 + 1) * b2, (b1 + 1) * b0, (b2 + 1) * b0};
    t_l0p[gg][0] = (uint8_t)gg;
    t_l0c[0][gg] = (T)(0.5 * ((b0 + 1) * (b0 + 1) + (b1 + 1) * (b1 + 1) + (b2 + 1) * (b2 + 1)));
    for (int q = 0; q < 6; ++q) {
      t_l0p[gg][1 + q] = (uint8_t)(cw[q] ? pos[q] : gg);
      t_l0c[1 + q][gg] = (T)(0.5 * cw[q]);
    }
    t_l0p[gg][7] = (uint8_t)gg;
  }
  for (int nn = tid; nn < Np; nn += 64 * WPB) {
    // position nn = layer j = alpha_3 of volume node nn, face-local (b0,b1,b2),
    // |b| = m = N - j; sources b - e_k in layer j + 1 (degree m - 1)
    const uint32_t ap = t_alpha[nn];
    const int b0 = ap & 255, b1 = (ap >> 8) & 255, b2 = (ap >> 16) & 255, j = ap >> 24;
    const int m = N - j;
    if (m == 0) {
      for (int k = 0; k < 3; ++k) {
        t_rsp[nn][k] = (uint16_t)nn;
        t_rsc[k][nn] = (T)0;
      }
      continue;
    }
    const int in0 = level_off(j + 1, N);
    t_rsp[nn][0] = (uint16_t)(b0 >= 1 ? in0 + tri_row(b2, m - 1) + b1 : nn);
    t_rsp[nn][1] = (uint16_t)(b1 >= 1 ? in0 + tri_row(b2, m - 1) + b1 - 1 : nn);
    t_rsp[nn][2] = (uint16_t)(b2 >= 1 ? in0 + tri_row(b2 - 1, m - 1) + b1 : nn);
    t_rsc[0][nn] = (T)((double)b0 / m);
    t_rsc[1][nn] = (T)((double)b1 / m);
    t_rsc[2][nn] = (T)((double)b2 / m);
  }
  __syncthreads();

  const int lane0 = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  // face item r of lane ln: element el, face f, position gg (false: none)
  auto face_item = [&](int ln, int r, int& el, int& f, int& gg) -> bool {
    const unsigned v = (unsigned)ln + 64u * (unsigned)r;
    const unsigned q = v / S::SF;  // el * 4 + f
    gg = (int)(v % S::SF);
    f = (int)(q & 3);
    el = (int)(q >> 2);
    return el < E && gg < Nfp;
  };
  const int64_t K = A.K;
  const int64_t KNp = K * Np;
  const int64_t G = (K + E - 1) / E;
  const int64_t GS = G * A.shots;
  const int xcd = blockIdx.x & 7;
  const int64_t g_lo = GS * xcd / 8, g_hi = GS * (xcd + 1) / 8;
  const int64_t wstride = (int64_t)(gridDim.x >> 3) * WPB;
  const T a_s = A.a_s, b_s = A.b_s, dt = A.dt;

  int64_t g = g_lo + (int64_t)(blockIdx.x >> 3) * WPB + w;
  AHeader<N, T> hd;
  if (g < g_hi) load_aheader<N, T>(hd, A, (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)g % (uint32_t)G) * E, lane0);

  for (; g < g_hi; g += wstride) {
    // lane-derived addresses are recomputed per group rather than hoisted
    // out of the loop (where they would hold registers for its whole life)
    int lane = lane0;
    asm volatile("" : "+v"(lane));
    const int64_t shot = (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)g / (uint32_t)G);
    const int64_t e0 = (g - shot * G) * E;
    const int64_t sb = shot * 4 * KNp;
    const int64_t zb = shot * K * 8 * Nfp;
    // this shot's arrays (uniform bases; in-shot offsets fit in 32 bits:
    // 4 K Np < 2^31 and 8 K Nfp < 2^32 for every order)
    T* const qb_s = A.qb + sb;
    T* const rb_s = A.rb + sb;
    const T* const recp_s = A.rec_p + shot * KNp;
    const T* const recj_s = A.rec_j + shot * A.nfaces * (2 * Nfp);
    const T* const zin_s = A.z_in + zb;
    T* const zout_s = A.z_out + zb;

    // ---- header of this group -> LDS; prefetch the next one -----------------------
    wave_sync();
#pragma unroll
    for (int r = 0; r < H::NG; ++r) {
      const int v = lane + 64 * r;
      if (v < E * H::GS) {
        if constexpr (H::kTG) {
          (&sgeo[w][0][0])[v] = hd.geo[r];
        } else {
          shg[H::kTG ? 0 : w][v] = hd.geo[r];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < S::NHE; ++r) {
      const int v = lane + 64 * r;
      if (v < E * 4) {
        she[w][v] = e0 + v / 4 < K ? hd.etoe[r] : -1;
        shf[w][v] = (uint8_t)hd.fo[r];
        shr[w][v] = hd.rf[r];
      }
    }
    wave_sync();
    // the group's loads are issued at raised wave priority (ahead of waves
    // busy with arithmetic), back to normal once they are all in flight
    __builtin_amdgcn_s_setprio(3);
    if (g + wstride < g_hi)
      load_aheader<N, T>(hd, A, (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)(g + wstride) % (uint32_t)G) * E, lane);

    // ---- issue every load of this group together --------------------------------
    // own adjoint state and recorded pressure right-hand side
    // (element-major fields: field f of node n of element e at e 4 Np + f Np + n)
    T qv[NPL][4], uv[NPL][4], pv[NPL];
    uint32_t noff[NPL];
#pragma unroll
    for (int r = 0; r < NPL; ++r) {
      const int v = lane + 64 * r;
      const int el = E == 1 ? 0 : v / Np;
      const int n = v - el * Np;
      const bool ok = (v < E * Np) && (e0 + el < K);
      // (lanes without a node read element 0 of the shot and discard it)
      noff[r] = ok ? (uint32_t)((e0 + el) * 4 * Np + n) : 0u;
      const T* qp = qb_s + noff[r];
      const T* up = rb_s + noff[r];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const T x = qp[f * Np], y = up[f * Np];
        qv[r][f] = ok ? x : (T)0;
        uv[r][f] = ok ? y : (T)0;
      }
      const T pr = recp_s[ok ? (uint32_t)((e0 + el) * Np + n) : 0u];
      pv[r] = ok ? pr : (T)0;
    }
    // per face item: the neighbour's face adjoint (pull) and the recorded jumps
    T zq[NFI][2], rjv[NFI][2];
#pragma unroll
    for (int r = 0; r < NFI; ++r) {
      zq[r][0] = zq[r][1] = rjv[r][0] = rjv[r][1] = 0;
      int el, f, gg;
      if (!face_item(lane, r, el, f, gg)) continue;
      const int64_t k = e0 + el;
      if (k >= K) continue;
      const int nb = she[w][el * 4 + f];
      const int info = shf[w][el * 4 + f];
      const int g2 = t_fperm[(info >> 2) * Nfp + gg];  // this node on the neighbour's face
      // the face's record, stored by the element with the lower index (or the
      // only one) on its own face nodes: [[p]] changes sign across the face,
      // the unit-normal velocity jump does not
      const bool own = nb < 0 || k <= nb;
      const T* rj = recj_s + ((uint32_t)shr[w][el * 4 + f] * (2 * Nfp) + (own ? gg : g2));
      const T jr = rj[0];
      rjv[r][0] = own ? jr : -jr;
      rjv[r][1] = rj[Nfp];
      if (A.pull && nb >= 0) {
        const T* zs = zin_s + (((uint32_t)nb * 4 + (info & 3)) * (2 * Nfp) + g2);
        zq[r][0] = zs[0];
        zq[r][1] = zs[Nfp];
      }
    }
    // gradient sums of this group (read-modify-write at the end)
    constexpr int NG = (E * 5 + 63) / 64;
    double gold[NG];
#pragma unroll
    for (int r = 0; r < NG; ++r) {
      const int v = lane + 64 * r;
      gold[r] = 0.0;
      if (v < E * 5 && e0 + v / 5 < K) {
        const int el = v / 5, c = v - 5 * el;
        gold[r] = c == 0 ? A.gk[shot * K + e0 + el] : A.gt[(shot * K + e0 + el) * 4 + c - 1];
      }
    }
    __builtin_amdgcn_s_setprio(0);

    // ---- geometry (FP64; FP32 groups loaded it with the header; the elements of
    // a ragged tail then hold element 0's, and nothing of theirs is stored) ----
    for (int v = lane; !H::kTG && v < E * 4; v += 64) {
      const int el = v >> 2, f = v & 3;
      const int64_t k = e0 + el;
      T* o = sgeo[w][el];
      if (k >= K) {  // ragged tail: neutral geometry, no neighbours
        for (int c = 0; c < 3; ++c) o[3 * f + c] = 0;
        if (f == 0) o[12] = 1;
        for (int c = 0; c < FS; ++c) o[16 + FS * f + c] = 1;
        continue;
      }
      const double* ge = shg[H::kTG ? 0 : w] + el * kGeoStride;
      double gx, gy, gz;
      if (f == 0) {
        gx = -(ge[0] + ge[3] + ge[6]);
        gy = -(ge[1] + ge[4] + ge[7]);
        gz = -(ge[2] + ge[5] + ge[8]);
      } else {
        gx = ge[3 * (f - 1) + 0];
        gy = ge[3 * (f - 1) + 1];
        gz = ge[3 * (f - 1) + 2];
      }
      o[3 * f + 0] = (T)gx;
      o[3 * f + 1] = (T)gy;
      o[3 * f + 2] = (T)gz;
      if (f == 0) o[12] = (T)ge[9];
      const double F = 2.0 * sqrt(gx * gx + gy * gy + gz * gz);
      T* fr = o + 16 + FS * f;
      fr[0] = (T)(-2.0 * gx);
      fr[1] = (T)(-2.0 * gy);
      fr[2] = (T)(-2.0 * gz);
      fr[3] = (T)ge[10 + f];     // a_p = kappa |g| / s
      fr[4] = (T)(0.5 * ge[9]);  // a_u = kappa / 2
      fr[5] = (T)ge[14 + f];     // b_u = s / (4 |g|)
      fr[6] = (T)F;
      fr[7] = (T)(1.0 / F);
      fr[8] = (T)(-ge[10 + f] / (4.0 * F * ge[14 + f]));  // -a_p / s, s = 4 |g| b_u
    }
    wave_sync();


    // ---- neighbour terms of the previous reverse stage -----------------------------
    if (A.pull) {
#pragma unroll
      for (int r = 0; r < NFI; ++r) {
        int el, f, gg;
        if (!face_item(lane, r, el, f, gg)) continue;
        // the neighbour's g is -(|g_nb|/|g_f|) g_f and zu carries |g_nb|:
        // the velocity adjoint gains -(g_f/|g_f|) zu
        sface[w][el][f][0][gg] = zq[r][0];
        sface[w][el][f][1][gg] = -zq[r][1] * sgeo[w][el][16 + FS * f + 7];
      }
      wave_sync();
#pragma unroll
      for (int r = 0; r < NPL; ++r) {
        const int v = lane + 64 * r;
        if (v >= E * Np) continue;
        const int el = E == 1 ? 0 : v / Np;
        const int n = v - el * Np;
        const uint32_t ap = t_alpha[n];
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          if ((ap >> (8 * f)) & 255) continue;
          const int gg = t_proj[n][f];
          const T* fr = sgeo[w][el] + 16 + FS * f;
          const T cp = sface[w][el][f][0][gg], cu = sface[w][el][f][1][gg];
          qv[r][0] += dt * cp;
          qv[r][1] += dt * fr[0] * cu;
          qv[r][2] += dt * fr[1] * cu;
          qv[r][3] += dt * fr[2] * cu;
        }
      }
    }

    // ---- u = rb + b_s qb; h_i = grad(lambda_i) . u_vel ------------------------------
    T kpart[NPL];
#pragma unroll
    for (int r = 0; r < NPL; ++r) {
      const int v = lane + 64 * r;
      kpart[r] = 0;
      if (v >= E * Np) continue;
      const int el = E == 1 ? 0 : v / Np;
      const int n = v - el * Np;
#pragma unroll
      for (int f = 0; f < 4; ++f) uv[r][f] += b_s * qv[r][f];
      su[w][el][0][n] = uv[r][0];
      const T* ge = sgeo[w][el];
#pragma unroll
      for (int i = 0; i < 4; ++i) sh[w][el][i][n] = ge[3 * i] * uv[r][1] + ge[3 * i + 1] * uv[r][2] + ge[3 * i + 2] * uv[r][3];
      kpart[r] = uv[r][0] * pv[r];
    }
    wave_sync();

    // ---- volume: transposed derivatives ---------------------------------------------
    T acc[NPL][4];
#pragma unroll
    for (int r = 0; r < NPL; ++r) {
#pragma unroll
      for (int f = 0; f < 4; ++f) acc[r][f] = 0;
      const int v = lane + 64 * r;
      if (v >= E * Np) continue;
      const int el = E == 1 ? 0 : v / Np;
      const int n = v - el * Np;
      const uint32_t ap = t_alpha[n];
      const int bi[4] = {(int)(ap & 255), (int)((ap >> 8) & 255), (int)((ap >> 16) & 255), (int)(ap >> 24)};
      const T* ge = sgeo[w][el];
      T tp[4], ph = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // (D^{iT} x)(beta) for x = u_p and x = h_i
        T a = (T)bi[i] * su[w][el][0][n];
        T b = (T)bi[i] * sh[w][el][i][n];
        if (bi[i] >= 1) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (j == i) continue;
            const int src = t_vnbr[n][3 * j + (i < j ? i : i - 1)];  // beta + e_j - e_i
            const T c = (T)(bi[j] + 1);
            a += c * su[w][el][0][src];
            b += c * sh[w][el][i][src];
          }
        }
        tp[i] = a;
        ph += b;
      }
      acc[r][0] = -ph;
#pragma unroll
      for (int d = 0; d < 3; ++d)
        acc[r][1 + d] = -ge[12] * (ge[d] * tp[0] + ge[3 + d] * tp[1] + ge[6 + d] * tp[2] + ge[9 + d] * tp[3]);
    }

    // ---- surface: L^{fT} on the face vectors, FB faces at a time ---------------------
    for (int fb0 = 0; fb0 < 4; fb0 += FB) {
      // layers: x_j(position) = ell_j x(alpha) over alpha with alpha_f = j
#pragma unroll
      for (int r = 0; r < NPL; ++r) {
        const int v = lane + 64 * r;
        if (v >= E * Np) continue;
        const int el = E == 1 ? 0 : v / Np;
        const int n = v - el * Np;
        const uint32_t ap = t_alpha[n];
#pragma unroll
        for (int fl = 0; fl < FB; ++fl) {
          const int f = fb0 + fl;
          const T* fr = sgeo[w][el] + 16 + FS * f;
          const T ell = t_ell[(ap >> (8 * f)) & 255];
          const int pos = t_proj[n][f];
          slev[w][el][fl][pos] = APair<T>{ell * uv[r][0], ell * (fr[0] * uv[r][1] + fr[1] * uv[r][2] + fr[2] * uv[r][3])};
        }
      }
      wave_sync();
      // Horner over the layers: y_j = x_j + E y_{j+1}, j = N-1 .. 0
      for (int j = N - 1; j >= 0; --j) {
        const int out0 = level_off(j, N);
        const int Tm = tri_of(N - j);
        const unsigned SM = a_item_stride(Tm, E * FB);
        for (unsigned v = lane; v < E * FB * SM; v += 64) {
          const unsigned s = v % SM;
          const unsigned rest = v / SM;  // = el * FB + face in the batch
          if (s >= (unsigned)Tm) continue;
          const unsigned nn = out0 + s;
          APair<T>* wv = &slev[w][0][0][0] + rest * Np;
          const T c0 = t_rsc[0][nn], c1 = t_rsc[1][nn], c2 = t_rsc[2][nn];
          const APair<T> x0 = wv[t_rsp[nn][0]], x1 = wv[t_rsp[nn][1]], x2 = wv[t_rsp[nn][2]];
          const APair<T> y = wv[nn];
          wv[nn] = APair<T>{y.p + c0 * x0.p + c1 * x1.p + c2 * x2.p, y.u + c0 * x0.u + c1 * x1.u + c2 * x2.u};
        }
        wave_sync();
      }
      // z = L_0 y_0 (L_0 symmetric)
      constexpr unsigned SL0 = a_item_stride(Nfp, E * FB);
      for (unsigned v = lane; v < E * FB * SL0; v += 64) {
        const unsigned gg = v % SL0;
        const unsigned rest = v / SL0;
        if (gg >= (unsigned)Nfp) continue;
        const APair<T>* sv = &slev[w][0][0][0] + rest * Np;
        T zp = 0, zu = 0;
#pragma unroll
        for (int q = 0; q < 7; ++q) {
          const T c = t_l0c[q][gg];
          const APair<T> x = sv[t_l0p[gg][q]];
          zp += c * x.p;
          zu += c * x.u;
        }
        (&sfl[w][0][0][0])[rest * Nfp + gg] = APair<T>{zp, zu};
      }
      wave_sync();
      // transposed flux on the face nodes of this batch
#pragma unroll
      for (int r = 0; r < NFI; ++r) {
        int el, f, gg;
        if (!face_item(lane, r, el, f, gg) || f < fb0 || f >= fb0 + FB) continue;
        const int64_t k = e0 + el;
        T dp = 0, du = 0, tau = 0;
        if (k < K) {
          const T* fr = sgeo[w][el] + 16 + FS * f;
          const APair<T> zz = sfl[w][el][f - fb0][gg];
          const T zp = zz.p, zu = zz.u;
          // sp = a_p [[p]] - a_u g.[[u]],  su = b_u g.[[u]] - [[p]]/2
          const T jbp = fr[3] * zp - (T)0.5 * zu;
          const T jbg = fr[5] * zu - fr[4] * zp;
          T* zo = zout_s + (((uint32_t)k * 4 + f) * (2 * Nfp) + gg);
          zo[0] = jbp;
          zo[Nfp] = fr[6] * jbg;
          const int nb = she[w][el * 4 + f];
          if (nb >= 0) {
            dp = -jbp;
            du = -jbg;
          } else if (A.bc == 0) {
            du = (T)(-2) * jbg;
          } else {
            dp = (T)(-2) * jbp;
          }
          // d/ds of the flux at fixed jumps: -a_p/s [[p]] and g.[[u]]/(4|g|), s = 4 |g| b_u
          // (the record holds g.[[u]] / |g|)
          tau = zp * fr[8] * rjv[r][0] + zu * rjv[r][1] * (T)0.25;
        }
        sface[w][el][f][0][gg] = dp;
        sface[w][el][f][1][gg] = du;
        sface[w][el][f][2][gg] = tau;
      }
      wave_sync();
      if constexpr (!kShuffleSums) {
        for (int v = lane; v < E * FB; v += 64) {
          const int el = v / FB, fl = v - el * FB;
          double t = 0.0;
          for (int gg = 0; gg < Nfp; ++gg) t += (double)sface[w][el][fb0 + fl][2][gg];
          sred[w][el][1 + fb0 + fl] = t;
        }
        wave_sync();
      }
    }
    if constexpr (kShuffleSums) {
      // tau terms of the four faces (kept in sface by every batch): one row
      // of 16 lanes per face
      const int f = lane >> 4, j = lane & 15;
      double t = 0.0;
      for (int gg = j; gg < Nfp; gg += 16) t += (double)sface[w][0][f][2][gg];
      t = row_sum16(t);
      if (j == 0) sred[w][0][1 + f] = t;
    }

    // ---- own face contributions ---------------------------------------------------
#pragma unroll
    for (int r = 0; r < NPL; ++r) {
      const int v = lane + 64 * r;
      if (v >= E * Np) continue;
      const int el = E == 1 ? 0 : v / Np;
      const int n = v - el * Np;
      const uint32_t ap = t_alpha[n];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        if ((ap >> (8 * f)) & 255) continue;
        const int gg = t_proj[n][f];
        const T* fr = sgeo[w][el] + 16 + FS * f;
        const T cp = sface[w][el][f][0][gg], cu = sface[w][el][f][1][gg];
        acc[r][0] += cp;
        acc[r][1] += fr[0] * cu;
        acc[r][2] += fr[1] * cu;
        acc[r][3] += fr[2] * cu;
      }
    }

    // ---- kappa part of the gradient: sum_n u_p P / kappa ------------------------------
    if constexpr (kShuffleSums) {
      double t = 0.0;  // lanes past the element hold zeros
#pragma unroll
      for (int r = 0; r < NPL; ++r) t += (double)kpart[r];
      t = row_sum16(t);
      t = (lane_f64(t, 0) + lane_f64(t, 16)) + (lane_f64(t, 32) + lane_f64(t, 48));
      if (lane == 0) sred[w][0][0] = t;
    } else {
#pragma unroll
      for (int r = 0; r < NPL; ++r) {
        const int v = lane + 64 * r;
        if (v >= E * Np) continue;
        const int el = E == 1 ? 0 : v / Np;
        const int n = v - el * Np;
        su[w][el][0][n] = kpart[r];
      }
      wave_sync();
      for (int el = lane; el < E; el += 64) {
        double t = 0.0;
        for (int n = 0; n < Np; ++n) t += (double)su[w][el][0][n];
        sred[w][el][0] = t;
      }
    }
    wave_sync();
#pragma unroll
    for (int r = 0; r < NG; ++r) {
      const int v = lane + 64 * r;
      if (v >= E * 5 || e0 + v / 5 >= K) continue;
      const int el = v / 5, c = v - 5 * el;
      const int64_t k = e0 + el;
      if (c == 0) {
        A.gk[shot * K + k] = gold[r] + (double)dt * sred[w][el][0] / (double)sgeo[w][el][12];
      } else {
        A.gt[(shot * K + k) * 4 + c - 1] = gold[r] + (double)dt * sred[w][el][c];
      }
    }

    // ---- update ------------------------------------------------------------------------
#pragma unroll
    for (int r = 0; r < NPL; ++r) {
      const int v = lane + 64 * r;
      const int el = E == 1 ? 0 : v / Np;
      if (v >= E * Np || e0 + el >= K) continue;
      T* const qo = qb_s + noff[r];
      T* const ro = rb_s + noff[r];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        qo[f * Np] = qv[r][f] + dt * acc[r][f];
        ro[f * Np] = a_s * uv[r][f];
      }
    }
  }
}

template <int N, typename T>
static hipError_t launch_adjoint_one(const AdjointArgs<T>& a, hipStream_t stream) {
  using S = AShape<N, T>;
  const int64_t groups = (a.K + S::E - 1) / S::E * a.shots;
  if (groups <= 0) return hipSuccess;
  static int resident = 0, cus = 0;
  if (resident == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return hipErrorInvalidDevice;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return hipErrorInvalidDevice;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, bb_adjoint_kernel<N, T>, 64 * S::WPB, 0) != hipSuccess)
      return hipErrorInvalidValue;
    resident = occ > 0 ? occ : 1;
  }
  const int64_t needed = (groups + S::WPB - 1) / S::WPB;
  int64_t grid = (int64_t)resident * cus;
  if (grid > needed) grid = needed;
  grid = ((grid + 7) / 8) * 8;
  (void)hipGetLastError();  // drop errors left by earlier, unrelated calls
  hipLaunchKernelGGL((bb_adjoint_kernel<N, T>), dim3((unsigned)grid), dim3(64 * S::WPB), 0, stream, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_stage(int N, const AdjointArgs<T>& a, hipStream_t stream) {
  switch (N) {
    case 1: return launch_adjoint_one<1, T>(a, stream);
    case 2: return launch_adjoint_one<2, T>(a, stream);
    case 3: return launch_adjoint_one<3, T>(a, stream);
    case 4: return launch_adjoint_one<4, T>(a, stream);
    case 5: return launch_adjoint_one<5, T>(a, stream);
    case 6: return launch_adjoint_one<6, T>(a, stream);
    case 7: return launch_adjoint_one<7, T>(a, stream);
    case 8: return launch_adjoint_one<8, T>(a, stream);
    case 9: return launch_adjoint_one<9, T>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_adjoint_stage<double>(int, const AdjointArgs<double>&, hipStream_t);
template hipError_t launch_adjoint_stage<float>(int, const AdjointArgs<float>&, hipStream_t);

// ---- small kernels around the reverse sweep ---------------------------------------------

// One thread per (shot, receiver, node).  The first receiver of an element
// adds the residuals of every receiver in that element, in receiver order, to
// the element's pressure coefficient: each coefficient has one writer (no
// atomics) and its sum keeps the order of the receivers.
template <typename T>
__global__ void inject_receivers_kernel(int Np, int64_t K, int64_t shots, int R, const int32_t* rec_elem,
                                        const T* rec_coef, const T* traces, const T* obs, T* qb) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= shots * R * Np) return;
  const int64_t sr = t / Np;
  const int n = (int)(t - sr * Np);
  const int64_t s = sr / R;
  const int r = (int)(sr - s * R);
  const int32_t e = rec_elem[r];
  if (e < 0 || e >= K) return;
  for (int r2 = 0; r2 < r; ++r2)
    if (rec_elem[r2] == e) return;  // an earlier receiver of this element adds for it
  T* const p = qb + s * 4 * K * Np + (int64_t)e * 4 * Np + n;  // pressure block of element e, shot s
  T acc = *p;
  for (int r2 = r; r2 < R; ++r2) {
    if (rec_elem[r2] != e) continue;
    const T res = traces[s * R + r2] - obs[s * R + r2];
    acc += res * rec_coef[(int64_t)r2 * Np + n];
  }
  *p = acc;
}

template <typename T>
hipError_t launch_inject_receivers(int Np, int64_t K, int64_t shots, int R, const int32_t* rec_elem,
                                   const T* rec_coef, const T* traces, const T* obs, T* qb, hipStream_t stream) {
  const int64_t n = shots * R * Np;
  if (n <= 0) return hipSuccess;
  (void)hipGetLastError();  // drop errors left by earlier, unrelated calls
  hipLaunchKernelGGL(inject_receivers_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, Np, K,
                     shots, R, rec_elem, rec_coef, traces, obs, qb);
  return hipGetLastError();
}

template hipError_t launch_inject_receivers<double>(int, int64_t, int64_t, int, const int32_t*, const double*,
                                                    const double*, const double*, double*, hipStream_t);
template hipError_t launch_inject_receivers<float>(int, int64_t, int64_t, int, const int32_t*, const float*,
                                                   const float*, const float*, float*, hipStream_t);

template <typename T>
__global__ __launch_bounds__(256) void misfit_kernel(int64_t n, const T* traces, const T* obs, double* J) {
  __shared__ double part[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double d = (double)traces[i] - (double)obs[i];
    s += d * d;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) J[0] = 0.5 * part[0];
}

template <typename T>
hipError_t launch_misfit(int64_t n, const T* traces, const T* obs, double* J, hipStream_t stream) {
  (void)hipGetLastError();  // drop errors left by earlier, unrelated calls
  hipLaunchKernelGGL(misfit_kernel<T>, dim3(1), dim3(256), 0, stream, n, traces, obs, J);
  return hipGetLastError();
}

template hipError_t launch_misfit<double>(int64_t, const double*, const double*, double*, hipStream_t);
template hipError_t launch_misfit<float>(int64_t, const float*, const float*, double*, hipStream_t);

__global__ void gradient_finalize_kernel(int64_t K, int64_t shots, const double* geo, const int32_t* etoe,
                                         const uint8_t* etofo, const double* gk, const double* gt, double* grad) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  const double c = sqrt(geo[k * kGeoStride + 9]);
  double total = 0.0;
  for (int64_t s = 0; s < shots; ++s) {
    double tau = 0.0;
    for (int f = 0; f < 4; ++f) {
      const int32_t nb = etoe[k * 4 + f];
      const double own = gt[(s * K + k) * 4 + f];
      if (nb < 0) {
        tau += 2.0 * own;
      } else {
        tau += own + gt[(s * K + nb) * 4 + (etofo[k * 4 + f] & 3)];
      }
    }
    total += gk[s * K + k] + tau / (2.0 * c);
  }
  grad[k] = total;
}

hipError_t launch_gradient_finalize(int64_t K, int64_t shots, const double* geo, const int32_t* etoe,
                                    const uint8_t* etofo, const double* gk, const double* gt, double* grad,
                                    hipStream_t stream) {
  if (K <= 0) return hipSuccess;
  (void)hipGetLastError();  // drop errors left by earlier, unrelated calls
  hipLaunchKernelGGL(gradient_finalize_kernel, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, stream, K, shots,
                     geo, etoe, etofo, gk, gt, grad);
  return hipGetLastError();
}

}  // namespace bbdg
