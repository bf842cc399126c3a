// Fused Bernstein-Bezier DG stage kernel for gfx950 (wave64).
//
// Work decomposition.  A workgroup holds WPB = 4 independent wavefronts (or,
// for the FP64 orders listed at Shape::TW, one team of TW waves).  Each team
// owns E consecutive elements at a time (E = its threads / Np, at least 1)
// and loops over element groups (persistent grid).  The waves of a
// workgroup share the order's index tables, loaded into LDS once; after that
// a one-wave team only synchronises with itself (LDS operations of a
// wavefront complete in issue order, so an LDS-only fence plus a wave
// barrier orders them while global loads stay in flight).  Consecutive workgroups land on
// different XCDs, so the element range is split into 8 contiguous parts, one
// per XCD, and each XCD's waves stride through their part: neighbouring
// elements are processed by the same XCD at about the same time and their
// face traces hit its L2.
//
// One latency round per element group: the group's connectivity/geometry
// header was prefetched during the previous group; own coefficients, LSRK
// residual and the neighbours' face traces are issued together, and the next
// header is prefetched behind them.
//
// Per element:
//   geometry, once: g_f = Fscale_f n_f = -2 grad(lambda_f), |g_f|, and the flux
//     weights of face f (tau_p = 2/(c+c'), tau_u = (c+c')/2, rho = 1);
//   volume (Algorithm 2, row form of Lemma 1 / Appendix A.1):
//     (D^i f)(alpha) = sum_j alpha_j f[alpha + e_i - e_j],
//     grad f = sum_{i=0..3} grad(lambda_i) D^i f;
//     rhs_p = -kappa div u, rhs_u = -grad p;
//   surface (Section 2 upwind flux, Section 3.1.2 factorisation L^f = E_L^f L_0):
//     on face node g: sp = kappa/2 (tau_p |g_f| [[p]] - g_f.[[u]]),
//                     su = 1/2 (tau_u g_f.[[u]]/|g_f| - [[p]]);
//     w_0 = L_0 s:  L_0[b,b] = 1/2 sum_k (b_k+1)^2, L_0[b, b+e_k-e_m] = 1/2 (b_k+1) b_m
//                   (the entries of ((N+1)^2/2) (E^{N+1}_N)^T E^{N+1}_N);
//     w_j = (E^{N-j+1}_{N-j})^T w_{j-1}, [E^T w](b) = sum_k (b_k+1)/(m+1) w(b+e_k)
//                   (the one-degree reductions of Algorithm 1);
//     rhs_p(alpha) += sum_f ell_{alpha_f} w^f_p,alpha_f(alpha without f),
//     rhs_u(alpha) += sum_f g_f ell_{alpha_f} w^f_u,alpha_f(alpha without f),
//     ell_j = (-1)^j C(N,j)/(1+j).
//   The rows of L_0 and of the reductions are spread over (vector, position)
//   pairs, vector = lane mod 2*FB; their coefficients and input positions come
//   from descriptor tables built in LDS once per workgroup.
//   LSRK4 update (fused): res = a res + dt rhs, q_out = q + b res.
// Fields ping-pong between q_in and q_out, so no stage overwrites a trace
// that another wave still reads.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "bb_common.hpp"
#include "bb_launch.hpp"

namespace bbdg {

// The two lifted vectors of a face (pressure flux, velocity flux) share every
// index and weight of L_0 and of the reductions, so they are stored and
// processed as one pair per position.
template <typename T>
struct alignas(2 * sizeof(T)) Pair {
  T p, u;
};

template <int N, typename T>
struct Shape {
  static constexpr int Np = np_of(N);
  static constexpr int Nfp = nfp_of(N);
  // waves that share one element group (the whole workgroup when > 1;
  // batched launches form such teams only with TW waves per workgroup)
  // (measured: teams pay off where one wave per group needs more than half
  // the register file, N >= 8 in FP64, or where they fill the lanes: three
  // waves at N = 8 leave 27 of 192 threads idle instead of 91 of 256; four
  // waves hold seven elements at N = 4, 245 of 256 nodes, where one wave
  // per element fills 35 of 64, and three at N = 6, 252 of 256 nodes, where
  // one wave fills 84 of 128)
  static constexpr int TW = (N == 4 || N == 6) ? 4 : (sizeof(T) == 8 ? (N >= 9 ? 4 : (N == 8 ? 3 : 1)) : 1);
  // faces per lift batch (bounds the LDS of the face vectors), for one-wave
  // teams and for workgroup teams (measured, 196,608 tets: all four faces in
  // one batch of a workgroup team instead of two batches of two save a
  // round of flux, L_0 and reduction barriers, 8 % at N = 8 and 4 % at N = 4
  // in FP64, although at N = 6 and 9 the larger LDS costs one workgroup per
  // CU and the two balance)
  static constexpr int FB1 = sizeof(T) == 8 ? (N >= 8 ? 1 : (N >= 6 ? 2 : 4)) : (N >= 8 ? 2 : 4);
  static constexpr int FBT = 4;
  // per-element derived geometry (type T): grad lambda_0..3 (12), kappa, pad,
  // then per face f at 16 + 6 f: g_x, g_y, g_z, a_p, a_u, b_u with
  //   sp = a_p [[p]] - a_u g.[[u]],  su = b_u g.[[u]] - [[p]]/2.
  static constexpr int GEO = 40;
  // register-lean variant for high orders: the LSRK residual is loaded after
  // the volume term and the own coefficients are re-read from LDS at the update
  static constexpr bool LATE_RES = sizeof(T) == 8 ? (N >= 6) : (N >= 8);
};

// Items (element, face, position < cnt) of the lift loops are laid out with a
// position stride of the next power of two when that costs no extra pass over
// the team's threads, so that decoding an item needs shifts, not divisions.
__host__ __device__ constexpr int pow2ceil(int x) {
  int p = 1;
  while (p < x) p *= 2;
  return p;
}
__host__ __device__ constexpr int item_stride(int cnt, int groups, int tpe) {
  return (groups * pow2ceil(cnt) + tpe - 1) / tpe == (groups * cnt + tpe - 1) / tpe ? pow2ceil(cnt) : cnt;
}

// Per-thread counts for a team of TW waves (TPE threads) working on one group.
template <int N, typename T, int TW>
struct Team {
  using S = Shape<N, T>;
  static constexpr int TPE = 64 * TW;
  // FP32 one-wave groups at N = 5 hold two elements interleaved: lane n takes
  // node n (and face item n) of both, so every index table of a node or a
  // face item is read and decoded once for the two elements.
  static constexpr bool IL = sizeof(T) == 4 && N == 5 && TW == 1;
  static constexpr int E = IL ? 2 : (TPE / S::Np > 1 ? TPE / S::Np : 1);  // elements per group
  static constexpr int NPL = IL ? E : (E * S::Np + TPE - 1) / TPE;         // nodes per thread
  static constexpr int SF = IL ? item_stride(S::Nfp, 4, 64) : item_stride(S::Nfp, E * 4, TPE);  // face-item stride
  static constexpr int NFE = IL ? (4 * SF + 63) / 64 : 1;                  // face-item passes per element
  static constexpr int NFI = IL ? E * NFE : (E * 4 * SF + TPE - 1) / TPE;  // face items per thread
  static constexpr int NHE = (E * 4 + TPE - 1) / TPE;
};

// Synchronisation of the threads that share an element group.  LDS operations
// of a wavefront complete in issue order, so for a one-wave team an LDS-only
// fence plus a wave barrier suffices; larger teams add a workgroup barrier.
// Neither waits for global loads in flight.
template <int TW>
__device__ __forceinline__ void team_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  if constexpr (TW > 1) {
    __builtin_amdgcn_s_barrier();
  } else {
    __builtin_amdgcn_wave_barrier();
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Occupancy target (waves per SIMD) that bounds the register allocation.
template <int N, typename T, int TW, int MODE, int WPB>
struct Occ {
  static constexpr bool kB = MODE >= kBatched;
  static constexpr bool kD = sizeof(T) == 8;
  static constexpr int f64[10] = {0, 2, 3, 4, 4, 4, 3, 3, 2, 2};
  static constexpr int f32[10] = {0, 3, 4, 5, 5, 5, 5, 4, 4, 3};
  // the batched kernel carries more stage state (buffers, coefficients, source)
  static constexpr int f64b[10] = {0, 2, 3, 4, 4, 4, 3, 3, 2, 2};
  static constexpr int f32b[10] = {0, 3, 4, 5, 5, 6, 4, 4, 3, 3};
  static constexpr int base = TW > 1 ? 4 : (kD ? (kB ? f64b[N] : f64[N]) : (kB ? f32b[N] : f32[N]));
  // batched shapes whose registers do not fit the base target (the compiler
  // spilled them to scratch memory) get one level less; a kernel that uses
  // scratch memory is not launched cooperatively (see kernel_residency)
  static constexpr bool kLess =
      kB && ((kD && N == 3 && WPB == 8) || (kD && N == 4 && WPB == 4 && MODE == kBatchedRecord) ||
             (kD && N == 6 && (WPB == 4 || (WPB == 8 && MODE == kBatchedRecord))) ||
             (!kD && N == 5 && MODE == kBatchedRecord) || (!kD && N == 9 && WPB == 4 && MODE == kBatchedRecord));
  static constexpr int value = kLess ? base - 1 : base;
};

template <int N>
struct Ell {
  static constexpr double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
  }
  // ell_j = (-1)^j C(N,j)/(1+j), j = 0..N (Section 3.1.2)
  static constexpr double value(int j) { return ((j & 1) ? -1.0 : 1.0) * binom(N, j) / (1.0 + j); }
};

// Header of an element group in registers (prefetched one group ahead): the
// per-element derived geometry in the element type, computed once on the
// host (kTGeoStride values), or, in FP64 where that larger header would take
// more registers per lane (element groups of 3, 7 or more elements), the
// double header from which the kernel derives it; and the connectivity.
// (Measured on 196,608 tets in FP64: the derived header is 1-2 % faster at
// N = 5..9 and 7 % on the cache-resident 24,576-tet mesh at N = 5, but 2 %
// slower at N = 4, whose seven-element groups need a second register.)
template <int N, typename T, int TW>
struct Header {
  static constexpr int NGT = (Team<N, T, TW>::E * kTGeoStride + Team<N, T, TW>::TPE - 1) / Team<N, T, TW>::TPE;
  static constexpr int NGD = (Team<N, T, TW>::E * kGeoStride + Team<N, T, TW>::TPE - 1) / Team<N, T, TW>::TPE;
  static constexpr bool kTG = sizeof(T) == 4 || NGT == NGD;
  static constexpr int GS = kTG ? kTGeoStride : kGeoStride;  // header words per element
  static constexpr int NG = (Team<N, T, TW>::E * GS + Team<N, T, TW>::TPE - 1) / Team<N, T, TW>::TPE;
  typename std::conditional<kTG, T, double>::type geo[NG];
  int32_t etoe[Team<N, T, TW>::NHE];
  uint32_t fo[Team<N, T, TW>::NHE];
};

template <int N, typename T, int TW>
__device__ __forceinline__ void load_header(Header<N, T, TW>& h, const StageArgs<T>& A, int64_t g, int tl) {
  using M = Team<N, T, TW>;
  using H = Header<N, T, TW>;
  const int64_t e0 = g * M::E;
#pragma unroll
  for (int r = 0; r < H::NG; ++r) {
    const int v = tl + M::TPE * r;
    int64_t idx = e0 * H::GS + v;
    if (v >= M::E * H::GS || idx >= A.K * H::GS) idx = 0;
    if constexpr (H::kTG) {
      h.geo[r] = A.tgeo[idx];
    } else {
      h.geo[r] = A.geo[idx];
    }
  }
#pragma unroll
  for (int r = 0; r < M::NHE; ++r) {
    const int v = tl + M::TPE * r;
    int64_t idx = e0 * 4 + v;
    if (v >= M::E * 4 || idx >= A.K * 4) idx = 0;
    h.etoe[r] = A.etoe[idx];
    h.fo[r] = A.etofo[idx];
  }
}

// Residual loads (read once, by the element itself): non-temporal with NT.
// Element offsets are 32-bit (4 K Np < 2^31 is enforced at create time); the
// byte address is formed in 64 bits, so fields larger than 4 GiB are fine.
template <bool NT, typename T>
__device__ __forceinline__ T ldn(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p); else return *p;
}

// Stores of the stage outputs; NT marks them non-temporal, which pays where
// the fields do not fit in the last-level caches.  (A compile-time choice: a
// run-time branch between the two stores is merged by the compiler into one
// plain store.)
template <bool NT, typename T>
__device__ __forceinline__ void st(T* p, T x) {
  if constexpr (NT) {
    __builtin_nontemporal_store(x, p);
  } else {
    *p = x;
  }
}

// Carpenter-Kennedy (5,4) 2N-storage coefficients (batched runs step inside
// the kernel): res = a_s res + dt rhs(t + c_s dt), q += b_s res.
__constant__ double kLsrkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                                 -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
__constant__ double kLsrkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                                 1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                                 2277821191437.0 / 14882151754819.0};
__constant__ double kLsrkC[5] = {0.0, 1432997174477.0 / 9575080441755.0, 2526269341429.0 / 6820363962896.0,
                                 2006345519317.0 / 3224310063776.0, 2802321613138.0 / 2924317926251.0};

// Grid-wide barrier of a persistent launch, with a bounded wait.
// Workgroup b arrives on the counter of its group b % 8; the last arrival of
// a group arrives on the top counter; the workgroups wait for the top counter
// to reach 8 (stage + 1).  A wait longer than `timeout` ticks of the
// constant-rate wall clock (a grid that is not co-resident) sets the sticky flag;
// every workgroup that finds the flag set leaves the barrier with false and
// ends, so the launch always drains.  One thread per workgroup releases
// (agent scope) after the workgroup barrier and acquires before the second
// one: fences are cumulative, so this covers the stores and loads of every
// wave of the workgroup, and each workgroup writes back and invalidates the
// XCD's L2 once per stage instead of once per wave.  Layout of sync (uint32 words, counters
// on separate 128-byte lines): [32 g] group g, [256] top, [288] flag.
constexpr int kSyncTop = 256, kSyncFlag = kSyncFlagWord;

__device__ __forceinline__ bool grid_barrier(uint32_t* sync, int64_t stage, uint64_t timeout, int* s_ok) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t groups = gridDim.x >> 3;  // workgroups per arrival group (gridDim.x % 8 == 0)
    const uint32_t round = (uint32_t)stage + 1;
    uint32_t* mine = sync + 32 * (blockIdx.x & 7);
    int ok = 1;
    if (__hip_atomic_fetch_add(mine, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 == groups * round) {
      // the group's last arrival passes the group's releases on to the top counter
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      __hip_atomic_fetch_add(sync + kSyncTop, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const int64_t t0 = wall_clock64();
    while (__hip_atomic_load(sync + kSyncTop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < 8 * round) {
      if (__hip_atomic_load(sync + kSyncFlag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
        ok = 0;
        break;
      }
      if ((uint64_t)(wall_clock64() - t0) > timeout) {
        __hip_atomic_store(sync + kSyncFlag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

// Ricker wavelet (1 - 2 pi^2 f0^2 s^2) exp(-pi^2 f0^2 s^2), s = t - tshift.
__device__ __forceinline__ double ricker(double t, double f0, double tshift) {
  const double a = 3.14159265358979323846 * f0 * (t - tshift);
  return (1.0 - 2.0 * a * a) * exp(-a * a);
}

// Waves per element team: batched launches form teams only when the team is
// the whole workgroup.
template <int N, typename T, int MODE, int WPB>
constexpr int team_waves() {
  return (MODE >= kBatched && WPB != Shape<N, T>::TW) ? 1 : Shape<N, T>::TW;
}

template <int N, typename T, int MODE, int WPB, bool NT = false>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(Occ<N, T, team_waves<N, T, MODE, WPB>(), MODE, WPB>::value)))
void bb_stage_kernel(StageArgs<T> A) {
  using S = Shape<N, T>;
  constexpr bool kBatch = (MODE == kBatched || MODE == kBatchedRecord);
  constexpr bool kRecord = (MODE == kBatchedRecord);  // stage record for the adjoint
  constexpr int TW = team_waves<N, T, MODE, WPB>();  // waves per element team
  static_assert(WPB % TW == 0 && (TW == 1 || TW == WPB), "a team is one wave or the whole workgroup");
  using M = Team<N, T, TW>;
  constexpr int TEAMS = WPB / TW, TPE = M::TPE;
  constexpr int Np = S::Np, Nfp = S::Nfp, E = M::E, NPL = M::NPL;
  constexpr int FB = TW > 1 ? S::FBT : S::FB1, GEO = S::GEO;
  constexpr bool kUpdate = (MODE == kStage || kBatch);
  // FP32 up to N = 6 keeps (h_i, p) pairs per node (one 8-byte read per
  // direction, 40-byte node stride free of bank conflicts); otherwise the
  // five values are stored field by field (less LDS)
  // (interleaved groups take the field-by-field layout: the pairs' LDS would
  // cost a workgroup per CU)
  constexpr bool kPairSq = sizeof(T) == 4 && N <= 6 && !M::IL;
  constexpr int SQW = kPairSq ? 10 : 5;  // words per node of sq
  constexpr bool kVol = (MODE != kRhsSurface);
  constexpr bool kSurf = (MODE != kRhsVolume);
  constexpr TabLayout L = tab_layout(N);

  // tables shared by the workgroup
  __shared__ uint16_t t_nbr[24 * Nfp];
  __shared__ uint16_t t_fnode[4 * Nfp];
  __shared__ uint32_t t_alpha[Np];
  __shared__ __attribute__((aligned(16))) uint16_t t_vnbr[Np][12];
  __shared__ __attribute__((aligned(8))) uint16_t t_proj[Np][4];
  __shared__ T t_ell[N + 1];
  // L_0 rows: input positions (diagonal first) and weights; reduction rows:
  // positions of b+e0 (b+e1 follows) and b+e2, and the weights (b_k+1)/(m+1)
  __shared__ __attribute__((aligned(16))) uint8_t t_l0p[Nfp][8];
  __shared__ T t_l0c[7][Nfp];
  __shared__ uint32_t t_lvp[Np];
  __shared__ T t_lvc[3][Np];
  // per-wave buffers
  // the element's coefficients, field-major in double, (p,u,v,w) packed into
  // one 16-byte vector per node in float
  // per node: p and h_i = grad(lambda_i) . u (i = 0..3), see kPairSq
  __shared__ __attribute__((aligned(16))) T sq[TEAMS][E][SQW][Np];
  __shared__ Pair<T> sfl[TEAMS][E][FB][Nfp];
  __shared__ Pair<T> slev[TEAMS][E][FB][Np];
  __shared__ __attribute__((aligned(16))) T sgeo[TEAMS][E][GEO];
  // FP32 groups take the derived geometry (float, computed once on the host)
  // straight into sgeo; FP64 groups stage the double header and derive it.
  // The header staging area is dead once geometry and h_i are derived, so it
  // shares memory with the lift layers when they are large enough.
  using H = Header<N, T, TW>;
  static_assert(!H::kTG || GEO == kTGeoStride, "sgeo holds the derived geometry layout");
  constexpr bool kAliasHg = H::kTG || sizeof(Pair<T>) * FB * Np >= sizeof(double) * kGeoStride;
  __shared__ double shg_own[kAliasHg ? 1 : TEAMS][kAliasHg ? 1 : E * kGeoStride];
  __shared__ int32_t she[TEAMS][E * 4];
  __shared__ uint8_t shf[TEAMS][E * 4];

  const int tid = threadIdx.x;
  for (int i = tid; i < 24 * Nfp; i += 64 * WPB) t_nbr[i] = A.tab[L.nbrnode + i];
  for (int i = tid; i < 4 * Nfp; i += 64 * WPB) t_fnode[i] = A.tab[L.fnode + i];
  for (int i = tid; i < Np; i += 64 * WPB) {
    const uint16_t* a = A.tab + L.alpha + 4 * i;
    t_alpha[i] = (uint32_t)a[0] | ((uint32_t)a[1] << 8) | ((uint32_t)a[2] << 16) | ((uint32_t)a[3] << 24);
#pragma unroll
    for (int p = 0; p < 12; ++p) t_vnbr[i][p] = A.tab[L.vnbr + 12 * i + p];
#pragma unroll
    for (int f = 0; f < 4; ++f) t_proj[i][f] = A.tab[L.proj + 4 * i + f];
  }
  if (tid <= N) {
    double e = 0.0;
#pragma unroll
    for (int j = 0; j <= N; ++j) e = (tid == j) ? Ell<N>::value(j) : e;
    t_ell[tid] = (T)e;
  }
  __syncthreads();
  for (int gg = tid; gg < Nfp; gg += 64 * WPB) {
    const uint32_t ap = t_alpha[gg];  // face-local (b0,b1,b2) = (a0,a1,a2) of node gg, a3 = 0
    const int b0 = ap & 255, b1 = (ap >> 8) & 255, b2 = (ap >> 16) & 255;
    const int row = tri_row(b2, N);
    const int rdn = b2 >= 1 ? tri_row(b2 - 1, N) : 0;
    const int rup = tri_row(b2 + 1, N);
    // neighbours b + e_k - e_m with weights 1/2 (b_k+1) b_m (zero weight -> own position)
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
  for (int nn = Nfp + tid; nn < Np; nn += 64 * WPB) {
    // position nn of a face-layered vector = volume node nn seen from face 3
    const uint32_t ap = t_alpha[nn];
    const int b0 = ap & 255, b1 = (ap >> 8) & 255, b2 = (ap >> 16) & 255, j = ap >> 24;
    const int m = N - j;
    const int in0 = level_off(j - 1, N);
    t_lvp[nn] = (uint32_t)(in0 + tri_row(b2, m + 1) + b1) | ((uint32_t)(in0 + tri_row(b2 + 1, m + 1) + b1) << 16);
    t_lvc[0][nn] = (T)((double)(b0 + 1) / (m + 1));
    t_lvc[1][nn] = (T)((double)(b1 + 1) / (m + 1));
    t_lvc[2][nn] = (T)((double)(b2 + 1) / (m + 1));
  }
  __syncthreads();

  const int lane0 = tid % TPE;                              // thread within the team
  const int w = __builtin_amdgcn_readfirstlane(tid / TPE);  // team index (uniform)
  // sq accessors: (p, h_i) of node n of element el, and the store of a node
  double* const shg_w = kAliasHg ? reinterpret_cast<double*>(&slev[w][0][0][0]) : &shg_own[kAliasHg ? 0 : w][0];
  auto sq_pair = [&](int el, int n, int i) -> Pair<T> {
    if constexpr (kPairSq) {
      // node layout: (h_0, p, h_1, p, h_2, p, h_3, p, pad, pad)
      const float2 x = *reinterpret_cast<const float2*>(&sq[w][el][0][0] + SQW * n + 2 * i);
      return Pair<T>{(T)x.y, (T)x.x};
    } else {
      return Pair<T>{sq[w][el][0][n], sq[w][el][1 + i][n]};
    }
  };
  auto sq_put = [&](int el, int n, T pv, const T* hv) {
    if constexpr (kPairSq) {
      float2* o = reinterpret_cast<float2*>(&sq[w][el][0][0] + SQW * n);
#pragma unroll
      for (int i = 0; i < 4; ++i) o[i] = make_float2(hv[i], pv);
    } else {
      sq[w][el][0][n] = pv;
#pragma unroll
      for (int i = 0; i < 4; ++i) sq[w][el][1 + i][n] = hv[i];
    }
  };
  // Node r of a thread: element el of the group and node n (false: none).
  auto node_of = [&](int ln, int r, int& el, int& n) -> bool {
    if constexpr (M::IL) {
      el = r;
      n = ln;
      return ln < Np;
    } else {
      const int v = ln + TPE * r;
      el = E == 1 ? 0 : v / Np;
      n = v - el * Np;
      return v < E * Np;
    }
  };
  // Face item r of a thread: position gg, face f, element el (false: none).
  auto face_item = [&](int ln, int r, unsigned& gg, int& f, unsigned& el) -> bool {
    if constexpr (M::IL) {
      const unsigned v = (unsigned)ln + 64u * (unsigned)(r % M::NFE);
      gg = v % M::SF;
      f = (int)(v / M::SF);
      el = (unsigned)(r / M::NFE);
      return f < 4 && gg < (unsigned)Nfp;
    } else {
      const unsigned v = (unsigned)ln + TPE * r;
      gg = v % M::SF;
      f = (int)((v / M::SF) % 4);
      el = v / (4 * M::SF);
      return el < (unsigned)E && gg < (unsigned)Nfp;
    }
  };
  const int64_t K = A.K;
  const int64_t KNp = K * Np;
  const int64_t G = (K + E - 1) / E;  // element groups per shot
  const int64_t GS = G * (kBatch ? A.shots : 1);
  // XCD-aware split of the element groups (gridDim.x is a multiple of 8)
  const int xcd = blockIdx.x & 7;
  const int64_t g_lo = GS * xcd / 8, g_hi = GS * (xcd + 1) / 8;
  const int64_t wstride = (int64_t)(gridDim.x >> 3) * TEAMS;
  const int64_t nst = kBatch ? A.nstages : 1;

  for (int64_t stage = 0; stage < nst; ++stage) {
  // stage constants: buffers, LSRK coefficients, source amplitude
  const int s5 = (int)(stage % 5);
  const T* qin_b = kBatch ? ((stage & 1) ? A.qalt : A.qout) : A.qin;
  T* qout_b = kBatch ? ((stage & 1) ? A.qout : A.qalt) : A.qout;
  const T rk_a = kBatch ? (T)kLsrkA[s5] : A.rk_a;
  const T rk_b = kBatch ? (T)kLsrkB[s5] : A.rk_b;
  const int read_res = kBatch ? (s5 != 0) : A.read_res;
  // the wavelet comes from a table: evaluating it here would keep its
  // constants in registers through the whole stage loop
  const T amp = (kBatch && A.src_elem) ? (T)A.amp[stage] : (T)0;

  int64_t g = g_lo + (int64_t)(blockIdx.x >> 3) * TEAMS + w;
  Header<N, T, TW> hd;
  // group g = shot * G + element group (shots * G < 2^32 is checked on the host)
  if (g < g_hi) load_header<N, T, TW>(hd, A, kBatch ? (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)g % (uint32_t)G) : g, lane0);

  for (; g < g_hi; g += wstride) {
    // (uniform per team: the division runs on the vector unit)
    const int64_t shot = kBatch ? (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)g / (uint32_t)G) : 0;
    const int64_t e0 = (g - shot * G) * E;
    const int64_t sb = shot * 4 * KNp;  // this shot's fields
    // element-major fields: element e holds p, u, v, w of its Np nodes in
    // one contiguous block of 4 Np values; field f of node n is at
    // e 4 Np + f Np + n, so one address per node serves all four fields
    const T* const qin_s = qin_b + sb;
    T* const res_s = A.res + (kUpdate ? sb : 0);
    T* const qout_s = qout_b + sb;
    // Lane-derived addresses are cheap to recompute; hiding the lane id from
    // loop-invariant code motion keeps them from being hoisted out of the
    // element loop and occupying (or spilling) registers for its whole life.
    int lane = lane0;
    asm volatile("" : "+v"(lane));

    // ---- header of this group -> LDS --------------------------------------
    team_sync<TW>();
#pragma unroll
    for (int r = 0; r < H::NG; ++r) {
      const int v = lane + TPE * r;
      if (v < E * H::GS) {
        if constexpr (H::kTG) {
          (&sgeo[w][0][0])[v] = hd.geo[r];
        } else {
          shg_w[v] = hd.geo[r];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < M::NHE; ++r) {
      const int v = lane + TPE * r;
      if (v < E * 4) {
        she[w][v] = hd.etoe[r];
        shf[w][v] = (uint8_t)hd.fo[r];
      }
    }
    team_sync<TW>();

    // ---- issue this group's loads: own q, residual, neighbour traces --------
    // (at raised wave priority, so that a wave about to start its memory
    // traffic gets the issue slots before waves busy with arithmetic)
    __builtin_amdgcn_s_setprio(3);
    T qv[NPL][4], rv[NPL][4];
    uint32_t noff[NPL];  // e 4 Np + n of the thread's nodes (field p)
#pragma unroll
    for (int r = 0; r < NPL; ++r) {
      int el, n;
      const bool ok = node_of(lane, r, el, n) && (e0 + el < K);
      noff[r] = ok ? (uint32_t)((e0 + el) * 4 * Np + n) : 0u;
      const T* qp = qin_s + noff[r];
#pragma unroll
      for (int f = 0; f < 4; ++f) qv[r][f] = qp[f * Np];
      if (kUpdate && read_res && !S::LATE_RES) {
        const T* rp = res_s + noff[r];
#pragma unroll
        for (int f = 0; f < 4; ++f) rv[r][f] = ldn<NT>(rp + f * Np);
      } else {
#pragma unroll
        for (int f = 0; f < 4; ++f) rv[r][f] = 0;
      }
    }
    T tr[M::NFI][4];
    if constexpr (kSurf) {
#pragma unroll
      for (int r = 0; r < M::NFI; ++r) {
        unsigned gg, el;
        int f;
        const bool item = face_item(lane, r, gg, f, el);
        uint32_t off = 0;
        if (item && e0 + el < K) {
          const int nb = she[w][el * 4 + f];
          const int info = shf[w][el * 4 + f];
          if (nb >= 0) off = (uint32_t)nb * (4 * Np) + t_nbr[((info & 3) * 6 + (info >> 2)) * Nfp + gg];
        }
        const T* tp = qin_s + off;
#pragma unroll
        for (int fl = 0; fl < 4; ++fl) tr[r][fl] = tp[fl * Np];
      }
    }
    // face numbers of the stage records, loaded with the group's data
    int32_t rfn[kRecord ? M::NFI : 1];
    if constexpr (kRecord) {
#pragma unroll
      for (int r = 0; r < M::NFI; ++r) {
        unsigned gg, el;
        int f;
        const bool item = face_item(lane, r, gg, f, el) && e0 + el < K;
        rfn[r] = A.rec_face[item ? (e0 + el) * 4 + f : 0];
      }
    }
    // ---- prefetch the next group's header -----------------------------------
    if (g + wstride < g_hi)
      load_header<N, T, TW>(hd, A, kBatch ? (int64_t)__builtin_amdgcn_readfirstlane((uint32_t)(g + wstride) % (uint32_t)G) : g + wstride, lane);
    __builtin_amdgcn_s_setprio(0);

    // ---- per-element derived geometry (one lane per element face; FP32
    // groups loaded it with the header) -----------------------------------------
    for (int v = lane; !H::kTG && v < E * 4; v += TPE) {
      const int el = v >> 2;
      const int f = v & 3;
      const double* ge = shg_w + el * kGeoStride;
      double gx, gy, gz;  // grad lambda_f
      if (f == 0) {
        gx = -(ge[0] + ge[3] + ge[6]);
        gy = -(ge[1] + ge[4] + ge[7]);
        gz = -(ge[2] + ge[5] + ge[8]);
      } else {
        gx = ge[3 * (f - 1) + 0];
        gy = ge[3 * (f - 1) + 1];
        gz = ge[3 * (f - 1) + 2];
      }
      T* o = sgeo[w][el];
      o[3 * f + 0] = (T)gx;
      o[3 * f + 1] = (T)gy;
      o[3 * f + 2] = (T)gz;
      if (f == 0) o[12] = (T)ge[9];
      T* fr = o + 16 + 6 * f;
      fr[0] = (T)(-2.0 * gx);
      fr[1] = (T)(-2.0 * gy);
      fr[2] = (T)(-2.0 * gz);
      fr[3] = (T)ge[10 + f];     // a_p
      fr[4] = (T)(0.5 * ge[9]);  // a_u = kappa / 2
      fr[5] = (T)ge[14 + f];     // b_u
    }

    // ---- own coefficients -> LDS -----------------------------------------------
    T hreg[NPL][4];  // h_i of the own nodes
#pragma unroll
    for (int r = 0; r < NPL; ++r) {
      int el, n;
      if (node_of(lane, r, el, n)) {
        T* hv = hreg[r];
        if constexpr (H::kTG) {
          // h_i from grad(lambda_i) of the derived geometry (in LDS since the last sync)
          const T* gt = sgeo[w][el];
#pragma unroll
          for (int i = 0; i < 4; ++i) hv[i] = gt[3 * i] * qv[r][1] + gt[3 * i + 1] * qv[r][2] + gt[3 * i + 2] * qv[r][3];
        } else {
          // h_i from grad(lambda_i) of the header (double, in LDS since the last sync)
          const double* hg = shg_w + el * kGeoStride;
#pragma unroll
          for (int i = 1; i < 4; ++i)
            hv[i] = (T)hg[3 * i - 3] * qv[r][1] + (T)hg[3 * i - 2] * qv[r][2] + (T)hg[3 * i - 1] * qv[r][3];
          hv[0] = (T)(-(hg[0] + hg[3] + hg[6])) * qv[r][1] + (T)(-(hg[1] + hg[4] + hg[7])) * qv[r][2] +
                  (T)(-(hg[2] + hg[5] + hg[8])) * qv[r][3];
        }
        sq_put(el, n, qv[r][0], hv);
      }
    }
    team_sync<TW>();

    // ---- volume term ------------------------------------------------------------
    T rhs[NPL][4];
#pragma unroll
    for (int r = 0; r < NPL; ++r) {
#pragma unroll
      for (int f = 0; f < 4; ++f) rhs[r][f] = 0;
    }
    if constexpr (kVol) {
#pragma unroll
      for (int r = 0; r < NPL; ++r) {
        int el, n;
        if (!node_of(lane, r, el, n)) continue;
        const uint32_t ap = t_alpha[n];
        const T av[4] = {(T)(ap & 255), (T)((ap >> 8) & 255), (T)((ap >> 16) & 255), (T)(ap >> 24)};
        int nb[12];
#pragma unroll
        for (int p = 0; p < 12; ++p) nb[p] = t_vnbr[n][p];
        // neighbour alpha + e_a - e_b: pair index 3a + (b < a ? b : b - 1)
        auto P = [&](int ai, int bi) { return nb[3 * ai + (bi < ai ? bi : bi - 1)]; };
        const T* ge = sgeo[w][el];
        // grad p = sum_i grad(lambda_i) D^i p; div u = sum_i D^i h_i (D^i is
        // linear and grad(lambda_i) is constant on the element)
        T Dp[4], div = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          T dp = av[i] * qv[r][0], dh = av[i] * hreg[r][i];
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            if (b == i) continue;
            const Pair<T> x = sq_pair(el, P(i, b), i);
            dp += av[b] * x.p;
            dh += av[b] * x.u;
          }
          Dp[i] = dp;
          div += dh;
        }
        T gp[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) gp[d] = ge[d] * Dp[0] + ge[3 + d] * Dp[1] + ge[6 + d] * Dp[2] + ge[9 + d] * Dp[3];
        rhs[r][0] = -ge[12] * div;
#pragma unroll
        for (int d = 0; d < 3; ++d) rhs[r][1 + d] = -gp[d];
      }
    }

    if constexpr (kUpdate && S::LATE_RES) {
      if (read_res) {
#pragma unroll
        for (int r = 0; r < NPL; ++r) {
          const T* rp = res_s + noff[r];
#pragma unroll
          for (int f = 0; f < 4; ++f) rv[r][f] = ldn<NT>(rp + f * Np);
        }
      }
    }

    // ---- surface term, FB faces at a time ------------------------------------------
    if constexpr (kSurf) {
#pragma unroll
      for (int fb0 = 0; fb0 < 4; fb0 += FB) {
        // flux on the face nodes of faces fb0 .. fb0+FB-1
#pragma unroll
        for (int r = 0; r < M::NFI; ++r) {
          unsigned gg, el;
          int f;
          if (!face_item(lane, r, gg, f, el) || f < fb0 || f >= fb0 + FB) continue;
          T sp = 0, su = 0;
          if (e0 + el < K) {
            const int n = t_fnode[f * Nfp + gg];
            // own trace: p and g_f . u = -2 h_f (g_f = -2 grad(lambda_f))
            const Pair<T> own = sq_pair(el, n, f);
            const T pm = own.p, gum = (T)(-2) * own.u;
            const T* fr = sgeo[w][el] + 16 + 6 * f;
            const T gx = fr[0], gy = fr[1], gz = fr[2];
            T jp, jgu;
            if (she[w][el * 4 + f] >= 0) {
              jp = tr[r][0] - pm;
              jgu = gx * tr[r][1] + gy * tr[r][2] + gz * tr[r][3] - gum;
            } else if (A.bc == 0) {  // rigid wall mirror
              jp = 0;
              jgu = (T)(-2) * gum;
            } else {  // pressure-release mirror
              jp = (T)(-2) * pm;
              jgu = 0;
            }
            sp = fr[3] * jp - fr[4] * jgu;
            su = fr[5] * jgu - (T)0.5 * jp;
            if constexpr (kRecord) {
              // one record per face, by the element with the lower index (or
              // the only one): [[p]], which the other side reads negated, and
              // the velocity jump along the unit normal, g_f.[[u]] / |g_f|,
              // the same from both sides.  Records are read once, by the
              // reverse sweep much later: non-temporal, so they do not evict
              // the fields from the caches.
              const int64_t k = e0 + el;
              const int nb = she[w][el * 4 + f];
              if (nb < 0 || k <= nb) {
                T* rj = A.rec_j + ((stage * A.shots + shot) * A.nfaces + rfn[r]) * (2 * Nfp) + gg;
                const T g2 = gx * gx + gy * gy + gz * gz;
                st<true>(rj, jp);
                if constexpr (sizeof(T) == 4) {
                  st<true>(rj + Nfp, jgu * rsqrtf(g2));
                } else {
                  st<true>(rj + Nfp, jgu / sqrt(g2));
                }
              }
            }
          }
          sfl[w][el][f - fb0][gg] = Pair<T>{sp, su};
        }
        team_sync<TW>();

        if constexpr (M::IL) {
          // w_0 = L_0 s, one row per (face, position) item, position fastest
          // (interleaved groups: an item's tables serve the LREP elements)
          constexpr unsigned LGR = M::IL ? FB : E * FB;  // face vectors per item space
          constexpr unsigned LREP = M::IL ? E : 1;       // elements sharing an item
          constexpr unsigned SL0 = item_stride(Nfp, LGR, TPE);
          for (unsigned v = lane; v < LGR * SL0; v += TPE) {
            const unsigned gg = v % SL0;
            const unsigned g0 = v / SL0;  // = el * FB + face in the batch (face in the batch if interleaved)
            if (gg >= Nfp) continue;
            const uint2 pp = *reinterpret_cast<const uint2*>(t_l0p[gg]);
            const unsigned pos[7] = {gg, (pp.x >> 8) & 255, (pp.x >> 16) & 255, pp.x >> 24,
                                     pp.y & 255, (pp.y >> 8) & 255, (pp.y >> 16) & 255};
            T c[7];
  #pragma unroll
            for (int q = 0; q < 7; ++q) c[q] = t_l0c[q][gg];
  #pragma unroll
            for (unsigned e2 = 0; e2 < LREP; ++e2) {
              const unsigned rest = g0 + e2 * FB;
              const Pair<T>* sv = &sfl[w][0][0][0] + rest * Nfp;
              T ap = 0, au = 0;
  #pragma unroll
              for (int q = 0; q < 7; ++q) {
                const Pair<T> x = sv[pos[q]];
                ap += c[q] * x.p;
                au += c[q] * x.u;
              }
              (&slev[w][0][0][0])[rest * Np + gg] = Pair<T>{ap, au};
            }
          }
          team_sync<TW>();

          // one-degree reductions, level j = 1..N, one row per (face, position) item
  #pragma unroll
          for (int j = 1; j <= N; ++j) {
            const int out0 = level_off(j, N);
            const int Tm = tri_of(N - j);
            const unsigned SM = item_stride(Tm, LGR, TPE);
            for (unsigned v = lane; v < LGR * SM; v += TPE) {
              const unsigned s = v % SM;
              const unsigned g0 = v / SM;  // = el * FB + face in the batch (face in the batch if interleaved)
              if (s >= (unsigned)Tm) continue;
              const unsigned nn = out0 + s;
              const uint32_t ip = t_lvp[nn];
              const unsigned i0 = ip & 0xffff, i2 = ip >> 16;
              const T c0 = t_lvc[0][nn], c1 = t_lvc[1][nn], c2 = t_lvc[2][nn];
  #pragma unroll
              for (unsigned e2 = 0; e2 < LREP; ++e2) {
                Pair<T>* wv = &slev[w][0][0][0] + (g0 + e2 * FB) * Np;
                const Pair<T> x0 = wv[i0], x1 = wv[i0 + 1], x2 = wv[i2];
                wv[nn] = Pair<T>{c0 * x0.p + c1 * x1.p + c2 * x2.p, c0 * x0.u + c1 * x1.u + c2 * x2.u};
              }
            }
            team_sync<TW>();
          }
        } else {
          // w_0 = L_0 s, one row per (face, position) item, position fastest
          constexpr unsigned SL0 = item_stride(Nfp, E * FB, TPE);
          for (unsigned v = lane; v < E * FB * SL0; v += TPE) {
            const unsigned gg = v % SL0;
            const unsigned rest = v / SL0;  // = el * FB + face in the batch
            if (gg >= Nfp) continue;
            const Pair<T>* sv = &sfl[w][0][0][0] + rest * Nfp;
            const uint2 pp = *reinterpret_cast<const uint2*>(t_l0p[gg]);
            const unsigned pos[7] = {gg, (pp.x >> 8) & 255, (pp.x >> 16) & 255, pp.x >> 24,
                                     pp.y & 255, (pp.y >> 8) & 255, (pp.y >> 16) & 255};
            T ap = 0, au = 0;
  #pragma unroll
            for (int q = 0; q < 7; ++q) {
              const T c = t_l0c[q][gg];
              const Pair<T> x = sv[pos[q]];
              ap += c * x.p;
              au += c * x.u;
            }
            (&slev[w][0][0][0])[rest * Np + gg] = Pair<T>{ap, au};
          }
          team_sync<TW>();

          // one-degree reductions, level j = 1..N, one row per (face, position) item
  #pragma unroll
          for (int j = 1; j <= N; ++j) {
            const int out0 = level_off(j, N);
            const int Tm = tri_of(N - j);
            const unsigned SM = item_stride(Tm, E * FB, TPE);
            for (unsigned v = lane; v < E * FB * SM; v += TPE) {
              const unsigned s = v % SM;
              const unsigned rest = v / SM;  // = el * FB + face in the batch
              if (s >= (unsigned)Tm) continue;
              const unsigned nn = out0 + s;
              Pair<T>* wv = &slev[w][0][0][0] + rest * Np;
              const uint32_t ip = t_lvp[nn];
              const unsigned i0 = ip & 0xffff, i2 = ip >> 16;
              const T c0 = t_lvc[0][nn], c1 = t_lvc[1][nn], c2 = t_lvc[2][nn];
              const Pair<T> x0 = wv[i0], x1 = wv[i0 + 1], x2 = wv[i2];
              wv[nn] = Pair<T>{c0 * x0.p + c1 * x1.p + c2 * x2.p, c0 * x0.u + c1 * x1.u + c2 * x2.u};
            }
            team_sync<TW>();
          }
        }

        // gather the lifted values of this batch into the nodes
#pragma unroll
        for (int r = 0; r < NPL; ++r) {
          int el, n;
          if (!node_of(lane, r, el, n)) continue;
          const uint32_t ap = t_alpha[n];
#pragma unroll
          for (int fl = 0; fl < FB; ++fl) {
            const int f = fb0 + fl;
            const T* fr = sgeo[w][el] + 16 + 6 * f;
            const int af = (ap >> (8 * f)) & 255;
            const int pos = t_proj[n][f];
            const T ell = t_ell[af];
            const Pair<T> x = slev[w][el][fl][pos];
            const T lp = ell * x.p;
            const T lu = ell * x.u;
            rhs[r][0] += lp;
            rhs[r][1] += fr[0] * lu;
            rhs[r][2] += fr[1] * lu;
            rhs[r][3] += fr[2] * lu;
          }
        }
        if (FB < 4) team_sync<TW>();
      }
    }

    // ---- point source of this shot (pressure equation) -------------------------------
    if constexpr (kBatch) {
      const int32_t se = A.src_elem ? A.src_elem[shot] : -1;
#pragma unroll
      for (int r = 0; r < NPL; ++r) {
        int el, n;
        if (node_of(lane, r, el, n) && e0 + el == se) rhs[r][0] += amp * A.src_coef[shot * Np + n];
      }
    }

    // ---- update / store -------------------------------------------------------------
#pragma unroll
    for (int r = 0; r < NPL; ++r) {
      int el, n;
      if (!node_of(lane, r, el, n) || e0 + el >= K) continue;
      T* const rp = res_s + noff[r];
      T* const op = qout_s + noff[r];
      if constexpr (kUpdate) {
        if constexpr (kRecord) st<true>(A.rec_p + ((stage * A.shots + shot) * KNp + (e0 + el) * Np + n), rhs[r][0]);
        const T dt = kBatch ? (T)A.dtd : A.dt;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const T rs = dt * rhs[r][f] + rk_a * rv[r][f];
          st<NT>(rp + f * Np, rs);
          st<NT>(op + f * Np, qv[r][f] + rk_b * rs);
        }
      } else {
#pragma unroll
        for (int f = 0; f < 4; ++f) st<NT>(op + f * Np, rhs[r][f]);
      }
    }
  }  // element groups

  if constexpr (kBatch) {
    __shared__ int s_ok;
    if (!grid_barrier(A.sync, stage, A.barrier_timeout, &s_ok)) return;
    // receivers read the pressure after the fifth stage of each step
    if (s5 == 4 && A.R > 0) {
      const int64_t items = A.shots * A.R;
      const int64_t step = stage / 5;
      for (int64_t it = (int64_t)blockIdx.x * (64 * WPB) + tid; it < items; it += (int64_t)gridDim.x * 64 * WPB) {
        const int64_t sh = it / A.R;
        const int rr = (int)(it - sh * A.R);
        const int32_t re = A.rec_elem[rr];
        T acc = (T)NAN;
        if (re >= 0 && re < K) {
          const T* pr = qout_b + sh * 4 * KNp + (int64_t)re * 4 * Np;  // p block of element re
          const T* cr = A.rec_coef + (int64_t)rr * Np;
          acc = 0;
#pragma unroll 8
          for (int n = 0; n < Np; ++n) acc += cr[n] * pr[n];
        }
        A.traces[(step * A.shots + sh) * A.R + rr] = acc;
      }
    }
  }
  }  // stages
}

__global__ __launch_bounds__(256) void wavelet_kernel(double* amp, int64_t n, double t0, int64_t step0, double dt,
                                                      double f0, double ts) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) amp[i] = ricker(t0 + (double)(step0 + i / 5) * dt + kLsrkC[i % 5] * dt, f0, ts);
}

hipError_t launch_wavelet(double* amp, int64_t nstages, double t0, int64_t step0, double dt, double f0, double ts,
                          hipStream_t stream) {
  if (nstages <= 0) return hipSuccess;
  if (!amp) return hipErrorInvalidValue;
  (void)hipGetLastError();
  hipLaunchKernelGGL(wavelet_kernel, dim3((unsigned)((nstages + 255) / 256)), dim3(256), 0, stream, amp, nstages, t0,
                     step0, dt, f0, ts);
  return hipGetLastError();
}

__global__ __launch_bounds__(64) void barrier_reset_kernel(uint32_t* sync) {
  // arrival counters and top counter; the sticky flag is kept
  for (int i = threadIdx.x; i < kSyncFlag; i += 64) sync[i] = 0u;
}

hipError_t launch_barrier_reset(uint32_t* sync, hipStream_t stream) {
  if (!sync) return hipErrorInvalidValue;
  (void)hipGetLastError();
  hipLaunchKernelGGL(barrier_reset_kernel, dim3(1), dim3(64), 0, stream, sync);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void poison_kernel(const uint32_t* sync, T* a, int64_t n) {
  if (sync[kSyncFlag] == 0u) return;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) a[i] = (T)NAN;
}

template <typename T>
hipError_t launch_poison(const uint32_t* sync, T* a, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  if (!sync || !a) return hipErrorInvalidValue;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 2048);
  (void)hipGetLastError();
  hipLaunchKernelGGL(poison_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, stream, sync, a, n);
  return hipGetLastError();
}

template hipError_t launch_poison<double>(const uint32_t*, double*, int64_t, hipStream_t);
template hipError_t launch_poison<float>(const uint32_t*, float*, int64_t, hipStream_t);

// Workgroups of a kernel that one CU holds at a time.  `api` is what the
// runtime's occupancy query reports; `bound` is derived here from the
// kernel's own resources, so that a cooperative grid never relies on the
// query alone:
//   VGPRs: 512 per SIMD lane, allocated in granules of 8, at most 8 waves per
//     SIMD; a workgroup of 4 or 8 waves puts the same number of waves on each
//     of the CU's 4 SIMDs; a two-wave workgroup is counted as if every such
//     workgroup used the same two SIMDs (the placement is not documented);
//   LDS: 160 KiB per CU, a workgroup's static LDS rounded up to 2 KiB;
//   scratch memory: a kernel that uses any is not proven co-resident (its
//     waves also need scratch space that the runtime sizes), bound 0;
//   at most 8 workgroups per CU for the persistent grids.
// The bound is min(api, the above).
struct Residency {
  int api = 0, bound = 0, vgprs = 0, lds = 0, scratch = 0, cus = 0;
  hipError_t err = hipSuccess;
};

template <int N, typename T, int MODE, int WPB, bool NT = false>
static const Residency& kernel_residency() {
  static Residency r;
  static bool done = false;
  if (done) return r;
  const void* fn = reinterpret_cast<const void*>(bb_stage_kernel<N, T, MODE, WPB, NT>);
  int dev = 0;
  r.err = hipGetDevice(&dev);
  if (r.err == hipSuccess) r.err = hipDeviceGetAttribute(&r.cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (r.err == hipSuccess)
    r.err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&r.api, bb_stage_kernel<N, T, MODE, WPB, NT>, 64 * WPB, 0);
  hipFuncAttributes fa{};
  if (r.err == hipSuccess) r.err = hipFuncGetAttributes(&fa, fn);
  if (r.err != hipSuccess) return r;  // not cached: the next call asks again
  r.vgprs = fa.numRegs;
  r.lds = (int)fa.sharedSizeBytes;
  r.scratch = (int)fa.localSizeBytes;
  int bound = 0;
  if (r.vgprs > 0 && r.scratch == 0) {
    const int per_simd = std::min(8, 512 / (((r.vgprs + 7) / 8) * 8));
    const int by_vgpr = WPB >= 4 ? per_simd * 4 / WPB : per_simd;
    const int by_lds = r.lds > 0 ? (160 * 1024) / (((r.lds + 2047) / 2048) * 2048) : 8;
    bound = std::min(std::min(by_vgpr, by_lds), std::min(8, r.api));
  }
  r.bound = std::max(bound, 0);
  done = true;
  return r;
}

// Grid of a persistent launch over `groups` element groups, `per_wg` groups
// per workgroup and pass: the co-resident workgroups, at most what has work,
// a multiple of 8 (one share per XCD).  Single-stage launches take the
// occupancy query's count (they need no co-residency: nothing waits across
// workgroups); cooperative (batched) launches take the derived bound and are
// refused when it is zero or the grid would fall below 8.
template <int N, typename T, int MODE, int WPB, bool NT = false>
static hipError_t resident_grid(int64_t groups, int per_wg, int64_t* grid_out) {
  const Residency& r = kernel_residency<N, T, MODE, WPB, NT>();
  if (r.err != hipSuccess) return r.err;
  const int per_cu = MODE >= kBatched ? r.bound : r.api;
  if (per_cu < 1) return MODE >= kBatched ? hipErrorCooperativeLaunchTooLarge : hipErrorInvalidConfiguration;
  const int64_t needed = (groups + per_wg - 1) / per_wg;  // workgroups with work
  int64_t grid = (int64_t)per_cu * r.cus;
  if (grid > ((needed + 7) / 8) * 8) grid = ((needed + 7) / 8) * 8;
  if (MODE >= kBatched) grid = grid / 8 * 8;  // stay within the co-resident bound
  else grid = ((grid + 7) / 8) * 8;
  if (grid < 8) return MODE >= kBatched ? hipErrorCooperativeLaunchTooLarge : (*grid_out = 8, hipSuccess);
  *grid_out = grid;
  return hipSuccess;
}

template <int N, typename T, int MODE, bool NT>
static hipError_t launch_one_nt(const StageArgs<T>& a, hipStream_t stream) {
  using S = Shape<N, T>;
  using M = Team<N, T, S::TW>;
  const int64_t groups = (a.K + M::E - 1) / M::E;
  if (groups <= 0) return hipSuccess;
  constexpr int WPB = S::TW > 1 ? S::TW : 4;
  int64_t grid = 0;
  const hipError_t e = resident_grid<N, T, MODE, WPB, NT>(groups, WPB / S::TW, &grid);
  if (e != hipSuccess) return e;
  (void)hipGetLastError();  // drop errors left by earlier, unrelated calls
  hipLaunchKernelGGL((bb_stage_kernel<N, T, MODE, WPB, NT>), dim3((unsigned)grid), dim3(64 * WPB), 0, stream, a);
  return hipGetLastError();
}

// Non-temporal output stores exist for the FP64 stage (the time-stepping
// path); right-hand-side evaluations and FP32 use plain stores.
template <int N, typename T, int MODE>
static hipError_t launch_one(const StageArgs<T>& a, hipStream_t stream) {
  if constexpr (MODE == kStage && sizeof(T) == 8) {
    if (a.nt_store) return launch_one_nt<N, T, MODE, true>(a, stream);
  }
  return launch_one_nt<N, T, MODE, false>(a, stream);
}

template <int N, typename T, int WPB, int MODE>
static hipError_t launch_batched_mode(const StageArgs<T>& a, hipStream_t stream) {
  using M = Team<N, T, team_waves<N, T, MODE, WPB>()>;
  const int64_t groups = (a.K + M::E - 1) / M::E * a.shots;
  if (groups <= 0 || a.nstages <= 0) return hipSuccess;
  int64_t grid = 0;
  const hipError_t e = resident_grid<N, T, MODE, WPB>(groups, WPB / team_waves<N, T, MODE, WPB>(), &grid);
  if (e != hipSuccess) return e;
  StageArgs<T> args = a;
  void* params[] = {&args};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(bb_stage_kernel<N, T, MODE, WPB>),
                                    dim3((unsigned)grid), dim3(64 * WPB), params, 0, stream);
}

template <int N, typename T, int WPB>
static hipError_t launch_batched_one(const StageArgs<T>& a, hipStream_t stream) {
  if (a.rec_p || a.rec_j) {
    if (!a.rec_p || !a.rec_j || !a.rec_face) return hipErrorInvalidValue;
    return launch_batched_mode<N, T, WPB, kBatchedRecord>(a, stream);
  }
  return launch_batched_mode<N, T, WPB, kBatched>(a, stream);
}

template <typename T>
hipError_t launch_batched(int N, int wpb, const StageArgs<T>& a, hipStream_t stream) {
  // One-wave workgroups are not offered: a cooperative launch of them hung
  // once (N = 5, FP32, 196,608 elements) for a reason not established.
#define BBDG_BATCH_CASE(NN)                                       \
  case NN:                                                        \
    if (wpb == 2) return launch_batched_one<NN, T, 2>(a, stream); \
    if (wpb == 4) return launch_batched_one<NN, T, 4>(a, stream); \
    if (wpb == 8) return launch_batched_one<NN, T, 8>(a, stream); \
    return hipErrorInvalidValue;
  switch (N) {
    BBDG_BATCH_CASE(1)
    BBDG_BATCH_CASE(2)
    BBDG_BATCH_CASE(3)
    BBDG_BATCH_CASE(4)
    BBDG_BATCH_CASE(5)
    BBDG_BATCH_CASE(6)
    BBDG_BATCH_CASE(7)
    BBDG_BATCH_CASE(8)
    BBDG_BATCH_CASE(9)
    default: return hipErrorInvalidValue;
  }
#undef BBDG_BATCH_CASE
}

template hipError_t launch_batched<double>(int, int, const StageArgs<double>&, hipStream_t);
template hipError_t launch_batched<float>(int, int, const StageArgs<float>&, hipStream_t);

template <int N, typename T, int WPB>
static hipError_t residency_of(int record, int out[6]) {
  const Residency& r = record ? kernel_residency<N, T, kBatchedRecord, WPB>() : kernel_residency<N, T, kBatched, WPB>();
  out[0] = r.api;
  out[1] = r.bound;
  out[2] = r.vgprs;
  out[3] = r.lds;
  out[4] = r.scratch;
  out[5] = r.cus;
  return r.err;
}

template <typename T>
hipError_t batched_residency(int N, int wpb, int record, int out[6]) {
#define BBDG_RES_CASE(NN)                                          \
  case NN:                                                         \
    if (wpb == 2) return residency_of<NN, T, 2>(record, out);      \
    if (wpb == 4) return residency_of<NN, T, 4>(record, out);      \
    if (wpb == 8) return residency_of<NN, T, 8>(record, out);      \
    return hipErrorInvalidValue;
  switch (N) {
    BBDG_RES_CASE(1)
    BBDG_RES_CASE(2)
    BBDG_RES_CASE(3)
    BBDG_RES_CASE(4)
    BBDG_RES_CASE(5)
    BBDG_RES_CASE(6)
    BBDG_RES_CASE(7)
    BBDG_RES_CASE(8)
    BBDG_RES_CASE(9)
    default: return hipErrorInvalidValue;
  }
#undef BBDG_RES_CASE
}

template hipError_t batched_residency<double>(int, int, int, int[6]);
template hipError_t batched_residency<float>(int, int, int, int[6]);

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
