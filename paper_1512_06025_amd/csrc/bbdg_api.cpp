// C ABI of libbbdg (declared in include/bbdg.h): argument validation, mesh
// geometry and connectivity, operator index tables, device residency of the
// per-element data, and the LSRK4 time loop around the fused stage kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/bbdg.h"
#include "bb_common.hpp"
#include "bb_launch.hpp"

using namespace bbdg;

struct bbdg_solver {
  int N = 0, dtype = 0, bc = 0, device = 0;
  int64_t K = 0;
  double* d_geo = nullptr;     // K x kGeoStride (see bb_common.hpp)
  int32_t* d_etoe = nullptr;   // K x 4
  uint8_t* d_etofo = nullptr;  // K x 4
  uint16_t* d_tab = nullptr;   // tab_layout(N).size
};

namespace {

// Carpenter-Kennedy (5,4) 2N-storage coefficients (the low-storage RK4 the
// paper uses, Section 4.2).
const double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
const double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};

std::vector<std::array<int, 4>> alphas(int N) {
  std::vector<std::array<int, 4>> out;
  for (int a3 = 0; a3 <= N; ++a3)
    for (int a2 = 0; a2 <= N - a3; ++a2)
      for (int a1 = 0; a1 <= N - a3 - a2; ++a1) out.push_back({N - a1 - a2 - a3, a1, a2, a3});
  return out;
}

// volume index of (a1, a2, a3) at order N
int vol_index(int N, int a1, int a2, int a3) { return level_off(a3, N) + tri_row(a2, N - a3) + a1; }

void face_verts(int f, int v[3]) {
  int m = 0;
  for (int i = 0; i < 4; ++i)
    if (i != f) v[m++] = i;
}

std::vector<uint16_t> build_tables(int N) {
  const TabLayout L = tab_layout(N);
  std::vector<uint16_t> t(L.size, 0);
  const auto A = alphas(N);
  for (int n = 0; n < L.Np; ++n) {
    for (int i = 0; i < 4; ++i) t[L.alpha + 4 * n + i] = (uint16_t)A[n][i];
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        if (a == b) continue;
        const int p = 3 * a + (b < a ? b : b - 1);
        int idx = n;
        if (A[n][b] >= 1) {
          std::array<int, 4> c = A[n];
          c[a] += 1;
          c[b] -= 1;
          idx = vol_index(N, c[1], c[2], c[3]);
        }
        t[L.vnbr + 12 * n + p] = (uint16_t)idx;
      }
    for (int f = 0; f < 4; ++f) {
      int fv[3];
      face_verts(f, fv);
      const int j = A[n][f];
      t[L.proj + 4 * n + f] = (uint16_t)(level_off(j, N) + tri_row(A[n][fv[2]], N - j) + A[n][fv[1]]);
    }
  }
  // face-local nodes (g0,g1,g2), g2 slowest
  std::vector<std::array<int, 3>> T;
  for (int g2 = 0; g2 <= N; ++g2)
    for (int g1 = 0; g1 <= N - g2; ++g1) T.push_back({N - g1 - g2, g1, g2});
  for (int f = 0; f < 4; ++f) {
    int fv[3];
    face_verts(f, fv);
    for (int g = 0; g < L.Nfp; ++g) {
      int a[4] = {0, 0, 0, 0};
      for (int m = 0; m < 3; ++m) a[fv[m]] = T[g][m];
      t[L.fnode + f * L.Nfp + g] = (uint16_t)vol_index(N, a[1], a[2], a[3]);
    }
  }
  for (int f2 = 0; f2 < 4; ++f2)
    for (int o = 0; o < 6; ++o)
      for (int g = 0; g < L.Nfp; ++g) {
        int gp[3];
        for (int m = 0; m < 3; ++m) gp[kPerm[o][m]] = T[g][m];
        const int local = tri_row(gp[2], N) + gp[1];
        t[L.nbrnode + (f2 * 6 + o) * L.Nfp + g] = t[L.fnode + f2 * L.Nfp + local];
      }
  return t;
}

bool finite_all(const double* x, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

int perm_inverse(int o) {
  int inv[3];
  for (int m = 0; m < 3; ++m) inv[kPerm[o][m]] = m;
  for (int q = 0; q < 6; ++q)
    if (kPerm[q][0] == inv[0] && kPerm[q][1] == inv[1] && kPerm[q][2] == inv[2]) return q;
  return -1;
}

size_t elem_size(int dtype) { return dtype == BBDG_F64 ? sizeof(double) : sizeof(float); }

template <typename T>
StageArgs<T> base_args(const bbdg_solver* s) {
  StageArgs<T> a{};
  a.geo = s->d_geo;
  a.etoe = s->d_etoe;
  a.etofo = s->d_etofo;
  a.tab = s->d_tab;
  a.K = s->K;
  a.bc = s->bc;
  return a;
}

template <typename T>
int run_typed(bbdg_solver* s, T* q, T* work, double dt, int64_t steps, hipStream_t st) {
  const int64_t n = 4 * s->K * (int64_t)np_of(s->N);
  T* res = work;
  T* other = work + n;
  T* cur = q;
  T* nxt = other;
  StageArgs<T> a = base_args<T>(s);
  a.res = res;
  a.dt = (T)dt;
  for (int64_t it = 0; it < steps; ++it) {
    for (int st5 = 0; st5 < 5; ++st5) {
      a.qin = cur;
      a.qout = nxt;
      a.rk_a = (T)kRkA[st5];
      a.rk_b = (T)kRkB[st5];
      a.read_res = (st5 != 0);
      if (launch_stage<T>(s->N, kStage, a, st) != hipSuccess) return BBDG_E_LAUNCH;
      std::swap(cur, nxt);
    }
  }
  if (cur != q) {
    if (hipMemcpyAsync(q, cur, n * sizeof(T), hipMemcpyDeviceToDevice, st) != hipSuccess)
      return BBDG_E_DEVICE;
  }
  return BBDG_OK;
}

void free_solver(bbdg_solver* s) {
  if (!s) return;
  if (s->d_geo) (void)hipFree(s->d_geo);
  if (s->d_etoe) (void)hipFree(s->d_etoe);
  if (s->d_etofo) (void)hipFree(s->d_etofo);
  if (s->d_tab) (void)hipFree(s->d_tab);
  delete s;
}

}  // namespace

extern "C" {

const char* bbdg_strerror(int code) {
  switch (code) {
    case BBDG_OK: return "ok";
    case BBDG_E_ARG: return "invalid argument";
    case BBDG_E_ORDER: return "order N outside 1..9";
    case BBDG_E_MESH: return "invalid mesh or connectivity";
    case BBDG_E_NONFINITE: return "non-finite input";
    case BBDG_E_DTYPE: return "unknown element type";
    case BBDG_E_BC: return "unknown boundary condition";
    case BBDG_E_DEVICE: return "HIP runtime error";
    case BBDG_E_LAUNCH: return "kernel launch failed";
    case BBDG_E_MODE: return "unknown right-hand-side mode";
    default: return "unknown error code";
  }
}

int bbdg_np(int N) {
  if (N < 1 || N > kMaxOrder) return BBDG_E_ORDER;
  return np_of(N);
}

int bbdg_alpha_table(int N, int32_t* alpha) {
  if (N < 1 || N > kMaxOrder) return BBDG_E_ORDER;
  if (!alpha) return BBDG_E_ARG;
  const auto A = alphas(N);
  for (size_t n = 0; n < A.size(); ++n)
    for (int i = 0; i < 4; ++i) alpha[4 * n + i] = A[n][i];
  return BBDG_OK;
}

int bbdg_mesh_geometry(int64_t K, int64_t Nv, const double* VX, const int32_t* EToV, double* geo,
                       int32_t* EToE, int8_t* EToF, int8_t* EToO) {
  if (K <= 0 || Nv < 4 || !VX || !EToV || !geo || !EToE || !EToF || !EToO) return BBDG_E_ARG;
  if (K > (int64_t)0x7ffffffe) return BBDG_E_ARG;
  if (!finite_all(VX, 3 * Nv)) return BBDG_E_NONFINITE;
  for (int64_t k = 0; k < K; ++k) {
    for (int i = 0; i < 4; ++i)
      if (EToV[4 * k + i] < 0 || EToV[4 * k + i] >= Nv) return BBDG_E_MESH;
    const double* X[4];
    for (int i = 0; i < 4; ++i) X[i] = VX + 3 * (int64_t)EToV[4 * k + i];
    // columns of the affine map (lambda_1..3) -> x - X0
    double Jm[3][3];
    for (int d = 0; d < 3; ++d)
      for (int c = 0; c < 3; ++c) Jm[d][c] = X[c + 1][d] - X[0][d];
    const double det = Jm[0][0] * (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) -
                       Jm[0][1] * (Jm[1][0] * Jm[2][2] - Jm[1][2] * Jm[2][0]) +
                       Jm[0][2] * (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]);
    if (!(det > 0.0)) return BBDG_E_MESH;
    // inverse rows = grad lambda_1..3 (cofactor form)
    double inv[3][3];
    inv[0][0] = (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) / det;
    inv[0][1] = (Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2]) / det;
    inv[0][2] = (Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1]) / det;
    inv[1][0] = (Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2]) / det;
    inv[1][1] = (Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0]) / det;
    inv[1][2] = (Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2]) / det;
    inv[2][0] = (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]) / det;
    inv[2][1] = (Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1]) / det;
    inv[2][2] = (Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0]) / det;
    for (int i = 0; i < 3; ++i)
      for (int d = 0; d < 3; ++d) geo[10 * k + 3 * i + d] = inv[i][d];
    geo[10 * k + 9] = 0.75 * (det / 6.0);  // J = V / |reference| with |reference| = 4/3
  }
  // face matching: sort (sorted vertex triple, element, face)
  struct FaceRec {
    int32_t v[3];
    int32_t k;
    int8_t f;
  };
  std::vector<FaceRec> faces((size_t)(4 * K));
  for (int64_t k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) {
      int fv[3];
      face_verts(f, fv);
      FaceRec r;
      for (int m = 0; m < 3; ++m) r.v[m] = EToV[4 * k + fv[m]];
      std::sort(r.v, r.v + 3);
      r.k = (int32_t)k;
      r.f = (int8_t)f;
      faces[(size_t)(4 * k + f)] = r;
    }
  std::sort(faces.begin(), faces.end(), [](const FaceRec& a, const FaceRec& b) {
    if (a.v[0] != b.v[0]) return a.v[0] < b.v[0];
    if (a.v[1] != b.v[1]) return a.v[1] < b.v[1];
    if (a.v[2] != b.v[2]) return a.v[2] < b.v[2];
    return a.k < b.k;
  });
  for (int64_t i = 0; i < 4 * K; ++i) {
    EToE[i] = -1;
    EToF[i] = -1;
    EToO[i] = -1;
  }
  auto same = [](const FaceRec& a, const FaceRec& b) {
    return a.v[0] == b.v[0] && a.v[1] == b.v[1] && a.v[2] == b.v[2];
  };
  size_t i = 0;
  while (i < faces.size()) {
    size_t j = i + 1;
    while (j < faces.size() && same(faces[i], faces[j])) ++j;
    if (j - i > 2) return BBDG_E_MESH;
    if (j - i == 2) {
      for (int side = 0; side < 2; ++side) {
        const FaceRec& me = faces[i + side];
        const FaceRec& ot = faces[i + 1 - side];
        int fa[3], fb[3];
        face_verts(me.f, fa);
        face_verts(ot.f, fb);
        int pi[3];
        for (int m = 0; m < 3; ++m) {
          pi[m] = -1;
          for (int mm = 0; mm < 3; ++mm)
            if (EToV[4 * (int64_t)me.k + fa[m]] == EToV[4 * (int64_t)ot.k + fb[mm]]) pi[m] = mm;
          if (pi[m] < 0) return BBDG_E_MESH;
        }
        int code = -1;
        for (int q = 0; q < 6; ++q)
          if (kPerm[q][0] == pi[0] && kPerm[q][1] == pi[1] && kPerm[q][2] == pi[2]) code = q;
        if (code < 0) return BBDG_E_MESH;
        const int64_t slot = 4 * (int64_t)me.k + me.f;
        EToE[slot] = ot.k;
        EToF[slot] = ot.f;
        EToO[slot] = (int8_t)code;
      }
    }
    i = j;
  }
  return BBDG_OK;
}

int bbdg_create(bbdg_solver** out, int N, int dtype, int64_t K, const int32_t* EToE, const int8_t* EToF,
                const int8_t* EToO, const double* geo, const double* c, int bc, int device) {
  if (!out) return BBDG_E_ARG;
  *out = nullptr;
  if (N < 1 || N > kMaxOrder) return BBDG_E_ORDER;
  if (dtype != BBDG_F64 && dtype != BBDG_F32) return BBDG_E_DTYPE;
  if (bc != BBDG_BC_RIGID && bc != BBDG_BC_PRESSURE_RELEASE) return BBDG_E_BC;
  if (K <= 0 || K > (int64_t)0x7ffffffe || !EToE || !EToF || !EToO || !geo || !c || device < 0)
    return BBDG_E_ARG;
  if (4 * K * (int64_t)np_of(N) >= kMaxFieldElems) return BBDG_E_ARG;
  if (!finite_all(geo, 10 * K) || !finite_all(c, K)) return BBDG_E_NONFINITE;
  for (int64_t k = 0; k < K; ++k) {
    if (!(geo[10 * k + 9] > 0.0)) return BBDG_E_MESH;
    if (!(c[k] > 0.0)) return BBDG_E_ARG;
    for (int f = 0; f < 4; ++f) {
      const int64_t slot = 4 * k + f;
      const int32_t nb = EToE[slot];
      if (nb < -1 || nb >= K) return BBDG_E_MESH;
      if (nb < 0) continue;
      const int f2 = EToF[slot], o = EToO[slot];
      if (f2 < 0 || f2 > 3 || o < 0 || o > 5) return BBDG_E_MESH;
      const int64_t back = 4 * (int64_t)nb + f2;
      if (EToE[back] != k || EToF[back] != f || EToO[back] != perm_inverse(o)) return BBDG_E_MESH;
    }
  }

  if (hipSetDevice(device) != hipSuccess) return BBDG_E_DEVICE;
  bbdg_solver* s = new (std::nothrow) bbdg_solver();
  if (!s) return BBDG_E_DEVICE;
  s->N = N;
  s->dtype = dtype;
  s->bc = bc;
  s->device = device;
  s->K = K;

  std::vector<double> dgeo((size_t)(kGeoStride * K));
  std::vector<uint8_t> fo((size_t)(4 * K));
  for (int64_t k = 0; k < K; ++k) {
    double* o = dgeo.data() + (size_t)(kGeoStride * k);
    for (int i = 0; i < 9; ++i) o[i] = geo[10 * k + i];
    o[9] = c[k] * c[k];
    for (int f = 0; f < 4; ++f) {
      const int64_t slot = 4 * k + f;
      fo[(size_t)slot] = EToE[slot] >= 0 ? (uint8_t)((EToF[slot] & 3) | (EToO[slot] << 2)) : 0;
      // grad lambda_f (lambda_0 = 1 - lambda_1 - lambda_2 - lambda_3)
      double gl[3];
      for (int d = 0; d < 3; ++d)
        gl[d] = f == 0 ? -(geo[10 * k + d] + geo[10 * k + 3 + d] + geo[10 * k + 6 + d]) : geo[10 * k + 3 * (f - 1) + d];
      const double gn = 2.0 * std::sqrt(gl[0] * gl[0] + gl[1] * gl[1] + gl[2] * gl[2]);
      const double cp = EToE[slot] >= 0 ? c[EToE[slot]] : c[k];
      o[10 + f] = c[k] * c[k] * gn / (c[k] + cp);  // kappa tau_p |g| / 2
      o[14 + f] = (c[k] + cp) / (4.0 * gn);         // tau_u / (2 |g|)
    }
  }
  const std::vector<uint16_t> tab = build_tables(N);
  bool ok = hipMalloc(&s->d_geo, dgeo.size() * sizeof(double)) == hipSuccess &&
            hipMalloc(&s->d_etoe, (size_t)(4 * K) * sizeof(int32_t)) == hipSuccess &&
            hipMalloc(&s->d_etofo, fo.size()) == hipSuccess &&
            hipMalloc(&s->d_tab, tab.size() * sizeof(uint16_t)) == hipSuccess;
  ok = ok && hipMemcpy(s->d_geo, dgeo.data(), dgeo.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(s->d_etoe, EToE, (size_t)(4 * K) * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(s->d_etofo, fo.data(), fo.size(), hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(s->d_tab, tab.data(), tab.size() * sizeof(uint16_t), hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    free_solver(s);
    return BBDG_E_DEVICE;
  }
  *out = s;
  return BBDG_OK;
}

int bbdg_info(const bbdg_solver* s, int* N, int* dtype, int64_t* K, int* Np) {
  if (!s) return BBDG_E_ARG;
  if (N) *N = s->N;
  if (dtype) *dtype = s->dtype;
  if (K) *K = s->K;
  if (Np) *Np = np_of(s->N);
  return BBDG_OK;
}

int bbdg_rhs(bbdg_solver* s, const void* q, void* rhs, int mode, void* stream) {
  if (!s || !q || !rhs) return BBDG_E_ARG;
  int km;
  switch (mode) {
    case BBDG_RHS_FULL: km = kRhsFull; break;
    case BBDG_RHS_VOLUME: km = kRhsVolume; break;
    case BBDG_RHS_SURFACE: km = kRhsSurface; break;
    default: return BBDG_E_MODE;
  }
  const size_t bytes = 4 * (size_t)s->K * np_of(s->N) * elem_size(s->dtype);
  const char* a = (const char*)q;
  const char* b = (const char*)rhs;
  if (a < b + bytes && b < a + bytes) return BBDG_E_ARG;
  if (hipSetDevice(s->device) != hipSuccess) return BBDG_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (s->dtype == BBDG_F64) {
    StageArgs<double> x = base_args<double>(s);
    x.qin = (const double*)q;
    x.qout = (double*)rhs;
    e = launch_stage<double>(s->N, km, x, st);
  } else {
    StageArgs<float> x = base_args<float>(s);
    x.qin = (const float*)q;
    x.qout = (float*)rhs;
    e = launch_stage<float>(s->N, km, x, st);
  }
  return e == hipSuccess ? BBDG_OK : BBDG_E_LAUNCH;
}

size_t bbdg_work_bytes(const bbdg_solver* s) {
  if (!s) return 0;
  return 2 * 4 * (size_t)s->K * np_of(s->N) * elem_size(s->dtype);
}

int bbdg_run(bbdg_solver* s, void* q, void* work, double t0, double dt, int64_t steps, void* stream) {
  if (!s || !q || !work || steps < 0) return BBDG_E_ARG;
  if (!std::isfinite(t0) || !std::isfinite(dt)) return BBDG_E_NONFINITE;
  if (((uintptr_t)work) % 256 != 0) return BBDG_E_ARG;
  const size_t bytes = 4 * (size_t)s->K * np_of(s->N) * elem_size(s->dtype);
  const char* a = (const char*)q;
  const char* w = (const char*)work;
  if (a < w + 2 * bytes && w < a + bytes) return BBDG_E_ARG;
  if (hipSetDevice(s->device) != hipSuccess) return BBDG_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  if (s->dtype == BBDG_F64) return run_typed<double>(s, (double*)q, (double*)work, dt, steps, st);
  return run_typed<float>(s, (float*)q, (float*)work, dt, steps, st);
}

int bbdg_copy_probe(const void* src, void* dst, size_t bytes, void* stream) {
  if (!src || !dst || bytes % 16 != 0) return BBDG_E_ARG;
  const char* a = (const char*)src;
  const char* b = (const char*)dst;
  if (a < b + bytes && b < a + bytes) return BBDG_E_ARG;
  if (((uintptr_t)src) % 16 != 0 || ((uintptr_t)dst) % 16 != 0) return BBDG_E_ARG;
  return launch_copy_probe(src, dst, bytes, (hipStream_t)stream) == hipSuccess ? BBDG_OK : BBDG_E_LAUNCH;
}

int bbdg_destroy(bbdg_solver* s) {
  if (!s) return BBDG_OK;
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  free_solver(s);
  return BBDG_OK;
}

}  // extern "C"
