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
  int basis = 0;  // 0 Bernstein-Bezier, 1 dense nodal comparator
  int64_t K = 0;
  void* d_dr = nullptr;    // nodal: [3][NpP][Kv] of the element type
  void* d_lift = nullptr;  // nodal: [NpP][Kl]
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
NodalArgs<T> nodal_args(const bbdg_solver* s);

template <typename T>
hipError_t launch_any(const bbdg_solver* s, int mode, const T* qin, T* qout, T* res, T rk_a, T rk_b, T dt,
                      int read_res, hipStream_t st) {
  if (s->basis == 0) {
    StageArgs<T> a = base_args<T>(s);
    a.qin = qin;
    a.qout = qout;
    a.res = res;
    a.rk_a = rk_a;
    a.rk_b = rk_b;
    a.dt = dt;
    a.read_res = read_res;
    return launch_stage<T>(s->N, mode, a, st);
  }
  NodalArgs<T> a = nodal_args<T>(s);
  a.qin = qin;
  a.qout = qout;
  a.res = res;
  a.rk_a = rk_a;
  a.rk_b = rk_b;
  a.dt = dt;
  a.read_res = read_res;
  return launch_nodal_stage<T>(s->N, mode, a, st);
}

template <typename T>
int run_typed(bbdg_solver* s, T* q, T* work, double dt, int64_t steps, hipStream_t st) {
  const int64_t n = 4 * s->K * (int64_t)np_of(s->N);
  T* res = work;
  T* cur = q;
  T* nxt = work + n;
  for (int64_t it = 0; it < steps; ++it) {
    for (int st5 = 0; st5 < 5; ++st5) {
      if (launch_any<T>(s, kStage, cur, nxt, res, (T)kRkA[st5], (T)kRkB[st5], (T)dt, st5 != 0, st) != hipSuccess)
        return BBDG_E_LAUNCH;
      std::swap(cur, nxt);
    }
  }
  if (cur != q) {
    if (hipMemcpyAsync(q, cur, n * sizeof(T), hipMemcpyDeviceToDevice, st) != hipSuccess) return BBDG_E_DEVICE;
  }
  return BBDG_OK;
}

// ---- dense nodal comparator operators --------------------------------------

double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

double fact(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

// In-place inverse of a dense n x n row-major matrix (Gauss-Jordan, partial pivoting).
bool invert(std::vector<double>& a, int n) {
  std::vector<double> inv((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)piv * n + c])) piv = r;
    if (a[(size_t)piv * n + c] == 0.0) return false;
    if (piv != c)
      for (int j = 0; j < n; ++j) {
        std::swap(a[(size_t)c * n + j], a[(size_t)piv * n + j]);
        std::swap(inv[(size_t)c * n + j], inv[(size_t)piv * n + j]);
      }
    const double d = 1.0 / a[(size_t)c * n + c];
    for (int j = 0; j < n; ++j) {
      a[(size_t)c * n + j] *= d;
      inv[(size_t)c * n + j] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        a[(size_t)r * n + j] -= f * a[(size_t)c * n + j];
        inv[(size_t)r * n + j] -= f * inv[(size_t)c * n + j];
      }
    }
  }
  a.swap(inv);
  return true;
}

std::vector<double> matmul(const std::vector<double>& a, const std::vector<double>& b, int n, int k, int m) {
  std::vector<double> c((size_t)n * m, 0.0);
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < k; ++l) {
      const double x = a[(size_t)i * k + l];
      if (x == 0.0) continue;
      for (int j = 0; j < m; ++j) c[(size_t)i * m + j] += x * b[(size_t)l * m + j];
    }
  return c;
}

// Bernstein-Vandermonde matrix of degree N on the equispaced lattice of a
// simplex with `dim`+1 barycentric coordinates: V[p][b] = B_b(lattice point p).
std::vector<double> vandermonde(const std::vector<std::vector<int>>& idx, int N) {
  const int n = (int)idx.size();
  std::vector<double> V((size_t)n * n);
  for (int p = 0; p < n; ++p)
    for (int b = 0; b < n; ++b) {
      double v = fact(N);
      for (size_t i = 0; i < idx[b].size(); ++i) {
        v /= fact(idx[b][i]);
        v *= std::pow((double)idx[p][i] / N, idx[b][i]);
      }
      V[(size_t)p * n + b] = v;
    }
  return V;
}

// Dense nodal operators of order N: Dr_i = V (D^i - D^0) V^{-1} (i = 1..3) and
// the lift [V L^f Vf^{-1}]_f with L^f = E_L^f L_0 from the closed forms of
// the factorisation (Section 3.1.2).  Returned padded to NodalDims.
bool nodal_operators(int N, std::vector<double>& dr, std::vector<double>& lift) {
  const NodalDims nd = nodal_dims(N);
  const int Np = np_of(N), Nfp = nfp_of(N);
  const auto A = alphas(N);
  std::vector<std::vector<int>> vidx(Np), fidx;
  for (int n = 0; n < Np; ++n) vidx[n] = {A[n][0], A[n][1], A[n][2], A[n][3]};
  for (int g2 = 0; g2 <= N; ++g2)
    for (int g1 = 0; g1 <= N - g2; ++g1) fidx.push_back({N - g1 - g2, g1, g2});
  std::vector<double> V = vandermonde(vidx, N), Vi = V;
  std::vector<double> Vf = vandermonde(fidx, N);
  if (!invert(Vi, Np) || !invert(Vf, Nfp)) return false;
  // barycentric derivatives in the BB basis (row form of Lemma 1)
  std::vector<double> Db[4];
  for (int i = 0; i < 4; ++i) {
    Db[i].assign((size_t)Np * Np, 0.0);
    for (int n = 0; n < Np; ++n)
      for (int j = 0; j < 4; ++j) {
        if (A[n][j] == 0) continue;
        std::array<int, 4> c = A[n];
        c[i] += 1;
        c[j] -= 1;
        Db[i][(size_t)n * Np + vol_index(N, c[1], c[2], c[3])] += A[n][j];
      }
  }
  dr.assign((size_t)3 * nd.NpP * nd.Kv, 0.0);
  for (int i = 1; i <= 3; ++i) {
    std::vector<double> d((size_t)Np * Np);
    for (size_t t = 0; t < d.size(); ++t) d[t] = Db[i][t] - Db[0][t];
    const std::vector<double> m = matmul(matmul(V, d, Np, Np, Np), Vi, Np, Np, Np);
    for (int r = 0; r < Np; ++r)
      for (int c = 0; c < Np; ++c) dr[((size_t)(i - 1) * nd.NpP + r) * nd.Kv + c] = m[(size_t)r * Np + c];
  }
  // L_0 on face-local indices
  std::vector<double> L0((size_t)Nfp * Nfp, 0.0);
  for (int a = 0; a < Nfp; ++a) {
    const auto& b = fidx[a];
    L0[(size_t)a * Nfp + a] = 0.5 * ((b[0] + 1) * (b[0] + 1) + (b[1] + 1) * (b[1] + 1) + (b[2] + 1) * (b[2] + 1));
    for (int k = 0; k < 3; ++k)
      for (int m = 0; m < 3; ++m) {
        if (k == m || b[m] == 0) continue;
        int c[3] = {b[0], b[1], b[2]};
        c[k] += 1;
        c[m] -= 1;
        L0[(size_t)a * Nfp + tri_row(c[2], N) + c[1]] += 0.5 * (b[k] + 1) * b[m];
      }
  }
  lift.assign((size_t)nd.NpP * nd.Kl, 0.0);
  for (int f = 0; f < 4; ++f) {
    int fv[3];
    face_verts(f, fv);
    // E_L^f (Np x Nfp): (-1)^{a_f}/(1+a_f) prod_m C(g_m, a_{v_m})
    std::vector<double> EL((size_t)Np * Nfp, 0.0);
    for (int n = 0; n < Np; ++n) {
      const int af = A[n][f];
      const double s = ((af & 1) ? -1.0 : 1.0) / (1.0 + af);
      for (int g = 0; g < Nfp; ++g) {
        double v = s;
        for (int m = 0; m < 3; ++m) v *= binom(fidx[g][m], A[n][fv[m]]);
        EL[(size_t)n * Nfp + g] = v;
      }
    }
    const std::vector<double> Lb = matmul(EL, L0, Np, Nfp, Nfp);
    const std::vector<double> Ln = matmul(matmul(V, Lb, Np, Np, Nfp), Vf, Np, Nfp, Nfp);
    for (int r = 0; r < Np; ++r)
      for (int g = 0; g < Nfp; ++g) lift[(size_t)r * nd.Kl + f * Nfp + g] = Ln[(size_t)r * Nfp + g];
  }
  return true;
}

template <typename T>
bool upload_as(const std::vector<double>& h, void** d) {
  std::vector<T> t(h.begin(), h.end());
  if (hipMalloc(d, t.size() * sizeof(T)) != hipSuccess) return false;
  return hipMemcpy(*d, t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
}

template <typename T>
NodalArgs<T> nodal_args(const bbdg_solver* s) {
  NodalArgs<T> a{};
  a.geo = s->d_geo;
  a.etoe = s->d_etoe;
  a.etofo = s->d_etofo;
  a.tab = s->d_tab;
  a.dr = (const T*)s->d_dr;
  a.lift = (const T*)s->d_lift;
  a.K = s->K;
  a.bc = s->bc;
  return a;
}

void free_solver(bbdg_solver* s) {
  if (!s) return;
  if (s->d_geo) (void)hipFree(s->d_geo);
  if (s->d_etoe) (void)hipFree(s->d_etoe);
  if (s->d_etofo) (void)hipFree(s->d_etofo);
  if (s->d_tab) (void)hipFree(s->d_tab);
  if (s->d_dr) (void)hipFree(s->d_dr);
  if (s->d_lift) (void)hipFree(s->d_lift);
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

static int create_impl(bbdg_solver** out, int N, int dtype, int64_t K, const int32_t* EToE, const int8_t* EToF,
                       const int8_t* EToO, const double* geo, const double* c, int bc, int device, int basis) {
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
  s->basis = basis;

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
  if (ok && basis == 1) {
    std::vector<double> dr, lift;
    if (!nodal_operators(N, dr, lift)) {
      free_solver(s);
      return BBDG_E_ARG;
    }
    ok = dtype == BBDG_F64 ? (upload_as<double>(dr, &s->d_dr) && upload_as<double>(lift, &s->d_lift))
                           : (upload_as<float>(dr, &s->d_dr) && upload_as<float>(lift, &s->d_lift));
  }
  if (!ok) {
    free_solver(s);
    return BBDG_E_DEVICE;
  }
  *out = s;
  return BBDG_OK;
}

int bbdg_create(bbdg_solver** out, int N, int dtype, int64_t K, const int32_t* EToE, const int8_t* EToF,
                const int8_t* EToO, const double* geo, const double* c, int bc, int device) {
  return create_impl(out, N, dtype, K, EToE, EToF, EToO, geo, c, bc, device, 0);
}

int bbdg_nodal_create(bbdg_solver** out, int N, int dtype, int64_t K, const int32_t* EToE, const int8_t* EToF,
                      const int8_t* EToO, const double* geo, const double* c, int bc, int device) {
  return create_impl(out, N, dtype, K, EToE, EToF, EToO, geo, c, bc, device, 1);
}

int bbdg_nodal_operators(int N, double* dr, double* lift) {
  if (N < 1 || N > kMaxOrder) return BBDG_E_ORDER;
  if (!dr || !lift) return BBDG_E_ARG;
  std::vector<double> d, l;
  if (!nodal_operators(N, d, l)) return BBDG_E_ARG;
  const NodalDims nd = nodal_dims(N);
  const int Np = np_of(N), Nfp = nfp_of(N);
  for (int i = 0; i < 3; ++i)
    for (int r = 0; r < Np; ++r)
      for (int c = 0; c < Np; ++c) dr[((size_t)i * Np + r) * Np + c] = d[((size_t)i * nd.NpP + r) * nd.Kv + c];
  for (int r = 0; r < Np; ++r)
    for (int c = 0; c < 4 * Nfp; ++c) lift[(size_t)r * 4 * Nfp + c] = l[(size_t)r * nd.Kl + c];
  return BBDG_OK;
}

int bbdg_basis(const bbdg_solver* s) {
  if (!s) return BBDG_E_ARG;
  return s->basis;
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
  if (s->dtype == BBDG_F64)
    e = launch_any<double>(s, km, (const double*)q, (double*)rhs, nullptr, 0.0, 0.0, 0.0, 0, st);
  else
    e = launch_any<float>(s, km, (const float*)q, (float*)rhs, nullptr, 0.f, 0.f, 0.f, 0, st);
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
