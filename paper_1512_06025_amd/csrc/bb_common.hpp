// Shared sizes and table layout of the Bernstein-Bezier DG kernels.
//
// Coefficient order: alpha = (a0,a1,a2,a3), |alpha| = N, a3 slowest, a2, a1
// fastest.  For a face f with local vertices (v0<v1<v2) a face-local node is
// (g0,g1,g2) = (alpha_v0, alpha_v1, alpha_v2) and face-local order is g2
// slowest, g1 fastest.  The same order describes the degree reductions of a
// face vector: "level j" of face f holds the degree N-j triangle that feeds
// the volume layer alpha_f = j, and the concatenation of all levels has the
// layout of a volume vector seen from face f.  Seen from face 3 this is the
// volume order itself.
#pragma once
#include <stdint.h>

namespace bbdg {

constexpr int kMaxOrder = 9;

constexpr int np_of(int N) { return (N + 1) * (N + 2) * (N + 3) / 6; }
constexpr int nfp_of(int N) { return (N + 1) * (N + 2) / 2; }
constexpr int tri_of(int m) { return (m + 1) * (m + 2) / 2; }
// position of (g1, g2) in a degree-m triangle: rows g2 = 0.. of length m+1-g2
constexpr int tri_row(int g2, int m) { return g2 * (m + 1) - g2 * (g2 - 1) / 2; }
// start of level j (alpha_f = j) in a face-layered volume vector of order N
constexpr int level_off(int j, int N) { return np_of(N) - np_of(N - j); }

// Device geometry per element (double): grad lambda_1, grad lambda_2,
// grad lambda_3 (x,y,z each), kappa = c^2, then for each face f the upwind
// flux weights a_p = kappa |g_f| / (c + c_f) and b_u = (c + c_f) / (4 |g_f|),
// where g_f = -2 grad(lambda_f) and c_f is the wavespeed across face f (the
// element's own c on boundary faces).
constexpr int kGeoStride = 18;

// Derived per-element geometry of Bernstein-Bezier solvers in the element
// type, computed once on the host in double from the header above (rounded
// once in FP32):
// grad lambda_0..3 (12 values; lambda_0 = 1 - lambda_1 - lambda_2 - lambda_3),
// kappa, 3 zeros, then for each face f at 16 + 6 f: g_f = -2 grad(lambda_f)
// (3 values), a_p, kappa / 2, b_u.
constexpr int kTGeoStride = 40;

// Derived per-element geometry of the FP32 reverse (adjoint) stage (float,
// computed on the host in double and rounded): grad lambda_0..3 (12 values),
// kappa, 3 zeros, then for each face f at 16 + 12 f: g_f (3 values), a_p,
// kappa / 2, b_u, F = |g_f|, 1 / F, -a_p / s with s = 4 F b_u, and 3 zeros.
constexpr int kAGeoStride = 64;

// Field arrays are addressed with 32-bit element offsets: 4 K Np < 2^31.
constexpr int64_t kMaxFieldElems = (int64_t)1 << 31;

// uint16 index tables of one order, one contiguous device buffer:
//   alpha   [Np][4]      multi-index components
//   vnbr    [Np][12]     volume index of alpha + e_a - e_b for the pair
//                        p = 3a + (b < a ? b : b - 1); the node itself when
//                        alpha_b = 0 (its weight alpha_b is then zero)
//   fnode   [4][Nfp]     volume index of face-local node g of face f
//   nbrnode [4][6][Nfp]  neighbour's volume index of own face-local node g,
//                        given the neighbour's face f' and orientation code o
//   proj    [Np][4]      position of node alpha in the face-layered vector of
//                        face f: level_off(alpha_f) + tri_row(alpha_v2) + alpha_v1
struct TabLayout {
  int Np, Nfp, alpha, vnbr, fnode, nbrnode, proj, fperm, size;
};

constexpr TabLayout tab_layout(int N) {
  TabLayout t{};
  t.Np = np_of(N);
  t.Nfp = nfp_of(N);
  t.alpha = 0;
  t.vnbr = t.alpha + 4 * t.Np;
  t.fnode = t.vnbr + 12 * t.Np;
  t.nbrnode = t.fnode + 4 * t.Nfp;
  t.proj = t.nbrnode + 24 * t.Nfp;
  t.fperm = t.proj + 4 * t.Np;
  t.size = t.fperm + 6 * t.Nfp;
  return t;
}

// Orientation codes: index of the permutation (pi(0), pi(1), pi(2)).
constexpr int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// Padded sizes of the dense nodal operators: rows to MFMA tiles of 16,
// contraction lengths to multiples of 4.
struct NodalDims {
  int NpP, Kv, Kl;
};
constexpr NodalDims nodal_dims(int N) {
  NodalDims d{};
  d.NpP = (np_of(N) + 15) / 16 * 16;
  d.Kv = (np_of(N) + 3) / 4 * 4;
  d.Kl = (4 * nfp_of(N) + 3) / 4 * 4;
  return d;
}

enum StageMode { kStage = 0, kRhsFull = 1, kRhsVolume = 2, kRhsSurface = 3, kBatched = 4, kBatchedRecord = 5 };

}  // namespace bbdg
