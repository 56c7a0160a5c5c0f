// Host-side checks of libpft under AddressSanitizer and UndefinedBehaviorSanitizer (host code only):
// the edge-sharing face order on random and broken meshes, and every entry point's synchronous
// argument validation (each call below returns before any GPU work). Exits non-zero on a failed check.
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "pft.h"

static int failures = 0;
#define CHECK(c)                                                           \
  do {                                                                     \
    if (!(c)) {                                                            \
      std::fprintf(stderr, "check failed (line %d): %s\n", __LINE__, #c); \
      ++failures;                                                          \
    }                                                                      \
  } while (0)

static void check_order(const std::vector<int32_t>& tris, int64_t nf, int64_t nv) {
  std::vector<int32_t> order(nf > 0 ? nf : 1);
  std::vector<uint8_t> meta(nf > 0 ? nf : 1);
  CHECK(pft_strip_order(tris.data(), nf, nv, order.data(), meta.data()) == PFT_OK);
  // traversal of position i: rotation r, then (b, a, c) when reversed (bit 3)
  auto trav = [&](int64_t i, int32_t* v) {
    const int32_t* f = &tris[3 * (int64_t)order[i]];
    const int r = meta[i] & 3;
    const bool rev = (meta[i] & 8) != 0;
    v[0] = f[(r + (rev ? 1 : 0)) % 3];
    v[1] = f[(r + (rev ? 0 : 1)) % 3];
    v[2] = f[(r + 2) % 3];
  };
  std::vector<int> seen(nf, 0);
  for (int64_t i = 0; i < nf; ++i) {
    CHECK(order[i] >= 0 && order[i] < nf);
    if (order[i] >= 0 && order[i] < nf) ++seen[order[i]];
    CHECK((meta[i] & 3) < 3 && (meta[i] & ~15) == 0);
    if ((meta[i] & 4) && i > 0) {  // edge 0 of this face is edge 1 of the previous face
      int32_t a[3], b[3];
      trav(i, a);
      trav(i - 1, b);
      CHECK((a[0] == b[1] && a[1] == b[2]) || (a[0] == b[2] && a[1] == b[1]));
    }
  }
  for (int64_t f = 0; f < nf; ++f) CHECK(seen[f] == 1);
}

int main() {
  std::mt19937 rng(7);
  // a closed strip of a cylinder: a grid of quads split into triangles
  for (int n : {1, 3, 17, 200}) {
    std::vector<int32_t> t;
    const int m = 12;
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < m; ++c) {
        const int a = r * m + c, b = r * m + (c + 1) % m, d = (r + 1) * m + c, e = (r + 1) * m + (c + 1) % m;
        t.insert(t.end(), {a, b, e, a, e, d});
      }
    check_order(t, (int64_t)t.size() / 3, (int64_t)(n + 1) * m);
  }
  // random indices, out-of-range and repeated ones, and faces repeated many times (non-manifold edges)
  for (int trial = 0; trial < 20; ++trial) {
    const int nv = 1 + (int)(rng() % 50), nf = (int)(rng() % 300);
    std::vector<int32_t> t(3 * (size_t)nf);
    for (auto& x : t) x = (int32_t)(rng() % (nv + 3)) - 1;
    check_order(t, nf, nv);
  }
  check_order({}, 0, 0);
  // the closed-mesh check on the same kinds of input (random, broken, empty)
  for (int trial = 0; trial < 10; ++trial) {
    const int nv = 1 + (int)(rng() % 40), nf = (int)(rng() % 200);
    std::vector<int32_t> t(3 * (size_t)nf);
    for (auto& x : t) x = (int32_t)(rng() % (nv + 3)) - 1;
    pft_mesh_check c;
    CHECK(pft_check_mesh(t.data(), nf, nv, &c) == PFT_OK);
    CHECK(c.bad_index >= 0 && c.open_edges >= 0 && c.nonmanifold_edges >= 0 && c.misoriented_edges >= 0);
  }
  {
    pft_mesh_check c;
    const int32_t tet[12] = {0, 2, 1, 0, 1, 3, 0, 3, 2, 1, 2, 3};
    CHECK(pft_check_mesh(tet, 4, 4, &c) == PFT_OK);
    CHECK(c.bad_index == 0 && c.open_edges == 0 && c.nonmanifold_edges == 0 && c.misoriented_edges == 0);
    CHECK(pft_check_mesh(tet, 3, 4, &c) == PFT_OK && c.open_edges == 3);
    CHECK(pft_check_mesh(nullptr, 2, 4, &c) == PFT_EINVAL);
    // the FP32C |Q| bound: a regular tetrahedron of circumradius 1 has faces of extent sqrt(8)/3
    const double a = 1.0 / std::sqrt(3.0);
    const double tv[12] = {a, a, a, a, -a, -a, -a, a, -a, -a, -a, a};
    double lim = 0.0;
    CHECK(pft_fp32c_q_limit(tv, PFT_F64, 4, tet, 4, &lim) == PFT_OK);
    CHECK(std::fabs(lim - PFT_FP32C_PHASE_MAX / (std::sqrt(8.0) / 3.0)) < 1e-12 * lim);
    const int32_t tet_bad[12] = {0, 2, 1, 0, 1, 3, 0, 3, 2, 1, 2, 40};
    CHECK(pft_fp32c_q_limit(tv, PFT_F64, 4, tet_bad, 4, &lim) == PFT_OK);
    CHECK(pft_fp32c_q_limit(tv, PFT_F64, 4, tet, 4, nullptr) == PFT_EINVAL);
    CHECK(pft_fp32c_q_limit(nullptr, PFT_F64, 0, nullptr, 0, &lim) == PFT_OK && std::isinf(lim));
  }
  CHECK(pft_strip_order(nullptr, 3, 3, nullptr, nullptr) == PFT_EINVAL);
  CHECK(pft_strip_order(nullptr, -1, 3, nullptr, nullptr) == PFT_EINVAL);

  // synchronous validation paths (no GPU work is reached)
  void* g = reinterpret_cast<void*>(0x10000);
  CHECK(pft_forward_3d(g, PFT_F64, -1, (const int32_t*)g, 1, g, PFT_F64, 4, PFT_FP64, g, nullptr, nullptr) ==
        PFT_EINVAL);
  CHECK(pft_forward_3d(g, PFT_F64, 3, (const int32_t*)g, 1, g, PFT_F64, 0, PFT_FP64, nullptr, nullptr, nullptr) ==
        PFT_OK);
  CHECK(pft_backward_3d(g, PFT_F64, 3, (const int32_t*)g, 1, g, PFT_F64, 4, PFT_FP64, nullptr, g, nullptr) ==
        PFT_EINVAL);
  const int64_t off_bad[3] = {0, 5, 3};
  CHECK(pft_forward_3d_poly(g, PFT_F64, 8, off_bad, (const int32_t*)g, 2, g, PFT_F64, 4, PFT_FP64, g, nullptr,
                            nullptr) == PFT_EINVAL);
  const int64_t reg_short[3] = {0, 4, 9};
  CHECK(pft_forward_3d_regions(g, PFT_F64, 8, (const int32_t*)g, 10, reg_short, 2, (const double*)g, g, PFT_F64, 4,
                               PFT_FP32C, g, nullptr, nullptr, nullptr, nullptr, nullptr) == PFT_EINVAL);
  CHECK(pft_q_order(g, PFT_F64, -1, (uint32_t*)g, nullptr) == PFT_EINVAL);
  CHECK(pft_intensity_loss_3d(g, PFT_F64, 8, (const int32_t*)g, 12, g, PFT_F64, 4, PFT_FP32C, nullptr,
                              (const double*)g, nullptr, nullptr, g, nullptr, nullptr, nullptr) == PFT_EINVAL);
  CHECK(pft_batch_forward(nullptr, PFT_FP64, g, nullptr, nullptr) == PFT_EINVAL);
  int64_t bad = 7, rep = 7;
  CHECK(pft_validate_mesh(nullptr, -1, 3, &bad, &rep, nullptr) == PFT_EINVAL);
  CHECK(pft_last_error() != nullptr && pft_version() != nullptr);
  if (failures) std::fprintf(stderr, "%d checks failed\n", failures);
  else std::printf("host checks passed\n");
  return failures ? 1 : 0;
}
