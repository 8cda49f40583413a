// Host driver of the library's CPU-side code, built with g++ under AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py (no GPU, no HIP).  Exercises
// argument validation, the host Gauss rule, the cluster lists, the node cube offsets and
// dV gather lists, and the FE mesh geometry, on ordinary, edge and invalid inputs, and
// checks the invariants each must keep.  Exits 0 when every check holds.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "host.h"
#include "sgq.h"

static int g_fail = 0;
#define CHECK(cond)                                                      \
  do {                                                                   \
    if (!(cond)) {                                                       \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++g_fail;                                                          \
    }                                                                    \
  } while (0)

static sgq_problem problem(int n, int nq, int n_proj, int precision) {
  sgq_problem p{};
  p.n[0] = p.n[1] = p.n[2] = n;
  p.h = 0.5;
  p.n_atoms = 10;
  p.n_proj = n_proj;
  p.proj_rc = 1.5;
  p.proj_rg = 0.5;
  p.n_nodes = nq;
  p.precision = precision;
  return p;
}

static void validation() {
  std::vector<int64_t> c = {0, 5, 64 * 64 * 64 - 1};
  std::vector<int32_t> hw = {16, 16, 0}, K = {60, 1, 128};
  sgq_problem p = problem(64, 3, 4, SGQ_FP32);
  CHECK(sgq_validate(&p, c.data(), hw.data(), K.data()) == SGQ_OK);
  CHECK(sgq_validate(nullptr, c.data(), hw.data(), K.data()) == SGQ_EINVAL);
  CHECK(sgq_validate(&p, nullptr, hw.data(), K.data()) == SGQ_EINVAL);
  CHECK(std::string(sgq_last_error()).size() > 0);
  std::vector<int32_t> bad = {16, 16, 29};           // 59 > 64 - 2*3
  CHECK(sgq_validate(&p, c.data(), bad.data(), K.data()) == SGQ_EINVAL);
  std::vector<int32_t> deep = {60, 129, 1};
  CHECK(sgq_validate(&p, c.data(), hw.data(), deep.data()) == SGQ_EINVAL);
  std::vector<int64_t> out = {0, -1, 3};
  CHECK(sgq_validate(&p, out.data(), hw.data(), K.data()) == SGQ_EINVAL);
  out[1] = 64 * 64 * 64;
  CHECK(sgq_validate(&p, out.data(), hw.data(), K.data()) == SGQ_EINVAL);
  sgq_problem q = problem(16, 1, 0, SGQ_FP64);
  std::vector<int64_t> c1 = {7};
  std::vector<int32_t> whole = {-1}, K1 = {30};
  CHECK(sgq_validate(&q, c1.data(), whole.data(), K1.data()) == SGQ_OK);
  q.h = 0.0;
  CHECK(sgq_validate(&q, c1.data(), whole.data(), K1.data()) == SGQ_EINVAL);
  q = problem(16, 0, 0, SGQ_FP64);
  CHECK(sgq_validate(&q, nullptr, nullptr, nullptr) == SGQ_OK);     // no nodes
  q.precision = 7;
  CHECK(sgq_validate(&q, nullptr, nullptr, nullptr) == SGQ_EINVAL);
  CHECK(sgq::box_half_width(1.5, 0.5) == 3);
}

static void gauss_rule() {
  std::mt19937_64 rng(5);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  for (int K : {1, 2, 3, 17, 64, 127, 128}) {
    std::vector<double> a(K), b(std::max(K - 1, 1)), th(K), w(K);
    for (auto& x : a) x = 3.0 * U(rng);
    for (auto& x : b) x = 0.05 + std::fabs(U(rng));
    CHECK(sgq_gauss_rule_host(a.data(), b.data(), K, th.data(), w.data()) == SGQ_OK);
    double sw = 0.0, swt = 0.0;
    for (int k = 0; k < K; ++k) {
      sw += w[k];
      swt += w[k] * th[k];
      if (k > 0) CHECK(th[k] >= th[k - 1]);
    }
    CHECK(std::fabs(sw - 1.0) < 1e-12);          // weights: squared first components
    CHECK(std::fabs(swt - a[0]) < 1e-11);        // first moment: T_11
  }
  double a[2] = {1.0, 2.0}, b[1] = {0.0}, th[2], w[2];
  CHECK(sgq_gauss_rule_host(a, b, 2, th, w) == SGQ_OK);   // decoupled: theta = a, w = (1, 0)
  CHECK(th[0] == 1.0 && th[1] == 2.0 && w[0] == 1.0 && w[1] == 0.0);
  CHECK(sgq_gauss_rule_host(a, b, 0, th, w) == SGQ_EINVAL);
  CHECK(sgq_gauss_rule_host(a, b, 129, th, w) == SGQ_EINVAL);
  CHECK(sgq_gauss_rule_host(a, nullptr, 2, th, w) == SGQ_EINVAL);
}

static void clusters() {
  const int32_t n[3] = {10, 12, 14};
  std::vector<int64_t> esp = {0, 5 + 10 * (6 + 12 * 7), 10 * 12 * 14 - 1, 3};
  std::vector<double> wt = {1.0, 32.0, 2.5, 4.0};
  int64_t nn = 0, nm = 0;
  CHECK(sgq_cluster_build(n, 0.5, esp.data(), 4, 1.0, wt.data(), 0, 0, nullptr, nullptr, nullptr,
                          nullptr, nullptr, &nn, &nm) == SGQ_OK);
  CHECK(nm == 4 * 33);                              // radius 2h: 33 points per ball
  std::vector<int64_t> nodes(nn), off(5);
  std::vector<int32_t> nesp(nn), mem(nm);
  std::vector<double> nw(nn);
  CHECK(sgq_cluster_build(n, 0.5, esp.data(), 4, 1.0, wt.data(), nn - 1, nm, nodes.data(),
                          nesp.data(), nw.data(), off.data(), mem.data(), &nn, &nm) == SGQ_EINVAL);
  CHECK(sgq_cluster_build(n, 0.5, esp.data(), 4, 1.0, wt.data(), nn, nm, nodes.data(), nesp.data(),
                          nw.data(), off.data(), mem.data(), &nn, &nm) == SGQ_OK);
  CHECK(std::is_sorted(nodes.begin(), nodes.end()));
  CHECK(std::adjacent_find(nodes.begin(), nodes.end()) == nodes.end());
  double total = 0.0;
  for (double x : nw) total += x;
  CHECK(std::fabs(total - (1.0 + 32.0 + 2.5 + 4.0)) < 1e-12);   // sum_p w_p = sum_q n_q
  for (int q = 0; q < 4; ++q) {
    CHECK(off[q + 1] - off[q] == 33);
    bool has_esp = false;
    for (int64_t i = off[q]; i < off[q + 1]; ++i) {
      CHECK(mem[i] >= 0 && mem[i] < nn);
      has_esp = has_esp || nodes[mem[i]] == esp[q];
      if (i > off[q]) CHECK(mem[i] > mem[i - 1]);
    }
    CHECK(has_esp);
  }
  for (int32_t x : nesp) CHECK(x >= 0 && x < 4);
  // a ball wider than the box holds each point once; radius 0 is the ESP alone
  const int32_t small[3] = {3, 3, 3};
  int64_t c0 = 13;
  CHECK(sgq_cluster_build(small, 0.5, &c0, 1, 10.0, nullptr, 0, 0, nullptr, nullptr, nullptr,
                          nullptr, nullptr, &nn, &nm) == SGQ_OK);
  CHECK(nn == 27 && nm == 27);
  CHECK(sgq_cluster_build(small, 0.5, &c0, 1, 0.0, nullptr, 0, 0, nullptr, nullptr, nullptr,
                          nullptr, nullptr, &nn, &nm) == SGQ_OK);
  CHECK(nn == 1 && nm == 1);
  int64_t outside = 27;
  CHECK(sgq_cluster_build(small, 0.5, &outside, 1, 1.0, nullptr, 0, 0, nullptr, nullptr, nullptr,
                          nullptr, nullptr, &nn, &nm) == SGQ_EINVAL);
  CHECK(sgq_cluster_build(small, -0.5, &c0, 1, 1.0, nullptr, 0, 0, nullptr, nullptr, nullptr,
                          nullptr, nullptr, &nn, &nm) == SGQ_EINVAL);
}

static void gather() {
  const int32_t n[3] = {20, 24, 28};
  std::mt19937_64 rng(9);
  std::vector<int32_t> center, hw;
  for (int q = 0; q < 40; ++q) {
    center.push_back((int32_t)(rng() % (20 * 24 * 28)));
    hw.push_back(q == 7 ? -1 : (int32_t)(rng() % 7));
  }
  center.push_back(0);                 // a cube that wraps on every axis
  hw.push_back(3);
  const int64_t ng = 20 * 24 * 28;
  std::vector<int64_t> off = sgq::cube_offsets(hw, ng);
  CHECK(off.size() == hw.size() + 1 && off[0] == 0);
  for (size_t q = 0; q < hw.size(); ++q) {
    const int64_t s = 2 * (int64_t)hw[q] + 1, npt = hw[q] < 0 ? ng : s * s * s;
    CHECK(off[q + 1] - off[q] >= npt && off[q + 1] - off[q] < npt + 4 && off[q + 1] % 4 == 0);
  }
  const int C = 8;
  std::vector<int32_t> start, list;
  sgq::gather_lists(n, center, hw, C, start, list);
  const int ncx = 3, ncy = 3, ncz = 4;
  CHECK((int)start.size() == ncx * ncy * ncz + 1);
  CHECK(start.back() == (int32_t)list.size());
  // every cube point's cell lists the node, once, in ascending node order
  std::vector<std::set<int>> cells(ncx * ncy * ncz);
  for (int k = 0; k < ncx * ncy * ncz; ++k) {
    for (int32_t e = start[k]; e < start[k + 1]; ++e) {
      CHECK(list[e] >= 0 && list[e] < (int)center.size());
      if (e > start[k]) CHECK(list[e] > list[e - 1]);
      cells[k].insert(list[e]);
    }
  }
  for (size_t q = 0; q < center.size(); ++q) {
    const int c = center[q], R = hw[q];
    const int cx = c % 20, cy = (c / 20) % 24, cz = c / (20 * 24);
    if (R < 0) {
      for (auto& s : cells) CHECK(s.count((int)q) == 1);
      continue;
    }
    for (int dz = -R; dz <= R; ++dz)
      for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
          const int x = ((cx + dx) % 20 + 20) % 20, y = ((cy + dy) % 24 + 24) % 24,
                    z = ((cz + dz) % 28 + 28) % 28;
          CHECK(cells[x / C + ncx * (y / C + ncy * (z / C))].count((int)q) == 1);
        }
  }
}

static void fe_mesh() {
  // the six Kuhn tetrahedra of a 4^3 cube on a 6^3 grid, one of them flipped, plus a
  // zero-volume tetrahedron
  const int32_t n[3] = {6, 6, 6};
  auto lin = [](int x, int y, int z) { return (int64_t)x + 6 * (y + 6 * z); };
  std::vector<int64_t> esp;
  for (int z = 0; z <= 1; ++z)
    for (int y = 0; y <= 1; ++y)
      for (int x = 0; x <= 1; ++x) esp.push_back(lin(4 * x, 4 * y, 4 * z));
  esp.push_back(lin(2, 0, 0));                       // on an edge: zero volume with 0, 1
  const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  std::vector<int32_t> tets;
  for (auto& p : perms) {
    int v = 0;
    tets.push_back(0);
    for (int i = 0; i < 3; ++i) {
      v |= 1 << p[i];
      tets.push_back(v);
    }
  }
  std::swap(tets[4], tets[5]);                       // flip the second one
  tets.insert(tets.end(), {0, 1, 8, 2});             // zero volume
  sgq::FeGeometry g;
  CHECK(sgq::fe_geometry(n, esp.data(), (int32_t)esp.size(), tets.data(), 7, 2, &g) == SGQ_OK);
  CHECK(g.kept == 6);
  for (int t = 0; t < 7; ++t) {
    const int32_t* v = g.tet.data() + 4 * t;
    long long D = 0;
    if (t < 6) {
      auto co = [&](int vv, int a) { return (long long)g.esp[4 * vv + a]; };
      long long u[3][3];
      for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 3; ++a) u[k][a] = co(v[k + 1], a) - co(v[0], a);
      D = u[0][0] * (u[1][1] * u[2][2] - u[1][2] * u[2][1]) -
          u[0][1] * (u[1][0] * u[2][2] - u[1][2] * u[2][0]) +
          u[0][2] * (u[1][0] * u[2][1] - u[1][1] * u[2][0]);
      CHECK(D == 64);                                // positively oriented, volume 64/6
    }
  }
  const int64_t nbk = (int64_t)g.nb[0] * g.nb[1] * g.nb[2];
  CHECK((int64_t)g.bstart.size() == nbk + 1);
  for (int64_t b = 0; b < nbk; ++b)
    for (int32_t e = g.bstart[b]; e < g.bstart[b + 1]; ++e) {
      CHECK(g.blist[e] >= 0 && g.blist[e] < 6);
      if (e > g.bstart[b]) CHECK(g.blist[e] > g.blist[e - 1]);
    }
  std::vector<int32_t> badv = {0, 1, 2, 99};
  CHECK(sgq::fe_geometry(n, esp.data(), (int32_t)esp.size(), badv.data(), 1, 2, &g) == SGQ_EINVAL);
  int64_t out_esp = 6 * 6 * 6;
  CHECK(sgq::fe_geometry(n, &out_esp, 1, nullptr, 0, 2, &g) == SGQ_EINVAL);
  CHECK(sgq::fe_geometry(n, esp.data(), (int32_t)esp.size(), tets.data(), 7, 5, &g) == SGQ_EINVAL);
  CHECK(sgq::fe_geometry(n, esp.data(), (int32_t)esp.size(), nullptr, 0, 1, &g) == SGQ_OK);
  CHECK(g.kept == 0);
}

int main() {
  validation();
  gauss_rule();
  clusters();
  gather();
  fe_mesh();
  if (g_fail) {
    std::fprintf(stderr, "%d checks failed\n", g_fail);
    return 1;
  }
  std::printf("host driver: all checks passed\n");
  return 0;
}
