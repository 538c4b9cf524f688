// Runs the library's host-side logic (parameter checks, plan, transport tables,
// tree checks) for a host-only build with AddressSanitizer and
// UndefinedBehaviorSanitizer. The library source is included whole so that the
// internal routines are reachable; no HIP runtime call is made. Exits nonzero
// on a wrong answer; the sanitizers abort on a finding.
#include "../../paper_2103_02903_amd/csrc/mrlbm.hip"

#include <cstdio>
#include <random>

#define EXPECT(x)                                                  \
  do {                                                             \
    if (!(x)) {                                                    \
      std::fprintf(stderr, "expected %s (line %d)\n", #x, __LINE__); \
      return 1;                                                    \
    }                                                              \
  } while (0)

static mrlbm_params base(int scheme, int jmin, int jmax) {
  mrlbm_params p;
  std::memset(&p, 0, sizeof p);
  p.scheme = scheme;
  p.jmin = jmin;
  p.jmax = jmax;
  p.precision = 4;
  p.lambda = scheme == MRLBM_D2Q4_EULER ? 5.0 : 1.0;
  p.eq_param = scheme == MRLBM_D2Q4_EULER ? 1.4 : 0.5;
  p.eps = 1e-3;
  p.mu_bar = 1.0;
  for (int h = 0; h < scheme_q(scheme); ++h) p.s[h] = conserved(scheme, h) ? 0.0 : 1.5;
  return p;
}

int main() {
  std::mt19937_64 gen(7);
  // parameter checks and plans over a sweep of valid and invalid sets
  int ok = 0;
  for (int scheme = 0; scheme <= 6; ++scheme)
    for (int jmin = 0; jmin <= 4; ++jmin)
      for (int jmax : {jmin, jmin + 3, 13, 14, 25, 26})
        for (int g = 0; g <= 4; ++g)
          for (int walls = 0; walls < 3; ++walls) {
            if (scheme < 1 || scheme > 5) {
              mrlbm_params p = base(1, 2, 5);
              p.scheme = scheme;
              size_t b = 0;
              EXPECT(mrlbm_workspace_size(&p, 1, &b) == MRLBM_ERR_INVALID);
              continue;
            }
            mrlbm_params p = base(scheme, jmin, jmax);
            p.gamma = g;
            p.metric = walls == 2 ? MRLBM_METRIC_L2 : MRLBM_METRIC_MAX;
            if (walls) p.bc[0] = p.bc[1] = MRLBM_BOUNCE_BACK;
            if (scheme == MRLBM_D3Q6) p.velocity[0] = 0.3;
            size_t b = 0;
            const int rc = mrlbm_workspace_size(&p, 1, &b);
            EXPECT(rc == MRLBM_OK || rc == MRLBM_ERR_INVALID);
            if (scheme == MRLBM_D3Q6)  // 3D: periodic, gamma = 1, jmax <= 8
              EXPECT((rc == MRLBM_OK) == (jmin >= 1 && jmax <= 8 && g <= 1 && walls == 0));
            if (rc == MRLBM_OK) {
              ++ok;
              EXPECT(b > 0);
              Plan P;
              make_plan(&p, 1, P);
              EXPECT(P.bytes == b);
            }
          }
  EXPECT(ok > 50);
  // a batch of uneven instances
  {
    std::vector<mrlbm_params> ps;
    for (int i = 0; i < 40; ++i) {
      mrlbm_params p = base(MRLBM_D2Q9, 3, 4 + (int)(gen() % 6));
      p.gamma = 2;
      p.metric = (int)(gen() % 2);
      if (i % 3 == 0) p.bc[2] = p.bc[3] = MRLBM_COPY;
      ps.push_back(p);
    }
    size_t b = 0;
    EXPECT(mrlbm_workspace_size(ps.data(), (int)ps.size(), &b) == MRLBM_OK);
    Plan P;
    make_plan(ps.data(), (int)ps.size(), P);
    EXPECT(P.B == 40 && P.gamma == 2 && P.any_walls);
  }
  // transport tables of every scheme, gamma and wall case
  for (int scheme = 1; scheme <= 4; ++scheme)
    for (int g = 1; g <= 3; ++g)
      for (int n = 1; n <= (scheme_dim(scheme) == 2 ? 10 : 16); ++n)
        for (int wc = 0; wc < (scheme_dim(scheme) == 2 ? 9 : 3); ++wc) {
          const int q = scheme_q(scheme), d = scheme_dim(scheme);
          std::vector<double> W((size_t)q * wide_ws(d, g)), C((size_t)q * wide_cs(d, g)), N((size_t)q * 2);
          EXPECT(mrlbm_transport_tables_general(scheme, n, g, wc % 3, wc / 3, W.data(), C.data(), N.data()) ==
                 MRLBM_OK);
          for (double w : W) EXPECT(std::isfinite(w));
        }
  {
    std::vector<double> W(9 * 25), C(9 * 36);
    for (int n = 1; n <= 13; ++n) EXPECT(mrlbm_transport_tables(MRLBM_D2Q9, n, W.data(), C.data()) == MRLBM_OK);
    EXPECT(mrlbm_transport_tables(MRLBM_D2Q9, 14, W.data(), C.data()) == MRLBM_ERR_INVALID);
  }
  // tree checks on trees built by hand: the full coarsest level, one refined
  // group, and a second refinement without its grading box
  for (int g = 1; g <= 3; ++g)
    for (int walls = 0; walls < 2; ++walls) {
      mrlbm_params p = base(MRLBM_D2Q9, 3, 6);
      p.gamma = g;
      if (walls) p.bc[0] = p.bc[1] = p.bc[2] = p.bc[3] = MRLBM_COPY;
      mrlbm_ctx c;
      c.p.assign(1, p);
      make_plan(&p, 1, c.P);
      const Inst<double> &I = c.P.inst[0];
      std::vector<uint8_t> t((size_t)I.total, 0);
      auto at = [&](int l, int x, int y) -> uint8_t & { return t[(size_t)(I.loff[l] - I.cbase + x + ((long long)y << l))]; };
      for (int y = 0; y < 8; ++y)
        for (int x = 0; x < 8; ++x) at(3, x, y) = 1;
      EXPECT(tree_is_graded(&c, 0, t.data()));
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) at(4, 2 * 3 + dx, 2 * 3 + dy) = 1;
      EXPECT(tree_is_graded(&c, 0, t.data()));
      std::vector<uint8_t> old = t;
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) at(5, 2 * 6 + dx, 2 * 6 + dy) = 1;
      // the parent (6, 6) of level 4 needs its box of half-width g at level 4
      EXPECT(!tree_is_graded(&c, 0, t.data()));
      EXPECT(refines_by_one(&c, 0, old.data(), old.data()));
      at(4, 5, 5) = 1;
      EXPECT(!tree_is_graded(&c, 0, t.data()));  // an incomplete sibling group
    }
  std::printf("host checks passed (%d valid parameter sets)\n", ok);
  return 0;
}
