// Kac-Ward plan builder (host only): the planar embedding of the bit-flip
// Ising model of the rotated surface code and the entries of its Kac-Ward
// matrix.  See kw_plan.hpp.
#include "kw_plan.hpp"

#include <cmath>
#include <cstring>
#include <map>
#include <utility>

namespace tnmld {

namespace {

bool xcheck(int d, int r, int c) {
  if (((r + c) & 1) != 0) return false;
  const bool bulk = r >= 0 && c >= 0 && r <= d - 2 && c <= d - 2;
  const bool tb = (r == -1 || r == d - 1) && c >= 0 && c <= d - 2;
  return bulk || tb;
}

// angle turned from direction a to direction b, in (-pi, pi]
double turn(double a, double b) {
  double t = std::fmod(b - a + M_PI, 2.0 * M_PI);
  if (t < 0) t += 2.0 * M_PI;
  return t - M_PI;
}

struct Pt {
  double x, y;
};

}  // namespace

std::string build_kw_plan(int d, KwPlan* out) {
  if (d < 3 || d > 31 || d % 2 == 0) return "d must be odd, 3 <= d <= 31";
  const int n = d * d, m = n - 1;
  // vertices: X-type checks at their corner centres, the two ghosts
  std::map<std::pair<int, int>, int> vid;
  std::vector<Pt> pos;
  for (int r = -1; r <= d - 1; ++r)
    for (int c = -1; c <= d - 1; ++c)
      if (xcheck(d, r, c)) {
        vid[{r, c}] = (int)pos.size();
        pos.push_back({c + 0.5, -(r + 0.5)});
      }
  const int mx = (int)pos.size();
  if (mx != m / 2) return "internal: X-type check count";
  const double ymid = -(d - 1) / 2.0;
  const int gl = (int)pos.size();
  pos.push_back({-2.0, ymid});
  const int gr = (int)pos.size();
  pos.push_back({d + 1.0, ymid});
  // undirected edges as polylines: qubit q (checks, or check and ghost through
  // a bend point beyond the boundary), then the ghost bond over the top
  struct Edge {
    int u, v;
    std::vector<Pt> pts;  // from u to v, including both ends
  };
  std::vector<Edge> E;
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c) {
      int cand[2][2];
      if (((r + c) & 1) == 0) {
        cand[0][0] = r - 1, cand[0][1] = c - 1, cand[1][0] = r, cand[1][1] = c;
      } else {
        cand[0][0] = r - 1, cand[0][1] = c, cand[1][0] = r, cand[1][1] = c - 1;
      }
      int ex[2], k = 0;
      for (int i = 0; i < 2; ++i)
        if (xcheck(d, cand[i][0], cand[i][1])) ex[k++] = vid[{cand[i][0], cand[i][1]}];
      if (k == 2) {
        E.push_back({ex[0], ex[1], {pos[ex[0]], pos[ex[1]]}});
      } else if (k == 1 && (c == 0 || c == d - 1)) {
        const bool left = c == 0;
        const Pt bendp{left ? -0.5 : d - 0.5, (double)-r};
        const int g = left ? gl : gr;
        E.push_back({ex[0], g, {pos[ex[0]], bendp, pos[g]}});
      } else {
        return "internal: qubit without a bond";
      }
    }
  E.push_back({gl, gr, {pos[gl], {-2.0, 3.0}, {d + 1.0, 3.0}, pos[gr]}});
  const int ne = (int)E.size(), N = 2 * ne;
  if (ne != n + 1) return "internal: edge count";
  // directed edges: start / end direction and the turning inside the edge
  std::vector<int> tail(N), head(N);
  std::vector<double> sdir(N), edir(N), bend(N);
  for (int e = 0; e < ne; ++e) {
    for (int rev = 0; rev < 2; ++rev) {
      std::vector<Pt> p = E[e].pts;
      if (rev) p.assign(E[e].pts.rbegin(), E[e].pts.rend());
      std::vector<double> dir;
      for (size_t i = 0; i + 1 < p.size(); ++i) dir.push_back(std::atan2(p[i + 1].y - p[i].y, p[i + 1].x - p[i].x));
      double b = 0.0;
      for (size_t i = 0; i + 1 < dir.size(); ++i) b += turn(dir[i], dir[i + 1]);
      const int a = 2 * e + rev;
      tail[a] = rev ? E[e].v : E[e].u;
      head[a] = rev ? E[e].u : E[e].v;
      sdir[a] = dir.front();
      edir[a] = dir.back();
      bend[a] = b;
    }
  }
  std::vector<std::vector<int>> outg(pos.size());
  for (int a = 0; a < N; ++a) outg[tail[a]].push_back(a);
  std::vector<KwEntry> ent;
  for (int a = 0; a < N; ++a)
    for (int b : outg[head[a]]) {
      if (b == (a ^ 1)) continue;
      const double phi = 0.5 * (turn(edir[a], sdir[b]) + bend[b]);
      KwEntry z{};
      z.row = (int16_t)a;
      z.col = (int16_t)b;
      z.edge = (int16_t)(b >> 1);
      z.re = std::cos(phi);
      z.im = std::sin(phi);
      ent.push_back(z);
    }
  // Z-type checks (syndrome bits 0 .. m/2 - 1): X string on column max(c, 0), rows 0..r
  std::vector<int8_t> zc;
  for (int r = -1; r <= d - 1; ++r)
    for (int c = -1; c <= d - 1; ++c) {
      const bool is_x = ((r + c) & 1) == 0;
      if (is_x) continue;
      const bool bulk = r >= 0 && c >= 0 && r <= d - 2 && c <= d - 2;
      const bool lr = (c == -1 || c == d - 1) && r >= 0 && r <= d - 2;
      if (!(bulk || lr)) continue;
      zc.push_back((int8_t)(c < 0 ? 0 : c));
      zc.push_back((int8_t)r);
    }
  if ((int)zc.size() != m) return "internal: Z-type check count";

  KwHeader h{};
  h.d = d;
  h.n = n;
  h.m = m;
  h.mx = mx;
  h.ne = ne;
  h.N = N;
  h.ld = (N + 15) / 16 * 16;
  h.nnz = (int)ent.size();
  h.log_pref = (double)(mx - n) * std::log(2.0);
  auto align8 = [](size_t x) { return (x + 7) / 8 * 8; };
  size_t off = align8(sizeof(KwHeader));
  h.nz_ofs = (int32_t)off;
  off = align8(off + ent.size() * sizeof(KwEntry));
  h.zcheck_ofs = (int32_t)off;
  off = align8(off + zc.size());
  h.bytes = (int32_t)off;
  out->h = h;
  out->blob.assign(off, 0);
  std::memcpy(out->blob.data(), &h, sizeof(h));
  std::memcpy(out->blob.data() + h.nz_ofs, ent.data(), ent.size() * sizeof(KwEntry));
  std::memcpy(out->blob.data() + h.zcheck_ofs, zc.data(), zc.size());
  return "";
}

}  // namespace tnmld
