// Specular path finder for 2.5-D scenes: vertical, axis-aligned wall faces
// spanning floor to ceiling, plus one floor plane (z = 0) and one ceiling
// plane (z = H), or open sky above the walls (H <= 0: an urban block whose
// buildings are taller than every path, which then has at most one ground
// reflection).  Such a scene's 3-D specular paths are exactly the 2-D
// specular paths of the floor plan (reflections off wall faces), each
// combined with a sequence of floor/ceiling reflections obtained by
// unfolding the vertical coordinate.
//
// Candidates come from shooting-and-bouncing rays in the plan from the Tx
// (Sec. II-F: candidate primitives from SBR, then exact chains by the image
// method): every ray segment after k bounces that passes within a reception
// radius of an Rx proposes its k-face prefix for that Rx.  Each distinct
// candidate is then validated exactly: the Tx is mirrored across the face
// lines, the path is traced back from the Rx through the images, every
// reflection point must fall inside its face, and every leg must be free of
// wall faces.
//
// Single-bounce diffuse paths (pd_run): per Rx, the surface samples seen
// from both the Tx and the Rx -- each on the front side of the sample's
// surface, the plan segment between them free of wall faces other than the
// sample's own.
//
// C ABI for ctypes: pf_run(...) computes and keeps the result, pf_count()
// and pf_fetch(...) copy it out, pf_free() releases it; pd_run / pd_fetch /
// pd_free likewise for the diffuse samples.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

struct Seg {
  int axis;       // 0: face on x = c (normal along x), 1: face on y = c
  double c;       // plane coordinate
  double lo, hi;  // extent along the other axis
  double nsign;   // +1 / -1: outward normal direction along `axis`
  int mat;
  int face;
};

struct Grid {
  double x0, y0, cell;
  int nx, ny;
  std::vector<int> start, items;  // CSR: cell -> segment ids
};

struct PathRec {
  int depth;
  float pts[8][3];
  float nrm[8][3];
  int mat[8];
  int face[8];
  double length;
};

// Candidate: an Rx and a wall-face prefix of up to kMaxWalls faces.
constexpr int kMaxWalls = 8;
struct Cand {
  int rx;
  int k;
  int f[kMaxWalls];
  bool operator<(const Cand& o) const {
    if (rx != o.rx) return rx < o.rx;
    if (k != o.k) return k < o.k;
    for (int j = 0; j < k; ++j)
      if (f[j] != o.f[j]) return f[j] < o.f[j];
    return false;
  }
  bool operator==(const Cand& o) const {
    if (rx != o.rx || k != o.k) return false;
    for (int j = 0; j < k; ++j)
      if (f[j] != o.f[j]) return false;
    return true;
  }
};

struct Result {
  std::vector<int64_t> off;
  std::vector<PathRec> paths;
};

Result* g_result = nullptr;

struct Diffuse {
  std::vector<int64_t> off;
  std::vector<int32_t> idx;
};

Diffuse* g_diffuse = nullptr;

inline double seg_coord_other(const Seg& s, double x, double y) { return s.axis == 0 ? y : x; }

// Intersection parameter t in (tmin, tmax) of ray o + t d with segment s, or
// -1.  Points on the segment ends count as hits (closed extents).
inline double hit_seg(const Seg& s, double ox, double oy, double dx, double dy, double tmin,
                      double tmax) {
  double o = s.axis == 0 ? ox : oy;
  double d = s.axis == 0 ? dx : dy;
  if (d == 0.0) return -1.0;
  double t = (s.c - o) / d;
  if (!(t > tmin && t < tmax)) return -1.0;
  double u = s.axis == 0 ? oy + t * dy : ox + t * dx;
  if (u < s.lo || u > s.hi) return -1.0;
  return t;
}

Grid build_grid(const std::vector<Seg>& segs, double x0, double y0, double x1, double y1,
                double cell) {
  Grid g;
  g.x0 = x0;
  g.y0 = y0;
  g.cell = cell;
  g.nx = std::max(1, (int)std::ceil((x1 - x0) / cell));
  g.ny = std::max(1, (int)std::ceil((y1 - y0) / cell));
  std::vector<std::vector<int>> lists((size_t)g.nx * g.ny);
  for (int i = 0; i < (int)segs.size(); ++i) {
    const Seg& s = segs[i];
    double ax0, ax1, ay0, ay1;
    if (s.axis == 0) {
      ax0 = ax1 = s.c;
      ay0 = s.lo;
      ay1 = s.hi;
    } else {
      ay0 = ay1 = s.c;
      ax0 = s.lo;
      ax1 = s.hi;
    }
    int cx0 = std::max(0, (int)std::floor((ax0 - x0) / cell - 1e-9));
    int cx1 = std::min(g.nx - 1, (int)std::floor((ax1 - x0) / cell + 1e-9));
    int cy0 = std::max(0, (int)std::floor((ay0 - y0) / cell - 1e-9));
    int cy1 = std::min(g.ny - 1, (int)std::floor((ay1 - y0) / cell + 1e-9));
    for (int cy = cy0; cy <= cy1; ++cy)
      for (int cx = cx0; cx <= cx1; ++cx) lists[(size_t)cy * g.nx + cx].push_back(i);
  }
  g.start.assign((size_t)g.nx * g.ny + 1, 0);
  for (size_t c = 0; c < lists.size(); ++c) g.start[c + 1] = g.start[c] + (int)lists[c].size();
  g.items.reserve(g.start.back());
  for (auto& l : lists) g.items.insert(g.items.end(), l.begin(), l.end());
  return g;
}

// Walk the grid cells along o + t d for t in [0, tmax] (Amanatides-Woo),
// calling f(cell_index, t_enter, t_exit); f returns false to stop.
template <class F>
void walk(const Grid& g, double ox, double oy, double dx, double dy, double tmax, F f) {
  double fx = (ox - g.x0) / g.cell, fy = (oy - g.y0) / g.cell;
  int cx = (int)std::floor(fx), cy = (int)std::floor(fy);
  int sx = dx > 0 ? 1 : (dx < 0 ? -1 : 0);
  int sy = dy > 0 ? 1 : (dy < 0 ? -1 : 0);
  double inf = 1e300;
  double tdx = sx ? g.cell / std::fabs(dx) : inf;
  double tdy = sy ? g.cell / std::fabs(dy) : inf;
  double tnx = sx > 0 ? ((cx + 1) - fx) * g.cell / dx : (sx < 0 ? (fx - cx) * g.cell / -dx : inf);
  double tny = sy > 0 ? ((cy + 1) - fy) * g.cell / dy : (sy < 0 ? (fy - cy) * g.cell / -dy : inf);
  double t = 0.0;
  while (t <= tmax) {
    double tn = std::min(tnx, tny);
    if (cx >= 0 && cy >= 0 && cx < g.nx && cy < g.ny) {
      if (!f(cy * g.nx + cx, t, std::min(tn, tmax))) return;
    } else if ((sx > 0 && cx >= g.nx) || (sx < 0 && cx < 0) || (sy > 0 && cy >= g.ny) ||
               (sy < 0 && cy < 0)) {
      return;
    }
    if (tnx < tny) {
      t = tnx;
      tnx += tdx;
      cx += sx;
    } else {
      t = tny;
      tny += tdy;
      cy += sy;
    }
  }
}

// First segment hit by the ray (excluding `skip`), within (eps, tmax].
int first_hit(const Grid& g, const std::vector<Seg>& segs, double ox, double oy, double dx,
              double dy, double tmax, int skip, double* t_hit) {
  int best = -1;
  double bt = tmax;
  walk(g, ox, oy, dx, dy, tmax, [&](int cell, double t0, double t1) {
    for (int k = g.start[cell]; k < g.start[cell + 1]; ++k) {
      int i = g.items[k];
      if (i == skip) continue;
      double t = hit_seg(segs[i], ox, oy, dx, dy, 1e-9, bt);
      if (t > 0 && t < bt) {
        bt = t;
        best = i;
      }
    }
    return !(best >= 0 && bt <= t1 + 1e-12);
  });
  *t_hit = bt;
  return best;
}

// True if the open segment a->b crosses a wall face other than skip1/skip2.
bool blocked(const Grid& g, const std::vector<Seg>& segs, double ax, double ay, double bx,
             double by, int skip1, int skip2) {
  double dx = bx - ax, dy = by - ay;
  double len = std::sqrt(dx * dx + dy * dy);
  if (len <= 0) return false;
  double ux = dx / len, uy = dy / len;
  bool hit = false;
  const double e = 1e-9;
  walk(g, ax, ay, ux, uy, len, [&](int cell, double, double) {
    for (int k = g.start[cell]; k < g.start[cell + 1]; ++k) {
      int i = g.items[k];
      if (i == skip1 || i == skip2) continue;
      double t = hit_seg(segs[i], ax, ay, ux, uy, e, len - e);
      if (t > 0) {
        hit = true;
        return false;
      }
    }
    return true;
  });
  return hit;
}

inline void mirror(const Seg& s, double& x, double& y) {
  if (s.axis == 0)
    x = 2 * s.c - x;
  else
    y = 2 * s.c - y;
}

// Exact 2-D image-method validation of a face sequence from tx to rx.
// Fills reflection points; returns false if the chain is not a valid path.
bool validate(const Grid& g, const std::vector<Seg>& segs, const int* seq, int k, double tx,
              double ty, double rx, double ry, double* px, double* py) {
  double ix[8], iy[8];
  ix[0] = tx;
  iy[0] = ty;
  for (int j = 0; j < k; ++j) {
    ix[j + 1] = ix[j];
    iy[j + 1] = iy[j];
    mirror(segs[seq[j]], ix[j + 1], iy[j + 1]);
  }
  double cx = rx, cy = ry;
  for (int j = k; j >= 1; --j) {
    const Seg& s = segs[seq[j - 1]];
    double dx = ix[j] - cx, dy = iy[j] - cy;
    double o = s.axis == 0 ? cx : cy;
    double d = s.axis == 0 ? dx : dy;
    if (std::fabs(d) < 1e-12) return false;
    double t = (s.c - o) / d;
    if (!(t > 1e-9 && t < 1 - 1e-9)) return false;
    double qx = cx + t * dx, qy = cy + t * dy;
    double u = s.axis == 0 ? qy : qx;
    if (u < s.lo || u > s.hi) return false;
    // the reflection must happen on the face's free side (outward normal)
    double side = (s.axis == 0 ? cx - s.c : cy - s.c) * s.nsign;
    if (side <= 0) return false;
    px[j - 1] = qx;
    py[j - 1] = qy;
    cx = qx;
    cy = qy;
  }
  // legs tx -> p1 -> ... -> pk -> rx must be unobstructed
  double ax = tx, ay = ty;
  int prev = -1;
  for (int j = 0; j <= k; ++j) {
    double bx = j < k ? px[j] : rx, by = j < k ? py[j] : ry;
    int cur = j < k ? seq[j] : -1;
    if (blocked(g, segs, ax, ay, bx, by, prev, cur)) return false;
    ax = bx;
    ay = by;
    prev = cur;
  }
  return true;
}

}  // namespace

extern "C" {

// walls: n_seg x [axis, c, lo, hi, nsign, mat, face] (doubles)
// Returns total path count (>= 0) or a negative error.
int64_t pf_run(const double* walls, int n_seg, double x0, double y0, double x1, double y1,
               double H, int floor_mat, int floor_face, int ceil_mat, int ceil_face,
               const double* tx, const double* rx, int n_rx, int max_depth, int64_t n_rays,
               double recv_factor, int n_threads, double cell) {
  if (max_depth < 0 || max_depth > kMaxWalls) return -1;
  if (n_threads > 0) omp_set_num_threads(n_threads);
  const bool open_sky = !(H > 0.0);
  std::vector<Seg> segs(n_seg);
  for (int i = 0; i < n_seg; ++i) {
    const double* w = walls + 7 * i;
    segs[i] = Seg{(int)w[0], w[1], w[2], w[3], w[4], (int)w[5], (int)w[6]};
  }
  Grid g = build_grid(segs, x0, y0, x1, y1, cell > 0.0 ? cell : 1.0);
  // Rx grid (CSR) for the reception test
  const double rcell = 1.0;
  Grid rg;
  rg.x0 = x0;
  rg.y0 = y0;
  rg.cell = rcell;
  rg.nx = std::max(1, (int)std::ceil((x1 - x0) / rcell));
  rg.ny = std::max(1, (int)std::ceil((y1 - y0) / rcell));
  {
    std::vector<int> cnt((size_t)rg.nx * rg.ny + 1, 0);
    std::vector<int> cell_of(n_rx);
    for (int r = 0; r < n_rx; ++r) {
      int cx = std::min(rg.nx - 1, std::max(0, (int)std::floor((rx[3 * r] - x0) / rcell)));
      int cy = std::min(rg.ny - 1, std::max(0, (int)std::floor((rx[3 * r + 1] - y0) / rcell)));
      cell_of[r] = cy * rg.nx + cx;
      cnt[cell_of[r] + 1]++;
    }
    for (size_t c = 0; c + 1 < cnt.size(); ++c) cnt[c + 1] += cnt[c];
    rg.start = cnt;
    rg.items.assign(n_rx, 0);
    std::vector<int> fill(cnt.begin(), cnt.end() - 1);
    for (int r = 0; r < n_rx; ++r) rg.items[fill[cell_of[r]]++] = r;
  }
  const double tx2x = tx[0], tx2y = tx[1];
  const double dtheta = 2.0 * M_PI / (double)n_rays;
  const int vmax = max_depth;  // at most max_depth wall reflections
  // ---- 1. SBR in the plan: (rx, prefix code) candidate pairs
  int nthr = omp_get_max_threads();
  std::vector<std::vector<Cand>> cand_thr(nthr);
  const double Lmax = 2.0 * ((x1 - x0) + (y1 - y0)) * 4.0;
#pragma omp parallel
  {
    auto& out = cand_thr[omp_get_thread_num()];
#pragma omp for schedule(dynamic, 1024)
    for (int64_t ri = 0; ri < n_rays; ++ri) {
      double th = ((double)ri + 0.5) * dtheta;
      double ox = tx2x, oy = tx2y, dx = std::cos(th), dy = std::sin(th);
      double Lpre = 0.0;
      int skip = -1;
      Cand cur;
      cur.k = 0;
      for (int k = 0; k <= vmax; ++k) {
        double thit;
        int hs = first_hit(g, segs, ox, oy, dx, dy, Lmax, skip, &thit);
        double seg_len = hs >= 0 ? thit : Lmax;
        // reception: Rx within r of this segment (three parallel cell walks)
        double rr = recv_factor * dtheta * (Lpre + seg_len);
        if (rr > 0.45 * rcell) rr = 0.45 * rcell;
        double nxp = -dy, nyp = dx;
        for (int off = -1; off <= 1; ++off) {
          double sx0 = ox + off * rr * nxp, sy0 = oy + off * rr * nyp;
          walk(rg, sx0, sy0, dx, dy, seg_len, [&](int cell, double, double) {
            for (int q = rg.start[cell]; q < rg.start[cell + 1]; ++q) {
              int r = rg.items[q];
              double vx = rx[3 * r] - ox, vy = rx[3 * r + 1] - oy;
              double t = vx * dx + vy * dy;
              if (t < 0 || t > seg_len) continue;
              double px = vx - t * dx, py = vy - t * dy;
              double rloc = recv_factor * dtheta * (Lpre + t);
              if (px * px + py * py <= rloc * rloc + 1e-18) {
                cur.rx = r;
                out.push_back(cur);
              }
            }
            return true;
          });
        }
        if (hs < 0 || k == vmax) break;
        // reflect
        cur.f[k] = hs;
        cur.k = k + 1;
        ox += thit * dx;
        oy += thit * dy;
        Lpre += thit;
        if (segs[hs].axis == 0)
          dx = -dx;
        else
          dy = -dy;
        skip = hs;
      }
    }
  }
  std::vector<Cand> cand;
  {
    size_t tot = 0;
    for (auto& v : cand_thr) tot += v.size();
    cand.reserve(tot + n_rx);
    for (auto& v : cand_thr) {
      cand.insert(cand.end(), v.begin(), v.end());
      std::vector<Cand>().swap(v);
    }
    for (int r = 0; r < n_rx; ++r) {  // line of sight
      Cand c;
      c.rx = r;
      c.k = 0;
      cand.push_back(c);
    }
  }
  std::sort(cand.begin(), cand.end());
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  std::vector<int64_t> cstart(n_rx + 1, 0);
  for (auto& c : cand) cstart[c.rx + 1]++;
  for (int r = 0; r < n_rx; ++r) cstart[r + 1] += cstart[r];

  // ---- 2. exact validation + vertical unfolding, per Rx
  std::vector<std::vector<PathRec>> per_rx(n_rx);
#pragma omp parallel for schedule(dynamic, 16)
  for (int r = 0; r < n_rx; ++r) {
    auto& out = per_rx[r];
    const double rxx = rx[3 * r], rxy = rx[3 * r + 1], rxz = rx[3 * r + 2];
    for (int64_t ci = cstart[r]; ci < cstart[r + 1]; ++ci) {
      const Cand& cd = cand[ci];
      int k = cd.k;
      int seq[kMaxWalls];
      for (int j = 0; j < k; ++j) seq[j] = cd.f[j];
      double px[8], py[8];
      if (!validate(g, segs, seq, k, tx2x, tx2y, rxx, rxy, px, py)) continue;
      // cumulative plan distance of each wall reflection
      double s_wall[8], S = 0.0;
      {
        double ax = tx2x, ay = tx2y;
        for (int j = 0; j < k; ++j) {
          S += std::hypot(px[j] - ax, py[j] - ay);
          s_wall[j] = S;
          ax = px[j];
          ay = py[j];
        }
        S += std::hypot(rxx - ax, rxy - ay);
      }
      // floor/ceiling sequences: kh reflections starting with the floor
      // (first = 0) or the ceiling (first = 1); under open sky at most one,
      // off the ground
      const int kh_max = open_sky ? std::min(1, max_depth - k) : max_depth - k;
      for (int kh = 0; kh <= kh_max; ++kh) {
        for (int first = 0; first < (kh == 0 || open_sky ? 1 : 2); ++first) {
          // unfolded Rx height and the crossed boundaries
          double zi;
          double bnd[8];
          if (kh == 0) {
            zi = rxz;
          } else if (open_sky) {  // the ground's image of the Rx
            zi = -rxz;
            bnd[0] = 0.0;
          } else if (first == 0) {  // down: copies below z = 0
            // copy n (1..kh) spans [-nH, -(n-1)H]
            zi = (kh % 2 == 1) ? -(kh - 1) * H - rxz : -kh * H + rxz;
            for (int n = 0; n < kh; ++n) bnd[n] = -n * H;
          } else {  // up: copies above z = H
            zi = (kh % 2 == 1) ? (kh + 1) * H - rxz : kh * H + rxz;
            for (int n = 0; n < kh; ++n) bnd[n] = (n + 1) * H;
          }
          double zt = tx[2];
          PathRec pr;
          pr.depth = k + kh;
          pr.length = std::sqrt(S * S + (zi - zt) * (zi - zt));
          // events: wall reflections at s_wall[j], z reflections at s_z[n]
          double s_z[8];
          for (int n = 0; n < kh; ++n) s_z[n] = S * (bnd[n] - zt) / (zi - zt);
          int a = 0, b = 0, e = 0;
          while (a < k || b < kh) {
            bool take_wall = b >= kh || (a < k && s_wall[a] < s_z[b]);
            double s = take_wall ? s_wall[a] : s_z[b];
            // plan position at arc length s
            double qx, qy;
            {
              double ax = tx2x, ay = tx2y, acc = 0.0;
              int j = 0;
              for (; j < k; ++j) {
                double L = s_wall[j] - acc;
                if (s <= s_wall[j]) break;
                acc = s_wall[j];
                ax = px[j];
                ay = py[j];
                (void)L;
              }
              double bx = j < k ? px[j] : rxx, by = j < k ? py[j] : rxy;
              double seglen = (j < k ? s_wall[j] : S) - acc;
              double f = seglen > 0 ? (s - acc) / seglen : 0.0;
              qx = ax + f * (bx - ax);
              qy = ay + f * (by - ay);
            }
            double zu = zt + (zi - zt) * (s / S);
            // fold the unfolded height back into [0, H] (mirror at z = 0
            // under open sky)
            double zf;
            if (open_sky) {
              zf = std::fabs(zu);
            } else {
              zf = std::fmod(zu, 2 * H);
              if (zf < 0) zf += 2 * H;
              if (zf > H) zf = 2 * H - zf;
            }
            if (take_wall) {
              const Seg& sg = segs[seq[a]];
              pr.pts[e][0] = (float)qx;
              pr.pts[e][1] = (float)qy;
              pr.pts[e][2] = (float)zf;
              pr.nrm[e][0] = (float)(sg.axis == 0 ? sg.nsign : 0.0);
              pr.nrm[e][1] = (float)(sg.axis == 1 ? sg.nsign : 0.0);
              pr.nrm[e][2] = 0.0f;
              pr.mat[e] = sg.mat;
              pr.face[e] = sg.face;
              ++a;
            } else {
              bool is_floor =
                  open_sky || std::fabs(std::fmod(std::fabs(bnd[b]), 2 * H)) < 0.5 * H;
              pr.pts[e][0] = (float)qx;
              pr.pts[e][1] = (float)qy;
              pr.pts[e][2] = (float)(is_floor ? 0.0 : H);
              pr.nrm[e][0] = 0.0f;
              pr.nrm[e][1] = 0.0f;
              pr.nrm[e][2] = is_floor ? 1.0f : -1.0f;
              pr.mat[e] = is_floor ? floor_mat : ceil_mat;
              pr.face[e] = is_floor ? floor_face : ceil_face;
              ++b;
            }
            ++e;
          }
          out.push_back(pr);
        }
      }
    }
    // deterministic order: (depth, face sequence, length)
    std::sort(out.begin(), out.end(), [](const PathRec& x, const PathRec& y) {
      if (x.depth != y.depth) return x.depth < y.depth;
      for (int j = 0; j < x.depth; ++j)
        if (x.face[j] != y.face[j]) return x.face[j] < y.face[j];
      return x.length < y.length;
    });
  }
  delete g_result;
  g_result = new Result();
  g_result->off.assign(n_rx + 1, 0);
  for (int r = 0; r < n_rx; ++r) g_result->off[r + 1] = g_result->off[r] + (int64_t)per_rx[r].size();
  g_result->paths.reserve(g_result->off[n_rx]);
  for (int r = 0; r < n_rx; ++r) {
    g_result->paths.insert(g_result->paths.end(), per_rx[r].begin(), per_rx[r].end());
    std::vector<PathRec>().swap(per_rx[r]);
  }
  return g_result->off[n_rx];
}

// Copy the result into interaction-major arrays (see synth/store.py).
int pf_fetch(int max_depth, int64_t* link_off, uint8_t* depth, float* pts, float* nrm,
             uint16_t* mat, int32_t* face, double* length) {
  if (!g_result) return -1;
  const int64_t P = (int64_t)g_result->paths.size();
  const int64_t n_links = (int64_t)g_result->off.size() - 1;
  std::memcpy(link_off, g_result->off.data(), sizeof(int64_t) * (n_links + 1));
  const int64_t DP = (int64_t)max_depth * P;
  for (int64_t p = 0; p < P; ++p) {
    const PathRec& r = g_result->paths[p];
    depth[p] = (uint8_t)r.depth;
    length[p] = r.length;
    for (int k = 0; k < max_depth; ++k) {
      int64_t i = (int64_t)k * P + p;
      bool on = k < r.depth;
      for (int c = 0; c < 3; ++c) {
        pts[c * DP + i] = on ? r.pts[k][c] : 0.0f;
        nrm[c * DP + i] = on ? r.nrm[k][c] : 0.0f;
      }
      mat[i] = on ? (uint16_t)r.mat[k] : 0;
      face[i] = on ? r.face[k] : -1;
    }
  }
  return 0;
}

void pf_free() {
  delete g_result;
  g_result = nullptr;
}

// Diffuse samples: points spts [n_s][3] with unit normals snrm [n_s][3] and
// the wall segment they lie on, sseg [n_s] (-1 for ground samples, which
// face +z).  For the Tx tx[3] and every Rx rx[n_rx][3], the samples with
// both end points strictly on their front side and both plan segments free
// of wall faces (other than the sample's own).  Returns the number of
// (Rx, sample) pairs; pd_fetch copies the CSR (off [n_rx+1], idx).
int64_t pd_run(const double* walls, int n_seg, double x0, double y0, double x1, double y1,
               const double* spts, const double* snrm, const int* sseg, int n_s,
               const double* tx, const double* rx, int n_rx, int n_threads, double cell) {
  if (n_threads > 0) omp_set_num_threads(n_threads);
  std::vector<Seg> segs(n_seg);
  for (int i = 0; i < n_seg; ++i) {
    const double* w = walls + 7 * i;
    segs[i] = Seg{(int)w[0], w[1], w[2], w[3], w[4], (int)w[5], (int)w[6]};
  }
  Grid g = build_grid(segs, x0, y0, x1, y1, cell > 0.0 ? cell : 1.0);
  auto front = [&](int s, const double* e) {
    const double* p = spts + 3 * s;
    const double* n = snrm + 3 * s;
    return (e[0] - p[0]) * n[0] + (e[1] - p[1]) * n[1] + (e[2] - p[2]) * n[2] > 0.0;
  };
  auto seen = [&](int s, const double* e) {
    const double* p = spts + 3 * s;
    return !blocked(g, segs, e[0], e[1], p[0], p[1], sseg[s], -1);
  };
  std::vector<int> vis_tx;
  {
    std::vector<char> v(n_s, 0);
#pragma omp parallel for schedule(dynamic, 256)
    for (int s = 0; s < n_s; ++s) v[s] = front(s, tx) && seen(s, tx);
    for (int s = 0; s < n_s; ++s)
      if (v[s]) vis_tx.push_back(s);
  }
  std::vector<std::vector<int32_t>> per_rx(n_rx);
#pragma omp parallel for schedule(dynamic, 4)
  for (int r = 0; r < n_rx; ++r) {
    const double* e = rx + 3 * r;
    for (int s : vis_tx)
      if (front(s, e) && seen(s, e)) per_rx[r].push_back(s);
  }
  delete g_diffuse;
  g_diffuse = new Diffuse();
  g_diffuse->off.assign(n_rx + 1, 0);
  for (int r = 0; r < n_rx; ++r) g_diffuse->off[r + 1] = g_diffuse->off[r] + per_rx[r].size();
  g_diffuse->idx.reserve(g_diffuse->off[n_rx]);
  for (int r = 0; r < n_rx; ++r) {
    g_diffuse->idx.insert(g_diffuse->idx.end(), per_rx[r].begin(), per_rx[r].end());
    std::vector<int32_t>().swap(per_rx[r]);
  }
  return g_diffuse->off[n_rx];
}

int pd_fetch(int64_t* off, int32_t* idx) {
  if (!g_diffuse) return -1;
  std::memcpy(off, g_diffuse->off.data(), sizeof(int64_t) * g_diffuse->off.size());
  std::memcpy(idx, g_diffuse->idx.data(), sizeof(int32_t) * g_diffuse->idx.size());
  return 0;
}

void pd_free() {
  delete g_diffuse;
  g_diffuse = nullptr;
}

}  // extern "C"
