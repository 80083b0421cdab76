// Seeded synthetic transparent scenes rasterised to per-pixel fragment lists (CSR).
//
// This module only produces INPUTS: triangles, a camera path, and the fragment
// lists a rasteriser would emit for them. It holds none of the compositing
// method's arithmetic, and both the CPU oracle and the GPU library consume its
// output as plain data.
//
// Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014). Every triangle, camera pose and shuffle is a
// pure function of (seed, stream, index), so any frame can be regenerated alone.
//
// Rasterisation rule: pixel centres at (x+0.5, y+0.5); vertices snapped to 1/256
// px; integer edge functions with a direction-antisymmetric tie rule, so a shared
// edge covers each pixel exactly once and a primitive emits at most one fragment
// per pixel. Depth is NDC z in [0,1], affine in screen space across a triangle.
// Within a pixel the list is in primitive order, optionally shuffled per pixel.
// Lists longer than max_per_pixel keep their max_per_pixel nearest fragments by
// (depth, primitive id); the rest are dropped and counted.

#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <cmath>
#include <vector>
#include <algorithm>

namespace {

inline uint64_t splitmix64(uint64_t& s) {
  s += 0x9E3779B97F4A7C15ull;
  uint64_t z = s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct Rng {
  uint64_t s;
  Rng(uint64_t seed, uint64_t stream, uint64_t index) {
    s = seed;
    uint64_t a = splitmix64(s) ^ (stream * 0xD1B54A32D192ED03ull);
    s = a;
    uint64_t b = splitmix64(s) ^ (index * 0x8CB92BA72F3D8DD7ull);
    s = b;
    splitmix64(s);
  }
  uint64_t next() { return splitmix64(s); }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
  double uniform(double lo, double hi) { return lo + (hi - lo) * uniform(); }
  double normal() {  // Box-Muller
    double u1 = uniform(), u2 = uniform();
    if (u1 < 1e-300) u1 = 1e-300;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

enum : uint64_t { ST_TRI = 1, ST_CAM = 2, ST_MOVE = 3, ST_SHUF = 4, ST_CLUSTER = 5 };

}  // namespace

extern "C" {

typedef struct {
  int32_t kind;            // 0 screen-space triangles, 1 world-space + perspective camera
  int32_t width, height;
  int32_t num_tris;        // static triangles
  int32_t num_moving;      // extra triangles with per-frame rigid motion (kind 1)
  int32_t num_frames;
  uint32_t max_per_pixel;  // 0 = unlimited
  int32_t shuffle;         // 1 = seeded per-pixel permutation of each list
  uint64_t seed;
  double alpha_lo, alpha_hi;
  double size_mu, size_sigma;   // kind 1: log-normal triangle radius (fraction of view depth)
  int32_t clusters;             // kind 1: number of cluster centres
  double cluster_frac;          // fraction of triangles drawn around cluster centres
  double cluster_radius;        // cluster spread (fraction of view depth)
  double depth_lo, depth_hi;    // kind 1: view-space distance range of triangle centres
  double fov_y_deg, z_near, z_far;
  double cam_rot_deg, cam_trans;    // per-frame camera motion bounds
  double move_rot_deg, move_trans;  // per-frame rigid motion bounds of moving triangles
  int32_t colour_mode;          // 0 iid U[0,1]; 1 colour correlated with depth; 2 object palette
  int32_t half_rgba;            // informational: caller stores RGBA as fp16
} sg_params;

typedef struct {
  uint64_t num_frags;
  uint64_t trimmed;
  uint32_t max_count;
  double mean_count;       // over all pixels
  uint32_t p99_count;
  uint32_t covered_pixels;
  uint32_t dropped_tris;   // triangles not drawn (behind the camera or outside depth range)
} sg_stats;

struct sg_scene;
}

struct Tri {
  double v[3][3];      // world (kind 1) or screen x,y,depth (kind 0)
  float rgba[4];
};

struct sg_scene {
  sg_params p;
  std::vector<Tri> tris;   // static then moving
  // last rasterised frame
  int frame = -1;
  std::vector<uint32_t> offsets;
  std::vector<float> depth;
  std::vector<float> rgba;
  std::vector<uint32_t> prim;
  double vp[16];
  sg_stats stats;
};

namespace {

// per-object material: base colour and opacity of object (cluster) `obj`
void object_material(const sg_params& p, int obj, double base[4]) {
  Rng r(p.seed, ST_CLUSTER + 100, (uint64_t)obj);
  for (int c = 0; c < 3; ++c) base[c] = r.uniform(0.05, 0.95);
  base[3] = r.uniform(p.alpha_lo, p.alpha_hi);
}

void colour_for(Rng& r, const sg_params& p, double depth01, float out[4], int obj = -1) {
  if (p.colour_mode == 2) {
    // object palette: the object's material with a small per-triangle variation
    double base[4];
    object_material(p, obj < 0 ? 0 : obj, base);
    for (int c = 0; c < 3; ++c)
      out[c] = (float)std::min(1.0, std::max(0.0, base[c] + 0.04 * (2.0 * r.uniform() - 1.0)));
    out[3] = (float)std::min(p.alpha_hi, std::max(p.alpha_lo, base[3] + 0.04 * (2.0 * r.uniform() - 1.0)));
    return;
  }
  if (p.colour_mode == 1) {
    // near fragments reddish, far fragments bluish, with noise
    double t = std::min(1.0, std::max(0.0, depth01));
    double base[3] = {0.9 - 0.7 * t, 0.3 + 0.3 * std::sin(3.14159 * t), 0.2 + 0.7 * t};
    for (int c = 0; c < 3; ++c) {
      double v = base[c] + 0.15 * (2.0 * r.uniform() - 1.0);
      out[c] = (float)std::min(1.0, std::max(0.0, v));
    }
  } else {
    for (int c = 0; c < 3; ++c) out[c] = (float)r.uniform();
  }
  out[3] = (float)r.uniform(p.alpha_lo, p.alpha_hi);
}

void build_triangles(sg_scene* s) {
  const sg_params& p = s->p;
  int total = p.num_tris + (p.kind == 1 ? p.num_moving : 0);
  s->tris.resize(total);
  if (p.kind == 0) {
    for (int i = 0; i < total; ++i) {
      Rng r(p.seed, ST_TRI, (uint64_t)i);
      Tri& t = s->tris[i];
      double zsum = 0;
      for (int k = 0; k < 3; ++k) {
        t.v[k][0] = r.uniform() * p.width;
        t.v[k][1] = r.uniform() * p.height;
        t.v[k][2] = r.uniform();
        zsum += t.v[k][2];
      }
      colour_for(r, p, zsum / 3.0, t.rgba, i % 8);
    }
    return;
  }
  // world space: camera at origin looking down -z at frame 0
  double tan_y = std::tan(p.fov_y_deg * 3.141592653589793 / 360.0);
  double tan_x = tan_y * (double)p.width / (double)p.height;
  int nc = std::max(1, p.clusters);
  std::vector<double> cc(3 * nc);
  for (int c = 0; c < nc; ++c) {
    Rng r(p.seed, ST_CLUSTER, (uint64_t)c);
    double d = r.uniform(p.depth_lo, p.depth_hi);
    cc[3 * c + 0] = r.uniform(-1.0, 1.0) * tan_x * d * 0.9;
    cc[3 * c + 1] = r.uniform(-1.0, 1.0) * tan_y * d * 0.9;
    cc[3 * c + 2] = -d;
  }
  for (int i = 0; i < total; ++i) {
    Rng r(p.seed, ST_TRI, (uint64_t)i);
    double cx, cy, cz, d;
    int obj = nc;  // scattered triangles share one background material
    if (p.clusters > 0 && r.uniform() < p.cluster_frac) {
      int c = (int)(r.next() % (uint64_t)nc);
      obj = c;
      d = -cc[3 * c + 2];
      cx = cc[3 * c + 0] + r.normal() * p.cluster_radius * d;
      cy = cc[3 * c + 1] + r.normal() * p.cluster_radius * d;
      cz = cc[3 * c + 2] + r.normal() * p.cluster_radius * d;
      cz = std::min(-p.depth_lo, std::max(-p.depth_hi, cz));
      d = -cz;
    } else {
      d = r.uniform(p.depth_lo, p.depth_hi);
      cx = r.uniform(-1.05, 1.05) * tan_x * d;
      cy = r.uniform(-1.05, 1.05) * tan_y * d;
      cz = -d;
    }
    double rad = d * std::exp(p.size_mu + p.size_sigma * r.normal());
    Tri& t = s->tris[i];
    for (int k = 0; k < 3; ++k) {
      // random direction on the unit sphere
      double z = r.uniform(-1.0, 1.0), phi = r.uniform(0.0, 6.283185307179586);
      double q = std::sqrt(std::max(0.0, 1.0 - z * z));
      t.v[k][0] = cx + rad * q * std::cos(phi);
      t.v[k][1] = cy + rad * q * std::sin(phi);
      t.v[k][2] = cz + rad * z;
    }
    double dep01 = (d - p.depth_lo) / std::max(1e-9, p.depth_hi - p.depth_lo);
    colour_for(r, p, dep01, t.rgba, obj);
  }
}

// row-major 4x4 products acting on column vectors
void mat_mul(const double* a, const double* b, double* o) {
  double t[16];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double s = 0;
      for (int k = 0; k < 4; ++k) s += a[4 * i + k] * b[4 * k + j];
      t[4 * i + j] = s;
    }
  std::memcpy(o, t, sizeof t);
}

void rot_axis(int axis, double ang, double* m) {
  double c = std::cos(ang), s = std::sin(ang);
  for (int i = 0; i < 16; ++i) m[i] = (i % 5 == 0) ? 1.0 : 0.0;
  int a = (axis + 1) % 3, b = (axis + 2) % 3;
  m[4 * a + a] = c; m[4 * a + b] = -s;
  m[4 * b + a] = s; m[4 * b + b] = c;
}

// Camera view-projection for frame t: accumulated seeded yaw/pitch/roll and
// translation steps, then a right-handed perspective with NDC z in [0,1].
void camera_vp(const sg_params& p, int frame, double* vp) {
  double yaw = 0, pitch = 0, roll = 0, pos[3] = {0, 0, 0};
  const double deg = 3.141592653589793 / 180.0;
  for (int f = 1; f <= frame; ++f) {
    Rng r(p.seed, ST_CAM, (uint64_t)f);
    yaw += r.uniform(-1.0, 1.0) * p.cam_rot_deg * deg;
    pitch += r.uniform(-1.0, 1.0) * p.cam_rot_deg * deg * 0.5;
    roll += r.uniform(-1.0, 1.0) * p.cam_rot_deg * deg * 0.25;
    for (int k = 0; k < 3; ++k) pos[k] += r.uniform(-1.0, 1.0) * p.cam_trans;
  }
  double ry[16], rx[16], rz[16], rot[16], tr[16], view[16];
  rot_axis(1, -yaw, ry);
  rot_axis(0, -pitch, rx);
  rot_axis(2, -roll, rz);
  mat_mul(rz, rx, rot);
  mat_mul(rot, ry, rot);
  for (int i = 0; i < 16; ++i) tr[i] = (i % 5 == 0) ? 1.0 : 0.0;
  tr[3] = -pos[0]; tr[7] = -pos[1]; tr[11] = -pos[2];
  mat_mul(rot, tr, view);
  double f = 1.0 / std::tan(p.fov_y_deg * deg * 0.5);
  double aspect = (double)p.width / (double)p.height;
  double n = p.z_near, fa = p.z_far;
  double proj[16] = {f / aspect, 0, 0, 0,
                     0, f, 0, 0,
                     0, 0, fa / (n - fa), n * fa / (n - fa),
                     0, 0, -1, 0};
  mat_mul(proj, view, vp);
}

// Per-frame rigid motion of a moving triangle: rotation about its centroid and a
// translation, accumulated from seeded steps.
void moving_vertices(const sg_params& p, const Tri& t, int idx, int frame, double out[3][3]) {
  double c[3] = {0, 0, 0};
  for (int k = 0; k < 3; ++k)
    for (int d = 0; d < 3; ++d) { out[k][d] = t.v[k][d]; c[d] += t.v[k][d] / 3.0; }
  const double deg = 3.141592653589793 / 180.0;
  for (int f = 1; f <= frame; ++f) {
    Rng r(p.seed, ST_MOVE, (uint64_t)idx * 4096u + (uint64_t)f);
    double ang = r.uniform(-1.0, 1.0) * p.move_rot_deg * deg;
    int axis = (int)(r.next() % 3u);
    double m[16];
    rot_axis(axis, ang, m);
    double tr[3];
    for (int d = 0; d < 3; ++d) tr[d] = r.uniform(-1.0, 1.0) * p.move_trans;
    for (int k = 0; k < 3; ++k) {
      double q[3], o[3];
      for (int d = 0; d < 3; ++d) q[d] = out[k][d] - c[d];
      for (int i = 0; i < 3; ++i) o[i] = m[4 * i] * q[0] + m[4 * i + 1] * q[1] + m[4 * i + 2] * q[2];
      for (int d = 0; d < 3; ++d) out[k][d] = c[d] + o[d] + tr[d];
    }
    for (int d = 0; d < 3; ++d) c[d] += tr[d];
  }
}

struct ScreenTri {
  int64_t X[3], Y[3];   // 1/256 px fixed point
  double z[3];
  int64_t area2;
  int x0, x1, y0, y1;   // inclusive pixel bbox, clipped
  bool live;
};

inline int64_t edge(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t px, int64_t py) {
  return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

inline bool edge_tie_in(int64_t ax, int64_t ay, int64_t bx, int64_t by) {
  int64_t dx = bx - ax, dy = by - ay;
  return dy > 0 || (dy == 0 && dx > 0);
}

void setup_screen(const sg_params& p, double sx[3], double sy[3], double sz[3], ScreenTri& st) {
  st.live = false;
  for (int k = 0; k < 3; ++k) {
    st.X[k] = (int64_t)std::llround(sx[k] * 256.0);
    st.Y[k] = (int64_t)std::llround(sy[k] * 256.0);
    st.z[k] = sz[k];
  }
  int64_t a = edge(st.X[0], st.Y[0], st.X[1], st.Y[1], st.X[2], st.Y[2]);
  if (a == 0) return;
  if (a < 0) {
    std::swap(st.X[1], st.X[2]); std::swap(st.Y[1], st.Y[2]); std::swap(st.z[1], st.z[2]);
    a = -a;
  }
  st.area2 = a;
  int64_t mnx = std::min({st.X[0], st.X[1], st.X[2]}), mxx = std::max({st.X[0], st.X[1], st.X[2]});
  int64_t mny = std::min({st.Y[0], st.Y[1], st.Y[2]}), mxy = std::max({st.Y[0], st.Y[1], st.Y[2]});
  // pixel x covers centre x*256+128
  auto lo = [](int64_t v) { int64_t t = v - 128; return t >= 0 ? (t + 255) / 256 : -((-t) / 256); };
  auto hi = [](int64_t v) { int64_t t = v - 128; return t >= 0 ? t / 256 : -((-t + 255) / 256); };
  int64_t x0 = std::max<int64_t>(0, lo(mnx)), x1 = std::min<int64_t>(p.width - 1, hi(mxx));
  int64_t y0 = std::max<int64_t>(0, lo(mny)), y1 = std::min<int64_t>(p.height - 1, hi(mxy));
  if (x0 > x1 || y0 > y1) return;
  st.x0 = (int)x0; st.x1 = (int)x1; st.y0 = (int)y0; st.y1 = (int)y1;
  st.live = true;
}

template <class Emit>
void raster_rows(const ScreenTri& st, int ylo, int yhi, Emit emit) {
  int y0 = std::max(st.y0, ylo), y1 = std::min(st.y1, yhi);
  if (y0 > y1) return;
  const bool t0 = edge_tie_in(st.X[1], st.Y[1], st.X[2], st.Y[2]);
  const bool t1 = edge_tie_in(st.X[2], st.Y[2], st.X[0], st.Y[0]);
  const bool t2 = edge_tie_in(st.X[0], st.Y[0], st.X[1], st.Y[1]);
  for (int y = y0; y <= y1; ++y) {
    int64_t py = (int64_t)y * 256 + 128;
    // Conservative x-span of the row from the three edge half-planes (floating
    // estimate widened by one pixel); the exact integer test below decides.
    double lo = st.x0, hi = st.x1;
    for (int e = 0; e < 3; ++e) {
      int a = (e + 1) % 3, b = (e + 2) % 3;
      double ax = (double)st.X[a], ay = (double)st.Y[a], bx = (double)st.X[b], by = (double)st.Y[b];
      // w(px) = (bx-ax)(py-ay) - (by-ay)(px-ax) >= 0
      double k = -(by - ay), c0 = (bx - ax) * ((double)py - ay) + (by - ay) * ax;
      if (k > 0) lo = std::max(lo, (-c0 / k - 128.0) / 256.0 - 1.0);
      else if (k < 0) hi = std::min(hi, (-c0 / k - 128.0) / 256.0 + 1.0);
      else if (c0 < 0) { lo = 1; hi = 0; }
    }
    if (lo > hi) continue;
    int xa = std::max(st.x0, (int)std::floor(lo)), xb = std::min(st.x1, (int)std::ceil(hi));
    for (int x = xa; x <= xb; ++x) {
      int64_t px = (int64_t)x * 256 + 128;
      int64_t w0 = edge(st.X[1], st.Y[1], st.X[2], st.Y[2], px, py);
      int64_t w1 = edge(st.X[2], st.Y[2], st.X[0], st.Y[0], px, py);
      int64_t w2 = edge(st.X[0], st.Y[0], st.X[1], st.Y[1], px, py);
      if (w0 < 0 || w1 < 0 || w2 < 0) continue;
      if ((w0 == 0 && !t0) || (w1 == 0 && !t1) || (w2 == 0 && !t2)) continue;
      double z = ((double)w0 * st.z[0] + (double)w1 * st.z[1] + (double)w2 * st.z[2]) / (double)st.area2;
      float zf = (float)z;
      if (zf < 0.f) zf = 0.f;
      if (zf > 1.f) zf = 1.f;
      emit(x, y, zf);
    }
  }
}

}  // namespace

extern "C" {

sg_scene* sg_create(const sg_params* p) {
  if (!p || p->width <= 0 || p->height <= 0 || p->num_tris < 0) return nullptr;
  sg_scene* s = new sg_scene();
  s->p = *p;
  build_triangles(s);
  return s;
}

void sg_destroy(sg_scene* s) { delete s; }

// Rasterise frame `frame` into the scene's internal buffers. Returns the number
// of fragments, or -1 on bad arguments.
int64_t sg_rasterize(sg_scene* s, int32_t frame) {
  if (!s || frame < 0) return -1;
  const sg_params& p = s->p;
  const int W = p.width, H = p.height;
  const size_t P = (size_t)W * H;
  int total = (int)s->tris.size();
  std::vector<ScreenTri> st(total);
  uint32_t dropped = 0;
  if (p.kind == 0) {
    for (int i = 0; i < 16; ++i) s->vp[i] = (i % 5 == 0) ? 1.0 : 0.0;
    for (int i = 0; i < total; ++i) {
      double sx[3], sy[3], sz[3];
      for (int k = 0; k < 3; ++k) { sx[k] = s->tris[i].v[k][0]; sy[k] = s->tris[i].v[k][1]; sz[k] = s->tris[i].v[k][2]; }
      setup_screen(p, sx, sy, sz, st[i]);
    }
  } else {
    camera_vp(p, frame, s->vp);
    for (int i = 0; i < total; ++i) {
      double v[3][3];
      if (i >= p.num_tris) moving_vertices(p, s->tris[i], i, frame, v);
      else std::memcpy(v, s->tris[i].v, sizeof v);
      double sx[3], sy[3], sz[3];
      bool ok = true;
      for (int k = 0; k < 3 && ok; ++k) {
        double c[4];
        for (int r = 0; r < 4; ++r)
          c[r] = s->vp[4 * r] * v[k][0] + s->vp[4 * r + 1] * v[k][1] + s->vp[4 * r + 2] * v[k][2] + s->vp[4 * r + 3];
        if (c[3] <= 1e-9) { ok = false; break; }
        double xn = c[0] / c[3], yn = c[1] / c[3], zn = c[2] / c[3];
        if (zn < 0.0 || zn > 1.0) { ok = false; break; }
        sx[k] = (xn + 1.0) * 0.5 * W;
        sy[k] = (1.0 - yn) * 0.5 * H;
        sz[k] = zn;
      }
      if (!ok) { st[i].live = false; ++dropped; continue; }
      setup_screen(p, sx, sy, sz, st[i]);
    }
  }
  // bands of rows, each walking the triangles in primitive order
  const int band = 8;
  const int nb = (H + band - 1) / band;
  std::vector<uint32_t> cnt(P, 0);
#pragma omp parallel for schedule(dynamic, 1)
  for (int b = 0; b < nb; ++b) {
    int ylo = b * band, yhi = std::min(H - 1, ylo + band - 1);
    for (int i = 0; i < total; ++i) {
      if (!st[i].live) continue;
      raster_rows(st[i], ylo, yhi, [&](int x, int y, float) { cnt[(size_t)y * W + x]++; });
    }
  }
  std::vector<uint64_t> off0(P + 1, 0);
  for (size_t i = 0; i < P; ++i) off0[i + 1] = off0[i] + cnt[i];
  uint64_t F0 = off0[P];
  std::vector<float> z0(F0), c0(4 * F0);
  std::vector<uint32_t> pr0(F0);
#pragma omp parallel for schedule(dynamic, 1)
  for (int b = 0; b < nb; ++b) {
    int ylo = b * band, yhi = std::min(H - 1, ylo + band - 1);
    std::vector<uint32_t> fill(W * (size_t)(yhi - ylo + 1), 0);
    for (int i = 0; i < total; ++i) {
      if (!st[i].live) continue;
      const float* col = s->tris[i].rgba;
      raster_rows(st[i], ylo, yhi, [&](int x, int y, float z) {
        size_t pix = (size_t)y * W + x;
        uint32_t& k = fill[(size_t)(y - ylo) * W + x];
        uint64_t at = off0[pix] + k++;
        z0[at] = z;
        std::memcpy(&c0[4 * at], col, 4 * sizeof(float));
        pr0[at] = (uint32_t)i;
      });
    }
  }
  // trim farthest-first, then shuffle
  std::vector<uint32_t> keep(P);
  const uint32_t mx = p.max_per_pixel;
  uint64_t trimmed = 0;
  std::vector<uint8_t> mark(F0, 1);
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : trimmed)
  for (size_t pix = 0; pix < P; ++pix) {
    uint32_t n = cnt[pix];
    if (mx == 0 || n <= mx) { keep[pix] = n; continue; }
    uint64_t b0 = off0[pix];
    std::vector<uint32_t> idx(n);
    for (uint32_t k = 0; k < n; ++k) idx[k] = k;
    std::sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) {
      float za = z0[b0 + a], zb = z0[b0 + b];
      if (za != zb) return za < zb;
      return pr0[b0 + a] < pr0[b0 + b];
    });
    for (uint32_t k = mx; k < n; ++k) mark[b0 + idx[k]] = 0;
    keep[pix] = mx;
    trimmed += n - mx;
  }
  s->offsets.assign(P + 1, 0);
  for (size_t i = 0; i < P; ++i) s->offsets[i + 1] = s->offsets[i] + keep[i];
  uint64_t F = s->offsets[P];
  s->depth.resize(F);
  s->rgba.resize(4 * F);
  s->prim.resize(F);
#pragma omp parallel for schedule(dynamic, 4096)
  for (size_t pix = 0; pix < P; ++pix) {
    uint64_t o = s->offsets[pix];
    uint32_t n = 0;
    for (uint64_t k = off0[pix]; k < off0[pix + 1]; ++k) {
      if (!mark[k]) continue;
      s->depth[o + n] = z0[k];
      std::memcpy(&s->rgba[4 * (o + n)], &c0[4 * k], 4 * sizeof(float));
      s->prim[o + n] = pr0[k];
      ++n;
    }
    if (p.shuffle && n > 1) {
      Rng r(p.seed, ST_SHUF, ((uint64_t)frame << 40) ^ (uint64_t)pix);
      for (uint32_t i = n - 1; i > 0; --i) {
        uint32_t j = (uint32_t)(r.next() % (uint64_t)(i + 1));
        std::swap(s->depth[o + i], s->depth[o + j]);
        std::swap(s->prim[o + i], s->prim[o + j]);
        for (int c = 0; c < 4; ++c) std::swap(s->rgba[4 * (o + i) + c], s->rgba[4 * (o + j) + c]);
      }
    }
  }
  // statistics
  sg_stats& S = s->stats;
  S.num_frags = F;
  S.trimmed = trimmed;
  S.dropped_tris = dropped;
  uint32_t mxc = 0, cov = 0;
  std::vector<uint64_t> hist(65537, 0);
  for (size_t i = 0; i < P; ++i) {
    uint32_t n = keep[i];
    mxc = std::max(mxc, n);
    cov += n > 0;
    hist[std::min<uint32_t>(n, 65536)]++;
  }
  S.max_count = mxc;
  S.covered_pixels = cov;
  S.mean_count = (double)F / (double)P;
  uint64_t acc = 0, target = (uint64_t)std::ceil(0.99 * (double)P);
  S.p99_count = 0;
  for (uint32_t n = 0; n <= 65536; ++n) {
    acc += hist[n];
    if (acc >= target) { S.p99_count = n; break; }
  }
  s->frame = frame;
  return (int64_t)F;
}

// Copy the last rasterised frame into caller buffers (any pointer may be NULL).
int32_t sg_fetch(const sg_scene* s, uint32_t* offsets, float* depth, float* rgba, uint32_t* prim,
                 double* vp, sg_stats* stats) {
  if (!s || s->frame < 0) return -1;
  const size_t P = (size_t)s->p.width * s->p.height;
  if (offsets) std::memcpy(offsets, s->offsets.data(), (P + 1) * sizeof(uint32_t));
  if (depth) std::memcpy(depth, s->depth.data(), s->depth.size() * sizeof(float));
  if (rgba) std::memcpy(rgba, s->rgba.data(), s->rgba.size() * sizeof(float));
  if (prim) std::memcpy(prim, s->prim.data(), s->prim.size() * sizeof(uint32_t));
  if (vp) std::memcpy(vp, s->vp, sizeof s->vp);
  if (stats) *stats = s->stats;
  return 0;
}

// Camera matrix of any frame without rasterising.
int32_t sg_camera(const sg_scene* s, int32_t frame, double* vp) {
  if (!s || frame < 0 || !vp) return -1;
  if (s->p.kind == 0) {
    for (int i = 0; i < 16; ++i) vp[i] = (i % 5 == 0) ? 1.0 : 0.0;
    return 0;
  }
  camera_vp(s->p, frame, vp);
  return 0;
}

// Seeded uniform numbers in [lo, hi) for data the method treats as input
// (initial network weights). Stream is separate from the scene's streams.
void sg_uniform(uint64_t seed, uint64_t stream, uint64_t n, double lo, double hi, double* out) {
  for (uint64_t i = 0; i < n; ++i) {
    Rng r(seed, 1000 + stream, i);
    out[i] = r.uniform(lo, hi);
  }
}

}  // extern "C"
