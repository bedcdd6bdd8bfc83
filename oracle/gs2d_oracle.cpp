// FP64 CPU oracle of the 2D Gaussian surfel rasterizer (forward and reverse mode).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call this
// file; only the test suite, the smoke check and the benchmark's CPU-baseline
// leg use it.  It shares no code, headers, tables or constants with the HIP
// library: every constant below is typed out here on its own.
//
// What it computes (paper: Sec. "2D Gaussian Splatting" and Sec. "Camera Pose
// Optimization"), written out as the plain definition, per pixel, in double:
//
//   * splat plane P(u,v) = mu + s_u t_u u + s_v t_v v                   (eq:Puv)
//   * camera-space frame H_c = T_cw H, columns s_u t_uc, s_v t_vc, mu_c (eq:hc)
//   * homography  M = K [s_u t_uc | s_v t_vc | mu_c], the 3x3 part of
//     W H_c with W the pinhole camera->image map                      (eq:homo, eq:wth)
//   * ray-splat intersection in uv space without inverting M: the pixel ray
//     (x, y) meets the plane where h_u.(u,v,1) = h_v.(u,v,1) = 0, with
//     h_u = M_0 - x M_2 and h_v = M_1 - y M_2, so (u,v,1) ~ h_u x h_v
//   * Gaussian weight G = exp(-(u^2+v^2)/2)
//   * depth-sorted front-to-back alpha blending of colour, depth, normal
//     t_nc = t_uc x t_vc and opacity (v = 1)                           (eq:alpha_blending)
//   * reverse mode to every surfel parameter, and the pose gradient in the
//     paper's form  d/dtau = sum_i [dL/dmu_c (I, -mu_c^x)] (+) [dL/dR_c
//     (0, -R_c[:,k]^x)]                                                (eq:derivatives)
//
// Conventions where the paper defers to the 2DGS rasterizer (each is a reading
// recorded with the project's design notes): pixel (x,y) sampled at integer
// coordinates; object-space low-pass filter rho = min(u^2+v^2, 2|p - c|^2) with
// the projected centre c (filter branch takes the depth of mu_c); include a
// (pixel, surfel) pair when rho <= 9 and depth >= z_near; alpha = min(0.99, o G)
// and pairs with alpha < 1/255 are skipped; compositing stops before the
// surfel that would bring transmittance below 1e-4; order is ascending
// (float32(mu_c.z), surfel index); background 0; depth is the blended camera z
// of the intersection, not divided by the opacity.
//
// Performance is not a goal: no SIMD, no tiles.  The only shortcut is a
// per-surfel conservative pixel rectangle, which a brute-force mode (every
// surfel tested at every pixel) checks bit-for-bit.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <array>
#include <vector>

namespace {

struct Cam {
  int width, height;
  double fx, fy, cx, cy;
};

struct Consts {
  double z_near;      // centre and per-pixel depth cut
  double rho_cutoff;  // include a pair when rho <= this
  double alpha_max;   // opacity clamp
  double alpha_min;   // skip pairs below this
  double t_min;       // stop before transmittance drops below this
  double filter_scale;  // rho2d = filter_scale * |p - c|^2
  int filter;         // 1: low-pass filter branch on
  int use_rect;       // 1: conservative rect; 0: brute force
};

typedef double V3[3];

inline void cross(const double* a, const double* b, double* o) {
  double x = a[1] * b[2] - a[2] * b[1];
  double y = a[2] * b[0] - a[0] * b[2];
  double z = a[0] * b[1] - a[1] * b[0];
  o[0] = x; o[1] = y; o[2] = z;
}
inline double dot(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline double rel(double a, double b) {
  double s = std::fabs(b) > 1e-300 ? std::fabs(b) : 1e-300;
  return std::fabs(a - b) / s;
}

struct Surf {
  bool culled;
  double mu_c[3], tuc[3], tvc[3], n[3], a[3], b[3];
  double M[3][3];  // rows M_0, M_1, M_2
  double su, sv, o, rgb[3];
  float key;       // float32(mu_c.z)
  double aabb[4];  // x0, x1, y0, y1 (exact 3-sigma ellipse box united with filter disc)
  int rect[4];     // inclusive pixel rect x0, x1, y0, y1 (empty when x0 > x1)
  double cull_margin;
};

// O1: per-surfel preprocessing (eq:hc, eq:wth).
void preprocess(const double* P, int64_t n, int64_t i, const Cam& cam, const double* T,
                const Consts& k, Surf& s) {
  double mu[3], tu[3], tv[3];
  for (int c = 0; c < 3; ++c) {
    mu[c] = P[(0 + c) * n + i];
    tu[c] = P[(3 + c) * n + i];
    tv[c] = P[(6 + c) * n + i];
  }
  s.su = P[9 * n + i];
  s.sv = P[10 * n + i];
  s.o = P[11 * n + i];
  for (int c = 0; c < 3; ++c) s.rgb[c] = P[(12 + c) * n + i];
  // T = [R | t], row-major 3x4
  for (int r = 0; r < 3; ++r) {
    s.mu_c[r] = T[r * 4 + 0] * mu[0] + T[r * 4 + 1] * mu[1] + T[r * 4 + 2] * mu[2] + T[r * 4 + 3];
    s.tuc[r] = T[r * 4 + 0] * tu[0] + T[r * 4 + 1] * tu[1] + T[r * 4 + 2] * tu[2];
    s.tvc[r] = T[r * 4 + 0] * tv[0] + T[r * 4 + 1] * tv[1] + T[r * 4 + 2] * tv[2];
  }
  cross(s.tuc, s.tvc, s.n);
  for (int c = 0; c < 3; ++c) {
    s.a[c] = s.su * s.tuc[c];
    s.b[c] = s.sv * s.tvc[c];
  }
  // M = K [a | b | mu_c]; K = [[fx,0,cx],[0,fy,cy],[0,0,1]]
  const double* col[3] = {s.a, s.b, s.mu_c};
  for (int j = 0; j < 3; ++j) {
    s.M[0][j] = cam.fx * col[j][0] + cam.cx * col[j][2];
    s.M[1][j] = cam.fy * col[j][1] + cam.cy * col[j][2];
    s.M[2][j] = col[j][2];
  }
  s.key = (float)s.mu_c[2];
  s.culled = false;
  s.rect[0] = 0; s.rect[1] = -1; s.rect[2] = 0; s.rect[3] = -1;
  s.cull_margin = rel(s.mu_c[2], k.z_near);
  if (!(s.mu_c[2] > k.z_near)) { s.culled = true; return; }
  // Dual conic of the 3-sigma disk u^2+v^2 <= 9: C* = M diag(9,9,-1) M^T.
  double C[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      C[r][c] = 9.0 * s.M[r][0] * s.M[c][0] + 9.0 * s.M[r][1] * s.M[c][1] - s.M[r][2] * s.M[c][2];
  double c22_scale = 9.0 * (s.M[2][0] * s.M[2][0] + s.M[2][1] * s.M[2][1]) + s.M[2][2] * s.M[2][2];
  s.cull_margin = std::min(s.cull_margin, std::fabs(C[2][2]) / c22_scale);
  // C*_22 < 0 exactly when the whole 3-sigma disk lies in front of the camera plane.
  if (!(C[2][2] < 0.0)) { s.culled = true; return; }
  double ex = C[0][2] / C[2][2], ey = C[1][2] / C[2][2];
  double hx = std::sqrt(std::max(0.0, ex * ex - C[0][0] / C[2][2]));
  double hy = std::sqrt(std::max(0.0, ey * ey - C[1][1] / C[2][2]));
  double x0 = ex - hx, x1 = ex + hx, y0 = ey - hy, y1 = ey + hy;
  if (k.filter) {
    double cx = s.M[0][2] / s.M[2][2], cy = s.M[1][2] / s.M[2][2];
    double r = std::sqrt(k.rho_cutoff / k.filter_scale);
    x0 = std::min(x0, cx - r); x1 = std::max(x1, cx + r);
    y0 = std::min(y0, cy - r); y1 = std::max(y1, cy + r);
  }
  s.aabb[0] = x0; s.aabb[1] = x1; s.aabb[2] = y0; s.aabb[3] = y1;
  // one pixel of slack on every side, then clip to the image
  double fx0 = std::floor(x0 - 1.0), fx1 = std::ceil(x1 + 1.0);
  double fy0 = std::floor(y0 - 1.0), fy1 = std::ceil(y1 + 1.0);
  fx0 = std::max(fx0, 0.0); fy0 = std::max(fy0, 0.0);
  fx1 = std::min(fx1, (double)(cam.width - 1)); fy1 = std::min(fy1, (double)(cam.height - 1));
  if (fx0 > fx1 || fy0 > fy1) { s.rect[0] = 0; s.rect[1] = -1; return; }
  s.rect[0] = (int)fx0; s.rect[1] = (int)fx1; s.rect[2] = (int)fy0; s.rect[3] = (int)fy1;
}

// O2: one (pixel, surfel) evaluation.
struct Hit {
  int64_t id;
  bool included;
  bool branch3d;
  bool clamped;
  double hu[3], hv[3], q[3];
  double u, v, rho, G, alpha, d, dx, dy;
};

void evaluate(const Surf& s, int64_t id, double x, double y, const Consts& k, Hit& h,
              double& fmargin, double& gmargin) {
  h.id = id;
  h.included = false;
  for (int c = 0; c < 3; ++c) {
    h.hu[c] = s.M[0][c] - x * s.M[2][c];
    h.hv[c] = s.M[1][c] - y * s.M[2][c];
  }
  cross(h.hu, h.hv, h.q);
  double rho3d = INFINITY;
  if (h.q[2] != 0.0) {
    h.u = h.q[0] / h.q[2];
    h.v = h.q[1] / h.q[2];
    rho3d = h.u * h.u + h.v * h.v;
  } else {
    h.u = h.v = 0.0;
  }
  double rho2d = INFINITY;
  double cx = s.M[0][2] / s.M[2][2], cy = s.M[1][2] / s.M[2][2];
  h.dx = x - cx;
  h.dy = y - cy;
  if (k.filter) rho2d = k.filter_scale * (h.dx * h.dx + h.dy * h.dy);
  if (rho3d <= rho2d) {
    h.branch3d = true;
    h.rho = rho3d;
    h.d = s.M[2][0] * h.u + s.M[2][1] * h.v + s.M[2][2];
  } else {
    h.branch3d = false;
    h.rho = rho2d;
    h.d = s.M[2][2];
  }
  if (!std::isfinite(h.rho)) return;
  double m_rho = rel(h.rho, k.rho_cutoff);
  if (m_rho < 0.5) { fmargin = std::min(fmargin, m_rho); gmargin = std::min(gmargin, m_rho); }
  if (!(h.rho <= k.rho_cutoff)) return;
  if (std::isfinite(rho3d) && std::isfinite(rho2d)) {
    // The branch switch changes the gradient always, and the value only where
    // the two branches' depths differ (they agree at the projected centre).
    double m_br = std::fabs(rho3d - rho2d) / std::max(std::max(rho3d, rho2d), 1e-300);
    double d3 = s.M[2][0] * h.u + s.M[2][1] * h.v + s.M[2][2];
    if (std::fabs(d3 - s.M[2][2]) > 1e-7 * std::fabs(s.M[2][2])) fmargin = std::min(fmargin, m_br);
    gmargin = std::min(gmargin, m_br);
  }
  double m_z = rel(h.d, k.z_near);
  fmargin = std::min(fmargin, m_z);
  gmargin = std::min(gmargin, m_z);
  if (!(h.d >= k.z_near)) return;
  h.G = std::exp(-0.5 * h.rho);
  double og = s.o * h.G;
  double m_amin = rel(og, k.alpha_min);
  fmargin = std::min(fmargin, m_amin);
  gmargin = std::min(gmargin, m_amin);
  gmargin = std::min(gmargin, rel(og, k.alpha_max));
  h.clamped = og > k.alpha_max;
  h.alpha = h.clamped ? k.alpha_max : og;
  if (h.alpha < k.alpha_min) return;
  h.included = true;
}

struct Scene {
  Cam cam;
  Consts k;
  int64_t n;
  std::vector<Surf> surf;
  std::vector<int64_t> order;                 // non-culled surfels by (key, index)
  std::vector<std::vector<int64_t>> rows;     // candidates per image row, in order
};

void build_scene(const double* P, int64_t n, const Cam& cam, const double* T, const Consts& k,
                 int nthreads, Scene& sc) {
  sc.cam = cam;
  sc.k = k;
  sc.n = n;
  sc.surf.resize((size_t)n);
  auto work = [&](int t) {
    for (int64_t i = t; i < n; i += nthreads) preprocess(P, n, i, cam, T, k, sc.surf[(size_t)i]);
  };
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t) th.emplace_back(work, t);
  for (auto& x : th) x.join();
  sc.order.clear();
  for (int64_t i = 0; i < n; ++i)
    if (!sc.surf[(size_t)i].culled) sc.order.push_back(i);
  // O3: ascending float32 depth, ties by surfel index
  std::stable_sort(sc.order.begin(), sc.order.end(), [&](int64_t a, int64_t b) {
    return sc.surf[(size_t)a].key < sc.surf[(size_t)b].key;
  });
  sc.rows.assign((size_t)cam.height, {});
  for (int64_t i : sc.order) {
    const Surf& s = sc.surf[(size_t)i];
    int y0 = k.use_rect ? s.rect[2] : 0, y1 = k.use_rect ? s.rect[3] : cam.height - 1;
    if (k.use_rect && s.rect[0] > s.rect[1]) continue;
    for (int y = y0; y <= y1; ++y) sc.rows[(size_t)y].push_back(i);
  }
}

// O4: composite one pixel.  Fills the included list (with the transmittance
// in front of each member) when `list` is non-null.
struct Entry {
  Hit h;
  double T;  // transmittance in front of this surfel
};

void composite_pixel(const Scene& sc, int x, int y, double out[8], double& t_final, int& count,
                     double& fm, double& gm, std::vector<Entry>* list) {
  for (int c = 0; c < 8; ++c) out[c] = 0.0;
  double T = 1.0;
  count = 0;
  fm = INFINITY;
  gm = INFINITY;
  double prev_z = NAN;
  for (int64_t i : sc.rows[(size_t)y]) {
    const Surf& s = sc.surf[(size_t)i];
    if (sc.k.use_rect && (x < s.rect[0] || x > s.rect[1])) continue;
    Hit h;
    evaluate(s, i, (double)x, (double)y, sc.k, h, fm, gm);
    if (!h.included) continue;
    double Tn = T * (1.0 - h.alpha);
    double m_t = rel(Tn, sc.k.t_min);
    fm = std::min(fm, m_t);
    gm = std::min(gm, m_t);
    // Order is decided on float32(mu_c.z) (ties by index).  A depth computed in
    // double lands on a different float32 key only if it sits on a float32
    // rounding boundary, so the order margin is the relative distance to the
    // nearest such boundary, scaled by 1e8 to share the 1e-5 exclusion threshold
    // (1e-13 relative is far above double rounding noise).
    {
      const double z = s.mu_c[2];
      const float f = (float)z;
      const double up = (double)std::nextafter(f, INFINITY), dn = (double)std::nextafter(f, -INFINITY);
      const double b1 = 0.5 * ((double)f + up), b0 = 0.5 * ((double)f + dn);
      const double m_o = 1e8 * std::min(std::fabs(z - b1), std::fabs(z - b0)) / std::fabs(z);
      fm = std::min(fm, m_o);
      gm = std::min(gm, m_o);
    }
    (void)prev_z;
    if (Tn < sc.k.t_min) break;
    double w = h.alpha * T;
    for (int c = 0; c < 3; ++c) out[c] += w * s.rgb[c];
    out[3] += w * h.d;
    for (int c = 0; c < 3; ++c) out[4 + c] += w * s.n[c];
    out[7] += w;
    if (list) list->push_back({h, T});
    T = Tn;
    ++count;
  }
  t_final = T;
}

template <class F>
void parallel_rows(int height, int nthreads, F f) {
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t)
    th.emplace_back([&, t]() {
      for (int y = t; y < height; y += nthreads) f(t, y);
    });
  for (auto& x : th) x.join();
}

}  // namespace

// O6, per surfel: the chain from the 16 summed screen terms A (dL/dM row-major,
// dL/dn, dL/drgb, dL/do) to the world-frame parameter gradient (15) and to the
// paper-form pose gradient of eq:derivatives (6).  Linear in A, so it also maps one
// pair's terms to that pair's share of every result.
void surfel_chain(const Surf& s, const Cam& cam, const double* R, const double* A, double outp[15],
                  double pose[6], double gmu_w[3], double gtu_w[3], double gtv_w[3]) {
  // dL/d[a b mu_c] = K^T dL/dM   (the paper's W^T dL/dT)
  double gA[3][3];
  for (int j = 0; j < 3; ++j) {
    double m0 = A[0 * 3 + j], m1 = A[1 * 3 + j], m2 = A[2 * 3 + j];
    gA[0][j] = cam.fx * m0;
    gA[1][j] = cam.fy * m1;
    gA[2][j] = cam.cx * m0 + cam.cy * m1 + m2;
  }
  double ga[3] = {gA[0][0], gA[1][0], gA[2][0]};
  double gb[3] = {gA[0][1], gA[1][1], gA[2][1]};
  double gmu[3] = {gA[0][2], gA[1][2], gA[2][2]};
  const double* gn = A + 9;
  // camera-frame tangent gradients: scale chain plus normal chain n = t_uc x t_vc
  double tmp[3], gtuc[3], gtvc[3];
  cross(s.tvc, gn, tmp);
  for (int cc = 0; cc < 3; ++cc) gtuc[cc] = s.su * ga[cc] + tmp[cc];
  cross(gn, s.tuc, tmp);
  for (int cc = 0; cc < 3; ++cc) gtvc[cc] = s.sv * gb[cc] + tmp[cc];
  double gsu = dot(s.tuc, ga), gsv = dot(s.tvc, gb);
  // world frame: g_world = R^T g_cam
  for (int cc = 0; cc < 3; ++cc) {
    gmu_w[cc] = R[0 * 4 + cc] * gmu[0] + R[1 * 4 + cc] * gmu[1] + R[2 * 4 + cc] * gmu[2];
    gtu_w[cc] = R[0 * 4 + cc] * gtuc[0] + R[1 * 4 + cc] * gtuc[1] + R[2 * 4 + cc] * gtuc[2];
    gtv_w[cc] = R[0 * 4 + cc] * gtvc[0] + R[1 * 4 + cc] * gtvc[1] + R[2 * 4 + cc] * gtvc[2];
  }
  for (int cc = 0; cc < 3; ++cc) {
    outp[0 + cc] = gmu_w[cc];
    outp[3 + cc] = gtu_w[cc];
    outp[6 + cc] = gtv_w[cc];
    outp[12 + cc] = A[12 + cc];
  }
  outp[9] = gsu;
  outp[10] = gsv;
  outp[11] = A[15];
  // Pose, paper form: dmu_c/dT = [I, -mu_c^x], dR_c/dT = [0, -R_c[:,k]^x]
  // with the columns of dL/dR_c = [dL/dt_uc (from H_c), dL/dt_vc, dL/dt_nc].
  double gcol0[3], gcol1[3];
  for (int cc = 0; cc < 3; ++cc) { gcol0[cc] = s.su * ga[cc]; gcol1[cc] = s.sv * gb[cc]; }
  double c1[3], c2[3], c3[3], c4[3];
  cross(s.mu_c, gmu, c1);
  cross(s.tuc, gcol0, c2);
  cross(s.tvc, gcol1, c3);
  cross(s.n, gn, c4);
  for (int cc = 0; cc < 3; ++cc) {
    pose[cc] = gmu[cc];
    pose[3 + cc] = c1[cc] + c2[cc] + c3[cc] + c4[cc];
  }
}

extern "C" {

struct OrcCamera {
  int32_t width, height;
  double fx, fy, cx, cy;
};

struct OrcConsts {
  double z_near, rho_cutoff, alpha_max, alpha_min, t_min, filter_scale;
  int32_t filter, use_rect;
};

static void unpack(const OrcCamera* c, const OrcConsts* k, Cam& cam, Consts& kk) {
  cam.width = c->width; cam.height = c->height;
  cam.fx = c->fx; cam.fy = c->fy; cam.cx = c->cx; cam.cy = c->cy;
  kk.z_near = k->z_near; kk.rho_cutoff = k->rho_cutoff; kk.alpha_max = k->alpha_max;
  kk.alpha_min = k->alpha_min; kk.t_min = k->t_min; kk.filter_scale = k->filter_scale;
  kk.filter = k->filter; kk.use_rect = k->use_rect;
}

// Per-surfel preprocessing results: culled flag, float32 depth key, exact box
// (x0, x1, y0, y1) and the relative margin of the culling decisions.
int orc_preprocess(const double* params, int64_t n, const OrcCamera* c, const double* pose,
                   const OrcConsts* k, int32_t* culled, float* key, double* aabb, int32_t* rect,
                   double* cull_margin) {
  Cam cam; Consts kk;
  unpack(c, k, cam, kk);
  for (int64_t i = 0; i < n; ++i) {
    Surf s;
    preprocess(params, n, i, cam, pose, kk, s);
    culled[i] = s.culled ? 1 : 0;
    key[i] = s.key;
    for (int j = 0; j < 4; ++j) {
      aabb[j * n + i] = s.culled ? NAN : s.aabb[j];
      rect[j * n + i] = s.rect[j];
    }
    cull_margin[i] = s.cull_margin;
  }
  return 0;
}

// Forward render.  Images are planar: rgb[3][H][W], depth[H][W], normal[3][H][W],
// alpha[H][W].  t_final, count, fmargin and gmargin are [H][W].
int orc_render(const double* params, int64_t n, const OrcCamera* c, const double* pose,
               const OrcConsts* k, int nthreads, double* rgb, double* depth, double* normal,
               double* alpha, double* t_final, int32_t* count, double* fmargin, double* gmargin) {
  Cam cam; Consts kk;
  unpack(c, k, cam, kk);
  if (nthreads < 1) nthreads = 1;
  Scene sc;
  build_scene(params, n, cam, pose, kk, nthreads, sc);
  const int64_t HW = (int64_t)cam.width * cam.height;
  parallel_rows(cam.height, nthreads, [&](int, int y) {
    for (int x = 0; x < cam.width; ++x) {
      double out[8], tf, fm, gm;
      int cnt;
      composite_pixel(sc, x, y, out, tf, cnt, fm, gm, nullptr);
      int64_t p = (int64_t)y * cam.width + x;
      for (int ch = 0; ch < 3; ++ch) rgb[ch * HW + p] = out[ch];
      depth[p] = out[3];
      for (int ch = 0; ch < 3; ++ch) normal[ch * HW + p] = out[4 + ch];
      alpha[p] = out[7];
      t_final[p] = tf;
      count[p] = cnt;
      fmargin[p] = fm;
      gmargin[p] = gm;
    }
  });
  return 0;
}

// Depth variants of the forward render (the depth channel's alternatives):
//  * depth_norm = D / O, the blended depth over the opacity (0 where O = 0);
//  * depth_median = the depth of the last composited intersection whose incoming
//    transmittance exceeds 1/2, i.e. where the accumulated opacity reaches one half
//    (the last composited one if it never does; 0 with none).
// margin[H][W] is the pixel's smallest relative margin to any decision of the render
// and to the median's T > 1/2 decisions.
int orc_depth_variants(const double* params, int64_t n, const OrcCamera* c, const double* pose,
                       const OrcConsts* k, int nthreads, double* depth_norm, double* depth_median,
                       double* margin) {
  Cam cam; Consts kk;
  unpack(c, k, cam, kk);
  if (nthreads < 1) nthreads = 1;
  Scene sc;
  build_scene(params, n, cam, pose, kk, nthreads, sc);
  std::vector<std::vector<Entry>> lists((size_t)nthreads);
  parallel_rows(cam.height, nthreads, [&](int t, int y) {
    std::vector<Entry>& list = lists[(size_t)t];
    for (int x = 0; x < cam.width; ++x) {
      double out[8], tf, fm, gm;
      int cnt;
      list.clear();
      composite_pixel(sc, x, y, out, tf, cnt, fm, gm, &list);
      const int64_t p = (int64_t)y * cam.width + x;
      depth_norm[p] = out[7] > 0.0 ? out[3] / out[7] : 0.0;
      double med = 0.0;
      for (const Entry& e : list) {
        fm = std::min(fm, rel(e.T, 0.5));
        if (e.T > 0.5) med = e.h.d;
      }
      depth_median[p] = med;
      margin[p] = fm;
    }
  });
  return 0;
}

// Per-surfel contribution to the rendered frame (eq:weight, eq:contribution): the
// sum over pixels of the surfel's blending weight w_k(p) = alpha_k T_k, over the same
// composited pairs as the forward.  contrib[n]; touched[n] (may be null) is set for
// every surfel evaluated at a pixel whose smallest decision margin (fmargin) is below
// `margin`, where a float32 renderer may composite a different set.  Per-thread sums
// are added in thread order.
int orc_contribution(const double* params, int64_t n, const OrcCamera* c, const double* pose,
                     const OrcConsts* k, int nthreads, double margin, double* contrib, uint8_t* touched) {
  Cam cam; Consts kk;
  unpack(c, k, cam, kk);
  if (nthreads < 1) nthreads = 1;
  Scene sc;
  build_scene(params, n, cam, pose, kk, nthreads, sc);
  std::vector<std::vector<double>> acc((size_t)nthreads, std::vector<double>((size_t)n, 0.0));
  std::vector<std::vector<uint8_t>> tch((size_t)nthreads, std::vector<uint8_t>(touched ? (size_t)n : 0, 0));
  parallel_rows(cam.height, nthreads, [&](int t, int y) {
    std::vector<Entry> list;
    for (int x = 0; x < cam.width; ++x) {
      list.clear();
      double out[8], tf, fm, gm;
      int cnt;
      composite_pixel(sc, x, y, out, tf, cnt, fm, gm, &list);
      for (const Entry& e : list) acc[(size_t)t][(size_t)e.h.id] += e.h.alpha * e.T;
      if (touched && fm < margin) {
        for (int64_t i : sc.rows[(size_t)y]) {
          const Surf& s = sc.surf[(size_t)i];
          if (!kk.use_rect || (x >= s.rect[0] && x <= s.rect[1])) tch[(size_t)t][(size_t)i] = 1;
        }
      }
    }
  });
  for (int64_t i = 0; i < n; ++i) {
    double sum = 0.0;
    uint8_t tt = 0;
    for (int t = 0; t < nthreads; ++t) {
      sum += acc[(size_t)t][(size_t)i];
      if (touched) tt |= tch[(size_t)t][(size_t)i];
    }
    contrib[i] = sum;
    if (touched) touched[i] = tt;
  }
  return 0;
}

// Reverse mode of the forward above for dL/d(images) given per pixel.
//
// d_params [15][n] (may be null): gradient to mu, t_u, t_v (world frame), s_u,
//   s_v, opacity, rgb, with the normal chain included.
// d_screen [16][n] (may be null): the per-surfel accumulations before the
//   camera chain: dL/dM (row-major 9), dL/dn (3), dL/drgb (3), dL/do (1).
// d_pose_paper[6]: (rho, phi) from the paper's per-splat Jacobians,
//   dL/dmu_c [I, -mu_c^x] plus the columns of dL/dR_c against [0, -R_c[:,k]^x].
// d_pose_identity[6]: the same quantity through the world-frame gradients,
//   rho = R sum g_mu, phi = sum mu_c x R g_mu + t_uc x R g_tu + t_vc x R g_tv.
// watch (H*W bytes, may be null) marks pixels; touched[n] (may be null) is set
//   for every surfel evaluated at a marked pixel.
int orc_backward(const double* params, int64_t n, const OrcCamera* c, const double* pose,
                 const OrcConsts* k, int nthreads, const double* g_rgb, const double* g_depth,
                 const double* g_normal, const double* g_alpha, double* d_params, double* d_screen,
                 double* d_pose_paper, double* d_pose_identity, const uint8_t* watch,
                 uint8_t* touched, double* d_scale, double* pose_scale, const uint8_t* scale_mask,
                 double* pose_scale_masked) {
  Cam cam; Consts kk;
  unpack(c, k, cam, kk);
  if (nthreads < 1) nthreads = 1;
  Scene sc;
  build_scene(params, n, cam, pose, kk, nthreads, sc);
  const int64_t HW = (int64_t)cam.width * cam.height;
  const int NA = 16;  // per surfel: g_M (9), g_n (3), g_rgb (3), g_o (1)
  std::vector<std::vector<double>> acc((size_t)nthreads, std::vector<double>((size_t)(NA * n), 0.0));
  // magnitude scales: the sums over pairs of |a pair's share of each result| (its
  // world-frame parameter gradient and paper-form pose gradient), over all pixels and
  // over the pixels of scale_mask
  const double* R = pose;  // rows of R are pose[0..2], pose[4..6], pose[8..10]
  const bool want_scale = d_scale || pose_scale || pose_scale_masked;
  std::vector<std::vector<double>> acc_abs((size_t)nthreads);
  std::vector<std::array<double, 12>> acc_pose_abs((size_t)nthreads);
  for (int t = 0; t < nthreads; ++t) {
    if (d_scale) acc_abs[(size_t)t].assign((size_t)(15 * n), 0.0);
    acc_pose_abs[(size_t)t].fill(0.0);
  }
  std::vector<std::vector<uint8_t>> tch((size_t)nthreads);
  if (touched)
    for (auto& v : tch) v.assign((size_t)n, 0);

  parallel_rows(cam.height, nthreads, [&](int t, int y) {
    std::vector<Entry> list;
    std::vector<double> A(NA);
    double* ac = acc[(size_t)t].data();
    for (int x = 0; x < cam.width; ++x) {
      int64_t p = (int64_t)y * cam.width + x;
      list.clear();
      double out[8], tf, fm, gm;
      int cnt;
      composite_pixel(sc, x, y, out, tf, cnt, fm, gm, &list);
      if (touched && watch && watch[p]) {
        for (int64_t i : sc.rows[(size_t)y]) {
          const Surf& s = sc.surf[(size_t)i];
          if (!kk.use_rect || (x >= s.rect[0] && x <= s.rect[1])) tch[(size_t)t][(size_t)i] = 1;
        }
      }
      double g[8];
      for (int ch = 0; ch < 3; ++ch) g[ch] = g_rgb ? g_rgb[ch * HW + p] : 0.0;
      g[3] = g_depth ? g_depth[p] : 0.0;
      for (int ch = 0; ch < 3; ++ch) g[4 + ch] = g_normal ? g_normal[ch * HW + p] : 0.0;
      g[7] = g_alpha ? g_alpha[p] : 0.0;
      const int m = (int)list.size();
      // suffix sums S_i = sum_{j>i} v_j w_j of every channel
      std::vector<double> suffix((size_t)(8 * (m + 1)), 0.0);
      for (int i = m - 1; i >= 0; --i) {
        const Entry& e = list[(size_t)i];
        const Surf& s = sc.surf[(size_t)e.h.id];
        double v[8] = {s.rgb[0], s.rgb[1], s.rgb[2], e.h.d, s.n[0], s.n[1], s.n[2], 1.0};
        double w = e.h.alpha * e.T;
        for (int ch = 0; ch < 8; ++ch)
          suffix[(size_t)(8 * i + ch)] = suffix[(size_t)(8 * (i + 1) + ch)] + v[ch] * w;
      }
      for (int i = 0; i < m; ++i) {
        const Entry& e = list[(size_t)i];
        const Hit& h = e.h;
        const Surf& s = sc.surf[(size_t)h.id];
        double v[8] = {s.rgb[0], s.rgb[1], s.rgb[2], h.d, s.n[0], s.n[1], s.n[2], 1.0};
        double w = h.alpha * e.T;
        // d out_ch / d alpha_i = v_i T_i - sum_{j>i} v_j w_j / (1 - alpha_i)
        double dL_dalpha = 0.0;
        for (int ch = 0; ch < 8; ++ch)
          dL_dalpha += g[ch] * (v[ch] * e.T - suffix[(size_t)(8 * (i + 1) + ch)] / (1.0 - h.alpha));
        std::fill(A.begin(), A.end(), 0.0);
        for (int ch = 0; ch < 3; ++ch) A[12 + ch] += w * g[ch];      // colour
        for (int ch = 0; ch < 3; ++ch) A[9 + ch] += w * g[4 + ch];   // normal
        double g_d = w * g[3];
        double dL_dG = 0.0;
        if (!h.clamped) {
          A[15] += h.G * dL_dalpha;
          dL_dG = s.o * dL_dalpha;
        }
        double dL_drho = -0.5 * h.G * dL_dG;
        double gM[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        if (h.branch3d) {
          // rho = u^2 + v^2, d = M_2 . (u, v, 1)
          double gu = 2.0 * h.u * dL_drho + s.M[2][0] * g_d;
          double gv = 2.0 * h.v * dL_drho + s.M[2][1] * g_d;
          gM[2][0] += h.u * g_d;
          gM[2][1] += h.v * g_d;
          gM[2][2] += g_d;
          // u = q0/q2, v = q1/q2
          double gq[3] = {gu / h.q[2], gv / h.q[2], -(gu * h.q[0] + gv * h.q[1]) / (h.q[2] * h.q[2])};
          // q = h_u x h_v
          double ghu[3], ghv[3];
          cross(h.hv, gq, ghu);
          cross(gq, h.hu, ghv);
          for (int cc = 0; cc < 3; ++cc) {
            gM[0][cc] += ghu[cc];
            gM[1][cc] += ghv[cc];
            gM[2][cc] += -(double)x * ghu[cc] - (double)y * ghv[cc];
          }
        } else {
          // rho = s |p - c|^2 with c = (M02/M22, M12/M22); d = M22
          double cx = s.M[0][2] / s.M[2][2], cy = s.M[1][2] / s.M[2][2];
          double gcx = -2.0 * kk.filter_scale * h.dx * dL_drho;
          double gcy = -2.0 * kk.filter_scale * h.dy * dL_drho;
          gM[0][2] += gcx / s.M[2][2];
          gM[1][2] += gcy / s.M[2][2];
          gM[2][2] += -(gcx * cx + gcy * cy) / s.M[2][2] + g_d;
        }
        for (int r = 0; r < 3; ++r)
          for (int cc = 0; cc < 3; ++cc) A[r * 3 + cc] += gM[r][cc];
        double* dst = ac + (size_t)(NA * h.id);
        for (int j = 0; j < NA; ++j) dst[j] += A[(size_t)j];
        if (want_scale) {
          double op[15], ps[6], w0[3], w1[3], w2[3];
          surfel_chain(s, cam, R, A.data(), op, ps, w0, w1, w2);
          if (d_scale) {
            double* da = acc_abs[(size_t)t].data() + (size_t)(15 * h.id);
            for (int j = 0; j < 15; ++j) da[j] += std::fabs(op[j]);
          }
          const bool masked = scale_mask && scale_mask[p];
          for (int j = 0; j < 6; ++j) {
            acc_pose_abs[(size_t)t][(size_t)j] += std::fabs(ps[j]);
            if (masked) acc_pose_abs[(size_t)t][(size_t)(6 + j)] += std::fabs(ps[j]);
          }
        }
      }
    }
  });

  // reduce the per-thread accumulators in thread order
  std::vector<double> tot((size_t)(NA * n), 0.0);
  for (int t = 0; t < nthreads; ++t)
    for (size_t j = 0; j < tot.size(); ++j) tot[j] += acc[(size_t)t][j];
  if (touched) {
    for (int64_t i = 0; i < n; ++i) {
      uint8_t f = 0;
      for (int t = 0; t < nthreads; ++t) f |= tch[(size_t)t][(size_t)i];
      touched[i] = f;
    }
  }

  double pp[6] = {0, 0, 0, 0, 0, 0}, pi[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t i = 0; i < n; ++i) {
    const Surf& s = sc.surf[(size_t)i];
    const double* A = &tot[(size_t)(NA * i)];
    if (d_screen)
      for (int j = 0; j < NA; ++j) d_screen[j * n + i] = A[j];
    double outp[15];
    for (int j = 0; j < 15; ++j) outp[j] = 0.0;
    if (!s.culled) {
      double ps[6], gmu_w[3], gtu_w[3], gtv_w[3];
      surfel_chain(s, cam, R, A, outp, ps, gmu_w, gtu_w, gtv_w);
      for (int j = 0; j < 6; ++j) pp[j] += ps[j];

      // Pose through the world-frame gradients (independent route)
      double Rg[3], Rtu[3], Rtv[3], c1[3], c2[3], c3[3];
      for (int r = 0; r < 3; ++r) {
        Rg[r] = R[r * 4 + 0] * gmu_w[0] + R[r * 4 + 1] * gmu_w[1] + R[r * 4 + 2] * gmu_w[2];
        Rtu[r] = R[r * 4 + 0] * gtu_w[0] + R[r * 4 + 1] * gtu_w[1] + R[r * 4 + 2] * gtu_w[2];
        Rtv[r] = R[r * 4 + 0] * gtv_w[0] + R[r * 4 + 1] * gtv_w[1] + R[r * 4 + 2] * gtv_w[2];
      }
      cross(s.mu_c, Rg, c1);
      cross(s.tuc, Rtu, c2);
      cross(s.tvc, Rtv, c3);
      for (int cc = 0; cc < 3; ++cc) {
        pi[cc] += Rg[cc];
        pi[3 + cc] += c1[cc] + c2[cc] + c3[cc];
      }
    }
    if (d_params)
      for (int j = 0; j < 15; ++j) d_params[j * n + i] = outp[j];
  }
  if (d_scale) {
    std::vector<double> sc15((size_t)(15 * n), 0.0);
    for (int t = 0; t < nthreads; ++t)
      for (size_t j = 0; j < sc15.size(); ++j) sc15[j] += acc_abs[(size_t)t][j];
    for (int64_t i = 0; i < n; ++i)
      for (int j = 0; j < 15; ++j) d_scale[j * n + i] = sc15[(size_t)(15 * i + j)];
  }
  if (pose_scale || pose_scale_masked) {
    double tot_abs[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int t = 0; t < nthreads; ++t)
      for (int j = 0; j < 12; ++j) tot_abs[j] += acc_pose_abs[(size_t)t][(size_t)j];
    for (int j = 0; j < 6; ++j) {
      if (pose_scale) pose_scale[j] = tot_abs[j];
      if (pose_scale_masked) pose_scale_masked[j] = tot_abs[6 + j];
    }
  }
  if (d_pose_paper)
    for (int j = 0; j < 6; ++j) d_pose_paper[j] = pp[j];
  if (d_pose_identity)
    for (int j = 0; j < 6; ++j) d_pose_identity[j] = pi[j];
  return 0;
}

}  // extern "C"
