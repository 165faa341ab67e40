// ECsim per-step particle hot path: plain, slow FP64 CPU oracle.
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call
// this file; only the test-suite, the smoke check and the CPU baseline of the
// benchmark do. It shares no source, header, table or helper with the GPU path.
//
// Every function below computes a definition from Sec. II of the paper
// ("Code structure") directly, in the paper's order, with plain loops:
//   * interpolation weights W_pN: linear (cloud-in-cell) in each dimension,
//     two nodes per dimension, eight in total (Sec. II after Eq. 1; Sec. III,
//     description of computeMoments);
//   * rotation matrix alpha_p (Eq. 2);
//   * hatted current J_sN (Eq. 1);
//   * mass matrices M_NN' for all 27 neighbour offsets (Eq. 3); the paper's
//     14 stored blocks are a view of these 27, obtained by symmetry;
//   * theta-scheme field equations (Eqs. 6-7), solved for E^{n+theta} with
//     restarted GMRES, then the field advance to n+1;
//   * particle mover (Eqs. 4, 5, 8);
//   * total energy, conserved by the scheme for theta = 1/2;
//   * diagnostic moments of the output routines (Sec. III, diagnostics for
//     I/O): charge density, charge current without the velocity rotation,
//     and the charge-weighted second velocity moment (pressure tensor).
// Units: Gaussian with 4 pi, c = 1, theta = 1/2. Node index
// ix + nx*(iy + ny*iz); periodic in all directions. Built with
// -O2 -fno-fast-math -ffp-contract=off.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kFourPi = 4.0 * kPi;
constexpr double kTheta = 0.5;
constexpr double kC = 1.0;

// ---------------------------------------------------------------------------
// forward-mode dual numbers (used only for the reference gradient)
// ---------------------------------------------------------------------------
constexpr int kND = 78;   // 3 x + 3 v + 24 E(pre) + 24 B(pre) + 24 B(post)
struct Dual {
  double v;
  double d[kND];
  Dual() : v(0) { std::memset(d, 0, sizeof d); }
  Dual(double a) : v(a) { std::memset(d, 0, sizeof d); }
};
inline Dual operator+(const Dual& a, const Dual& b) { Dual r(a.v + b.v); for (int i = 0; i < kND; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r(a.v - b.v); for (int i = 0; i < kND; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
inline Dual operator-(const Dual& a) { Dual r(-a.v); for (int i = 0; i < kND; ++i) r.d[i] = -a.d[i]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r(a.v * b.v); for (int i = 0; i < kND; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r(a.v / b.v);
  double ib2 = 1.0 / (b.v * b.v);
  for (int i = 0; i < kND; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) * ib2;
  return r;
}
inline Dual operator+(const Dual& a, double b) { Dual r(a); r.v += b; return r; }
inline Dual operator+(double b, const Dual& a) { return a + b; }
inline Dual operator-(const Dual& a, double b) { Dual r(a); r.v -= b; return r; }
inline Dual operator-(double b, const Dual& a) { return Dual(b) - a; }
inline Dual operator*(const Dual& a, double b) { Dual r(a.v * b); for (int i = 0; i < kND; ++i) r.d[i] = a.d[i] * b; return r; }
inline Dual operator*(double b, const Dual& a) { return a * b; }
inline Dual operator/(const Dual& a, double b) { Dual r(a.v / b); for (int i = 0; i < kND; ++i) r.d[i] = a.d[i] / b; return r; }
inline Dual& operator+=(Dual& a, const Dual& b) { a = a + b; return a; }

inline double value(double a) { return a; }
inline double value(const Dual& a) { return a.v; }

// ---------------------------------------------------------------------------
// grid
// ---------------------------------------------------------------------------
struct Grid {
  int n[3];
  double h[3];
  double dt;
  double V() const { return h[0] * h[1] * h[2]; }
  int64_t nn() const { return (int64_t)n[0] * n[1] * n[2]; }
  double L(int d) const { return n[d] * h[d]; }
  int64_t node(int64_t ix, int64_t iy, int64_t iz) const {
    ix %= n[0]; if (ix < 0) ix += n[0];
    iy %= n[1]; if (iy < 0) iy += n[1];
    iz %= n[2]; if (iz < 0) iz += n[2];
    return ix + (int64_t)n[0] * (iy + (int64_t)n[1] * iz);
  }
};

inline Grid make_grid(const int32_t* n, const double* h, double dt) {
  Grid g;
  for (int d = 0; d < 3; ++d) { g.n[d] = n[d]; g.h[d] = h[d]; }
  g.dt = dt;
  return g;
}

// Offset index in the 27-block storage: (ox+1) + 3 (oy+1) + 9 (oz+1).
inline int off27(int ox, int oy, int oz) { return (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1); }

// The 14 stored offsets: 0, then the 13 offsets whose first non-zero component,
// scanning z, y, x, is positive. Order: (0,0,0); (1,0,0); (-1..1, 1, 0);
// (-1..1 in x, -1..1 in y, 1).
void canonical14(int o[14][3]) {
  int k = 0;
  o[k][0] = 0; o[k][1] = 0; o[k][2] = 0; ++k;
  o[k][0] = 1; o[k][1] = 0; o[k][2] = 0; ++k;
  for (int ox = -1; ox <= 1; ++ox) { o[k][0] = ox; o[k][1] = 1; o[k][2] = 0; ++k; }
  for (int oy = -1; oy <= 1; ++oy)
    for (int ox = -1; ox <= 1; ++ox) { o[k][0] = ox; o[k][1] = oy; o[k][2] = 1; ++k; }
}

// ---------------------------------------------------------------------------
// interpolation: linear weights between the two nearest nodes per dimension
// ---------------------------------------------------------------------------
template <class T>
struct Stencil {
  int64_t lo[3];   // index of the lower node N^- in each dimension
  T w[3][2];       // w[d][0] weight of N^-, w[d][1] weight of N^+ = N^- + 1
};

template <class T>
Stencil<T> stencil(const Grid& g, const T x[3]) {
  Stencil<T> s;
  for (int d = 0; d < 3; ++d) {
    T u = x[d] / g.h[d];
    double fl = std::floor(value(u));
    s.lo[d] = (int64_t)fl;
    T xi = u - fl;
    s.w[d][0] = 1.0 - xi;
    s.w[d][1] = xi;
  }
  return s;
}

template <class T>
T corner_weight(const Stencil<T>& s, int ax, int ay, int az) {
  return s.w[0][ax] * s.w[1][ay] * s.w[2][az];
}

template <class T>
int64_t corner_node(const Grid& g, const Stencil<T>& s, int ax, int ay, int az) {
  return g.node(s.lo[0] + ax, s.lo[1] + ay, s.lo[2] + az);
}

// F_p = sum over the 8 corners of W_a F_N[node(a)], F given as [3][Nn].
template <class T>
void gather(const Grid& g, const Stencil<T>& s, const double* F, T out[3]) {
  const int64_t nn = g.nn();
  for (int c = 0; c < 3; ++c) out[c] = T(0.0);
  for (int az = 0; az < 2; ++az)
    for (int ay = 0; ay < 2; ++ay)
      for (int ax = 0; ax < 2; ++ax) {
        T w = corner_weight(s, ax, ay, az);
        int64_t nd = corner_node(g, s, ax, ay, az);
        for (int c = 0; c < 3; ++c) out[c] = out[c] + w * F[c * nn + nd];
      }
}

// Rotation matrix of Eq. 2 for the Lorentz force q(E + v x B) (c = 1):
//   alpha = (I - beta [B x] + beta^2 B B^T) / (1 + beta^2 |B|^2),
// with [B x] u = B x u, so that alpha u solves  vbar - beta vbar x B = u.
template <class T>
void rotation(const T B[3], double beta, T a[9]) {
  T bx = beta * B[0], by = beta * B[1], bz = beta * B[2];
  T den = 1.0 + (bx * bx + by * by + bz * bz);
  // I + beta^2 B B^T
  a[0] = 1.0 + bx * bx; a[1] = bx * by;       a[2] = bx * bz;
  a[3] = by * bx;       a[4] = 1.0 + by * by; a[5] = by * bz;
  a[6] = bz * bx;       a[7] = bz * by;       a[8] = 1.0 + bz * bz;
  // - beta [B x]:  [B x] = [[0,-Bz,By],[Bz,0,-Bx],[-By,Bx,0]]
  a[1] = a[1] + bz; a[2] = a[2] - by;
  a[3] = a[3] - bz; a[5] = a[5] + bx;
  a[6] = a[6] + by; a[7] = a[7] - bx;
  for (int i = 0; i < 9; ++i) a[i] = a[i] / den;
}

template <class T>
void matvec(const T a[9], const T u[3], T out[3]) {
  for (int i = 0; i < 3; ++i) out[i] = a[3 * i] * u[0] + a[3 * i + 1] * u[1] + a[3 * i + 2] * u[2];
}

// Position push with periodic wrap into [0, L); a result that rounds to L is 0.
template <class T>
T wrap_position(T x, double L) {
  double k = std::floor(value(x) / L);
  T r = x - k * L;
  if (value(r) >= L) r = r - L;
  if (value(r) < 0.0) r = r + L;
  if (value(r) >= L) r = T(0.0);
  return r;
}

// Mover of Eqs. 4, 5 and 8 for one particle: gathers E^{n+theta} and B^n at
// x^{n-1/2}, vbar = alpha (v + beta E_p), v^{n+1} = 2 vbar - v^n,
// x^{n+1/2} = x^{n-1/2} + dt v^{n+1}. In a reduced (1D or 2D) run the
// positions along the dimensions of a single cell stay where they are: the
// mover's fixPosition step (Sec. III) keeps particles on their line or plane;
// the velocity keeps all three components.
template <class T>
void move_one(const Grid& g, double beta, T x[3], T v[3], const T Ep[3], const T Bp[3]) {
  T a[9];
  rotation(Bp, beta, a);
  T u[3], vb[3];
  for (int c = 0; c < 3; ++c) u[c] = v[c] + beta * Ep[c];
  matvec(a, u, vb);
  for (int c = 0; c < 3; ++c) v[c] = 2.0 * vb[c] - v[c];
  for (int c = 0; c < 3; ++c)
    if (g.n[c] > 1) x[c] = wrap_position(x[c] + g.dt * v[c], g.L(c));
}

// Neumaier-compensated sum.
struct KSum {
  double s = 0.0, c = 0.0;
  void add(double y) {
    double t = s + y;
    if (std::fabs(s) >= std::fabs(y)) c += (s - t) + y; else c += (y - t) + s;
    s = t;
  }
  double get() const { return s + c; }
};

// ---------------------------------------------------------------------------
// staggered grid operators (E, J on nodes; B on cell centres)
// ---------------------------------------------------------------------------
// Cell c = (cx, cy, cz) spans [c h, (c+1) h); its centre carries B_C. Node g
// sits at g h. Each derivative is the average of the four edge differences
// parallel to that axis, which makes curl_N the transpose of curl_C.
void curl_C(const Grid& g, const double* E, double* out) {
  const int64_t nn = g.nn();
  for (int cz = 0; cz < g.n[2]; ++cz)
    for (int cy = 0; cy < g.n[1]; ++cy)
      for (int cx = 0; cx < g.n[0]; ++cx) {
        double d[3][3] = {{0}};   // d[axis][component]
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) {
            for (int comp = 0; comp < 3; ++comp) {
              const double* F = E + comp * nn;
              d[0][comp] += F[g.node(cx + 1, cy + a, cz + b)] - F[g.node(cx, cy + a, cz + b)];
              d[1][comp] += F[g.node(cx + a, cy + 1, cz + b)] - F[g.node(cx + a, cy, cz + b)];
              d[2][comp] += F[g.node(cx + a, cy + b, cz + 1)] - F[g.node(cx + a, cy + b, cz)];
            }
          }
        for (int ax = 0; ax < 3; ++ax)
          for (int comp = 0; comp < 3; ++comp) d[ax][comp] /= 4.0 * g.h[ax];
        int64_t c = g.node(cx, cy, cz);
        out[0 * nn + c] = d[1][2] - d[2][1];
        out[1 * nn + c] = d[2][0] - d[0][2];
        out[2 * nn + c] = d[0][1] - d[1][0];
      }
}

void curl_N(const Grid& g, const double* B, double* out) {
  const int64_t nn = g.nn();
  for (int gz = 0; gz < g.n[2]; ++gz)
    for (int gy = 0; gy < g.n[1]; ++gy)
      for (int gx = 0; gx < g.n[0]; ++gx) {
        // the 8 cells around node g are g - 1 + a, a in {0,1}^3
        double d[3][3] = {{0}};
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) {
            for (int comp = 0; comp < 3; ++comp) {
              const double* F = B + comp * nn;
              d[0][comp] += F[g.node(gx, gy - 1 + a, gz - 1 + b)] - F[g.node(gx - 1, gy - 1 + a, gz - 1 + b)];
              d[1][comp] += F[g.node(gx - 1 + a, gy, gz - 1 + b)] - F[g.node(gx - 1 + a, gy - 1, gz - 1 + b)];
              d[2][comp] += F[g.node(gx - 1 + a, gy - 1 + b, gz)] - F[g.node(gx - 1 + a, gy - 1 + b, gz - 1)];
            }
          }
        for (int ax = 0; ax < 3; ++ax)
          for (int comp = 0; comp < 3; ++comp) d[ax][comp] /= 4.0 * g.h[ax];
        int64_t c = g.node(gx, gy, gz);
        out[0 * nn + c] = d[1][2] - d[2][1];
        out[1 * nn + c] = d[2][0] - d[0][2];
        out[2 * nn + c] = d[0][1] - d[1][0];
      }
}

// node value = mean of the 8 cell-centred values around the node
void centres_to_nodes(const Grid& g, const double* BC, double* BN) {
  const int64_t nn = g.nn();
  for (int gz = 0; gz < g.n[2]; ++gz)
    for (int gy = 0; gy < g.n[1]; ++gy)
      for (int gx = 0; gx < g.n[0]; ++gx) {
        int64_t nd = g.node(gx, gy, gz);
        for (int comp = 0; comp < 3; ++comp) {
          double s = 0.0;
          for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
              for (int c = 0; c < 2; ++c) s += BC[comp * nn + g.node(gx - 1 + a, gy - 1 + b, gz - 1 + c)];
          BN[comp * nn + nd] = s / 8.0;
        }
      }
}

// (M E)_g = sum over the 27 offsets o of M27[g][o] E[g + o], M27 as [27][9][Nn].
void mass_apply27(const Grid& g, const double* M27, const double* E, double* y) {
  const int64_t nn = g.nn();
  for (int gz = 0; gz < g.n[2]; ++gz)
    for (int gy = 0; gy < g.n[1]; ++gy)
      for (int gx = 0; gx < g.n[0]; ++gx) {
        int64_t nd = g.node(gx, gy, gz);
        double acc[3] = {0, 0, 0};
        for (int oz = -1; oz <= 1; ++oz)
          for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
              int k = off27(ox, oy, oz);
              int64_t nb = g.node(gx + ox, gy + oy, gz + oz);
              for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                  acc[i] += M27[((int64_t)k * 9 + 3 * i + j) * nn + nd] * E[j * nn + nb];
            }
        for (int i = 0; i < 3; ++i) y[i * nn + nd] = acc[i];
      }
}

// The implicit field operator of Eqs. 6-7 after eliminating B^{n+theta}:
//   A E = E + (c theta dt)^2 curl_N curl_C E + 4 pi theta dt (M E).
struct FieldOp {
  const Grid& g;
  const double* M27;
  std::vector<double> tc, tn, tm;
  explicit FieldOp(const Grid& gg, const double* m) : g(gg), M27(m), tc(3 * gg.nn()), tn(3 * gg.nn()), tm(3 * gg.nn()) {}
  void apply(const double* E, double* out) {
    const int64_t n3 = 3 * g.nn();
    const double ctd = kC * kTheta * g.dt;
    curl_C(g, E, tc.data());
    curl_N(g, tc.data(), tn.data());
    mass_apply27(g, M27, E, tm.data());
    for (int64_t i = 0; i < n3; ++i) out[i] = E[i] + ctd * ctd * tn[i] + kFourPi * kTheta * g.dt * tm[i];
  }
};

double dot(const double* a, const double* b, int64_t n) {
  KSum s;
  for (int64_t i = 0; i < n; ++i) s.add(a[i] * b[i]);
  return s.get();
}

// Restarted GMRES(m), modified Gram-Schmidt, Givens rotations, no
// preconditioner; stops when ||b - A x||_2 <= tol ||b||_2 (true residual).
int gmres(FieldOp& op, const double* b, double* x, int64_t n, double tol, int m, int maxit,
          double* rel_out) {
  std::vector<double> r(n), w(n), V((size_t)(m + 1) * n), H((size_t)(m + 1) * m), cs(m), sn(m), e(m + 1), yv(m);
  const double bnorm = std::sqrt(dot(b, b, n));
  if (bnorm == 0.0) { for (int64_t i = 0; i < n; ++i) x[i] = 0.0; *rel_out = 0.0; return 0; }
  int it = 0;
  double rel = 0.0;
  while (true) {
    op.apply(x, w.data());
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - w[i];
    double beta = std::sqrt(dot(r.data(), r.data(), n));
    rel = beta / bnorm;
    if (rel <= tol || it >= maxit) break;
    for (int64_t i = 0; i < n; ++i) V[i] = r[i] / beta;
    std::fill(e.begin(), e.end(), 0.0);
    e[0] = beta;
    int j = 0;
    for (; j < m && it < maxit; ++j, ++it) {
      op.apply(&V[(size_t)j * n], w.data());
      for (int i = 0; i <= j; ++i) {
        double hij = dot(w.data(), &V[(size_t)i * n], n);
        H[(size_t)i * m + j] = hij;
        for (int64_t k = 0; k < n; ++k) w[k] -= hij * V[(size_t)i * n + k];
      }
      double hn = std::sqrt(dot(w.data(), w.data(), n));
      H[(size_t)(j + 1) * m + j] = hn;
      if (hn > 0.0)
        for (int64_t k = 0; k < n; ++k) V[(size_t)(j + 1) * n + k] = w[k] / hn;
      for (int i = 0; i < j; ++i) {
        double t = cs[i] * H[(size_t)i * m + j] + sn[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)(i + 1) * m + j] = -sn[i] * H[(size_t)i * m + j] + cs[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = t;
      }
      double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
      double rr = std::hypot(a, bb);
      cs[j] = a / rr; sn[j] = bb / rr;
      H[(size_t)j * m + j] = rr;
      H[(size_t)(j + 1) * m + j] = 0.0;
      e[j + 1] = -sn[j] * e[j];
      e[j] = cs[j] * e[j];
      if (std::fabs(e[j + 1]) <= tol * bnorm * 0.5 || hn == 0.0) { ++j; ++it; break; }
    }
    // back substitution on the j x j triangle
    for (int i = j - 1; i >= 0; --i) {
      double s = e[i];
      for (int k = i + 1; k < j; ++k) s -= H[(size_t)i * m + k] * yv[k];
      yv[i] = s / H[(size_t)i * m + i];
    }
    for (int i = 0; i < j; ++i)
      for (int64_t k = 0; k < n; ++k) x[k] += yv[i] * V[(size_t)i * n + k];
  }
  *rel_out = rel;
  return it;
}

// Eqs. 1 and 3 for one particle at position xp with velocity vp: J += its
// current q vhat W_N / V, M27 += its 64 corner-pair blocks.
void deposit_particle(const Grid& g, double beta, double qp, const double xp[3], const double vp[3],
                      const double* B_node, double* J, double* M27) {
  const int64_t nn = g.nn();
  const double V = g.V();
  Stencil<double> s = stencil(g, xp);
  double Bp[3];
  gather(g, s, B_node, Bp);
  double a[9];
  rotation(Bp, beta, a);
  double vhat[3];
  matvec(a, vp, vhat);
  // Eq. 1: J_N += q_p vhat_p W_pN / V_N
  for (int az = 0; az < 2; ++az)
    for (int ay = 0; ay < 2; ++ay)
      for (int ax = 0; ax < 2; ++ax) {
        double w = corner_weight(s, ax, ay, az);
        int64_t nd = corner_node(g, s, ax, ay, az);
        for (int c = 0; c < 3; ++c) J[c * nn + nd] += qp * vhat[c] * w / V;
      }
  // Eq. 3: M_{N N'} += beta_p q_p alpha_p W_pN' W_pN / V_N for every ordered
  // pair of corners (a, b); N = node(a), N' = node(b), offset o = b - a.
  for (int az = 0; az < 2; ++az)
    for (int ay = 0; ay < 2; ++ay)
      for (int ax = 0; ax < 2; ++ax)
        for (int bz = 0; bz < 2; ++bz)
          for (int by = 0; by < 2; ++by)
            for (int bx = 0; bx < 2; ++bx) {
              double wa = corner_weight(s, ax, ay, az);
              double wb = corner_weight(s, bx, by, bz);
              int64_t nd = corner_node(g, s, ax, ay, az);
              int k = off27(bx - ax, by - ay, bz - az);
              for (int ij = 0; ij < 9; ++ij)
                M27[((int64_t)k * 9 + ij) * nn + nd] += beta * qp * a[ij] * wb * wa / V;
            }
}

// Eqs. 4, 5 and 8 for particle p of [3][np] arrays x, v, in place.
void move_particle(const Grid& g, double beta, int64_t np, int64_t p, double* x, double* v, const double* E_node,
                   const double* B_node) {
  double xp[3] = {x[p], x[np + p], x[2 * np + p]};
  double vp[3] = {v[p], v[np + p], v[2 * np + p]};
  Stencil<double> s = stencil(g, xp);
  double Ep[3], Bp[3];
  gather(g, s, E_node, Ep);
  gather(g, s, B_node, Bp);
  move_one(g, beta, xp, vp, Ep, Bp);
  for (int c = 0; c < 3; ++c) { x[c * np + p] = xp[c]; v[c * np + p] = vp[c]; }
}

}  // namespace

// ===========================================================================
// C interface (ctypes). Arrays are host pointers, owned by the caller.
// Particle positions and velocities are [3][np] structure of arrays; node
// fields [3][Nn]; M27 [27][9][Nn] with offset index (ox+1)+3(oy+1)+9(oz+1)
// and component index 3i+j.
// ===========================================================================
extern "C" {

// Interpolation stencil of one particle: lower node index per dimension and
// the 8 weights W_a, a = ax + 2 ay + 4 az.
void oracle_weights(const int32_t* n, const double* h, const double* x, int64_t* lo, double* W) {
  Grid g = make_grid(n, h, 0.0);
  Stencil<double> s = stencil(g, x);
  for (int d = 0; d < 3; ++d) lo[d] = s.lo[d];
  for (int az = 0; az < 2; ++az)
    for (int ay = 0; ay < 2; ++ay)
      for (int ax = 0; ax < 2; ++ax) W[ax + 2 * ay + 4 * az] = corner_weight(s, ax, ay, az);
}

// Field at the particle positions: out [3][np].
void oracle_gather(const int32_t* n, const double* h, int64_t np, const double* x, const double* F, double* out) {
  Grid g = make_grid(n, h, 0.0);
  for (int64_t p = 0; p < np; ++p) {
    double xp[3] = {x[p], x[np + p], x[2 * np + p]};
    Stencil<double> s = stencil(g, xp);
    double f[3];
    gather(g, s, F, f);
    for (int c = 0; c < 3; ++c) out[c * np + p] = f[c];
  }
}

void oracle_alpha(const double* B, double beta, double* a) { rotation(B, beta, a); }

// Diagnostic moments (Sec. III, diagnostics for I/O), accumulated (+=):
//   rho [Nn]:   sum_p q_p W_pN / V_N                 (charge density)
//   Jd  [3][Nn]: sum_p q_p v_p W_pN / V_N            (current, no rotation)
//   P   [6][Nn]: sum_p q_p v_i v_j W_pN / V_N, components xx, xy, xz, yy,
//                yz, zz (charge-weighted second velocity moment)
// at the particles' positions x with velocities v as given.
void oracle_diagnostics(const int32_t* n, const double* h, int64_t np, const double* x, const double* v,
                        const double* q, double q_const, double* rho, double* Jd, double* P) {
  Grid g = make_grid(n, h, 1.0);
  const int64_t nn = g.nn();
  const double V = g.V();
  const int pi[6] = {0, 0, 0, 1, 1, 2}, pj[6] = {0, 1, 2, 1, 2, 2};
  for (int64_t p = 0; p < np; ++p) {
    const double qp = q ? q[p] : q_const;
    double xp[3] = {x[p], x[np + p], x[2 * np + p]};
    double vp[3] = {v[p], v[np + p], v[2 * np + p]};
    Stencil<double> s = stencil(g, xp);
    for (int az = 0; az < 2; ++az)
      for (int ay = 0; ay < 2; ++ay)
        for (int ax = 0; ax < 2; ++ax) {
          const double w = corner_weight(s, ax, ay, az);
          const int64_t nd = corner_node(g, s, ax, ay, az);
          rho[nd] += qp * w / V;
          for (int c = 0; c < 3; ++c) Jd[c * nn + nd] += qp * vp[c] * w / V;
          for (int c = 0; c < 6; ++c) P[c * nn + nd] += qp * vp[pi[c]] * vp[pj[c]] * w / V;
        }
  }
}

// Moments of Eqs. 1 and 3, accumulated (+=) into J [3][Nn] and M27 [27][9][Nn].
// q: per-particle charge (or NULL to use q_const). B_node: node magnetic field.
void oracle_moments(const int32_t* n, const double* h, double dt, int64_t np, const double* x,
                    const double* v, const double* q, double q_const, double qom,
                    const double* B_node, double* J, double* M27) {
  Grid g = make_grid(n, h, dt);
  const double beta = qom * dt / 2.0;
  for (int64_t p = 0; p < np; ++p) {
    const double qp = q ? q[p] : q_const;
    double xp[3] = {x[p], x[np + p], x[2 * np + p]};
    double vp[3] = {v[p], v[np + p], v[2 * np + p]};
    deposit_particle(g, beta, qp, xp, vp, B_node, J, M27);
  }
}

// The 14 stored blocks as a view of the 27: M14[k][ij][g] = M27[o_k][ij][g].
void oracle_m14_from_m27(const int32_t* n, const double* M27, double* M14) {
  const int64_t nn = (int64_t)n[0] * n[1] * n[2];
  int o[14][3];
  canonical14(o);
  for (int k = 0; k < 14; ++k) {
    int k27 = off27(o[k][0], o[k][1], o[k][2]);
    std::memcpy(M14 + (int64_t)k * 9 * nn, M27 + (int64_t)k27 * 9 * nn, sizeof(double) * 9 * nn);
  }
}

void oracle_canonical14(int32_t* out) {
  int o[14][3];
  canonical14(o);
  for (int k = 0; k < 14; ++k)
    for (int d = 0; d < 3; ++d) out[3 * k + d] = o[k][d];
}

void oracle_mass_apply27(const int32_t* n, const double* M27, const double* E, double* y) {
  double h[3] = {1, 1, 1};
  Grid g = make_grid(n, h, 0.0);
  mass_apply27(g, M27, E, y);
}

// Mover of Eqs. 4, 5, 8, in place on x [3][np] and v [3][np].
void oracle_move(const int32_t* n, const double* h, double dt, int64_t np, double* x, double* v,
                 double qom, const double* E_node, const double* B_node) {
  Grid g = make_grid(n, h, dt);
  const double beta = qom * dt / 2.0;
  for (int64_t p = 0; p < np; ++p) move_particle(g, beta, np, p, x, v, E_node, B_node);
}

// The mover and then the moments at the moved positions (the particle pass
// of one step, as timed for the CPU baseline), over `threads` threads: each
// thread moves a contiguous share of the particles in place and deposits them
// into its own zeroed J and M27; the thread grids are then added into J and
// M27 (+=) in thread order, so the result does not depend on scheduling.
// threads = 1 runs the same code on one thread. Returns the threads used.
int oracle_move_moments_threads(const int32_t* n, const double* h, double dt, int64_t np, double* x, double* v,
                                const double* q, double q_const, double qom, const double* E_node,
                                const double* B_node, const double* B_next, double* J, double* M27,
                                int threads) {
  Grid g = make_grid(n, h, dt);
  const int64_t nn = g.nn();
  const double beta = qom * dt / 2.0;
  if (threads < 1) threads = 1;
  std::vector<std::vector<double>> Jt(threads), Mt(threads);
  int used = 1;
#pragma omp parallel num_threads(threads)
  {
    int t = 0, nt = 1;
#ifdef _OPENMP
    t = omp_get_thread_num();
    nt = omp_get_num_threads();
#endif
#pragma omp single
    used = nt;
    Jt[t].assign((size_t)3 * nn, 0.0);
    Mt[t].assign((size_t)27 * 9 * nn, 0.0);
    const int64_t p0 = np * t / nt, p1 = np * (t + 1) / nt;
    for (int64_t p = p0; p < p1; ++p) {
      move_particle(g, beta, np, p, x, v, E_node, B_node);
      const double qp = q ? q[p] : q_const;
      double xp[3] = {x[p], x[np + p], x[2 * np + p]};
      double vp[3] = {v[p], v[np + p], v[2 * np + p]};
      deposit_particle(g, beta, qp, xp, vp, B_next, Jt[t].data(), Mt[t].data());
    }
#pragma omp barrier
    // fixed-order reduction: every entry sums the thread grids in order 0..nt-1
#pragma omp for schedule(static)
    for (int64_t i = 0; i < 27 * 9 * nn; ++i) {
      double s = M27[i];
      for (int u = 0; u < nt; ++u) s += Mt[u][i];
      M27[i] = s;
    }
#pragma omp for schedule(static)
    for (int64_t i = 0; i < 3 * nn; ++i) {
      double s = J[i];
      for (int u = 0; u < nt; ++u) s += Jt[u][i];
      J[i] = s;
    }
  }
  return used;
}

void oracle_curl_C(const int32_t* n, const double* h, const double* E, double* out) {
  Grid g = make_grid(n, h, 0.0);
  curl_C(g, E, out);
}

void oracle_curl_N(const int32_t* n, const double* h, const double* B, double* out) {
  Grid g = make_grid(n, h, 0.0);
  curl_N(g, B, out);
}

void oracle_centres_to_nodes(const int32_t* n, const double* BC, double* BN) {
  double h[3] = {1, 1, 1};
  Grid g = make_grid(n, h, 0.0);
  centres_to_nodes(g, BC, BN);
}

// out = A E for the implicit field operator.
void oracle_field_operator(const int32_t* n, const double* h, double dt, const double* M27,
                           const double* E, double* out) {
  Grid g = make_grid(n, h, dt);
  FieldOp op(g, M27);
  op.apply(E, out);
}

// Right-hand side b = E^n - 4 pi theta dt J + c theta dt curl_N B_C^n.
void oracle_field_rhs(const int32_t* n, const double* h, double dt, const double* J,
                      const double* E_n, const double* BC_n, double* b) {
  Grid g = make_grid(n, h, dt);
  const int64_t n3 = 3 * g.nn();
  std::vector<double> cb(n3);
  curl_N(g, BC_n, cb.data());
  for (int64_t i = 0; i < n3; ++i)
    b[i] = E_n[i] - kFourPi * kTheta * dt * J[i] + kC * kTheta * dt * cb[i];
}

// Solves A E^{n+theta} = b (GMRES from E^n), then advances the fields:
// B_C^{n+theta} = B_C^n - c theta dt curl_C E^{n+theta},
// E^{n+1} = E^{n+theta}/theta + (theta-1)/theta E^n, same for B.
// Outputs E_theta, E_next, BC_next ([3][Nn] each); returns iterations, or -1
// if the tolerance was not reached in maxit iterations.
int oracle_field_solve(const int32_t* n, const double* h, double dt, const double* M27, const double* J,
                       const double* E_n, const double* BC_n, double tol, int restart, int maxit,
                       double* E_theta, double* E_next, double* BC_next, double* rel_resid) {
  Grid g = make_grid(n, h, dt);
  const int64_t n3 = 3 * g.nn();
  std::vector<double> b(n3), cc(n3);
  oracle_field_rhs(n, h, dt, J, E_n, BC_n, b.data());
  FieldOp op(g, M27);
  for (int64_t i = 0; i < n3; ++i) E_theta[i] = E_n[i];
  int it = gmres(op, b.data(), E_theta, n3, tol, restart, maxit, rel_resid);
  curl_C(g, E_theta, cc.data());
  for (int64_t i = 0; i < n3; ++i) {
    double bt = BC_n[i] - kC * kTheta * dt * cc[i];
    BC_next[i] = bt / kTheta + (kTheta - 1.0) / kTheta * BC_n[i];
    E_next[i] = E_theta[i] / kTheta + (kTheta - 1.0) / kTheta * E_n[i];
  }
  return (*rel_resid <= tol) ? it : -1;
}

// Energies: K = sum 1/2 m_p |v_p|^2 with m_p = q_p / (q/m); W_E = V/(8 pi) sum E_N^2;
// W_B = V/(8 pi) sum B_C^2. Compensated sums.
double oracle_kinetic(int64_t np, const double* v, const double* q, double q_const, double qom) {
  KSum s;
  for (int64_t p = 0; p < np; ++p) {
    double m = (q ? q[p] : q_const) / qom;
    double v2 = v[p] * v[p] + v[np + p] * v[np + p] + v[2 * np + p] * v[2 * np + p];
    s.add(0.5 * m * v2);
  }
  return s.get();
}

double oracle_field_energy(const int32_t* n, const double* h, const double* F) {
  const int64_t n3 = 3 * (int64_t)n[0] * n[1] * n[2];
  KSum s;
  for (int64_t i = 0; i < n3; ++i) s.add(F[i] * F[i]);
  return h[0] * h[1] * h[2] / (8.0 * kPi) * s.get();
}

// Reference gradient of L = <gJ, J> + <gM, M14> through mover -> moments,
// both with the same node field B, for the particles of one species.
// Forward-mode dual numbers seeded on each particle's own x, v and on the 72
// local stencil field values; the local Jacobian is scattered to the grids.
// gx, gv: [3][np] (overwritten); gE, gB: [3][Nn] (accumulated).
void oracle_grad(const int32_t* n, const double* h, double dt, int64_t np, const double* x,
                 const double* v, const double* q, double q_const, double qom,
                 const double* E_node, const double* B_node, const double* gJ, const double* gM,
                 double* gx, double* gv, double* gE, double* gB) {
  Grid g = make_grid(n, h, dt);
  const int64_t nn = g.nn();
  const double V = g.V();
  const double beta = qom * dt / 2.0;
  int o14[14][3];
  canonical14(o14);
  int k14_of27[27];
  for (int i = 0; i < 27; ++i) k14_of27[i] = -1;
  for (int k = 0; k < 14; ++k) k14_of27[off27(o14[k][0], o14[k][1], o14[k][2])] = k;

  for (int64_t p = 0; p < np; ++p) {
    const double qp = q ? q[p] : q_const;
    Dual X[3], Vv[3];
    for (int c = 0; c < 3; ++c) {
      X[c] = Dual(x[c * np + p]); X[c].d[c] = 1.0;
      Vv[c] = Dual(v[c * np + p]); Vv[c].d[3 + c] = 1.0;
    }
    // pre-move stencil and seeded local field values
    Stencil<Dual> s0 = stencil(g, X);
    Dual Ep[3], Bp[3];
    int64_t pre_nodes[8];
    for (int c = 0; c < 3; ++c) { Ep[c] = Dual(0.0); Bp[c] = Dual(0.0); }
    for (int az = 0; az < 2; ++az)
      for (int ay = 0; ay < 2; ++ay)
        for (int ax = 0; ax < 2; ++ax) {
          int a = ax + 2 * ay + 4 * az;
          int64_t nd = corner_node(g, s0, ax, ay, az);
          pre_nodes[a] = nd;
          Dual w = corner_weight(s0, ax, ay, az);
          for (int c = 0; c < 3; ++c) {
            Dual Ev(E_node[c * nn + nd]); Ev.d[6 + 3 * a + c] = 1.0;
            Dual Bv(B_node[c * nn + nd]); Bv.d[30 + 3 * a + c] = 1.0;
            Ep[c] = Ep[c] + w * Ev;
            Bp[c] = Bp[c] + w * Bv;
          }
        }
    move_one(g, beta, X, Vv, Ep, Bp);
    // post-move moments
    Stencil<Dual> s1 = stencil(g, X);
    Dual B1[3];
    int64_t post_nodes[8];
    for (int c = 0; c < 3; ++c) B1[c] = Dual(0.0);
    for (int az = 0; az < 2; ++az)
      for (int ay = 0; ay < 2; ++ay)
        for (int ax = 0; ax < 2; ++ax) {
          int a = ax + 2 * ay + 4 * az;
          int64_t nd = corner_node(g, s1, ax, ay, az);
          post_nodes[a] = nd;
          Dual w = corner_weight(s1, ax, ay, az);
          for (int c = 0; c < 3; ++c) {
            Dual Bv(B_node[c * nn + nd]); Bv.d[54 + 3 * a + c] = 1.0;
            B1[c] = B1[c] + w * Bv;
          }
        }
    Dual al[9];
    rotation(B1, beta, al);
    Dual vhat[3];
    matvec(al, Vv, vhat);
    Dual loss(0.0);
    for (int az = 0; az < 2; ++az)
      for (int ay = 0; ay < 2; ++ay)
        for (int ax = 0; ax < 2; ++ax) {
          Dual w = corner_weight(s1, ax, ay, az);
          int64_t nd = post_nodes[ax + 2 * ay + 4 * az];
          for (int c = 0; c < 3; ++c) loss = loss + gJ[c * nn + nd] * (qp * vhat[c] * w / V);
        }
    for (int az = 0; az < 2; ++az)
      for (int ay = 0; ay < 2; ++ay)
        for (int ax = 0; ax < 2; ++ax)
          for (int bz = 0; bz < 2; ++bz)
            for (int by = 0; by < 2; ++by)
              for (int bx = 0; bx < 2; ++bx) {
                int k = k14_of27[off27(bx - ax, by - ay, bz - az)];
                if (k < 0) continue;   // the mirrored pair carries this block
                Dual wa = corner_weight(s1, ax, ay, az);
                Dual wb = corner_weight(s1, bx, by, bz);
                int64_t nd = post_nodes[ax + 2 * ay + 4 * az];
                for (int ij = 0; ij < 9; ++ij)
                  loss = loss + gM[((int64_t)k * 9 + ij) * nn + nd] * (beta * qp * al[ij] * wb * wa / V);
              }
    for (int c = 0; c < 3; ++c) {
      gx[c * np + p] = loss.d[c];
      gv[c * np + p] = loss.d[3 + c];
    }
    for (int a = 0; a < 8; ++a)
      for (int c = 0; c < 3; ++c) {
        gE[c * nn + pre_nodes[a]] += loss.d[6 + 3 * a + c];
        gB[c * nn + pre_nodes[a]] += loss.d[30 + 3 * a + c];
        gB[c * nn + post_nodes[a]] += loss.d[54 + 3 * a + c];
      }
  }
}

// Per-particle loss l_p of the composite (mover -> moments), plain FP64, used
// by finite-difference checks as a sum of per-particle differences.
void oracle_particle_loss(const int32_t* n, const double* h, double dt, int64_t np, const double* x,
                          const double* v, const double* q, double q_const, double qom,
                          const double* E_node, const double* B_node, const double* gJ,
                          const double* gM, double* lp) {
  Grid g = make_grid(n, h, dt);
  const int64_t nn = g.nn();
  const double V = g.V();
  const double beta = qom * dt / 2.0;
  int o14[14][3];
  canonical14(o14);
  int k14_of27[27];
  for (int i = 0; i < 27; ++i) k14_of27[i] = -1;
  for (int k = 0; k < 14; ++k) k14_of27[off27(o14[k][0], o14[k][1], o14[k][2])] = k;
  for (int64_t p = 0; p < np; ++p) {
    const double qp = q ? q[p] : q_const;
    double X[3] = {x[p], x[np + p], x[2 * np + p]};
    double Vv[3] = {v[p], v[np + p], v[2 * np + p]};
    Stencil<double> s0 = stencil(g, X);
    double Ep[3], Bp[3];
    gather(g, s0, E_node, Ep);
    gather(g, s0, B_node, Bp);
    move_one(g, beta, X, Vv, Ep, Bp);
    Stencil<double> s1 = stencil(g, X);
    double B1[3];
    gather(g, s1, B_node, B1);
    double al[9];
    rotation(B1, beta, al);
    double vhat[3];
    matvec(al, Vv, vhat);
    double loss = 0.0;
    for (int az = 0; az < 2; ++az)
      for (int ay = 0; ay < 2; ++ay)
        for (int ax = 0; ax < 2; ++ax) {
          double w = corner_weight(s1, ax, ay, az);
          int64_t nd = corner_node(g, s1, ax, ay, az);
          for (int c = 0; c < 3; ++c) loss += gJ[c * nn + nd] * (qp * vhat[c] * w / V);
        }
    for (int az = 0; az < 2; ++az)
      for (int ay = 0; ay < 2; ++ay)
        for (int ax = 0; ax < 2; ++ax)
          for (int bz = 0; bz < 2; ++bz)
            for (int by = 0; by < 2; ++by)
              for (int bx = 0; bx < 2; ++bx) {
                int k = k14_of27[off27(bx - ax, by - ay, bz - az)];
                if (k < 0) continue;
                double wa = corner_weight(s1, ax, ay, az);
                double wb = corner_weight(s1, bx, by, bz);
                int64_t nd = corner_node(g, s1, ax, ay, az);
                for (int ij = 0; ij < 9; ++ij)
                  loss += gM[((int64_t)k * 9 + ij) * nn + nd] * (beta * qp * al[ij] * wb * wa / V);
              }
    lp[p] = loss;
  }
}

}  // extern "C"
