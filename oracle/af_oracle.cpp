// af_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, FP64 CPU implementation of one forward-Euler stage (and the
// SSP-RK3 step built from it) of the positivity-preserving Active Flux scheme
// for 2D ideal MHD with the Godunov-Powell source term (Duan, Chandrashekar,
// Klingenberg, arXiv 2506.04857).  It exists to check the HIP library: only
// the test suite, the smoke check and the CPU-baseline leg of the benchmark
// may load it.  It shares no code, header or table with the HIP path.
//
// Every step follows the paper in the paper's order; each function names the
// passage it implements.  Where the paper is silent or garbled the reading
// taken is stated at the function (the list of readings is kept with the
// design notes of the repository).  Compile with -ffp-contract=off: no fused
// multiply-adds, plain IEEE double arithmetic, std::sqrt / std::exp.
//
// Index convention (0-based):
//   A(i,j)  cell average of cell (i,j),            i in [0,nx), j in [0,ny)
//   X(k,j)  point value at (x_{k-1/2}, y_j)        (left vertical face of cell k)
//   Y(i,l)  point value at (x_i, y_{l-1/2})        (bottom horizontal face of cell i)
//   V(k,l)  point value at (x_{k-1/2}, y_{l-1/2})  (lower-left vertex of cell (k,l))
// Periodic directions hold n entries per point set; an outflow direction holds
// n+1.  Storage: structure of arrays, component-major, x fastest:
//   cell [8][ny][nx], xface [8][ny][nxp], yface [8][nyp][nx], vert [8][nyp][nxp].
// Conservative variables in the paper's order U = (rho, rho v1, rho v2, rho v3,
// B1, B2, B3, E).

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

// ------------------------------------------------------------ scalar type
// The plain build computes in double.  Built with -DORC_TANGENT=n the same
// code runs on forward-mode dual numbers that carry n directional
// derivatives beside each value (the tangent oracle, the reference for the
// adjoint).  Every decision -- a guard, a max or min, the sign taken by an
// absolute value, a Newton stopping test -- is taken on the value, so the
// derivatives are those of the branch the value takes.  Conventions: ties in
// max and min go to the first argument (std::max / std::min do this), |x| has
// derivative +1 at x = 0, and sqrt has derivative 0 at 0.
#ifdef ORC_TANGENT
namespace tangent {
constexpr int ND = ORC_TANGENT;
struct Dual {
  double v;
  double d[ND];
  Dual() : v(0.0) { for (int q = 0; q < ND; ++q) d[q] = 0.0; }
  Dual(double x) : v(x) { for (int q = 0; q < ND; ++q) d[q] = 0.0; }  // NOLINT: implicit on purpose
  Dual& operator+=(const Dual& o) { v += o.v; for (int q = 0; q < ND; ++q) d[q] += o.d[q]; return *this; }
  Dual& operator-=(const Dual& o) { v -= o.v; for (int q = 0; q < ND; ++q) d[q] -= o.d[q]; return *this; }
};
inline Dual operator-(const Dual& a) { Dual r; r.v = -a.v; for (int q = 0; q < ND; ++q) r.d[q] = -a.d[q]; return r; }
inline Dual operator+(const Dual& a, const Dual& b) { Dual r; r.v = a.v + b.v; for (int q = 0; q < ND; ++q) r.d[q] = a.d[q] + b.d[q]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r; r.v = a.v - b.v; for (int q = 0; q < ND; ++q) r.d[q] = a.d[q] - b.d[q]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) {
  Dual r;
  r.v = a.v * b.v;
  for (int q = 0; q < ND; ++q) r.d[q] = a.d[q] * b.v + a.v * b.d[q];
  return r;
}
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r;
  r.v = a.v / b.v;
  for (int q = 0; q < ND; ++q) r.d[q] = (a.d[q] - r.v * b.d[q]) / b.v;
  return r;
}
inline Dual operator+(const Dual& a, double b) { return a + Dual(b); }
inline Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
inline Dual operator-(const Dual& a, double b) { return a - Dual(b); }
inline Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
inline Dual operator*(const Dual& a, double b) { return a * Dual(b); }
inline Dual operator*(double a, const Dual& b) { return Dual(a) * b; }
inline Dual operator/(const Dual& a, double b) { return a / Dual(b); }
inline Dual operator/(double a, const Dual& b) { return Dual(a) / b; }
inline bool operator<(const Dual& a, const Dual& b) { return a.v < b.v; }
inline bool operator>(const Dual& a, const Dual& b) { return a.v > b.v; }
inline bool operator<=(const Dual& a, const Dual& b) { return a.v <= b.v; }
inline bool operator>=(const Dual& a, const Dual& b) { return a.v >= b.v; }
inline Dual sqrt(const Dual& a) {
  Dual r;
  r.v = std::sqrt(a.v);
  for (int q = 0; q < ND; ++q) r.d[q] = r.v > 0.0 ? a.d[q] / (2.0 * r.v) : 0.0;
  return r;
}
inline Dual exp(const Dual& a) {
  Dual r;
  r.v = std::exp(a.v);
  for (int q = 0; q < ND; ++q) r.d[q] = a.d[q] * r.v;
  return r;
}
inline Dual fabs(const Dual& a) { return a.v < 0.0 ? -a : a; }
inline double val(const Dual& a) { return a.v; }
}  // namespace tangent
typedef tangent::Dual real;
using tangent::val;
#else
typedef double real;
inline double val(double x) { return x; }
#endif

namespace {

using std::exp;
using std::fabs;
using std::sqrt;

constexpr int NV = 8;
typedef std::array<real, NV> Vec;

struct Grid {
  int nx, ny, nxp, nyp, bcx, bcy;  // bc: 0 periodic, 1 outflow
  double dx, dy, gamma, kappa;
};

// ---------------------------------------------------------------- boundary
// Periodic wrap, or (outflow) even mirror extension across the boundary:
// a cell index mirrors about the boundary face, a node index about the
// boundary node.  Valid for overshoots up to n (stencils need at most 3).
int cell_index(int i, int n, int bc) {
  if (bc == 0) { i %= n; return i < 0 ? i + n : i; }
  if (i < 0) return -1 - i;
  if (i >= n) return 2 * n - 1 - i;
  return i;
}
int node_index(int k, int n, int bc) {
  if (bc == 0) { k %= n; return k < 0 ? k + n : k; }
  if (k < 0) return -k;
  if (k > n) return 2 * n - k;
  return k;
}

struct StateView {
  const real *a, *x, *y, *v;
};

struct Access {
  const Grid& g;
  StateView s;
  Vec A(int i, int j) const {
    const int I = cell_index(i, g.nx, g.bcx), J = cell_index(j, g.ny, g.bcy);
    Vec u;
    for (int c = 0; c < NV; ++c) u[c] = s.a[((size_t)c * g.ny + J) * g.nx + I];
    return u;
  }
  Vec X(int k, int j) const {
    const int K = node_index(k, g.nx, g.bcx), J = cell_index(j, g.ny, g.bcy);
    Vec u;
    for (int c = 0; c < NV; ++c) u[c] = s.x[((size_t)c * g.ny + J) * g.nxp + K];
    return u;
  }
  Vec Y(int i, int l) const {
    const int I = cell_index(i, g.nx, g.bcx), L = node_index(l, g.ny, g.bcy);
    Vec u;
    for (int c = 0; c < NV; ++c) u[c] = s.y[((size_t)c * g.nyp + L) * g.nx + I];
    return u;
  }
  Vec V(int k, int l) const {
    const int K = node_index(k, g.nx, g.bcx), L = node_index(l, g.ny, g.bcy);
    Vec u;
    for (int c = 0; c < NV; ++c) u[c] = s.v[((size_t)c * g.nyp + L) * g.nxp + K];
    return u;
  }
};

// ----------------------------------------------------------------- physics
// Pressure from the conservative variables, Section 1 (EOS of the perfect gas)
// and the admissible set of Section 3:
//   p = (gamma-1) (E - |rho v|^2 / (2 rho) - |B|^2 / 2).
real pressure(const Vec& U, double gamma) {
  const real m2 = U[1] * U[1] + U[2] * U[2] + U[3] * U[3];
  const real b2 = U[4] * U[4] + U[5] * U[5] + U[6] * U[6];
  return (gamma - 1.0) * (U[7] - m2 / (2.0 * U[0]) - b2 / 2.0);
}

// Physical fluxes F1 (dir 0) and F2 (dir 1), Section 1.
Vec flux(const Vec& U, double gamma, int dir) {
  const real rho = U[0];
  const real v1 = U[1] / rho, v2 = U[2] / rho, v3 = U[3] / rho;
  const real B1 = U[4], B2 = U[5], B3 = U[6], E = U[7];
  const real p = pressure(U, gamma);
  const real pt = p + (B1 * B1 + B2 * B2 + B3 * B3) / 2.0;
  const real vB = v1 * B1 + v2 * B2 + v3 * B3;
  Vec F;
  if (dir == 0) {
    F[0] = rho * v1;
    F[1] = rho * v1 * v1 - B1 * B1 + pt;
    F[2] = rho * v1 * v2 - B1 * B2;
    F[3] = rho * v1 * v3 - B1 * B3;
    F[4] = 0.0;
    F[5] = v1 * B2 - B1 * v2;
    F[6] = v1 * B3 - B1 * v3;
    F[7] = (E + pt) * v1 - B1 * vB;
  } else {
    F[0] = rho * v2;
    F[1] = rho * v1 * v2 - B1 * B2;
    F[2] = rho * v2 * v2 - B2 * B2 + pt;
    F[3] = rho * v2 * v3 - B2 * B3;
    F[4] = v2 * B1 - B2 * v1;
    F[5] = 0.0;
    F[6] = v2 * B3 - B2 * v3;
    F[7] = (E + pt) * v2 - B2 * vB;
  }
  return F;
}

// Godunov-Powell source vector Psi = (0, B, v, v.B), eq. (gp_src).
Vec psi(const Vec& U) {
  const real v1 = U[1] / U[0], v2 = U[2] / U[0], v3 = U[3] / U[0];
  Vec P;
  P[0] = 0.0;
  P[1] = U[4];
  P[2] = U[5];
  P[3] = U[6];
  P[4] = v1;
  P[5] = v2;
  P[6] = v3;
  P[7] = v1 * U[4] + v2 * U[5] + v3 * U[6];
  return P;
}

// Fast magnetosonic speed c_{f,l}, eq. (cf).  A negative inner discriminant
// (round-off only) is clamped to zero.
real fast_speed(const Vec& U, double gamma, int dir) {
  const real rho = U[0];
  const real c2 = gamma * pressure(U, gamma) / rho;
  const real b2 = (U[4] * U[4] + U[5] * U[5] + U[6] * U[6]) / rho;
  const real Bl = U[4 + dir];
  const real s = c2 + b2;
  real disc = s * s - 4.0 * c2 * Bl * Bl / rho;
  if (disc < 0.0) disc = 0.0;
  return sqrt(0.5 * (s + sqrt(disc)));
}

// Spectral radius of dF_l/dU: |v_l| + c_{f,l} (Section 2.3).
real spectral_radius(const Vec& U, double gamma, int dir) {
  return fabs(U[1 + dir] / U[0]) + fast_speed(U, gamma, dir);
}

// alpha_{l,*}(U, Ut) of the Lemma (Wu's bound), Section 3.1.
real alpha_star(const Vec& U, const Vec& Ut, double gamma, int dir) {
  const real sa = sqrt(U[0]), sb = sqrt(Ut[0]);
  const real va = U[1 + dir] / U[0], vb = Ut[1 + dir] / Ut[0];
  const real t1 = std::max(fabs(va), fabs(sa * va + sb * vb) / (sa + sb));
  const real t2 = std::max(fast_speed(U, gamma, dir), fast_speed(Ut, gamma, dir));
  const real d1 = U[4] - Ut[4], d2 = U[5] - Ut[5], d3 = U[6] - Ut[6];
  const real t3 = sqrt(d1 * d1 + d2 * d2 + d3 * d3) / (sa + sb);
  return t1 + t2 + t3;
}

// LLF viscosity: the Lemma's lower bound taken with equality.
real alpha_llf(const Vec& U, const Vec& Ut, double gamma, int dir) {
  return std::max(std::max(spectral_radius(U, gamma, dir), spectral_radius(Ut, gamma, dir)),
                  std::max(alpha_star(U, Ut, gamma, dir), alpha_star(Ut, U, gamma, dir)));
}

// LLF numerical flux, eq. (2d_llf_flux):
//   F^LLF(U, Ut) = 1/2 [F(U) + F(Ut) - alpha (Ut - U)].
Vec llf_flux(const Vec& U, const Vec& Ut, double gamma, int dir) {
  const real al = alpha_llf(U, Ut, gamma, dir);
  const Vec Fa = flux(U, gamma, dir), Fb = flux(Ut, gamma, dir);
  Vec F;
  for (int c = 0; c < NV; ++c) F[c] = 0.5 * (Fa[c] + Fb[c] - al * (Ut[c] - U[c]));
  return F;
}

bool in_G(const Vec& U, double gamma) { return U[0] > 0.0 && pressure(U, gamma) > 0.0; }

// ---------------------------------------------------------- counters
struct Counters {
  int64_t n_llf_not_admissible = 0;  // first-order LLF states outside G
  int64_t n_newton = 0;              // vertex root solves (flux limiter step 2)
  int64_t newton_iters_max = 0;
  int64_t n_fallback = 0;            // round-off fallback uses
  int64_t n_not_admissible = 0;      // final DoFs outside G
  int64_t n_theta_active = 0;        // interfaces with theta < 1 (flux limiter)
  int64_t n_point_limited = 0;       // point values changed by the scaling limiter
  int64_t n_centre_limited = 0;      // centre values changed by their limiter
  int64_t n_source_limited = 0;      // cells with a source coefficient < 1
  double min_theta = 1.0;
  void merge(const Counters& o) {
    n_llf_not_admissible += o.n_llf_not_admissible;
    n_newton += o.n_newton;
    newton_iters_max = std::max(newton_iters_max, o.newton_iters_max);
    n_fallback += o.n_fallback;
    n_not_admissible += o.n_not_admissible;
    n_theta_active += o.n_theta_active;
    n_point_limited += o.n_point_limited;
    n_centre_limited += o.n_centre_limited;
    n_source_limited += o.n_source_limited;
    min_theta = std::min(min_theta, o.min_theta);
  }
};

constexpr double EPS_FLOOR = 1e-13;   // lower bounds for rho and p
constexpr double LAMBDA_REG = 1e-12;  // regulariser of the density box
constexpr double SHRINK = 1e-8;       // round-off fallback step 2^m * 1e-8

// Round-off fallback of the closing remark of Section 4.  Reading: the
// limiters aim at rho >= eps_rho, p >= eps_p; the fallback fires only when
// round-off leaves the blended state outside G itself (rho > 0, p > 0 fails),
// as happens when the variables' scales differ a lot.  It shrinks the
// coefficient by 2^m 1e-8, m = 0..9 (each trial from the original value),
// until the state is in G; theta = 0 (the safe state) otherwise.
// make(theta) builds the blended state.
template <class Make>
real shrink_until_admissible(real theta, double gamma, Make make, Counters& cnt) {
  if (in_G(make(theta), gamma) || theta <= 0.0) return theta;
  ++cnt.n_fallback;
  for (int m = 0; m < 10; ++m) {
    const real t = std::max<real>(theta - std::ldexp(SHRINK, m), 0.0);
    if (in_G(make(t), gamma)) return t;
  }
  return 0.0;
}

// ----------------------------------------------- scaling limiters (points)
// Scaling limiter for a point value, Section 3.3: blend the high-order state
// UH with the safe state UL.  Step (1) changes the density only, step (2)
// blends the whole state.  The two fractions are guarded: each applies only
// when the bound is violated, so its denominator is positive.
Vec point_scaling_limiter(const Vec& UH, const Vec& UL, double gamma, Counters& cnt) {
  const real rhoL = UL[0], pL = pressure(UL, gamma);
  const real eps_rho = std::min<real>(EPS_FLOOR, rhoL);
  const real eps_p = std::min<real>(EPS_FLOOR, pL);
  real th1 = 1.0;
  if (UH[0] < eps_rho) th1 = (rhoL - eps_rho) / (rhoL - UH[0]);
  Vec Us = UH;
  Us[0] = th1 * UH[0] + (1.0 - th1) * rhoL;
  const real ps = pressure(Us, gamma);
  real th2 = 1.0;
  if (ps < eps_p) th2 = (pL - eps_p) / (pL - ps);
  if (th1 < 1.0 || th2 < 1.0) ++cnt.n_point_limited;
  auto make = [&](real t) {
    Vec W;
    for (int c = 0; c < NV; ++c) W[c] = t * Us[c] + (1.0 - t) * UL[c];
    return W;
  };
  th2 = shrink_until_admissible(th2, gamma, make, cnt);
  return make(th2);
}

// Limiter of the centre value, Remark rmk:cell_center: the limited centre is
// of the printed form theta~ Uc + (1 - theta~) Abar, one coefficient for the
// whole state.  Reading: theta~ = theta_rho * theta_p, found like the point
// limiter's two steps -- first the whole state is blended towards the cell
// average until rho >= eps_rho, then again until p >= eps_p; eps from the
// cell average.  The round-off fallback of the closing remark of Section 4
// acts on theta_p.
Vec centre_limiter(const Vec& Uc, const Vec& A, double gamma, Counters& cnt) {
  const real rhoA = A[0], pA = pressure(A, gamma);
  const real eps_rho = std::min<real>(EPS_FLOOR, rhoA);
  const real eps_p = std::min<real>(EPS_FLOOR, pA);
  real th1 = 1.0;
  if (Uc[0] < eps_rho) th1 = (rhoA - eps_rho) / (rhoA - Uc[0]);
  Vec Ur;
  for (int c = 0; c < NV; ++c) Ur[c] = th1 * Uc[c] + (1.0 - th1) * A[c];
  const real pr = pressure(Ur, gamma);
  real th2 = 1.0;
  if (pr < eps_p) th2 = (pA - eps_p) / (pA - pr);
  if (th1 < 1.0 || th2 < 1.0) ++cnt.n_centre_limited;
  auto make = [&](real t) {
    Vec W;
    for (int c = 0; c < NV; ++c) W[c] = t * Ur[c] + (1.0 - t) * A[c];
    return W;
  };
  th2 = shrink_until_admissible(th2, gamma, make, cnt);
  return make(th2);
}

// Centre value of the bi-parabolic reconstruction (Section 2.1),
//   Uc = (36 Abar - 4 (sum of the face midpoints) - (sum of the vertices)) / 16,
// then limited towards the cell average.
Vec centre_value(const Access& acc, int i, int j, double gamma, Counters& cnt) {
  const Vec A = acc.A(i, j);
  const Vec Xl = acc.X(i, j), Xr = acc.X(i + 1, j);
  const Vec Yd = acc.Y(i, j), Yu = acc.Y(i, j + 1);
  const Vec Vdl = acc.V(i, j), Vdr = acc.V(i + 1, j), Vul = acc.V(i, j + 1), Vur = acc.V(i + 1, j + 1);
  Vec Uc;
  for (int c = 0; c < NV; ++c) {
    const real faces = (Xl[c] + Xr[c]) + (Yd[c] + Yu[c]);
    const real corners = (Vdl[c] + Vdr[c]) + (Vul[c] + Vur[c]);
    Uc[c] = (36.0 * A[c] - 4.0 * faces - corners) / 16.0;
  }
  return centre_limiter(Uc, A, gamma, cnt);
}

// ------------------------------------------- point value update (Sec. 2.3)
// Flux-vector-split derivative along one line, D+F+ + D-F-, with the
// one-sided operators of eq. (2d_fd) and F+- = 1/2 (F +- alpha U).  The
// five stencil states w[0..4] sit at offsets -h, -h/2, 0, +h/2, +h.
// alpha is the maximal spectral radius over the stencil.  Also returns the
// central derivative 1/2 (D+ B_l + D- B_l) of the normal field component.
void fvs_derivative(const Vec w[5], double gamma, int dir, double h, Vec& R, real& dB) {
  Vec F[5];
  real alpha = 0.0;
  for (int m = 0; m < 5; ++m) {
    F[m] = flux(w[m], gamma, dir);
    alpha = std::max(alpha, spectral_radius(w[m], gamma, dir));
  }
  for (int c = 0; c < NV; ++c) {
    real Fp[5], Fm[5];
    for (int m = 0; m < 5; ++m) {
      Fp[m] = 0.5 * (F[m][c] + alpha * w[m][c]);
      Fm[m] = 0.5 * (F[m][c] - alpha * w[m][c]);
    }
    const real Dp = (Fp[0] - 4.0 * Fp[1] + 3.0 * Fp[2]) / h;
    const real Dm = (-3.0 * Fm[2] + 4.0 * Fm[3] - Fm[4]) / h;
    R[c] = Dp + Dm;
  }
  const int b = 4 + dir;
  const real Bp = (w[0][b] - 4.0 * w[1][b] + 3.0 * w[2][b]) / h;
  const real Bm = (-3.0 * w[2][b] + 4.0 * w[3][b] - w[4][b]) / h;
  dB = 0.5 * (Bp + Bm);
}

// First-order LLF scheme for a point value, Section 3.3: four neighbour
// states, LLF fluxes of eq. (2d_llf_flux) divided by the mesh sizes, and the
// central divergence over 2 dx, 2 dy times Psi(U), exactly as printed (the
// face-to-vertex pairs are half a cell apart but divided by the full size).
Vec point_llf(const Vec& U, const Vec& L, const Vec& R, const Vec& D, const Vec& Up, double dt,
              const Grid& g) {
  const Vec FR = llf_flux(U, R, g.gamma, 0), FL = llf_flux(L, U, g.gamma, 0);
  const Vec FU = llf_flux(U, Up, g.gamma, 1), FD = llf_flux(D, U, g.gamma, 1);
  const real divB = (R[4] - L[4]) / (2.0 * g.dx) + (Up[5] - D[5]) / (2.0 * g.dy);
  const Vec P = psi(U);
  Vec W;
  for (int c = 0; c < NV; ++c)
    W[c] = U[c] - dt / g.dx * (FR[c] - FL[c]) - dt / g.dy * (FU[c] - FD[c]) - dt * divB * P[c];
  return W;
}

struct CentreField {
  // limited centre values for cells [-2, nx+2) x [-2, ny+2)
  int nx, ny;
  std::vector<Vec> v;
  const Vec& at(int i, int j) const { return v[(size_t)(j + 2) * (nx + 4) + (i + 2)]; }
};

// Vertex V(k,l): FVS in x and in y, Section 2.3.
Vec vertex_high(const Access& acc, int k, int l, double dt, const Grid& g, Vec& U) {
  U = acc.V(k, l);
  const Vec wx[5] = {acc.V(k - 1, l), acc.Y(k - 1, l), U, acc.Y(k, l), acc.V(k + 1, l)};
  const Vec wy[5] = {acc.V(k, l - 1), acc.X(k, l - 1), U, acc.X(k, l), acc.V(k, l + 1)};
  Vec R1, R2;
  real d1, d2;
  fvs_derivative(wx, g.gamma, 0, g.dx, R1, d1);
  fvs_derivative(wy, g.gamma, 1, g.dy, R2, d2);
  const real divB = d1 + d2;
  const Vec P = psi(U);
  Vec H;
  for (int c = 0; c < NV; ++c) H[c] = U[c] + dt * (-R1[c] - R2[c] - divB * P[c]);
  return H;
}

// Vertical face X(k,j): FVS in x, central D2 F2 in y, Section 2.3.
Vec xface_high(const Access& acc, const CentreField& C, int k, int j, double dt, const Grid& g,
               Vec& U) {
  U = acc.X(k, j);
  const Vec wx[5] = {acc.X(k - 1, j), C.at(k - 1, j), U, C.at(k, j), acc.X(k + 1, j)};
  Vec R1;
  real d1;
  fvs_derivative(wx, g.gamma, 0, g.dx, R1, d1);
  const Vec Vd = acc.V(k, j), Vu = acc.V(k, j + 1);
  const Vec Fd = flux(Vd, g.gamma, 1), Fu = flux(Vu, g.gamma, 1);
  const real d2 = (Vu[5] - Vd[5]) / g.dy;
  const real divB = d1 + d2;
  const Vec P = psi(U);
  Vec H;
  for (int c = 0; c < NV; ++c) {
    const real R2 = (Fu[c] - Fd[c]) / g.dy;
    H[c] = U[c] + dt * (-R1[c] - R2 - divB * P[c]);
  }
  return H;
}

// Horizontal face Y(i,l): central D1 F1 in x, FVS in y, Section 2.3.
Vec yface_high(const Access& acc, const CentreField& C, int i, int l, double dt, const Grid& g,
               Vec& U) {
  U = acc.Y(i, l);
  const Vec wy[5] = {acc.Y(i, l - 1), C.at(i, l - 1), U, C.at(i, l), acc.Y(i, l + 1)};
  Vec R2;
  real d2;
  fvs_derivative(wy, g.gamma, 1, g.dy, R2, d2);
  const Vec Vl = acc.V(i, l), Vr = acc.V(i + 1, l);
  const Vec Fl = flux(Vl, g.gamma, 0), Fr = flux(Vr, g.gamma, 0);
  const real d1 = (Vr[4] - Vl[4]) / g.dx;
  const real divB = d1 + d2;
  const Vec P = psi(U);
  Vec H;
  for (int c = 0; c < NV; ++c) {
    const real R1 = (Fr[c] - Fl[c]) / g.dx;
    H[c] = U[c] + dt * (-R1 - R2[c] - divB * P[c]);
  }
  return H;
}

// ----------------------------------------------- cell average (Sec. 2.2)
// Simpson flux at x-interface k of row j: [F1(V(k,j)) + 4 F1(X(k,j)) + F1(V(k,j+1))] / 6.
Vec simpson_x(const Access& acc, int k, int j, double gamma) {
  const Vec a = flux(acc.V(k, j), gamma, 0), b = flux(acc.X(k, j), gamma, 0),
            c = flux(acc.V(k, j + 1), gamma, 0);
  Vec F;
  for (int q = 0; q < NV; ++q) F[q] = (a[q] + 4.0 * b[q] + c[q]) / 6.0;
  return F;
}
// Simpson flux at y-interface l of column i: [F2(V(i,l)) + 4 F2(Y(i,l)) + F2(V(i+1,l))] / 6.
Vec simpson_y(const Access& acc, int i, int l, double gamma) {
  const Vec a = flux(acc.V(i, l), gamma, 1), b = flux(acc.Y(i, l), gamma, 1),
            c = flux(acc.V(i + 1, l), gamma, 1);
  Vec F;
  for (int q = 0; q < NV; ++q) F[q] = (a[q] + 4.0 * b[q] + c[q]) / 6.0;
  return F;
}

// Powell source of the cell average, eq. (semi_av_src): 3x3 Simpson
// (Gauss-Lobatto) quadrature of (div B) Psi on the cell's own nine points,
// with the derivatives of eq. (2d_fd) at each point.  The first index a runs
// in x (left, centre, right), the second b in y (bottom, middle, top).
Vec cell_source(const Access& acc, const CentreField& C, int i, int j, const Grid& g) {
  Vec S9[3][3];  // [a][b]
  S9[0][0] = acc.V(i, j);
  S9[1][0] = acc.Y(i, j);
  S9[2][0] = acc.V(i + 1, j);
  S9[0][1] = acc.X(i, j);
  S9[1][1] = C.at(i, j);
  S9[2][1] = acc.X(i + 1, j);
  S9[0][2] = acc.V(i, j + 1);
  S9[1][2] = acc.Y(i, j + 1);
  S9[2][2] = acc.V(i + 1, j + 1);
  const double w[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
  auto d3 = [](int at, real u0, real u1, real u2) {
    if (at == 0) return -3.0 * u0 + 4.0 * u1 - u2;  // D^-
    if (at == 1) return u2 - u0;                    // D (central)
    return u0 - 4.0 * u1 + 3.0 * u2;                // D^+
  };
  Vec S{};
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b) {
      const real dB1 = d3(a, S9[0][b][4], S9[1][b][4], S9[2][b][4]) / g.dx;
      const real dB2 = d3(b, S9[a][0][5], S9[a][1][5], S9[a][2][5]) / g.dy;
      const real divB = dB1 + dB2;
      const Vec P = psi(S9[a][b]);
      for (int q = 0; q < NV; ++q) S[q] += w[a] * w[b] * divB * P[q];
    }
  }
  return S;
}

// Shock sensor of Section 3.4 for one cell, from cell averages only:
// phi1 (Jameson on the total pressure, per direction), phi2 (modified
// Ducros), phi3 (relative discrete divergence, as printed).
struct Sensor {
  real phi1x, phi1y, phi2, phi3;
};
Sensor cell_sensor(const Access& acc, int i, int j, const Grid& g) {
  const Vec c = acc.A(i, j);
  const Vec l = acc.A(i - 1, j), r = acc.A(i + 1, j), d = acc.A(i, j - 1), u = acc.A(i, j + 1);
  auto pt = [&](const Vec& U) {
    return pressure(U, g.gamma) + (U[4] * U[4] + U[5] * U[5] + U[6] * U[6]) / 2.0;
  };
  const real ptc = pt(c), ptl = pt(l), ptr = pt(r), ptd = pt(d), ptu = pt(u);
  Sensor s;
  s.phi1x = fabs(ptr - 2.0 * ptc + ptl) / fabs(ptr + 2.0 * ptc + ptl);
  s.phi1y = fabs(ptu - 2.0 * ptc + ptd) / fabs(ptu + 2.0 * ptc + ptd);
  const real divv = (r[1] / r[0] - l[1] / l[0]) / (2.0 * g.dx) + (u[2] / u[0] - d[2] / d[0]) / (2.0 * g.dy);
  const real curlv = (r[2] / r[0] - l[2] / l[0]) / (2.0 * g.dx) - (u[1] / u[0] - d[1] / d[0]) / (2.0 * g.dy);
  s.phi2 = std::max<real>(-divv / sqrt(divv * divv + curlv * curlv + 1e-40), 0.0);
  s.phi3 = fabs(r[4] - l[4] + u[5] - d[5]) / (fabs(c[4] + c[5]) + 1e-40);
  return s;
}

real sensor_theta(const Sensor& L, const Sensor& R, bool xdir, double kappa) {
  const real p1 = xdir ? std::max(L.phi1x, R.phi1x) : std::max(L.phi1y, R.phi1y);
  const real p2 = std::max(L.phi2, R.phi2);
  const real p3 = std::max(L.phi3, R.phi3);
  return exp(-kappa * (p1 * p2 + p3));
}

// The pressure condition along the ray A1 + r D written as the cubic of
// Section 3.2: q(r) = rho(r) [E(r) - |B(r)|^2/2 - eps_p/(gamma-1)] - |m(r)|^2/2,
// which is rho(r) (p(r) - eps_p) / (gamma-1): same sign as p - eps_p while
// rho > 0, but without the pole of p at rho = 0.  Returns q and dq/dr.
void pressure_cubic(const Vec& A1, const Vec& D, real r, double gamma, real eps_p, real& q, real& dq) {
  Vec W;
  for (int c = 0; c < NV; ++c) W[c] = A1[c] + r * D[c];
  const real b2 = W[4] * W[4] + W[5] * W[5] + W[6] * W[6];
  const real m2 = W[1] * W[1] + W[2] * W[2] + W[3] * W[3];
  const real e = W[7] - b2 / 2.0 - eps_p / (gamma - 1.0);
  q = W[0] * e - m2 / 2.0;
  const real de = D[7] - (W[4] * D[4] + W[5] * D[5] + W[6] * D[6]);
  dq = D[0] * e + W[0] * de - (W[1] * D[1] + W[2] * D[2] + W[3] * D[3]);
}

// Step (2), second bullet, of Section 3.2: for an infeasible vertex of the
// density box, the r in (0,1) with p(A1 + r D) = eps_p, i.e. the largest r
// keeping the vertex feasible (the pressure is concave along the ray, so the
// root in (0,1) is unique).  Reading: Newton's method on the cubic q above,
// started at r = 1 and kept inside the bracket [lo, hi] with q(lo) >= 0 > q(hi)
// (a step leaving it is replaced by the midpoint); stop when the step is
// <= 1e-13, at most 50 steps.
real vertex_root(const Vec& A1, const Vec& D, double gamma, real eps_p, int& iters) {
  real lo = 0.0, hi = 1.0, r = 1.0;
  iters = 0;
  for (int it = 0; it < 50; ++it) {
    real q, dq;
    pressure_cubic(A1, D, r, gamma, eps_p, q, dq);
    ++iters;
    if (q >= 0.0) lo = r; else hi = r;
    real rn = r - q / dq;
    if (!(rn >= lo && rn <= hi)) rn = 0.5 * (lo + hi);
    const real step = fabs(rn - r);
    r = rn;
    if (step <= 1e-13) break;
  }
  return r;
}

// Step (2) of the parametrized flux limiter, Section 3.2: the density box
// Lambda^rho and the pressure shrink over the 15 non-trivial vertices.
// H[0..3] = H_L, H_R, H_D, H_U.  Returns Lambda[0..3].
void flux_limiter_box(const Vec& A1, const Vec H[4], double gamma, real eps_rho, real eps_p,
                      real Lambda[4], Counters& cnt, real* before_fallback = nullptr) {
  real neg = 0.0;
  for (int I = 0; I < 4; ++I)
    if (H[I][0] < 0.0) neg += H[I][0];
  real Lr[4];
  for (int I = 0; I < 4; ++I) {
    Lr[I] = 1.0;
    if (H[I][0] < 0.0) Lr[I] = std::min<real>(1.0, (A1[0] - eps_rho) / (LAMBDA_REG - neg));
  }
  real rmin[4] = {1.0, 1.0, 1.0, 1.0};
  bool any_root = false;
  for (int k = 1; k < 16; ++k) {
    Vec D{};
    for (int I = 0; I < 4; ++I)
      if (k & (1 << I))
        for (int c = 0; c < NV; ++c) D[c] += Lr[I] * H[I][c];
    Vec W;
    for (int c = 0; c < NV; ++c) W[c] = A1[c] + D[c];
    real r = 1.0;
    if (pressure(W, gamma) < eps_p) {
      int it = 0;
      r = vertex_root(A1, D, gamma, eps_p, it);
      ++cnt.n_newton;
      cnt.newton_iters_max = std::max<int64_t>(cnt.newton_iters_max, it);
      any_root = true;
    }
    for (int I = 0; I < 4; ++I)
      if (k & (1 << I)) rmin[I] = std::min(rmin[I], r);
  }
  for (int I = 0; I < 4; ++I) Lambda[I] = Lr[I] * rmin[I];
  if (before_fallback)
    for (int I = 0; I < 4; ++I) before_fallback[I] = Lambda[I];
  if (!any_root) return;  // the box corners are exactly the vertices checked above
  // Round-off fallback on the final box: all 15 corners must lie in G.
  auto box_ok = [&](const real L[4]) {
    for (int k = 1; k < 16; ++k) {
      Vec D{};
      for (int I = 0; I < 4; ++I)
        if (k & (1 << I))
          for (int c = 0; c < NV; ++c) D[c] += L[I] * H[I][c];
      Vec W;
      for (int c = 0; c < NV; ++c) W[c] = A1[c] + D[c];
      if (!in_G(W, gamma)) return false;
    }
    return true;
  };
  if (box_ok(Lambda)) return;
  ++cnt.n_fallback;
  for (int m = 0; m < 10; ++m) {
    real L[4];
    for (int I = 0; I < 4; ++I) L[I] = std::max<real>(Lambda[I] - std::ldexp(SHRINK, m), 0.0);
    if (box_ok(L)) {
      for (int I = 0; I < 4; ++I) Lambda[I] = L[I];
      return;
    }
  }
  for (int I = 0; I < 4; ++I) Lambda[I] = 0.0;
}

// Per-cell data of the cell-average update, for cells [-1, nx+1) x [-1, ny+1).
struct CellWork {
  Vec A, S_s, S_llf;
  Vec FsL, FsR, FsD, FsU;      // sensor-blended high-order fluxes at the 4 interfaces
  Vec FlL, FlR, FlD, FlU;      // LLF fluxes at the 4 interfaces
  real theta_src;
  real Lambda[4];            // L, R, D, U
};

// Steps (1) and (2) of the parametrized flux limiter, Section 3.2, for one
// cell: the first-order LLF update of eq. (2d_llf), the source coefficient
// theta_{i,j}, the state A^{Lim,1} and the box Lambda_{L,R,D,U}.  Fills
// w.theta_src and w.Lambda; returns whether the LLF update is in G.
bool cell_limiter(CellWork& w, double dt, double dx, double dy, double gamma, Counters& cnt, Vec* A1_out = nullptr) {
  const double ldx = dt / dx, ldy = dt / dy;
  Vec Allf, Asrc;
  for (int c = 0; c < NV; ++c) {
    const real G = w.A[c] - ldx * (w.FlR[c] - w.FlL[c]) - ldy * (w.FlU[c] - w.FlD[c]);
    Allf[c] = G - dt * w.S_llf[c];
    Asrc[c] = G - dt * w.S_s[c];
  }
  const bool llf_ok = in_G(Allf, gamma);
  const real rhoL = Allf[0], pL = pressure(Allf, gamma);
  const real eps_rho = std::min<real>(EPS_FLOOR, rhoL);
  const real eps_p = std::min<real>(EPS_FLOOR, pL);
  // Step (1): limit the source term.
  real th = 1.0;
  const real psrc = pressure(Asrc, gamma);
  if (psrc < eps_p) {
    th = (pL - eps_p) / (pL - psrc);
    ++cnt.n_source_limited;
  }
  auto make = [&](real t) {
    Vec W;
    for (int c = 0; c < NV; ++c) W[c] = t * Asrc[c] + (1.0 - t) * Allf[c];
    return W;
  };
  th = shrink_until_admissible(th, gamma, make, cnt);
  w.theta_src = th;
  const Vec A1 = make(th);
  if (A1_out) *A1_out = A1;
  // Step (2): anti-diffusive fluxes and the box of admissible coefficients.
  Vec H[4];
  for (int c = 0; c < NV; ++c) {
    H[0][c] = ldx * (w.FsL[c] - w.FlL[c]);
    H[1][c] = -ldx * (w.FsR[c] - w.FlR[c]);
    H[2][c] = ldy * (w.FsD[c] - w.FlD[c]);
    H[3][c] = -ldy * (w.FsU[c] - w.FlU[c]);
  }
  flux_limiter_box(A1, H, gamma, eps_rho, eps_p, w.Lambda, cnt);
  return llf_ok;
}

// -------------------------------------------------------------- FE stage
struct Stage {
  const Grid& g;
  Access acc;
  double dt;
  Counters cnt;

  // out = a * Un + b * FE(Uk), for all four DoF sets.
  void run(StateView un, real* const out[4], double a, double b, int nthreads);
};

inline size_t cidx(const Grid& g, int c, int i, int j) { return ((size_t)c * g.ny + j) * g.nx + i; }
inline size_t xidx(const Grid& g, int c, int k, int j) { return ((size_t)c * g.ny + j) * g.nxp + k; }
inline size_t yidx(const Grid& g, int c, int i, int l) { return ((size_t)c * g.nyp + l) * g.nx + i; }
inline size_t vidx(const Grid& g, int c, int k, int l) { return ((size_t)c * g.nyp + l) * g.nxp + k; }

void Stage::run(StateView un, real* const out[4], double a, double b, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  const int nx = g.nx, ny = g.ny, nxp = g.nxp, nyp = g.nyp;
  const bool first = (a == 0.0 && b == 1.0);
  auto combine = [&](real un_v, real fe) { return first ? fe : a * un_v + b * fe; };

  // Centre values (limited) on cells [-2, nx+2) x [-2, ny+2).
  CentreField C;
  C.nx = nx;
  C.ny = ny;
  C.v.resize((size_t)(nx + 4) * (ny + 4));
  std::vector<Counters> tc(256);
#pragma omp parallel for schedule(static)
  for (int j = -2; j < ny + 2; ++j) {
    Counters cc, ghost;
    for (int i = -2; i < nx + 2; ++i) {
      const bool interior = (i >= 0 && i < nx && j >= 0 && j < ny);
      C.v[(size_t)(j + 2) * (nx + 4) + (i + 2)] = centre_value(acc, i, j, g.gamma, interior ? cc : ghost);
    }
#ifdef _OPENMP
    tc[omp_get_thread_num()].merge(cc);
#else
    tc[0].merge(cc);
#endif
  }

  // ---- point values
#pragma omp parallel for schedule(static)
  for (int l = 0; l < nyp; ++l) {
    Counters cc;
    for (int k = 0; k < nxp; ++k) {
      Vec U;
      const Vec H = vertex_high(acc, k, l, dt, g, U);
      const Vec L = point_llf(U, acc.V(k - 1, l), acc.V(k + 1, l), acc.V(k, l - 1), acc.V(k, l + 1), dt, g);
      if (!in_G(L, g.gamma)) ++cc.n_llf_not_admissible;
      const Vec W = point_scaling_limiter(H, L, g.gamma, cc);
      if (!in_G(W, g.gamma)) ++cc.n_not_admissible;
      for (int c = 0; c < NV; ++c) {
        const size_t id = vidx(g, c, k, l);
        out[3][id] = combine(un.v[id], W[c]);
      }
    }
#ifdef _OPENMP
    tc[omp_get_thread_num()].merge(cc);
#else
    tc[0].merge(cc);
#endif
  }
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j) {
    Counters cc;
    for (int k = 0; k < nxp; ++k) {
      Vec U;
      const Vec H = xface_high(acc, C, k, j, dt, g, U);
      const Vec L = point_llf(U, acc.X(k - 1, j), acc.X(k + 1, j), acc.V(k, j), acc.V(k, j + 1), dt, g);
      if (!in_G(L, g.gamma)) ++cc.n_llf_not_admissible;
      const Vec W = point_scaling_limiter(H, L, g.gamma, cc);
      if (!in_G(W, g.gamma)) ++cc.n_not_admissible;
      for (int c = 0; c < NV; ++c) {
        const size_t id = xidx(g, c, k, j);
        out[1][id] = combine(un.x[id], W[c]);
      }
    }
#ifdef _OPENMP
    tc[omp_get_thread_num()].merge(cc);
#else
    tc[0].merge(cc);
#endif
  }
#pragma omp parallel for schedule(static)
  for (int l = 0; l < nyp; ++l) {
    Counters cc;
    for (int i = 0; i < nx; ++i) {
      Vec U;
      const Vec H = yface_high(acc, C, i, l, dt, g, U);
      const Vec L = point_llf(U, acc.V(i, l), acc.V(i + 1, l), acc.Y(i, l - 1), acc.Y(i, l + 1), dt, g);
      if (!in_G(L, g.gamma)) ++cc.n_llf_not_admissible;
      const Vec W = point_scaling_limiter(H, L, g.gamma, cc);
      if (!in_G(W, g.gamma)) ++cc.n_not_admissible;
      for (int c = 0; c < NV; ++c) {
        const size_t id = yidx(g, c, i, l);
        out[2][id] = combine(un.y[id], W[c]);
      }
    }
#ifdef _OPENMP
    tc[omp_get_thread_num()].merge(cc);
#else
    tc[0].merge(cc);
#endif
  }

  // ---- cell averages
  // Sensor on cells [-2, nx+2) x [-2, ny+2).
  const int sw = nx + 4;
  std::vector<Sensor> sen((size_t)(nx + 4) * (ny + 4));
#pragma omp parallel for schedule(static)
  for (int j = -2; j < ny + 2; ++j)
    for (int i = -2; i < nx + 2; ++i) sen[(size_t)(j + 2) * sw + (i + 2)] = cell_sensor(acc, i, j, g);
  auto S_at = [&](int i, int j) -> const Sensor& { return sen[(size_t)(j + 2) * sw + (i + 2)]; };

  // Interface quantities for x-interfaces k in [-1, nx+2), rows j in [-1, ny+1),
  // and y-interfaces l in [-1, ny+2), columns i in [-1, nx+1).
  const int xw = nx + 3, yw = nx + 2;
  std::vector<Vec> FsX((size_t)xw * (ny + 2)), FlX((size_t)xw * (ny + 2));
  std::vector<real> tsX((size_t)xw * (ny + 2));
  std::vector<Vec> FsY((size_t)yw * (ny + 3)), FlY((size_t)yw * (ny + 3));
  std::vector<real> tsY((size_t)yw * (ny + 3));
#pragma omp parallel for schedule(static)
  for (int j = -1; j < ny + 1; ++j)
    for (int k = -1; k < nx + 2; ++k) {
      const size_t id = (size_t)(j + 1) * xw + (k + 1);
      const Vec Fh = simpson_x(acc, k, j, g.gamma);
      const Vec Fl = llf_flux(acc.A(k - 1, j), acc.A(k, j), g.gamma, 0);
      const real ts = sensor_theta(S_at(k - 1, j), S_at(k, j), true, g.kappa);
      Vec Fs;
      for (int c = 0; c < NV; ++c) Fs[c] = ts * Fh[c] + (1.0 - ts) * Fl[c];
      FsX[id] = Fs;
      FlX[id] = Fl;
      tsX[id] = ts;
    }
#pragma omp parallel for schedule(static)
  for (int l = -1; l < ny + 2; ++l)
    for (int i = -1; i < nx + 1; ++i) {
      const size_t id = (size_t)(l + 1) * yw + (i + 1);
      const Vec Fh = simpson_y(acc, i, l, g.gamma);
      const Vec Fl = llf_flux(acc.A(i, l - 1), acc.A(i, l), g.gamma, 1);
      const real ts = sensor_theta(S_at(i, l - 1), S_at(i, l), false, g.kappa);
      Vec Fs;
      for (int c = 0; c < NV; ++c) Fs[c] = ts * Fh[c] + (1.0 - ts) * Fl[c];
      FsY[id] = Fs;
      FlY[id] = Fl;
      tsY[id] = ts;
    }
  auto xid = [&](int k, int j) { return (size_t)(j + 1) * xw + (k + 1); };
  auto yid = [&](int i, int l) { return (size_t)(l + 1) * yw + (i + 1); };

  // Per-cell limiter on cells [-1, nx+1) x [-1, ny+1).
  const int cw = nx + 2;
  std::vector<CellWork> cwk((size_t)(nx + 2) * (ny + 2));
#pragma omp parallel for schedule(static)
  for (int j = -1; j < ny + 1; ++j) {
    Counters cc;
    for (int i = -1; i < nx + 1; ++i) {
      const bool interior = (i >= 0 && i < nx && j >= 0 && j < ny);
      CellWork& w = cwk[(size_t)(j + 1) * cw + (i + 1)];
      w.A = acc.A(i, j);
      w.FsL = FsX[xid(i, j)];
      w.FsR = FsX[xid(i + 1, j)];
      w.FlL = FlX[xid(i, j)];
      w.FlR = FlX[xid(i + 1, j)];
      w.FsD = FsY[yid(i, j)];
      w.FsU = FsY[yid(i, j + 1)];
      w.FlD = FlY[yid(i, j)];
      w.FlU = FlY[yid(i, j + 1)];
      // Sources: high order (eq. semi_av_src), LLF (central divergence of the
      // cell averages), and the sensor blend with the smallest interface theta.
      const Vec S = cell_source(acc, C, i, j, g);
      const Vec Al = acc.A(i - 1, j), Ar = acc.A(i + 1, j), Ad = acc.A(i, j - 1), Au = acc.A(i, j + 1);
      const real divBbar = (Ar[4] - Al[4]) / (2.0 * g.dx) + (Au[5] - Ad[5]) / (2.0 * g.dy);
      const Vec P = psi(w.A);
      const real ts_ij = std::min(std::min(tsX[xid(i, j)], tsX[xid(i + 1, j)]),
                                    std::min(tsY[yid(i, j)], tsY[yid(i, j + 1)]));
      for (int c = 0; c < NV; ++c) {
        w.S_llf[c] = divBbar * P[c];
        w.S_s[c] = ts_ij * S[c] + (1.0 - ts_ij) * w.S_llf[c];
      }
      Counters dummy;
      if (interior && !cell_limiter(w, dt, g.dx, g.dy, g.gamma, cc)) ++cc.n_llf_not_admissible;
      if (!interior) cell_limiter(w, dt, g.dx, g.dy, g.gamma, dummy);
    }
#ifdef _OPENMP
    tc[omp_get_thread_num()].merge(cc);
#else
    tc[0].merge(cc);
#endif
  }
  auto cwat = [&](int i, int j) -> const CellWork& { return cwk[(size_t)(j + 1) * cw + (i + 1)]; };

  // Step (3) and the limited update, eq. (2d_av_limited), in flux form.
  const double ldx = dt / g.dx, ldy = dt / g.dy;
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j) {
    Counters cc;
    for (int i = 0; i < nx; ++i) {
      const CellWork& w = cwat(i, j);
      const real thL = std::min(cwat(i - 1, j).Lambda[1], w.Lambda[0]);
      const real thR = std::min(w.Lambda[1], cwat(i + 1, j).Lambda[0]);
      const real thD = std::min(cwat(i, j - 1).Lambda[3], w.Lambda[2]);
      const real thU = std::min(w.Lambda[3], cwat(i, j + 1).Lambda[2]);
      // count each interface once: the left and bottom ones of the cell
      if (thL < 1.0) ++cc.n_theta_active;
      if (thD < 1.0) ++cc.n_theta_active;
      if ((g.bcx == 1 && i == nx - 1) && thR < 1.0) ++cc.n_theta_active;
      if ((g.bcy == 1 && j == ny - 1) && thU < 1.0) ++cc.n_theta_active;
      cc.min_theta = std::min(cc.min_theta, val(std::min(std::min(thL, thR), std::min(thD, thU))));
      Vec Anew;
      for (int c = 0; c < NV; ++c) {
        const real FL = thL * w.FsL[c] + (1.0 - thL) * w.FlL[c];
        const real FR = thR * w.FsR[c] + (1.0 - thR) * w.FlR[c];
        const real FD = thD * w.FsD[c] + (1.0 - thD) * w.FlD[c];
        const real FU = thU * w.FsU[c] + (1.0 - thU) * w.FlU[c];
        const real S = w.theta_src * w.S_s[c] + (1.0 - w.theta_src) * w.S_llf[c];
        Anew[c] = w.A[c] - ldx * (FR - FL) - ldy * (FU - FD) - dt * S;
      }
      if (!in_G(Anew, g.gamma)) ++cc.n_not_admissible;
      for (int c = 0; c < NV; ++c) {
        const size_t id = cidx(g, c, i, j);
        out[0][id] = combine(un.a[id], Anew[c]);
      }
    }
#ifdef _OPENMP
    tc[omp_get_thread_num()].merge(cc);
#else
    tc[0].merge(cc);
#endif
  }
  for (auto& t : tc) cnt.merge(t);
}

// Time step: dt = min(CFL / max over all DoFs of (rho_1/dx + rho_2/dy), t_remaining).
real compute_dt(const Grid& g, StateView s, double cfl, double t_remaining) {
  double mx = 0.0;
  auto visit = [&](const real* base, int w, int h) {
    double m = 0.0;
#pragma omp parallel for reduction(max : m) schedule(static)
    for (int j = 0; j < h; ++j)
      for (int i = 0; i < w; ++i) {
        Vec U;
        for (int c = 0; c < NV; ++c) U[c] = base[((size_t)c * h + j) * w + i];
        const double q = val(spectral_radius(U, g.gamma, 0)) / g.dx + val(spectral_radius(U, g.gamma, 1)) / g.dy;
        m = std::max(m, q);
      }
    mx = std::max(mx, m);
  };
  visit(s.a, g.nx, g.ny);
  visit(s.x, g.nxp, g.ny);
  visit(s.y, g.nx, g.nyp);
  visit(s.v, g.nxp, g.nyp);
  double dt = cfl / mx;
  if (dt > t_remaining) dt = t_remaining;
  return dt;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

typedef struct {
  int32_t nx, ny;
  double x0, x1, y0, y1;
  double gamma, cfl, kappa;
  int32_t bc_x, bc_y;
  int32_t nthreads;  // 0: OpenMP default
} orc_params;

typedef struct {
  int64_t n_llf_not_admissible, n_newton, newton_iters_max, n_fallback, n_not_admissible, n_theta_active;
  int64_t n_point_limited, n_centre_limited, n_source_limited;
  double min_theta;
} orc_counters;

static Grid make_grid(const orc_params* p) {
  Grid g;
  g.nx = p->nx;
  g.ny = p->ny;
  g.bcx = p->bc_x;
  g.bcy = p->bc_y;
  g.nxp = p->nx + (p->bc_x == 1 ? 1 : 0);
  g.nyp = p->ny + (p->bc_y == 1 ? 1 : 0);
  g.dx = (p->x1 - p->x0) / p->nx;
  g.dy = (p->y1 - p->y0) / p->ny;
  g.gamma = p->gamma;
  g.kappa = p->kappa;
  return g;
}

static void export_counters(const Counters& c, orc_counters* o) {
  if (!o) return;
  o->n_llf_not_admissible += c.n_llf_not_admissible;
  o->n_newton += c.n_newton;
  o->newton_iters_max = std::max(o->newton_iters_max, c.newton_iters_max);
  o->n_fallback += c.n_fallback;
  o->n_not_admissible += c.n_not_admissible;
  o->n_theta_active += c.n_theta_active;
  o->n_point_limited += c.n_point_limited;
  o->n_centre_limited += c.n_centre_limited;
  o->n_source_limited += c.n_source_limited;
  o->min_theta = std::min(o->min_theta, c.min_theta);
}

#ifdef ORC_TANGENT
// ---- tangent build: values with ORC_TANGENT directional derivatives.
// A state with derivatives is 4 value arrays (cell, xface, yface, vert) and
// 4 derivative arrays laid out [ORC_TANGENT][size of the set].
static const double RK_A[3] = {0.0, 0.75, 1.0 / 3.0};
static const double RK_B[3] = {1.0, 0.25, 2.0 / 3.0};

static void set_sizes(const Grid& g, size_t n[4]) {
  n[0] = (size_t)NV * g.nx * g.ny;
  n[1] = (size_t)NV * g.nxp * g.ny;
  n[2] = (size_t)NV * g.nx * g.nyp;
  n[3] = (size_t)NV * g.nxp * g.nyp;
}
static void pack(const double* v, const double* d, size_t n, std::vector<real>& out) {
  out.resize(n);
  for (size_t i = 0; i < n; ++i) {
    out[i] = real(v[i]);
    for (int q = 0; q < tangent::ND; ++q) out[i].d[q] = d[(size_t)q * n + i];
  }
}
static void unpack(const std::vector<real>& in, double* v, double* d) {
  const size_t n = in.size();
  for (size_t i = 0; i < n; ++i) {
    v[i] = in[i].v;
    for (int q = 0; q < tangent::ND; ++q) d[(size_t)q * n + i] = in[i].d[q];
  }
}

int orc_t_nd(void) { return tangent::ND; }

// out = a_k Un + b_k FE(Uk) and its directional derivatives; dt is fixed.
int orc_t_stage(const orc_params* p, int k, const double* const* un, const double* const* dun,
                const double* const* uk, const double* const* duk, double* const* out, double* const* dout,
                double dt) {
  if (!p || k < 0 || k > 2 || p->nx < 4 || p->ny < 4) return -1;
  const Grid g = make_grid(p);
  size_t n[4];
  set_sizes(g, n);
  std::vector<real> vn[4], vk[4], vo[4];
  real* po[4];
  for (int q = 0; q < 4; ++q) {
    pack(un[q], dun[q], n[q], vn[q]);
    pack(uk[q], duk[q], n[q], vk[q]);
    vo[q].resize(n[q]);
    po[q] = vo[q].data();
  }
  Stage st{g, Access{g, StateView{vk[0].data(), vk[1].data(), vk[2].data(), vk[3].data()}}, dt, Counters()};
  st.run(StateView{vn[0].data(), vn[1].data(), vn[2].data(), vn[3].data()}, po, RK_A[k], RK_B[k], p->nthreads);
  for (int q = 0; q < 4; ++q) unpack(vo[q], out[q], dout[q]);
  return 0;
}

// nsteps SSP-RK3 steps in place with the given time steps dts[nsteps] (the
// step sizes are data, not differentiated).
int orc_t_run(const orc_params* p, int nsteps, const double* dts, double* const* u, double* const* du) {
  if (!p || nsteps < 0 || p->nx < 4 || p->ny < 4) return -1;
  const Grid g = make_grid(p);
  size_t n[4];
  set_sizes(g, n);
  std::vector<real> s0[4], s1[4], s2[4];
  real *p0[4], *p1[4], *p2[4];
  for (int q = 0; q < 4; ++q) {
    pack(u[q], du[q], n[q], s0[q]);
    s1[q].resize(n[q]);
    s2[q].resize(n[q]);
    p0[q] = s0[q].data();
    p1[q] = s1[q].data();
    p2[q] = s2[q].data();
  }
  const StateView v0{p0[0], p0[1], p0[2], p0[3]}, v1{p1[0], p1[1], p1[2], p1[3]}, v2{p2[0], p2[1], p2[2], p2[3]};
  for (int s = 0; s < nsteps; ++s) {
    Stage a{g, Access{g, v0}, dts[s], Counters()};
    a.run(v0, p1, RK_A[0], RK_B[0], p->nthreads);
    Stage b{g, Access{g, v1}, dts[s], Counters()};
    b.run(v0, p2, RK_A[1], RK_B[1], p->nthreads);
    Stage c{g, Access{g, v2}, dts[s], Counters()};
    c.run(v0, p1, RK_A[2], RK_B[2], p->nthreads);
    for (int q = 0; q < 4; ++q) std::copy(s1[q].begin(), s1[q].end(), s0[q].begin());
  }
  for (int q = 0; q < 4; ++q) unpack(s0[q], u[q], du[q]);
  return 0;
}
// Limiter building blocks with derivatives (for function-level checks of
// the adjoint).  Derivative arrays are [ORC_TANGENT][n] for n inputs.
static Vec tvec(const double* v, const double* d, int n, int off) {
  Vec u;
  for (int c = 0; c < NV; ++c) {
    u[c] = real(v[off + c]);
    for (int q = 0; q < tangent::ND; ++q) u[c].d[q] = d[(size_t)q * n + off + c];
  }
  return u;
}

// Point scaling limiter: UH, UL (8 each) -> out (8).
void orc_t_point_limiter(const double* UH, const double* dUH, const double* UL, const double* dUL, double gamma,
                         double* out, double* dout, int64_t* n_fallback) {
  Counters c;
  const Vec w = point_scaling_limiter(tvec(UH, dUH, NV, 0), tvec(UL, dUL, NV, 0), gamma, c);
  for (int k = 0; k < NV; ++k) {
    out[k] = w[k].v;
    for (int q = 0; q < tangent::ND; ++q) dout[(size_t)q * NV + k] = w[k].d[q];
  }
  if (n_fallback) *n_fallback = c.n_fallback;
}

// Flux limiter steps (1)-(2) for one cell: inputs A (8), F (8 x 8: FsL, FsR,
// FsD, FsU, FlL, FlR, FlD, FlU), S (2 x 8: S_s, S_llf), packed as one
// vector x[88] with derivatives dx[ND][88] -> theta_src, Lambda[4].
void orc_t_cell_limiter(const double* x, const double* dx_, double dt, double dx, double dy, double gamma,
                        double* th, double* dth, double* Lam, double* dLam, int64_t* n_fallback) {
  const int n = 88;
  CellWork w;
  w.A = tvec(x, dx_, n, 0);
  Vec* fs[8] = {&w.FsL, &w.FsR, &w.FsD, &w.FsU, &w.FlL, &w.FlR, &w.FlD, &w.FlU};
  for (int k = 0; k < 8; ++k) *fs[k] = tvec(x, dx_, n, 8 + 8 * k);
  w.S_s = tvec(x, dx_, n, 72);
  w.S_llf = tvec(x, dx_, n, 80);
  Counters c;
  cell_limiter(w, dt, dx, dy, gamma, c);
  *th = w.theta_src.v;
  for (int q = 0; q < tangent::ND; ++q) dth[q] = w.theta_src.d[q];
  for (int I = 0; I < 4; ++I) {
    Lam[I] = w.Lambda[I].v;
    for (int q = 0; q < tangent::ND; ++q) dLam[(size_t)q * 4 + I] = w.Lambda[I].d[q];
  }
  if (n_fallback) *n_fallback = c.n_fallback;
}
#else
// out = a_k Un + b_k FE(Uk) with (a,b) = (0,1), (3/4,1/4), (1/3,2/3).
// Each state is given as 4 pointers: cell, xface, yface, vert.
int orc_stage(const orc_params* p, int k, const double* const* un, const double* const* uk,
              double* const* out, double dt, orc_counters* cnt) {
  if (!p || k < 0 || k > 2 || p->nx < 4 || p->ny < 4) return -1;
  const Grid g = make_grid(p);
  static const double A[3] = {0.0, 0.75, 1.0 / 3.0};
  static const double B[3] = {1.0, 0.25, 2.0 / 3.0};
  Stage st{g, Access{g, StateView{uk[0], uk[1], uk[2], uk[3]}}, dt, Counters()};
  st.run(StateView{un[0], un[1], un[2], un[3]}, out, A[k], B[k], p->nthreads);
  export_counters(st.cnt, cnt);
  return 0;
}

double orc_dt(const orc_params* p, const double* const* u, double t_remaining) {
  const Grid g = make_grid(p);
#ifdef _OPENMP
  if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
#endif
  return compute_dt(g, StateView{u[0], u[1], u[2], u[3]}, p->cfl, t_remaining);
}

// One SSP-RK3 step in place.  dt is computed from U^n (or taken from
// *dt_inout when fixed_dt != 0) and returned in *dt_inout.
int orc_step(const orc_params* p, double* const* u, double t_remaining, int fixed_dt, double* dt_inout,
             orc_counters* cnt) {
  const Grid g = make_grid(p);
  const size_t n[4] = {(size_t)NV * g.nx * g.ny, (size_t)NV * g.nxp * g.ny, (size_t)NV * g.nx * g.nyp,
                       (size_t)NV * g.nxp * g.nyp};
  double dt = fixed_dt ? *dt_inout : orc_dt(p, u, t_remaining);
  std::vector<double> s1[4], s2[4];
  double *p1[4], *p2[4];
  for (int q = 0; q < 4; ++q) {
    s1[q].resize(n[q]);
    s2[q].resize(n[q]);
    p1[q] = s1[q].data();
    p2[q] = s2[q].data();
  }
  const double* cu[4] = {u[0], u[1], u[2], u[3]};
  const double* c1[4] = {p1[0], p1[1], p1[2], p1[3]};
  const double* c2[4] = {p2[0], p2[1], p2[2], p2[3]};
  int rc = orc_stage(p, 0, cu, cu, p1, dt, cnt);
  if (rc) return rc;
  rc = orc_stage(p, 1, cu, c1, p2, dt, cnt);
  if (rc) return rc;
  rc = orc_stage(p, 2, cu, c2, p1, dt, cnt);
  if (rc) return rc;
  for (int q = 0; q < 4; ++q) std::memcpy(u[q], p1[q], n[q] * sizeof(double));
  *dt_inout = dt;
  return 0;
}

// ---- building blocks, exposed for the pins
double orc_pressure(const double* U, double gamma) {
  Vec u;
  std::memcpy(u.data(), U, sizeof(Vec));
  return pressure(u, gamma);
}
void orc_flux(const double* U, double gamma, int dir, double* F) {
  Vec u;
  std::memcpy(u.data(), U, sizeof(Vec));
  const Vec f = flux(u, gamma, dir);
  std::memcpy(F, f.data(), sizeof(Vec));
}
double orc_fast_speed(const double* U, double gamma, int dir) {
  Vec u;
  std::memcpy(u.data(), U, sizeof(Vec));
  return fast_speed(u, gamma, dir);
}
double orc_spectral_radius(const double* U, double gamma, int dir) {
  Vec u;
  std::memcpy(u.data(), U, sizeof(Vec));
  return spectral_radius(u, gamma, dir);
}
double orc_alpha_llf(const double* U, const double* Ut, double gamma, int dir) {
  Vec a, b;
  std::memcpy(a.data(), U, sizeof(Vec));
  std::memcpy(b.data(), Ut, sizeof(Vec));
  return alpha_llf(a, b, gamma, dir);
}
void orc_llf_flux(const double* U, const double* Ut, double gamma, int dir, double* F) {
  Vec a, b;
  std::memcpy(a.data(), U, sizeof(Vec));
  std::memcpy(b.data(), Ut, sizeof(Vec));
  const Vec f = llf_flux(a, b, gamma, dir);
  std::memcpy(F, f.data(), sizeof(Vec));
}
// FVS derivative along a 5-point line: w is [5][8] row-major.
void orc_fvs_derivative(const double* w, double gamma, int dir, double h, double* R, double* dB) {
  Vec ws[5];
  for (int m = 0; m < 5; ++m) std::memcpy(ws[m].data(), w + 8 * m, sizeof(Vec));
  Vec r;
  fvs_derivative(ws, gamma, dir, h, r, *dB);
  std::memcpy(R, r.data(), sizeof(Vec));
}
void orc_point_limiter(const double* UH, const double* UL, double gamma, double* out, int64_t* n_fallback) {
  Vec h, l;
  std::memcpy(h.data(), UH, sizeof(Vec));
  std::memcpy(l.data(), UL, sizeof(Vec));
  Counters c;
  const Vec w = point_scaling_limiter(h, l, gamma, c);
  std::memcpy(out, w.data(), sizeof(Vec));
  if (n_fallback) *n_fallback = c.n_fallback;
}
// Flux limiter step (2): A1[8], H[4][8] -> Lambda[4].
// Lambda_pre[4] (may be null): the box before the round-off fallback.
void orc_flux_limiter_box(const double* A1, const double* H, double gamma, double eps_rho, double eps_p,
                          double* Lambda, int64_t* n_newton, int64_t* iters_max, int64_t* n_fallback,
                          double* Lambda_pre) {
  Vec a;
  std::memcpy(a.data(), A1, sizeof(Vec));
  Vec h[4];
  for (int I = 0; I < 4; ++I) std::memcpy(h[I].data(), H + 8 * I, sizeof(Vec));
  Counters c;
  flux_limiter_box(a, h, gamma, eps_rho, eps_p, Lambda, c, Lambda_pre);
  if (n_newton) *n_newton = c.n_newton;
  if (iters_max) *iters_max = c.newton_iters_max;
  if (n_fallback) *n_fallback = c.n_fallback;
}
// Limiter of a centre value Uc towards the cell average A.
void orc_centre_limiter(const double* Uc, const double* A, double gamma, double* out, int64_t* n_fallback) {
  Vec u, a;
  std::memcpy(u.data(), Uc, sizeof(Vec));
  std::memcpy(a.data(), A, sizeof(Vec));
  Counters c;
  const Vec w = centre_limiter(u, a, gamma, c);
  std::memcpy(out, w.data(), sizeof(Vec));
  if (n_fallback) *n_fallback = c.n_fallback;
}
double orc_vertex_root(const double* A1, const double* D, double gamma, double eps_p, int* iters) {
  Vec a, d;
  std::memcpy(a.data(), A1, sizeof(Vec));
  std::memcpy(d.data(), D, sizeof(Vec));
  return vertex_root(a, d, gamma, eps_p, *iters);
}

// First-order point LLF update from four neighbour states.
void orc_point_llf(const double* U, const double* L, const double* R, const double* D, const double* Up, double dt,
                   double dx, double dy, double gamma, double* out) {
  Vec u, l, r, d, up;
  std::memcpy(u.data(), U, sizeof(Vec));
  std::memcpy(l.data(), L, sizeof(Vec));
  std::memcpy(r.data(), R, sizeof(Vec));
  std::memcpy(d.data(), D, sizeof(Vec));
  std::memcpy(up.data(), Up, sizeof(Vec));
  Grid g{};
  g.dx = dx;
  g.dy = dy;
  g.gamma = gamma;
  const Vec w = point_llf(u, l, r, d, up, dt, g);
  std::memcpy(out, w.data(), sizeof(Vec));
}

// Simpson interface flux of a state: dir 0 -> x-interface k of row j,
// dir 1 -> y-interface l = j of column i = k.
void orc_simpson(const orc_params* p, const double* const* u, int dir, int k, int j, double* out) {
  const Grid g = make_grid(p);
  Access acc{g, StateView{u[0], u[1], u[2], u[3]}};
  const Vec f = dir == 0 ? simpson_x(acc, k, j, g.gamma) : simpson_y(acc, k, j, g.gamma);
  std::memcpy(out, f.data(), sizeof(Vec));
}

// Steps (1)-(2) of the flux limiter for one cell.  F: [8] fluxes in the order
// FsL, FsR, FsD, FsU, FlL, FlR, FlD, FlU (each 8 values); S: S_s then S_llf.
// Outputs theta_src, Lambda[4] and A^{Lim,1}[8].
void orc_cell_limiter(const double* A, const double* F, const double* S, double dt, double dx, double dy,
                      double gamma, double* theta_src, double* Lambda, double* A1, int64_t* n_fallback) {
  CellWork w;
  std::memcpy(w.A.data(), A, sizeof(Vec));
  Vec* fs[8] = {&w.FsL, &w.FsR, &w.FsD, &w.FsU, &w.FlL, &w.FlR, &w.FlD, &w.FlU};
  for (int q = 0; q < 8; ++q) std::memcpy(fs[q]->data(), F + 8 * q, sizeof(Vec));
  std::memcpy(w.S_s.data(), S, sizeof(Vec));
  std::memcpy(w.S_llf.data(), S + 8, sizeof(Vec));
  Counters c;
  Vec a1;
  cell_limiter(w, dt, dx, dy, gamma, c, &a1);
  *theta_src = w.theta_src;
  for (int I = 0; I < 4; ++I) Lambda[I] = w.Lambda[I];
  std::memcpy(A1, a1.data(), sizeof(Vec));
  if (n_fallback) *n_fallback = c.n_fallback;
}

// Per-cell quantities of one state, for the pins: limited centre values
// [8][ny][nx], the 9-point source S [8][ny][nx], sensor (phi1x, phi1y, phi2,
// phi3) [4][ny][nx].
void orc_cell_diagnostics(const orc_params* p, const double* const* u, double* centre, double* source,
                          double* sensor) {
  const Grid g = make_grid(p);
  Access acc{g, StateView{u[0], u[1], u[2], u[3]}};
  CentreField C;
  C.nx = g.nx;
  C.ny = g.ny;
  C.v.resize((size_t)(g.nx + 4) * (g.ny + 4));
  Counters cc;
  for (int j = -2; j < g.ny + 2; ++j)
    for (int i = -2; i < g.nx + 2; ++i) C.v[(size_t)(j + 2) * (g.nx + 4) + (i + 2)] = centre_value(acc, i, j, g.gamma, cc);
  for (int j = 0; j < g.ny; ++j)
    for (int i = 0; i < g.nx; ++i) {
      const Vec& c = C.at(i, j);
      const Vec S = cell_source(acc, C, i, j, g);
      const Sensor s = cell_sensor(acc, i, j, g);
      for (int q = 0; q < NV; ++q) {
        if (centre) centre[cidx(g, q, i, j)] = c[q];
        if (source) source[cidx(g, q, i, j)] = S[q];
      }
      if (sensor) {
        const size_t plane = (size_t)g.nx * g.ny, id = (size_t)j * g.nx + i;
        sensor[id] = s.phi1x;
        sensor[plane + id] = s.phi1y;
        sensor[2 * plane + id] = s.phi2;
        sensor[3 * plane + id] = s.phi3;
      }
    }
}

// The two discrete divergences recorded for the Orszag-Tang example
// (Section 4): div1 sums |div B| at the nine points of every cell, with the
// same derivatives and weights as the source of eq. (semi_av_src) (limited
// centre values), times dx dy; div2 sums, per cell, one sixth of the
// absolute Simpson edge integral of B . n (the Gauss-Green form), times
// dx dy, as printed.
void orc_divb(const orc_params* p, const double* const* u, double* out2) {
  const Grid g = make_grid(p);
  Access acc{g, StateView{u[0], u[1], u[2], u[3]}};
  CentreField C;
  C.nx = g.nx;
  C.ny = g.ny;
  C.v.resize((size_t)(g.nx + 4) * (g.ny + 4));
  Counters cc;
  for (int j = -2; j < g.ny + 2; ++j)
    for (int i = -2; i < g.nx + 2; ++i) C.v[(size_t)(j + 2) * (g.nx + 4) + (i + 2)] = centre_value(acc, i, j, g.gamma, cc);
  const double w[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
  auto d3 = [](int at, double u0, double u1, double u2) {
    if (at == 0) return -3.0 * u0 + 4.0 * u1 - u2;
    if (at == 1) return u2 - u0;
    return u0 - 4.0 * u1 + 3.0 * u2;
  };
  double div1 = 0.0, div2 = 0.0;
  for (int j = 0; j < g.ny; ++j)
    for (int i = 0; i < g.nx; ++i) {
      Vec S9[3][3];  // [a][b]: a along x, b along y
      S9[0][0] = acc.V(i, j);
      S9[1][0] = acc.Y(i, j);
      S9[2][0] = acc.V(i + 1, j);
      S9[0][1] = acc.X(i, j);
      S9[1][1] = C.at(i, j);
      S9[2][1] = acc.X(i + 1, j);
      S9[0][2] = acc.V(i, j + 1);
      S9[1][2] = acc.Y(i, j + 1);
      S9[2][2] = acc.V(i + 1, j + 1);
      double cell1 = 0.0;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          const double dB1 = d3(a, S9[0][b][4], S9[1][b][4], S9[2][b][4]) / g.dx;
          const double dB2 = d3(b, S9[a][0][5], S9[a][1][5], S9[a][2][5]) / g.dy;
          cell1 += std::fabs(dB1 + dB2) * w[a] * w[b];
        }
      div1 += cell1 * g.dx * g.dy;
      const double right = S9[2][0][4] + 4.0 * S9[2][1][4] + S9[2][2][4];
      const double left = S9[0][0][4] + 4.0 * S9[0][1][4] + S9[0][2][4];
      const double top = S9[0][2][5] + 4.0 * S9[1][2][5] + S9[2][2][5];
      const double bottom = S9[0][0][5] + 4.0 * S9[1][0][5] + S9[2][0][5];
      div2 += std::fabs((right - left) + (top - bottom)) / 6.0 * g.dx * g.dy;
    }
  out2[0] = div1;
  out2[1] = div2;
}

#endif  // ORC_TANGENT

}  // extern "C"
