// FP64 reference ("oracle") for the batched rigid-body physics step.
//
// TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline
// leg of the benchmark load this library.  It shares no code with the GPU library:
// it parses the model blob with its own reader and computes every phase itself, in
// plain loops, in double precision (or in forward-mode dual numbers for reference
// derivatives).
//
// The paper (MuJoCo Playground) runs the MuJoCo/MJX step but does not restate its
// algorithms; the phases below follow the textbook definitions they come from:
//   * spatial algebra, forward kinematics, RNEA, CRBA and the sparse LTDL factorisation
//     of the joint-space inertia: Featherstone, Rigid Body Dynamics Algorithms (2008),
//     ch. 2, 4, 5, 6 (Table 5.1 RNEA, Table 6.2 CRBA, sec. 6.5 LTDL);
//   * the convex soft-constraint contact model (cost, impedance, reference
//     acceleration): Todorov, "Convex and analytically-invertible dynamics with
//     contacts and constraints", ICRA 2014, with MuJoCo's documented parameter
//     conventions (solref, solimp);
//   * Newton's method with an exact line search on a convex piecewise quadratic:
//     Nocedal & Wright, Numerical Optimization, ch. 3 and 6;
//   * closest points between primitives: Ericson, Real-Time Collision Detection, ch. 5.
// The paper fixes the knobs: solver iterations and line-search iterations (Table
// tab:dm_control_envs) and the PD actuator mapping (eq. pd_mapping).
//
// Conventions: quaternions are w-first; a free joint's qpos is (position, quaternion)
// and its qvel is (world linear velocity of the body origin, body-frame angular
// velocity).  Spatial vectors are in world-aligned Plucker coordinates at the world
// origin: motion [angular; linear], force [moment; force].

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <string>
#include <thread>
#include <vector>

namespace mjo {

// --------------------------------------------------------------------------- duals
struct Dual {
  double v = 0.0, d = 0.0;
  Dual() = default;
  Dual(double x) : v(x), d(0.0) {}  // NOLINT: implicit on purpose
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
inline Dual& operator/=(Dual& a, Dual b) { a = a / b; return a; }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
inline bool operator==(Dual a, Dual b) { return a.v == b.v; }
inline bool operator!=(Dual a, Dual b) { return a.v != b.v; }
inline Dual sqrt(Dual a) {
  double s = std::sqrt(a.v);
  return {s, s > 0.0 ? a.d / (2.0 * s) : 0.0};
}
inline Dual sin(Dual a) { return {std::sin(a.v), std::cos(a.v) * a.d}; }
inline Dual cos(Dual a) { return {std::cos(a.v), -std::sin(a.v) * a.d}; }
inline Dual fabs(Dual a) { return a.v < 0.0 ? -a : a; }
inline Dual pow(Dual a, double p) {
  return {std::pow(a.v, p), p * std::pow(a.v, p - 1.0) * a.d};
}
inline bool isfinite(Dual a) { return std::isfinite(a.v) && std::isfinite(a.d); }
inline bool isfinite(double a) { return std::isfinite(a); }
inline double val(double x) { return x; }
inline double val(Dual x) { return x.v; }

// ------------------------------------------------------- operation-counting scalar
// Counts floating-point operations (+ - * / and elementary functions, one each) of the
// reference algorithm; used to report the algorithmic work of one step.  g_flops counts
// every operation of these plain dense loops; g_flops_nz only those whose operands are
// all nonzero: a product with an exact zero (a structural zero of the dense Jacobian or
// mass matrix, an inactive row's force) and a sum with an exact zero are free to an
// implementation that skips them, so g_flops_nz is the algorithmic count.
thread_local long long g_flops = 0;
thread_local long long g_flops_nz = 0;
struct Cnt {
  double v = 0.0;
  Cnt() = default;
  Cnt(double x) : v(x) {}  // NOLINT: implicit on purpose
};
inline void count_op(double a, double b) {
  g_flops++;
  if (a != 0.0 && b != 0.0) g_flops_nz++;
}
inline Cnt operator+(Cnt a, Cnt b) { count_op(a.v, b.v); return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { count_op(a.v, b.v); return Cnt(a.v - b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt operator*(Cnt a, Cnt b) { count_op(a.v, b.v); return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { count_op(a.v, 1.0); return Cnt(a.v / b.v); }
inline Cnt& operator+=(Cnt& a, Cnt b) { a = a + b; return a; }
inline Cnt& operator-=(Cnt& a, Cnt b) { a = a - b; return a; }
inline Cnt& operator*=(Cnt& a, Cnt b) { a = a * b; return a; }
inline Cnt& operator/=(Cnt& a, Cnt b) { a = a / b; return a; }
inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }
inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
inline bool operator<=(Cnt a, Cnt b) { return a.v <= b.v; }
inline bool operator>=(Cnt a, Cnt b) { return a.v >= b.v; }
inline bool operator==(Cnt a, Cnt b) { return a.v == b.v; }
inline bool operator!=(Cnt a, Cnt b) { return a.v != b.v; }
inline Cnt sqrt(Cnt a) { count_op(a.v, 1.0); return Cnt(std::sqrt(a.v)); }
inline Cnt sin(Cnt a) { count_op(1.0, 1.0); return Cnt(std::sin(a.v)); }
inline Cnt cos(Cnt a) { count_op(1.0, 1.0); return Cnt(std::cos(a.v)); }
inline Cnt fabs(Cnt a) { return Cnt(std::fabs(a.v)); }
inline Cnt pow(Cnt a, double p) { count_op(1.0, 1.0); return Cnt(std::pow(a.v, p)); }
inline bool isfinite(Cnt a) { return std::isfinite(a.v); }
inline double val(Cnt x) { return x.v; }

using std::cos;
using std::fabs;
using std::pow;
using std::sin;
using std::sqrt;

template <class T> inline T tmin(T a, T b) { return b < a ? b : a; }
template <class T> inline T tmax(T a, T b) { return a < b ? b : a; }
template <class T> inline T clamp(T x, T lo, T hi) { return tmin(tmax(x, lo), hi); }

// ------------------------------------------------------------------ 3-vector algebra
template <class T> inline T dot3(const T* a, const T* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
template <class T> inline void cross3(const T* a, const T* b, T* r) {
  T x = a[1] * b[2] - a[2] * b[1];
  T y = a[2] * b[0] - a[0] * b[2];
  T z = a[0] * b[1] - a[1] * b[0];
  r[0] = x; r[1] = y; r[2] = z;
}
template <class T> inline T norm3(const T* a) { return sqrt(dot3(a, a)); }
// r = R v, R row-major 3x3
template <class T, class U> inline void matvec(const T* R, const U* v, T* r) {
  T x = R[0] * v[0] + R[1] * v[1] + R[2] * v[2];
  T y = R[3] * v[0] + R[4] * v[1] + R[5] * v[2];
  T z = R[6] * v[0] + R[7] * v[1] + R[8] * v[2];
  r[0] = x; r[1] = y; r[2] = z;
}
// r = R^T v
template <class T> inline void matTvec(const T* R, const T* v, T* r) {
  T x = R[0] * v[0] + R[3] * v[1] + R[6] * v[2];
  T y = R[1] * v[0] + R[4] * v[1] + R[7] * v[2];
  T z = R[2] * v[0] + R[5] * v[1] + R[8] * v[2];
  r[0] = x; r[1] = y; r[2] = z;
}
template <class T, class U> inline void matmul(const T* A, const U* B, T* C) {
  T out[9];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      out[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
  for (int k = 0; k < 9; k++) C[k] = out[k];
}
// rotation matrix of a unit quaternion (w, x, y, z)
template <class T> inline void quat2mat(const T* q, T* R) {
  T w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
}
// rotation by angle about a unit axis (Rodrigues)
template <class T> inline void axis_angle(const T* a, T ang, T* R) {
  T c = cos(ang), s = sin(ang), t = 1.0 - c;
  R[0] = c + t * a[0] * a[0];        R[1] = t * a[0] * a[1] - s * a[2]; R[2] = t * a[0] * a[2] + s * a[1];
  R[3] = t * a[0] * a[1] + s * a[2]; R[4] = c + t * a[1] * a[1];        R[5] = t * a[1] * a[2] - s * a[0];
  R[6] = t * a[0] * a[2] - s * a[1]; R[7] = t * a[1] * a[2] + s * a[0]; R[8] = c + t * a[2] * a[2];
}
template <class T> inline void quatmul(const T* a, const T* b, T* r) {
  T w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  T x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  T y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  T z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
  r[0] = w; r[1] = x; r[2] = y; r[3] = z;
}

// ------------------------------------------------------------- spatial algebra (RBDA 2)
// motion cross: [w1; v1] x [w2; v2] = [w1 x w2; w1 x v2 + v1 x w2]
template <class T> inline void crossm(const T* m1, const T* m2, T* r) {
  T a[3], b[3], c[3];
  cross3(m1, m2, a);
  cross3(m1, m2 + 3, b);
  cross3(m1 + 3, m2, c);
  for (int i = 0; i < 3; i++) { r[i] = a[i]; r[3 + i] = b[i] + c[i]; }
}
// force cross: [w; v] x* [n; f] = [w x n + v x f; w x f]
template <class T> inline void crossf(const T* m, const T* f, T* r) {
  T a[3], b[3], c[3];
  cross3(m, f, a);
  cross3(m + 3, f + 3, b);
  cross3(m, f + 3, c);
  for (int i = 0; i < 3; i++) { r[i] = a[i] + b[i]; r[3 + i] = c[i]; }
}
// spatial inertia at the world origin, stored as
//   [m, h (= m c, 3), I_O (xx yy zz xy xz yz)]
// applied to a motion [w; v]:  [I_O w + h x v;  m v - h x w]   (RBDA 2.13)
template <class T> inline void inertia_apply(const T* I, const T* mv, T* f) {
  const T m = I[0];
  const T* h = I + 1;
  const T* J = I + 4;
  const T* w = mv;
  const T* v = mv + 3;
  T hv[3], hw[3];
  cross3(h, v, hv);
  cross3(h, w, hw);
  T n0 = J[0] * w[0] + J[3] * w[1] + J[4] * w[2];
  T n1 = J[3] * w[0] + J[1] * w[1] + J[5] * w[2];
  T n2 = J[4] * w[0] + J[5] * w[1] + J[2] * w[2];
  f[0] = n0 + hv[0]; f[1] = n1 + hv[1]; f[2] = n2 + hv[2];
  f[3] = m * v[0] - hw[0]; f[4] = m * v[1] - hw[1]; f[5] = m * v[2] - hw[2];
}
template <class T> inline T dot6(const T* a, const T* b) {
  T s = 0.0;
  for (int i = 0; i < 6; i++) s += a[i] * b[i];
  return s;
}

// -------------------------------------------------------------------------- model
enum { JFREE = 0, JSLIDE = 1, JHINGE = 2 };
enum { GPLANE = 0, GSPHERE = 1, GCAPSULE = 2, GBOX = 3, GHFIELD = 4 };
enum { AMOTOR = 0, APD = 1 };
enum { ST_NONFINITE = 1, ST_OVERFLOW = 2, ST_NODESCENT = 4 };
static const int CON_SIZE = 20;  // exported contact record (see mjo_api.h)

struct Model {
  int nbody = 0, njnt = 0, ngeom = 0, npair = 0, nu = 0, nq = 0, nv = 0;
  int iterations = 0, ls_iterations = 0, nconmax = 0;
  double dt = 0, grav[3] = {0, 0, 0}, solref[2] = {0, 0}, solimp[5] = {0, 0, 0, 0, 0};
  double tolerance = 0;
  std::vector<int> body_parent;
  std::vector<double> body_pos, body_quat, body_mass, body_ipos, body_inertia;
  std::vector<int> jnt_type, jnt_body, jnt_limited;
  std::vector<double> jnt_pos, jnt_axis, jnt_damping, jnt_armature, jnt_range,
      jnt_frictionloss;
  std::vector<int> geom_type, geom_body;
  std::vector<double> geom_size, geom_pos, geom_quat, geom_friction;
  std::vector<int> pair_g1, pair_g2;
  std::vector<int> pair_condim;  // 1 frictionless (1 row); 3 sliding (4 rows); 4 + torsion
                                 // (6 rows); 6 + rolling (10 rows): two pyramid edges a
                                 // friction direction
  std::vector<double> pair_mu, pair_mu_torsion, pair_mu_rolling;
  std::vector<int> act_type, act_jnt;
  std::vector<double> act_gear, act_kp, act_kd, act_range, act_qdef;
  int neq = 0;
  int cone = 0;  // friction cone: 0 pyramidal (edges), 1 elliptic (the contact frame's rows)
  int integrator = 0;  // 0: semi-implicit Euler; 1: with implicit damping; 2: also implicit
                       // PD position gains; 3: classic fourth-order Runge-Kutta
  // heightfield: nrow x ncol elevations in [0, 1] over [-sx, sx] x [-sy, sy], z = sz h
  int hf_nrow = 0, hf_ncol = 0;
  double hf_size[3] = {0, 0, 0};
  std::vector<double> hf_data;
  std::vector<int> eq_type, eq_b1, eq_b2;
  std::vector<double> eq_a1, eq_a2;  // anchor in body1's / body2's frame
  std::vector<double> eq_relR;       // weld: body2's reference orientation in body1's frame
  int neqrow = 0;                    // 3 rows per connect, 6 per weld
  std::vector<double> qpos0;
  // derived
  std::vector<int> jnt_qposadr, jnt_dofadr, body_jntadr, body_jntnum, body_dofadr, body_dofnum;
  std::vector<int> dof_body, dof_jnt, dof_parent;
  std::vector<double> dof_damping, dof_armature, dof_frictionloss;
  std::vector<double> body_invweight;
  std::vector<double> dof_invweight;  // (M^-1)_kk at qpos0
  int nlimit = 0;                     // limited joints
  int nfric = 0;                      // dofs with friction loss (one row each, always)
};

struct Reader {
  const uint8_t* p;
  size_t n, off = 0;
  bool ok = true;
  template <class X> void read(X* dst, size_t count) {
    size_t bytes = sizeof(X) * count;
    if (off + bytes > n) { ok = false; return; }
    std::memcpy(dst, p + off, bytes);
    off += bytes;
  }
};

// ------------------------------------------------------------------------ world data
template <class T> struct Contact {
  T dist = 0.0;
  T pos[3];
  T frame[9];  // rows: normal (geom1 -> geom2), tangent 1, tangent 2
  T mu = 0.0, mu_t = 0.0, mu_r = 0.0;  // sliding, torsional and rolling coefficients
  int pair = -1, sub = -1, g1 = -1, g2 = -1;
  int condim = 3, row = 0;  // its contact dimension and first row
};

template <class T> struct Data {
  std::vector<T> qpos, qvel, qacc_ws, ctrl;
  std::vector<T> xpos, xmat, xipos, cinert;     // bodies
  std::vector<T> cdof, cdof_dot, cvel;          // dofs / bodies
  std::vector<T> gpos, gmat;                    // geoms
  std::vector<T> M, qLD, qfrc_bias, qfrc_act, qfrc_pass, qfrc_smooth, qacc_smooth;
  std::vector<Contact<T>> con;
  int nrow = 0;
  std::vector<T> J, aref, D, efc_force, qfrc_con;
  std::vector<double> fl;  // per row: friction-loss bound, 0 for a one-sided row
  std::vector<T> qacc;
  std::vector<T> qacc_int;  // acceleration the integrator applies (differs with implicit damping)
  std::vector<T> H;  // dense Cholesky factor of the last Newton Hessian
  // elliptic cone blocks: a contact's first row, its rows (condim) and sliding mu; per row,
  // the ratio mu_j / mu of its friction coefficient to the sliding one (1 on the normal)
  // and whether it belongs to such a block
  std::vector<int> cone_row0, cone_nd;
  std::vector<T> cone_mu, row_ratio;
  std::vector<char> in_cone;
  int status = 0;
  int newton_iters = 0;
  void alloc(const Model& m) {
    qpos.assign(m.nq, 0.0); qvel.assign(m.nv, 0.0); qacc_ws.assign(m.nv, 0.0);
    ctrl.assign(m.nu, 0.0);
    xpos.assign(3 * m.nbody, 0.0); xmat.assign(9 * m.nbody, 0.0);
    xipos.assign(3 * m.nbody, 0.0); cinert.assign(10 * m.nbody, 0.0);
    cdof.assign(6 * m.nv, 0.0); cdof_dot.assign(6 * m.nv, 0.0); cvel.assign(6 * m.nbody, 0.0);
    gpos.assign(3 * m.ngeom, 0.0); gmat.assign(9 * m.ngeom, 0.0);
    M.assign(m.nv * m.nv, 0.0); qLD.assign(m.nv * m.nv, 0.0);
    qfrc_bias.assign(m.nv, 0.0); qfrc_act.assign(m.nv, 0.0); qfrc_pass.assign(m.nv, 0.0);
    qfrc_smooth.assign(m.nv, 0.0); qacc_smooth.assign(m.nv, 0.0);
    qacc.assign(m.nv, 0.0); qfrc_con.assign(m.nv, 0.0); qacc_int.assign(m.nv, 0.0);
    H.assign(m.nv * m.nv, 0.0);
  }
};

// ------------------------------------------------------------------ A1: kinematics
// Bodies in tree order.  A body's frame is placed on its parent's frame, then its joints
// act in declaration order: a hinge rotates the frame about its world axis through its
// world anchor, a slide translates along its world axis, a free joint sets the pose.
// The motion subspace of each dof is stored at the world origin (RBDA ch. 4).
template <class T> void kinematics(const Model& m, Data<T>& d) {
  for (int k = 0; k < 3; k++) d.xpos[k] = 0.0;
  for (int k = 0; k < 9; k++) d.xmat[k] = (k % 4 == 0) ? 1.0 : 0.0;
  for (int b = 1; b < m.nbody; b++) {
    const int p = m.body_parent[b];
    T pos[3], R[9], Rq[9];
    matvec(&d.xmat[9 * p], &m.body_pos[3 * b], pos);
    for (int k = 0; k < 3; k++) pos[k] += d.xpos[3 * p + k];
    T qb[4] = {m.body_quat[4 * b], m.body_quat[4 * b + 1], m.body_quat[4 * b + 2],
               m.body_quat[4 * b + 3]};
    quat2mat(qb, Rq);
    matmul(&d.xmat[9 * p], Rq, R);
    for (int jj = 0; jj < m.body_jntnum[b]; jj++) {
      const int j = m.body_jntadr[b] + jj;
      const int qa = m.jnt_qposadr[j], da = m.jnt_dofadr[j];
      T* S = &d.cdof[6 * da];
      if (m.jnt_type[j] == JFREE) {
        for (int k = 0; k < 3; k++) pos[k] = d.qpos[qa + k];
        T q[4] = {d.qpos[qa + 3], d.qpos[qa + 4], d.qpos[qa + 5], d.qpos[qa + 6]};
        T n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        for (int k = 0; k < 4; k++) q[k] = q[k] / n;
        quat2mat(q, R);
        for (int i = 0; i < 3; i++) {  // translation dofs: [0; e_i]
          for (int k = 0; k < 6; k++) S[6 * i + k] = 0.0;
          S[6 * i + 3 + i] = 1.0;
        }
        for (int i = 0; i < 3; i++) {  // rotation dofs: [R e_i; x × R e_i]
          T r[3] = {R[i], R[3 + i], R[6 + i]};
          T* s = S + 6 * (3 + i);
          s[0] = r[0]; s[1] = r[1]; s[2] = r[2];
          cross3(pos, r, s + 3);
        }
      } else if (m.jnt_type[j] == JSLIDE) {
        T ax[3];
        matvec(R, &m.jnt_axis[3 * j], ax);
        for (int k = 0; k < 3; k++) pos[k] += ax[k] * d.qpos[qa];
        S[0] = S[1] = S[2] = 0.0;
        S[3] = ax[0]; S[4] = ax[1]; S[5] = ax[2];
      } else {  // hinge
        T ax[3], anc[3], off[3];
        matvec(R, &m.jnt_axis[3 * j], ax);
        matvec(R, &m.jnt_pos[3 * j], off);
        for (int k = 0; k < 3; k++) anc[k] = pos[k] + off[k];
        T Rj[9];
        axis_angle(ax, d.qpos[qa], Rj);
        matmul(Rj, R, R);
        matvec(R, &m.jnt_pos[3 * j], off);
        for (int k = 0; k < 3; k++) pos[k] = anc[k] - off[k];
        S[0] = ax[0]; S[1] = ax[1]; S[2] = ax[2];
        cross3(anc, ax, S + 3);
      }
    }
    for (int k = 0; k < 3; k++) d.xpos[3 * b + k] = pos[k];
    for (int k = 0; k < 9; k++) d.xmat[9 * b + k] = R[k];
    // centre of mass and spatial inertia at the world origin
    T c[3];
    matvec(R, &m.body_ipos[3 * b], c);
    for (int k = 0; k < 3; k++) { c[k] += pos[k]; d.xipos[3 * b + k] = c[k]; }
    const double* Ib = &m.body_inertia[6 * b];
    double Il[9] = {Ib[0], Ib[3], Ib[4], Ib[3], Ib[1], Ib[5], Ib[4], Ib[5], Ib[2]};
    T RI[9], Iw[9], Rt[9];
    matmul(R, Il, RI);
    for (int i = 0; i < 3; i++)
      for (int k = 0; k < 3; k++) Rt[3 * i + k] = R[3 * k + i];
    matmul(RI, Rt, Iw);
    const double mass = m.body_mass[b];
    T cc = dot3(c, c);
    T* ci = &d.cinert[10 * b];
    ci[0] = mass;
    for (int k = 0; k < 3; k++) ci[1 + k] = mass * c[k];
    ci[4] = Iw[0] + mass * (cc - c[0] * c[0]);
    ci[5] = Iw[4] + mass * (cc - c[1] * c[1]);
    ci[6] = Iw[8] + mass * (cc - c[2] * c[2]);
    ci[7] = Iw[1] - mass * c[0] * c[1];
    ci[8] = Iw[2] - mass * c[0] * c[2];
    ci[9] = Iw[5] - mass * c[1] * c[2];
  }
  for (int g = 0; g < m.ngeom; g++) {
    const int b = m.geom_body[g];
    T off[3], Rg[9];
    matvec(&d.xmat[9 * b], &m.geom_pos[3 * g], off);
    for (int k = 0; k < 3; k++) d.gpos[3 * g + k] = d.xpos[3 * b + k] + off[k];
    T qg[4] = {m.geom_quat[4 * g], m.geom_quat[4 * g + 1], m.geom_quat[4 * g + 2],
               m.geom_quat[4 * g + 3]};
    T n = sqrt(qg[0] * qg[0] + qg[1] * qg[1] + qg[2] * qg[2] + qg[3] * qg[3]);
    for (int k = 0; k < 4; k++) qg[k] = qg[k] / n;
    quat2mat(qg, Rg);
    matmul(&d.xmat[9 * b], Rg, &d.gmat[9 * g]);
  }
}

// -------------------------------------------------- A2: body velocities, dS/dt (RBDA 5)
// The subspace of a hinge or slide is fixed in the frame reached after that joint, so
// its rate is V x S with V the velocity accumulated up to and including the joint.
// A free joint's translation subspaces are fixed in the world (rate 0); its rotation
// subspaces turn with the body (rate V_body x S).
template <class T> void velocities(const Model& m, Data<T>& d) {
  for (int k = 0; k < 6; k++) d.cvel[k] = 0.0;
  for (int b = 1; b < m.nbody; b++) {
    T V[6];
    for (int k = 0; k < 6; k++) V[k] = d.cvel[6 * m.body_parent[b] + k];
    for (int jj = 0; jj < m.body_jntnum[b]; jj++) {
      const int j = m.body_jntadr[b] + jj;
      const int da = m.jnt_dofadr[j];
      if (m.jnt_type[j] == JFREE) {
        for (int i = 0; i < 6; i++)
          for (int k = 0; k < 6; k++) V[k] += d.cdof[6 * (da + i) + k] * d.qvel[da + i];
        for (int i = 0; i < 3; i++)
          for (int k = 0; k < 6; k++) d.cdof_dot[6 * (da + i) + k] = 0.0;
        for (int i = 3; i < 6; i++) crossm(V, &d.cdof[6 * (da + i)], &d.cdof_dot[6 * (da + i)]);
      } else {
        for (int k = 0; k < 6; k++) V[k] += d.cdof[6 * da + k] * d.qvel[da];
        crossm(V, &d.cdof[6 * da], &d.cdof_dot[6 * da]);
      }
    }
    for (int k = 0; k < 6; k++) d.cvel[6 * b + k] = V[k];
  }
}

// ------------------------------------------------- A5: recursive Newton-Euler (RBDA 5.3)
// tau = M(q) qacc + c(q, qvel); the world accelerates at -gravity so gravity is included.
template <class T>
void rne(const Model& m, const Data<T>& d, const T* qacc, T* tau) {
  std::vector<T> acc(6 * m.nbody, 0.0), frc(6 * m.nbody, 0.0);
  acc[0] = acc[1] = acc[2] = 0.0;
  for (int k = 0; k < 3; k++) acc[3 + k] = -m.grav[k];
  for (int b = 1; b < m.nbody; b++) {
    T A[6];
    for (int k = 0; k < 6; k++) A[k] = acc[6 * m.body_parent[b] + k];
    for (int i = 0; i < m.body_dofnum[b]; i++) {
      const int k0 = m.body_dofadr[b] + i;
      for (int k = 0; k < 6; k++) {
        A[k] += d.cdof_dot[6 * k0 + k] * d.qvel[k0];
        if (qacc) A[k] += d.cdof[6 * k0 + k] * qacc[k0];
      }
    }
    for (int k = 0; k < 6; k++) acc[6 * b + k] = A[k];
    T IA[6], IV[6], VxIV[6];
    inertia_apply(&d.cinert[10 * b], A, IA);
    inertia_apply(&d.cinert[10 * b], &d.cvel[6 * b], IV);
    crossf(&d.cvel[6 * b], IV, VxIV);
    for (int k = 0; k < 6; k++) frc[6 * b + k] = IA[k] + VxIV[k];
  }
  for (int b = m.nbody - 1; b > 0; b--) {
    const int p = m.body_parent[b];
    if (p > 0)
      for (int k = 0; k < 6; k++) frc[6 * p + k] += frc[6 * b + k];
  }
  for (int i = 0; i < m.nv; i++) tau[i] = dot6(&d.cdof[6 * i], &frc[6 * m.dof_body[i]]);
}

// ------------------------------------------------------------ A3: CRBA (RBDA Table 6.2)
// Composite inertia of each subtree; M_ij = S_j . (Ic_{body(i)} S_i) for every dof j that
// is an ancestor-or-self of dof i; armature on the diagonal.
template <class T> void crba(const Model& m, Data<T>& d) {
  std::vector<T> Ic(d.cinert);
  for (int b = m.nbody - 1; b > 0; b--) {
    const int p = m.body_parent[b];
    if (p > 0)
      for (int k = 0; k < 10; k++) Ic[10 * p + k] += Ic[10 * b + k];
  }
  std::fill(d.M.begin(), d.M.end(), T(0.0));
  for (int i = 0; i < m.nv; i++) {
    T F[6];
    inertia_apply(&Ic[10 * m.dof_body[i]], &d.cdof[6 * i], F);
    for (int j = i; j >= 0; j = m.dof_parent[j]) {
      T v = dot6(&d.cdof[6 * j], F);
      d.M[i * m.nv + j] = v;
      d.M[j * m.nv + i] = v;
    }
    d.M[i * m.nv + i] += m.dof_armature[i];
  }
}

// ---------------------------------------------------- A4: sparse LTDL (RBDA sec. 6.5)
// M = L^T D L with L unit lower triangular and the dof-tree sparsity (no fill-in).
// Result in qLD: strictly lower part = L, diagonal = D.
template <class T> void factor_ltdl(const Model& m, const std::vector<T>& M, std::vector<T>& LD) {
  const int n = m.nv;
  LD = M;
  for (int k = n - 1; k >= 0; k--) {
    const T Dk = LD[k * n + k];
    for (int i = m.dof_parent[k]; i >= 0; i = m.dof_parent[i]) {
      const T a = LD[k * n + i] / Dk;
      for (int j = i; j >= 0; j = m.dof_parent[j]) LD[i * n + j] -= a * LD[k * n + j];
      LD[k * n + i] = a;
    }
  }
}
// x = M^{-1} b using the LTDL factors
template <class T> void solve_ltdl(const Model& m, const std::vector<T>& LD, const T* b, T* x) {
  const int n = m.nv;
  std::vector<T> y(b, b + n);
  for (int k = n - 1; k >= 0; k--)  // L^T y = b
    for (int i = m.dof_parent[k]; i >= 0; i = m.dof_parent[i]) y[i] -= LD[k * n + i] * y[k];
  for (int k = 0; k < n; k++) y[k] = y[k] / LD[k * n + k];  // D
  for (int k = 0; k < n; k++)  // L x = y
    for (int i = m.dof_parent[k]; i >= 0; i = m.dof_parent[i]) y[k] -= LD[k * n + i] * y[i];
  for (int k = 0; k < n; k++) x[k] = y[k];
}

// -------------------------------------------------------- A0: actuation and passive
// Motor: tau = gear * u.  Position actuator (eq. pd_mapping):
//   tau = kp (q_default + gear * u - q) - kd qdot,  u clamped to ctrlrange.
// Joint damping: tau = -b qdot (explicit, evaluated at the start of the step).
template <class T> void actuation(const Model& m, Data<T>& d) {
  for (int i = 0; i < m.nv; i++) {
    d.qfrc_act[i] = 0.0;
    d.qfrc_pass[i] = -m.dof_damping[i] * d.qvel[i];
  }
  for (int a = 0; a < m.nu; a++) {
    const int j = m.act_jnt[a];
    const int qa = m.jnt_qposadr[j], da = m.jnt_dofadr[j];
    T u = clamp(d.ctrl[a], T(m.act_range[2 * a]), T(m.act_range[2 * a + 1]));
    if (m.act_type[a] == AMOTOR) {
      d.qfrc_act[da] += m.act_gear[a] * u;
    } else {
      d.qfrc_act[da] += m.act_kp[a] * (m.act_qdef[a] + m.act_gear[a] * u - d.qpos[qa]) -
                        m.act_kd[a] * d.qvel[da];
    }
  }
}

// --------------------------------------------------------------- A7: collision
// Contact: signed distance (negative = penetration), position midway between the two
// surface points, normal from geom 1 toward geom 2.  Emitted iff dist < 0.
template <class T> struct Cand {
  T dist;
  T pos[3];
  T n[3];
  int sub;
};

template <class T>
void add_cand(std::vector<Cand<T>>& out, T dist, const T* pos, const T* n, int sub) {
  Cand<T> c;
  c.dist = dist;
  for (int k = 0; k < 3; k++) { c.pos[k] = pos[k]; c.n[k] = n[k]; }
  c.sub = sub;
  out.push_back(c);
}

// sphere (centre c, radius r) against a plane (point p0, unit normal n)
template <class T>
void sphere_plane(const T* p0, const T* n, const T* c, T r, int sub, std::vector<Cand<T>>& out) {
  T rel[3] = {c[0] - p0[0], c[1] - p0[1], c[2] - p0[2]};
  T dist = dot3(n, rel) - r;
  if (dist < 0.0) {
    T pos[3];
    for (int k = 0; k < 3; k++) pos[k] = c[k] - n[k] * (r + 0.5 * dist);
    add_cand(out, dist, pos, n, sub);
  }
}

// two spheres; the normal points from sphere 1 to sphere 2
template <class T>
void sphere_sphere(const T* c1, T r1, const T* c2, T r2, int sub, std::vector<Cand<T>>& out) {
  T dv[3] = {c2[0] - c1[0], c2[1] - c1[1], c2[2] - c1[2]};
  T L = norm3(dv);
  T n[3];
  if (L > 1e-12) {
    for (int k = 0; k < 3; k++) n[k] = dv[k] / L;
  } else {
    n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
  }
  T dist = L - r1 - r2;
  if (dist < 0.0) {
    T pos[3];
    for (int k = 0; k < 3; k++) pos[k] = c1[k] + n[k] * (r1 + 0.5 * dist);
    add_cand(out, dist, pos, n, sub);
  }
}

// closest point parameter on segment a + t u (t in [0,1]) to point p
template <class T> T seg_point_param(const T* a, const T* u, const T* p) {
  T uu = dot3(u, u);
  T ap[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
  if (uu < 1e-30) return T(0.0);
  return clamp(dot3(ap, u) / uu, T(0.0), T(1.0));
}

// closest points of segments p0 + s d1 and q0 + t d2 (Ericson 5.1.9); parallel segments
// take the midpoint of the overlap of segment 2's projection on segment 1
template <class T>
void seg_seg(const T* p0, const T* d1, const T* q0, const T* d2, T& s, T& t) {
  T r[3] = {p0[0] - q0[0], p0[1] - q0[1], p0[2] - q0[2]};
  T a = dot3(d1, d1), e = dot3(d2, d2), f = dot3(d2, r);
  T c = dot3(d1, r), b = dot3(d1, d2);
  T den = a * e - b * b;
  if (den > 1e-6 * a * e) {
    s = clamp((b * f - c * e) / den, T(0.0), T(1.0));
    t = (b * s + f) / e;
    if (t < 0.0) {
      t = 0.0;
      s = clamp(-c / a, T(0.0), T(1.0));
    } else if (t > 1.0) {
      t = 1.0;
      s = clamp((b - c) / a, T(0.0), T(1.0));
    }
  } else {
    T s0 = clamp(-c / a, T(0.0), T(1.0));
    T s1 = clamp((b - c) / a, T(0.0), T(1.0));
    s = 0.5 * (s0 + s1);
    t = clamp((b * s + f) / e, T(0.0), T(1.0));
  }
}

// signed distance of a point p (box frame) to a box of half extents h, and its gradient
template <class T> T box_sdf(const T* p, const double* h, T* grad) {
  T q[3], o[3];
  bool outside = false;
  for (int k = 0; k < 3; k++) {
    q[k] = fabs(p[k]) - h[k];
    o[k] = tmax(q[k], T(0.0));
    if (q[k] > 0.0) outside = true;
  }
  if (outside) {
    T L = norm3(o);
    if (grad)
      for (int k = 0; k < 3; k++) grad[k] = (p[k] < 0.0 ? -1.0 : 1.0) * o[k] / L;
    return L;
  }
  int ax = 0;
  for (int k = 1; k < 3; k++)
    if (q[k] > q[ax]) ax = k;
  if (grad) {
    grad[0] = grad[1] = grad[2] = 0.0;
    grad[ax] = p[ax] < 0.0 ? -1.0 : 1.0;
  }
  return q[ax];
}

// box (centre c, rotation R, half extents h) against a sphere at world point p:
// returns sdf and the outward box normal (world) at p
template <class T>
T box_point(const T* c, const T* R, const double* h, const T* p, T* nworld) {
  T rel[3] = {p[0] - c[0], p[1] - c[1], p[2] - c[2]}, pl[3], g[3];
  matTvec(R, rel, pl);
  T s = box_sdf(pl, h, g);
  matvec(R, g, nworld);
  return s;
}

// capsule segment a + t u (t in [0, 1]) against a box.  In box coordinates the segment is
// P(t) = p0 + t v, and the box's signed distance f(t) along it is convex and piecewise
// smooth: its pieces change where a coordinate crosses -h_k, 0 or h_k and, inside the
// box, where the largest face distance changes hands (|P_i| - h_i = |P_j| - h_j).  On a
// piece outside the box f^2 is the sum, over the coordinates beyond their slab, of
// (|P_k| - h_k)^2: a quadratic in t with a closed-form minimiser.  Inside, f is linear.
// So the minimiser set of f over [0, 1] is found exactly among the breakpoints and the
// pieces' stationary points: the points whose f equals the minimum (to g_cb_eq of the
// segment's scale, a rounding allowance) span it.  Candidates: the segment's ends and
// the minimiser set's ends (both when it is a stretch, as for a capsule lying on a face;
// one point otherwise), de-duplicated within g_cb_dup in t; the two deepest penetrating
// ones are kept.  Normal from capsule to box.
// mjo_set_capsule_box_tolerances changes g_cb_eq and g_cb_dup (tests only: the contacts
// must not depend on them).
static double g_cb_eq = 1e-12, g_cb_dup = 1e-6;
template <class T>
void capsule_box(const T* a, const T* u, T r, const T* c, const T* R, const double* h,
                 std::vector<Cand<T>>& out) {
  T rel[3] = {a[0] - c[0], a[1] - c[1], a[2] - c[2]}, p0[3], v[3];
  matTvec(R, rel, p0);
  matTvec(R, u, v);
  auto f = [&](T t) {
    T p[3] = {p0[0] + t * v[0], p0[1] + t * v[1], p0[2] + t * v[2]};
    return box_sdf(p, h, (T*)nullptr);
  };
  std::vector<T> ts = {T(0.0), T(1.0)};
  auto add = [&](T t) {
    if (t > 0.0 && t < 1.0) ts.push_back(t);
  };
  for (int k = 0; k < 3; k++)
    if (v[k] != 0.0)
      for (double q : {-h[k], 0.0, h[k]}) add((T(q) - p0[k]) / v[k]);
  for (int i = 0; i < 3; i++)
    for (int j = i + 1; j < 3; j++)
      for (double si : {-1.0, 1.0})
        for (double sj : {-1.0, 1.0}) {  // si P_i - h_i = sj P_j - h_j
          const T den = si * v[i] - sj * v[j];
          if (den != 0.0) add((T(h[i] - h[j]) - si * p0[i] + sj * p0[j]) / den);
        }
  std::sort(ts.begin(), ts.end(), [](const T& x, const T& y) { return x < y; });
  const size_t nb = ts.size();
  for (size_t k = 0; k + 1 < nb; k++) {  // stationary point of each outside piece
    const T mid = 0.5 * (ts[k] + ts[k + 1]);
    T num = 0.0, den = 0.0;
    for (int i = 0; i < 3; i++) {
      const T pi = p0[i] + mid * v[i];
      if (!(fabs(pi) > h[i])) continue;
      const T s = pi < 0.0 ? T(-1.0) : T(1.0);
      num += (s * p0[i] - h[i]) * s * v[i];
      den += v[i] * v[i];
    }
    if (den > 0.0) {
      const T t = -num / den;
      if (t > ts[k] && t < ts[k + 1]) ts.push_back(t);
    }
  }
  T fmin = f(ts[0]);
  for (const T& t : ts) fmin = tmin(fmin, f(t));
  const double eq = g_cb_eq * (val(norm3(v)) + h[0] + h[1] + h[2]);
  T tlo = 1.0, thi = 0.0;
  for (const T& t : ts)
    if (f(t) <= fmin + eq) {
      tlo = tmin(tlo, t);
      thi = tmax(thi, t);
    }
  T ts4[4] = {T(0.0), T(1.0), tlo, thi};
  bool keep[4] = {true, true, true, true};
  const double tdup = g_cb_dup;
  for (int k = 2; k < 4; k++)
    if (fabs(ts4[k] - 0.0) < tdup || fabs(ts4[k] - 1.0) < tdup) keep[k] = false;
  if (keep[2] && keep[3] && fabs(ts4[3] - ts4[2]) < tdup) keep[3] = false;
  T depth[4];
  T nrm[4][3];
  T pts[4][3];
  for (int k = 0; k < 4; k++) {
    if (!keep[k]) continue;
    T p[3] = {a[0] + ts4[k] * u[0], a[1] + ts4[k] * u[1], a[2] + ts4[k] * u[2]};
    T nb[3];
    T sd = box_point(c, R, h, p, nb);
    depth[k] = sd - r;
    for (int i = 0; i < 3; i++) { nrm[k][i] = -nb[i]; pts[k][i] = p[i] - 0.5 * (r + sd) * nb[i]; }
    if (!(depth[k] < 0.0)) keep[k] = false;
  }
  // two deepest (ties to the lower candidate index), emitted in candidate order
  int sel[2] = {-1, -1};
  for (int s = 0; s < 2; s++) {
    int best = -1;
    for (int k = 0; k < 4; k++) {
      if (!keep[k] || k == sel[0]) continue;
      if (best < 0 || depth[k] < depth[best]) best = k;
    }
    sel[s] = best;
  }
  for (int k = 0; k < 4; k++)
    if (k == sel[0] || k == sel[1]) add_cand(out, depth[k], pts[k], nrm[k], k);
}

// closest point of triangle (a, b, c) to p: the projection onto the triangle's plane
// when it falls inside (all barycentric weights >= 0), else the nearest of the three
// edges' closest points
template <class T>
void tri_closest(const T* a, const T* b, const T* c, const T* p, T* q) {
  T ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
  T ac[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
  T ap[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
  T n[3];
  cross3(ab, ac, n);
  T nn = dot3(n, n);
  T h = dot3(ap, n) / nn;
  T pp[3] = {p[0] - h * n[0], p[1] - h * n[1], p[2] - h * n[2]};  // projection
  // barycentric weights of the projection: areas of the sub-triangles against n
  const T* v[3] = {a, b, c};
  T w[3];
  for (int k = 0; k < 3; k++) {
    const T* e0 = v[(k + 1) % 3];
    const T* e1 = v[(k + 2) % 3];
    T d0[3] = {e0[0] - pp[0], e0[1] - pp[1], e0[2] - pp[2]};
    T d1[3] = {e1[0] - pp[0], e1[1] - pp[1], e1[2] - pp[2]};
    T cr[3];
    cross3(d0, d1, cr);
    w[k] = dot3(cr, n) / nn;
  }
  if (w[0] >= 0.0 && w[1] >= 0.0 && w[2] >= 0.0) {
    for (int k = 0; k < 3; k++) q[k] = pp[k];
    return;
  }
  T best = 0.0;
  for (int e = 0; e < 3; e++) {
    const T* s0 = v[e];
    const T* s1 = v[(e + 1) % 3];
    T u[3] = {s1[0] - s0[0], s1[1] - s0[1], s1[2] - s0[2]};
    T t = seg_point_param(s0, u, p);
    T x[3] = {s0[0] + t * u[0], s0[1] + t * u[1], s0[2] + t * u[2]};
    T dx[3] = {p[0] - x[0], p[1] - x[1], p[2] - x[2]};
    T dd = dot3(dx, dx);
    if (e == 0 || dd < best) {
      best = dd;
      for (int k = 0; k < 3; k++) q[k] = x[k];
    }
  }
}

// sphere (geom 1: centre c, radius r) against the heightfield surface (geom 2, pose
// (xg, Rg)): the nearest point q of the triangles of the grid cells that the sphere's
// footprint overlaps (first in cell and triangle order on ties).  Signed distance
// = +-|c - q| - r, negative when c lies below the nearest triangle's plane; the normal
// points from the sphere into the surface; the position is midway between the surfaces.
template <class T>
void sphere_hfield(const Model& m, const T* xg, const T* Rg, const T* c, T r,
                   std::vector<Cand<T>>& out) {
  const int nr = m.hf_nrow, nc = m.hf_ncol;
  const double sx = m.hf_size[0], sy = m.hf_size[1], sz = m.hf_size[2];
  const double dx = 2.0 * sx / (nc - 1), dy = 2.0 * sy / (nr - 1);
  T rel[3] = {c[0] - xg[0], c[1] - xg[1], c[2] - xg[2]};
  T cl[3];
  matTvec(Rg, rel, cl);  // centre in the heightfield's frame
  auto vert = [&](int i, int j, T* v) {
    v[0] = -sx + dx * j; v[1] = -sy + dy * i; v[2] = sz * m.hf_data[(size_t)i * nc + j];
  };
  const int j0 = std::max(0, (int)std::floor(val((cl[0] - r + sx) / dx)));
  const int j1 = std::min(nc - 2, (int)std::floor(val((cl[0] + r + sx) / dx)));
  const int i0 = std::max(0, (int)std::floor(val((cl[1] - r + sy) / dy)));
  const int i1 = std::min(nr - 2, (int)std::floor(val((cl[1] + r + sy) / dy)));
  bool found = false;
  T bestd = 0.0, bq[3], bn[3];
  for (int i = i0; i <= i1; i++)
    for (int j = j0; j <= j1; j++) {
      T v00[3], v01[3], v10[3], v11[3];
      vert(i, j, v00); vert(i, j + 1, v01); vert(i + 1, j, v10); vert(i + 1, j + 1, v11);
      const T* tris[2][3] = {{v00, v01, v11}, {v00, v11, v10}};
      for (int k = 0; k < 2; k++) {
        T q[3];
        tri_closest(tris[k][0], tris[k][1], tris[k][2], cl, q);
        T dq[3] = {cl[0] - q[0], cl[1] - q[1], cl[2] - q[2]};
        T dd = dot3(dq, dq);
        if (!found || dd < bestd) {
          found = true;
          bestd = dd;
          for (int a = 0; a < 3; a++) bq[a] = q[a];
          T e1[3] = {tris[k][1][0] - tris[k][0][0], tris[k][1][1] - tris[k][0][1],
                     tris[k][1][2] - tris[k][0][2]};
          T e2[3] = {tris[k][2][0] - tris[k][0][0], tris[k][2][1] - tris[k][0][1],
                     tris[k][2][2] - tris[k][0][2]};
          cross3(e1, e2, bn);
        }
      }
    }
  if (!found) return;
  T L = sqrt(bestd);
  T nl = norm3(bn);
  for (int a = 0; a < 3; a++) bn[a] = bn[a] / nl;  // upward unit normal of that triangle
  T dq[3] = {cl[0] - bq[0], cl[1] - bq[1], cl[2] - bq[2]};
  const bool below = dot3(bn, dq) < 0.0;
  T dist = (below ? -L : L) - r;
  if (!(dist < 0.0)) return;
  T nloc[3];  // from the sphere into the surface
  if (L > 1e-12) {
    for (int a = 0; a < 3; a++) nloc[a] = (below ? dq[a] : -dq[a]) / L;
  } else {
    for (int a = 0; a < 3; a++) nloc[a] = -bn[a];
  }
  T n[3], qw[3];
  matvec(Rg, nloc, n);
  matvec(Rg, bq, qw);
  T pos[3];
  for (int a = 0; a < 3; a++) {
    qw[a] += xg[a];
    pos[a] = 0.5 * (c[a] + r * n[a] + qw[a]);
  }
  add_cand(out, dist, pos, n, 0);
}

template <class T> void collide_pair(const Model& m, const Data<T>& d, int pi, std::vector<Cand<T>>& out) {
  const int g1 = m.pair_g1[pi], g2 = m.pair_g2[pi];
  const int t1 = m.geom_type[g1], t2 = m.geom_type[g2];
  const T* x1 = &d.gpos[3 * g1];
  const T* R1 = &d.gmat[9 * g1];
  const T* x2 = &d.gpos[3 * g2];
  const T* R2 = &d.gmat[9 * g2];
  const double* s1 = &m.geom_size[3 * g1];
  const double* s2 = &m.geom_size[3 * g2];
  T z1[3] = {R1[2], R1[5], R1[8]};  // local z axes
  T z2[3] = {R2[2], R2[5], R2[8]};
  if (t1 == GPLANE) {
    if (t2 == GSPHERE) {
      sphere_plane(x1, z1, x2, T(s2[0]), 0, out);
    } else if (t2 == GCAPSULE) {
      for (int e = 0; e < 2; e++) {
        T sg = e == 0 ? -1.0 : 1.0;
        T c[3];
        for (int k = 0; k < 3; k++) c[k] = x2[k] + sg * s2[1] * z2[k];
        sphere_plane(x1, z1, c, T(s2[0]), e, out);
      }
    } else if (t2 == GBOX) {
      T dist[8], cor[8][3];
      for (int k = 0; k < 8; k++) {
        T loc[3] = {T((k & 1) ? s2[0] : -s2[0]), T((k & 2) ? s2[1] : -s2[1]),
                    T((k & 4) ? s2[2] : -s2[2])};
        T w[3];
        matvec(R2, loc, w);
        for (int i = 0; i < 3; i++) cor[k][i] = x2[i] + w[i];
        T rel[3] = {cor[k][0] - x1[0], cor[k][1] - x1[1], cor[k][2] - x1[2]};
        dist[k] = dot3(z1, rel);
      }
      // up to 4 deepest penetrating corners, ties to the lower corner index
      bool used[8] = {false};
      for (int s = 0; s < 4; s++) {
        int best = -1;
        for (int k = 0; k < 8; k++) {
          if (used[k] || !(dist[k] < 0.0)) continue;
          if (best < 0 || dist[k] < dist[best]) best = k;
        }
        if (best < 0) break;
        used[best] = true;
      }
      for (int k = 0; k < 8; k++) {
        if (!used[k]) continue;
        T pos[3];
        for (int i = 0; i < 3; i++) pos[i] = cor[k][i] - 0.5 * dist[k] * z1[i];
        add_cand(out, dist[k], pos, z1, k);
      }
    }
  } else if (t1 == GSPHERE) {
    if (t2 == GSPHERE) {
      sphere_sphere(x1, T(s1[0]), x2, T(s2[0]), 0, out);
    } else if (t2 == GCAPSULE) {
      T a[3], u[3];
      for (int k = 0; k < 3; k++) { a[k] = x2[k] - s2[1] * z2[k]; u[k] = 2.0 * s2[1] * z2[k]; }
      T t = seg_point_param(a, u, x1);
      T q[3] = {a[0] + t * u[0], a[1] + t * u[1], a[2] + t * u[2]};
      sphere_sphere(x1, T(s1[0]), q, T(s2[0]), 0, out);
    } else if (t2 == GHFIELD) {
      sphere_hfield(m, x2, R2, x1, T(s1[0]), out);
    } else if (t2 == GBOX) {
      T nb[3];
      T sd = box_point(x2, R2, s2, x1, nb);
      T dist = sd - s1[0];
      if (dist < 0.0) {
        T pos[3], n[3];
        for (int k = 0; k < 3; k++) { n[k] = -nb[k]; pos[k] = x1[k] - 0.5 * (s1[0] + sd) * nb[k]; }
        add_cand(out, dist, pos, n, 0);
      }
    }
  } else if (t1 == GCAPSULE) {
    T a[3], u[3];
    for (int k = 0; k < 3; k++) { a[k] = x1[k] - s1[1] * z1[k]; u[k] = 2.0 * s1[1] * z1[k]; }
    if (t2 == GCAPSULE) {
      T b[3], w[3];
      for (int k = 0; k < 3; k++) { b[k] = x2[k] - s2[1] * z2[k]; w[k] = 2.0 * s2[1] * z2[k]; }
      T s, t;
      seg_seg(a, u, b, w, s, t);
      T p[3] = {a[0] + s * u[0], a[1] + s * u[1], a[2] + s * u[2]};
      T q[3] = {b[0] + t * w[0], b[1] + t * w[1], b[2] + t * w[2]};
      sphere_sphere(p, T(s1[0]), q, T(s2[0]), 0, out);
    } else if (t2 == GBOX) {
      capsule_box(a, u, T(s1[0]), x2, R2, s2, out);
    }
  }
}

// contact frame: tangent 1 from the world axis least aligned with the normal (lowest
// index on ties), tangent 2 = n x t1
template <class T> void contact_frame(const T* n, T* frame) {
  int ax = 0;
  for (int k = 1; k < 3; k++)
    if (fabs(n[k]) < fabs(n[ax])) ax = k;
  T e[3] = {0.0, 0.0, 0.0};
  e[ax] = 1.0;
  T en = n[ax];
  T t1[3] = {e[0] - en * n[0], e[1] - en * n[1], e[2] - en * n[2]};
  T L = norm3(t1);
  for (int k = 0; k < 3; k++) t1[k] = t1[k] / L;
  T t2[3];
  cross3(n, t1, t2);
  for (int k = 0; k < 3; k++) { frame[k] = n[k]; frame[3 + k] = t1[k]; frame[6 + k] = t2[k]; }
}

// all pairs in list order; on overflow keep the nconmax deepest (ties to the earlier
// contact) and restore list order
template <class T> void collision(const Model& m, Data<T>& d) {
  d.con.clear();
  std::vector<Contact<T>> all;
  for (int pi = 0; pi < m.npair; pi++) {
    std::vector<Cand<T>> cand;
    collide_pair(m, d, pi, cand);
    for (auto& c : cand) {
      Contact<T> k;
      k.dist = c.dist;
      for (int i = 0; i < 3; i++) k.pos[i] = c.pos[i];
      contact_frame(c.n, k.frame);
      k.mu = m.pair_mu[pi];
      k.pair = pi; k.sub = c.sub; k.g1 = m.pair_g1[pi]; k.g2 = m.pair_g2[pi];
      k.condim = m.pair_condim[pi];
      k.mu_t = m.pair_mu_torsion[pi];
      k.mu_r = m.pair_mu_rolling[pi];
      all.push_back(k);
    }
  }
  if ((int)all.size() > m.nconmax) {
    d.status |= ST_OVERFLOW;
    std::vector<int> idx(all.size());
    for (size_t i = 0; i < idx.size(); i++) idx[i] = (int)i;
    std::stable_sort(idx.begin(), idx.end(),
                     [&](int x, int y) { return all[x].dist < all[y].dist; });
    idx.resize(m.nconmax);
    std::sort(idx.begin(), idx.end());
    for (int i : idx) d.con.push_back(all[i]);
  } else {
    d.con = all;
  }
}

// ------------------------------------------------------- A8: constraint rows
// translational Jacobian of the point x rigidly attached to body b: 3 x nv, column k is
// S_k^lin + S_k^ang x x for every dof k on the path from b to the root
template <class T> void point_jac(const Model& m, const Data<T>& d, int b, const T* x, T* J) {
  for (int i = 0; i < 3 * m.nv; i++) J[i] = 0.0;
  for (; b > 0; b = m.body_parent[b]) {
    for (int i = 0; i < m.body_dofnum[b]; i++) {
      const int k = m.body_dofadr[b] + i;
      const T* S = &d.cdof[6 * k];
      T wx[3];
      cross3(S, x, wx);
      for (int r = 0; r < 3; r++) J[r * m.nv + k] = S[3 + r] + wx[r];
    }
  }
}

// angular Jacobian (3 x nv, world frame) of body b: the rotation axes of the dofs on
// its path to the root
template <class T> void body_angjac(const Model& m, const Data<T>& d, int b, T* J) {
  for (int i = 0; i < 3 * m.nv; i++) J[i] = 0.0;
  for (; b > 0; b = m.body_parent[b]) {
    for (int i = 0; i < m.body_dofnum[b]; i++) {
      const int k = m.body_dofadr[b] + i;
      for (int r = 0; r < 3; r++) J[r * m.nv + k] = d.cdof[6 * k + r];
    }
  }
}

// impedance d(r) from solimp = (dmin, dmax, width, mid, power)
template <class T> T impedance(const Model& m, T r) {
  const double dmin = m.solimp[0], dmax = m.solimp[1], width = m.solimp[2];
  const double mid = m.solimp[3], power = m.solimp[4];
  T x = tmin(fabs(r) / width, T(1.0));
  T y;
  if (x <= mid) y = pow(x, power) / std::pow(mid, power - 1.0);
  else y = 1.0 - pow(1.0 - x, power) / std::pow(1.0 - mid, power - 1.0);
  return dmin + y * (dmax - dmin);
}

// Pyramidal cone with 4 edges per contact, rows ordered (+t1, -t1, +t2, -t2):
//   J_e = J_n +- mu J_t;  aref = -b (J_e qvel) - k d(r) r;  R = (1-d)/d * A, D = 1/R,
//   k = 1/(dmax^2 tc^2 zeta^2), b = 2/(dmax tc) with (tc, zeta) = solref, tc >= 2 dt,
//   A = (1 + mu^2)(w(b1) + w(b2)) with w the bodies' translational inverse weights.
//
// Joint limits follow the contacts, one row per limited hinge or slide joint whose
// coordinate lies outside its range, in joint order: distance r = q - lo (row J = e_k)
// or r = hi - q (J = -e_k), the same aref, impedance and R with A = (M^-1)_kk at qpos0.
// Then one friction-loss row per dof k with a bound F_k > 0, always present: J = e_k,
// r = 0 (so d = d(0) and aref = -b qvel_k), the same A; its force is limited to
// [-F_k, F_k] (dry joint friction, Todorov 2014's box-constrained rows).
// Then three two-sided rows per connect equality, always present: with p1, p2 the
// anchor's world positions through body1 and body2, row k has J = e_k^T (J_p(b1, p1) -
// J_p(b2, p2)), r = (p1 - p2)_k, and A = w(b1) + w(b2); its force is unbounded.  A weld
// adds three rotational rows after its three translational ones (see below).
template <class T> void constraint_rows(const Model& m, Data<T>& d) {
  const int nc = (int)d.con.size(), n = m.nv;
  std::vector<int> lim_dof;
  std::vector<double> lim_sign;
  std::vector<T> lim_dist;
  for (int j = 0; j < m.njnt; j++) {
    if (!m.jnt_limited[j]) continue;
    const T q = d.qpos[m.jnt_qposadr[j]];
    const T rlo = q - m.jnt_range[2 * j], rhi = m.jnt_range[2 * j + 1] - q;
    if (rlo < 0.0) { lim_dof.push_back(m.jnt_dofadr[j]); lim_sign.push_back(1.0); lim_dist.push_back(rlo); }
    else if (rhi < 0.0) { lim_dof.push_back(m.jnt_dofadr[j]); lim_sign.push_back(-1.0); lim_dist.push_back(rhi); }
  }
  const int nl = (int)lim_dof.size();
  // contact rows: a pyramid's edges, an elliptic cone's frame rows (condim of them), or
  // one normal row without friction
  int nrc = 0;
  for (int c = 0; c < nc; c++) {
    d.con[c].row = nrc;
    const int cd = d.con[c].condim;
    nrc += (cd == 1 || m.cone == 1) ? cd : 2 * (cd - 1);
  }
  d.nrow = nrc + nl + m.nfric + m.neqrow;
  d.J.assign(d.nrow * n, 0.0);
  d.aref.assign(d.nrow, 0.0);
  d.D.assign(d.nrow, 0.0);
  d.fl.assign(d.nrow, 0.0);
  d.cone_row0.clear();
  d.cone_nd.clear();
  d.cone_mu.clear();
  d.row_ratio.assign(d.nrow, T(1.0));
  d.in_cone.assign(d.nrow, 0);
  const double tc = std::max(m.solref[0], 2.0 * m.dt), zeta = m.solref[1];
  const double dmax = m.solimp[1];
  const double K = 1.0 / (dmax * dmax * tc * tc * zeta * zeta);
  const double B = 2.0 / (dmax * tc);
  std::vector<T> J1(3 * n), J2(3 * n), Jc(3 * n);
  for (int c = 0; c < nc; c++) {
    const Contact<T>& k = d.con[c];
    const int b1 = m.geom_body[k.g1], b2 = m.geom_body[k.g2];
    point_jac(m, d, b2, k.pos, J2.data());
    point_jac(m, d, b1, k.pos, J1.data());
    for (int r = 0; r < 3; r++)
      for (int i = 0; i < n; i++) {
        T s = 0.0;
        for (int a = 0; a < 3; a++) s += k.frame[3 * r + a] * (J2[a * n + i] - J1[a * n + i]);
        Jc[r * n + i] = s;
      }
    const T imp = impedance(m, k.dist);
    if (k.condim == 1) {
      // frictionless: one row along the normal, J = J_n, A = w1 + w2
      const double A1 = std::max(m.body_invweight[b1] + m.body_invweight[b2], 1e-15);
      const int row = k.row;
      T jv = 0.0;
      for (int i = 0; i < n; i++) {
        d.J[row * n + i] = Jc[i];
        jv += Jc[i] * d.qvel[i];
      }
      d.aref[row] = -B * jv - K * imp * k.dist;
      d.D[row] = 1.0 / ((1.0 - imp) / imp * A1);
      continue;
    }
    // friction directions: the two tangents (mu); with condim >= 4 the spin about the
    // normal, n . (w2 - w1) (mu_t); with condim 6 the rolling about the tangents,
    // t_k . (w2 - w1) (mu_r).
    std::vector<T> Ja(3 * n, T(0.0));
    if (k.condim >= 4) {
      body_angjac(m, d, b2, J2.data());
      body_angjac(m, d, b1, J1.data());
      for (int r = 0; r < 3; r++)
        for (int i = 0; i < n; i++) {
          T s = 0.0;
          for (int a = 0; a < 3; a++) s += k.frame[3 * r + a] * (J2[a * n + i] - J1[a * n + i]);
          Ja[r * n + i] = s;
        }
    }
    const int ndir = k.condim - 1;
    if (m.cone == 1) {
      // Elliptic cone: the contact frame's rows (normal, then one per friction direction)
      // with the normal's impedance.  The normal row has aref = -b (J_n qvel) - k d(r) r
      // and R_n = (1-d)/d (w1 + w2); a friction row, with no distance, aref = -b (J qvel)
      // and R = R_n (mu / mu_j)^2, mu the sliding coefficient: in the coordinates
      // e_j mu_j / mu the rows share D_n and the cone is round (see cone_eval).
      const double A1 = std::max(m.body_invweight[b1] + m.body_invweight[b2], 1e-15);
      const T Dn = 1.0 / ((1.0 - imp) / imp * A1);
      d.cone_row0.push_back(k.row);
      d.cone_nd.push_back(k.condim);
      d.cone_mu.push_back(k.mu);
      for (int e = 0; e < k.condim; e++) {
        const int row = k.row + e;
        const T* Jr = e == 0 ? &Jc[0] : (e < 3 ? &Jc[e * n] : (e == 3 ? &Ja[0] : &Ja[(e - 3) * n]));
        const T mu_e = e < 3 ? k.mu : (e == 3 ? k.mu_t : k.mu_r);
        const T ratio = e == 0 ? T(1.0) : mu_e / k.mu;
        T jv = 0.0;
        for (int i = 0; i < n; i++) {
          d.J[row * n + i] = Jr[i];
          jv += Jr[i] * d.qvel[i];
        }
        d.aref[row] = e == 0 ? -B * jv - K * imp * k.dist : -B * jv;
        d.D[row] = Dn * ratio * ratio;
        d.row_ratio[row] = ratio;
        d.in_cone[row] = 1;
      }
      continue;
    }
    // Pyramid: each friction direction gives the edges J_n + mu J_dir and J_n - mu J_dir.
    const double A = std::max((1.0 + val(k.mu) * val(k.mu)) *
                                  (m.body_invweight[b1] + m.body_invweight[b2]), 1e-15);
    const T R = (1.0 - imp) / imp * A;
    for (int e = 0; e < 2 * ndir; e++) {
      const int row = k.row + e, dir = e / 2;
      const T* Jd = dir < 2 ? &Jc[(1 + dir) * n] : (dir == 2 ? &Ja[0] : &Ja[(dir - 2) * n]);
      const T mu = dir < 2 ? k.mu : (dir == 2 ? k.mu_t : k.mu_r);
      const T sg = (e % 2 == 0) ? mu : -mu;
      T jv = 0.0;
      for (int i = 0; i < n; i++) {
        d.J[row * n + i] = Jc[i] + sg * Jd[i];
        jv += d.J[row * n + i] * d.qvel[i];
      }
      d.aref[row] = -B * jv - K * imp * k.dist;
      d.D[row] = 1.0 / R;
    }
  }
  for (int l = 0; l < nl; l++) {
    const int row = nrc + l, k = lim_dof[l];
    d.J[row * n + k] = lim_sign[l];
    const T imp = impedance(m, lim_dist[l]);
    const double A = std::max(m.dof_invweight[k], 1e-15);
    const T R = (1.0 - imp) / imp * A;
    d.aref[row] = -B * (lim_sign[l] * d.qvel[k]) - K * imp * lim_dist[l];
    d.D[row] = 1.0 / R;
  }
  int row = nrc + nl;
  for (int k = 0; k < n; k++) {
    if (!(m.dof_frictionloss[k] > 0.0)) continue;
    d.J[row * n + k] = 1.0;
    const T imp = impedance(m, T(0.0));
    const double A = std::max(m.dof_invweight[k], 1e-15);
    d.aref[row] = -B * d.qvel[k];
    d.D[row] = 1.0 / ((1.0 - imp) / imp * A);
    d.fl[row] = m.dof_frictionloss[k];
    row++;
  }
  for (int q = 0; q < m.neq; q++) {
    const int b1 = m.eq_b1[q], b2 = m.eq_b2[q];
    T p1[3], p2[3];
    matvec(&d.xmat[9 * b1], &m.eq_a1[3 * q], p1);
    matvec(&d.xmat[9 * b2], &m.eq_a2[3 * q], p2);
    for (int k = 0; k < 3; k++) { p1[k] += d.xpos[3 * b1 + k]; p2[k] += d.xpos[3 * b2 + k]; }
    point_jac(m, d, b1, p1, J1.data());
    point_jac(m, d, b2, p2, J2.data());
    const double A = std::max(m.body_invweight[b1] + m.body_invweight[b2], 1e-15);
    for (int k = 0; k < 3; k++, row++) {
      T jv = 0.0;
      for (int i = 0; i < n; i++) {
        d.J[row * n + i] = J1[k * n + i] - J2[k * n + i];
        jv += d.J[row * n + i] * d.qvel[i];
      }
      const T r = p1[k] - p2[k];
      const T imp = impedance(m, r);
      d.aref[row] = -B * jv - K * imp * r;
      d.D[row] = 1.0 / ((1.0 - imp) / imp * A);
      d.fl[row] = INFINITY;  // two-sided: the quadratic piece everywhere
    }
    if (m.eq_type[q] != 1) continue;
    // weld: body2's orientation relative to body1 held at the reference Q.  The error
    // rotation E = R1 Q R2^T is I when held; its residual r = vee(E - E^T) / 2 = sin(theta)
    // axis (world frame), whose rate at E = I is w1 - w2: J = J_w(b1) - J_w(b2).
    T E[9], RQ[9];
    const T* R1 = &d.xmat[9 * b1];
    const T* R2 = &d.xmat[9 * b2];
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) {
        T v = 0.0;
        for (int k = 0; k < 3; k++) v += R1[3 * i + k] * m.eq_relR[9 * q + 3 * k + j];
        RQ[3 * i + j] = v;
      }
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) {
        T v = 0.0;
        for (int k = 0; k < 3; k++) v += RQ[3 * i + k] * R2[3 * j + k];
        E[3 * i + j] = v;
      }
    const T rr[3] = {0.5 * (E[7] - E[5]), 0.5 * (E[2] - E[6]), 0.5 * (E[3] - E[1])};
    body_angjac(m, d, b1, J1.data());
    body_angjac(m, d, b2, J2.data());
    for (int k = 0; k < 3; k++, row++) {
      T jv = 0.0;
      for (int i = 0; i < n; i++) {
        d.J[row * n + i] = J1[k * n + i] - J2[k * n + i];
        jv += d.J[row * n + i] * d.qvel[i];
      }
      const T imp = impedance(m, rr[k]);
      d.aref[row] = -B * jv - K * imp * rr[k];
      d.D[row] = 1.0 / ((1.0 - imp) / imp * A);
      d.fl[row] = INFINITY;
    }
  }
}

// ---------------------------------------------------------- A9: Newton contact solve
// Minimise F(a) = 1/2 (a - a0)^T M (a - a0) + sum_i s_i(J_i a - aref_i), with
//   s_i(e) = 1/2 D_i min(0, e)^2                       for a one-sided row,
//   s_i(e) = 1/2 D_i e^2 if |D_i e| <= F_i, else F_i |e| - F_i^2 / (2 D_i)
//                                                      for a friction-loss row (bound F_i),
//   s_i(e) = 1/2 D_i e^2                               for an equality row (F_i = inf),
// the largest of -f e - f^2 / (2 D) over the row's admissible forces f (f >= 0, or
// |f| <= F).  F is strictly convex and piecewise quadratic (M is SPD).
template <class T> struct Solver {
  const Model& m;
  Data<T>& d;
  const int n, nr;
  Solver(const Model& m_, Data<T>& d_) : m(m_), d(d_), n(m_.nv), nr(d_.nrow) {}

  T jrow(int i, const T* a) const {
    T s = 0.0;
    for (int k = 0; k < n; k++) s += d.J[i * n + k] * a[k];
    return s;
  }
  // s_i(e), its derivative, and whether e lies on the row's quadratic piece
  T srow(int i, T e) const {
    const double F = d.fl[i];
    if (F == 0.0) return e < 0.0 ? T(0.5 * d.D[i] * e * e) : T(0.0);
    if (std::isinf(F) || fabs(d.D[i] * e) <= F) return 0.5 * d.D[i] * e * e;
    return F * fabs(e) - F * F / (2.0 * d.D[i]);
  }
  T dsrow(int i, T e) const {
    const double F = d.fl[i];
    if (F == 0.0) return e < 0.0 ? T(d.D[i] * e) : T(0.0);
    const T v = d.D[i] * e;
    return v > F ? T(F) : (v < -F ? T(-F) : v);
  }
  bool quad(int i, T e) const {
    const double F = d.fl[i];
    return F == 0.0 ? e < 0.0 : (std::isinf(F) || fabs(d.D[i] * e) < F);
  }
  // Elliptic cone block b at e (its rows' J a - aref): cost s, row forces f (so that
  // ds/de = -f) and, when Hb is given, the Hessian d2s/de2 (nd x nd, row-major).
  // The block's rows share D = D_n in the coordinates x = (e_n, e_j mu_j / mu), where the
  // friction cone is round: K = {g : |g_t| <= mu g_n}.  The soft-constraint cost is
  //   s(e) = max over g in K of  -g.x - |g|^2 / (2 D)  =  |P_K(-D x)|^2 / (2 D),
  // whose maximiser g = P_K(-D x) is the Euclidean projection onto K, in three zones
  // with T = |x_t|:
  //   separated  e_n >= mu T:   g = 0;
  //   sticking   mu e_n + T <= 0: g = -D x (every row on its quadratic);
  //   sliding    otherwise:      g on the cone's surface, g_n = c psi with
  //              psi = mu T - e_n > 0, c = D / (1 + mu^2), g_t = -mu g_n x_t / T, and
  //              s = c psi^2 / 2 (its Hessian: c (a a^T + psi mu/T (I - t t^T) on the
  //              friction coordinates), a = (-1, mu t), t = x_t / T).
  // Physical forces f_j = g_j mu_j / mu; the Hessian maps back by the same scaling.
  void cone_eval(int b, const T* e, T& cost_out, T* f, T* Hb) const {
    const int r0 = d.cone_row0[b], nd = d.cone_nd[b];
    const T mu = d.cone_mu[b], D = d.D[r0];
    T x[6];
    T T2 = 0.0;
    x[0] = e[0];
    for (int j = 1; j < nd; j++) {
      x[j] = e[j] * d.row_ratio[r0 + j];
      T2 += x[j] * x[j];
    }
    const T Tn = sqrt(T2);
    T g[6];
    T Hs[36];
    for (int j = 0; j < nd * nd; j++) Hs[j] = 0.0;
    if (!(x[0] < mu * Tn)) {  // separated
      cost_out = 0.0;
      for (int j = 0; j < nd; j++) g[j] = 0.0;
    } else if (mu * x[0] + Tn <= 0.0) {  // sticking
      cost_out = 0.5 * D * (x[0] * x[0] + T2);
      for (int j = 0; j < nd; j++) {
        g[j] = -D * x[j];
        Hs[j * nd + j] = D;
      }
    } else {  // sliding on the cone's surface
      const T psi = mu * Tn - x[0], c = D / (1.0 + mu * mu);
      cost_out = 0.5 * c * psi * psi;
      g[0] = c * psi;
      T a[6];
      a[0] = -1.0;
      for (int j = 1; j < nd; j++) {
        g[j] = -mu * g[0] * x[j] / Tn;
        a[j] = mu * x[j] / Tn;
      }
      const T w2 = c * psi * mu / Tn;
      for (int i = 0; i < nd; i++)
        for (int j = 0; j < nd; j++) {
          T v = c * a[i] * a[j];
          if (i > 0 && j > 0) v += w2 * ((i == j ? 1.0 : 0.0) - x[i] * x[j] / T2);
          Hs[i * nd + j] = v;
        }
    }
    for (int j = 0; j < nd; j++) f[j] = g[j] * d.row_ratio[r0 + j];
    if (Hb)
      for (int i = 0; i < nd; i++)
        for (int j = 0; j < nd; j++)
          Hb[i * nd + j] = Hs[i * nd + j] * d.row_ratio[r0 + i] * d.row_ratio[r0 + j];
  }
  T cone_cost(int b, const T* a) const {
    const int r0 = d.cone_row0[b], nd = d.cone_nd[b];
    T e[6], f[6], c;
    for (int j = 0; j < nd; j++) e[j] = jrow(r0 + j, a) - d.aref[r0 + j];
    cone_eval(b, e, c, f, nullptr);
    return c;
  }
  T cost(const T* a) const {
    std::vector<T> da(n), Mda(n);
    for (int k = 0; k < n; k++) da[k] = a[k] - d.qacc_smooth[k];
    T c = 0.0;
    for (int i = 0; i < n; i++) {
      T s = 0.0;
      for (int k = 0; k < n; k++) s += d.M[i * n + k] * da[k];
      c += 0.5 * da[i] * s;
    }
    for (int i = 0; i < nr; i++)
      if (!d.in_cone[i]) c += srow(i, jrow(i, a) - d.aref[i]);
    for (size_t b = 0; b < d.cone_row0.size(); b++) c += cone_cost((int)b, a);
    return c;
  }
  // gradient and Hessian with the active set at a
  void grad_hess(const T* a, T* g, T* H) const {
    for (int i = 0; i < n; i++) {
      T s = 0.0;
      for (int k = 0; k < n; k++) s += d.M[i * n + k] * (a[k] - d.qacc_smooth[k]);
      g[i] = s;
      for (int k = 0; k < n; k++) H[i * n + k] = d.M[i * n + k];
    }
    for (int r = 0; r < nr; r++) {
      if (d.in_cone[r]) continue;
      T e = jrow(r, a) - d.aref[r];
      const T* Jr = &d.J[r * n];
      const T ds = dsrow(r, e);
      for (int i = 0; i < n; i++) g[i] += ds * Jr[i];
      if (!quad(r, e)) continue;
      for (int i = 0; i < n; i++)
        for (int k = 0; k < n; k++) H[i * n + k] += d.D[r] * Jr[i] * Jr[k];
    }
    // elliptic cone blocks: g += J_c^T (-f), H += J_c^T Hb J_c
    for (size_t b = 0; b < d.cone_row0.size(); b++) {
      const int r0 = d.cone_row0[b], nd = d.cone_nd[b];
      T e[6], f[6], Hb[36], c;
      for (int j = 0; j < nd; j++) e[j] = jrow(r0 + j, a) - d.aref[r0 + j];
      cone_eval((int)b, e, c, f, Hb);
      for (int j = 0; j < nd; j++)
        for (int i = 0; i < n; i++) g[i] -= f[j] * d.J[(r0 + j) * n + i];
      for (int p = 0; p < nd; p++)
        for (int q = 0; q < nd; q++) {
          if (Hb[p * nd + q] == 0.0) continue;
          for (int i = 0; i < n; i++)
            for (int k = 0; k < n; k++)
              H[i * n + k] += Hb[p * nd + q] * d.J[(r0 + p) * n + i] * d.J[(r0 + q) * n + k];
        }
    }
  }
  // exact minimiser of phi(alpha) = F(a + alpha delta) over alpha >= 0 when the model
  // has elliptic cone blocks: phi is convex and C^1 but no longer piecewise quadratic.
  // phi' (nondecreasing, negative at 0) is bracketed by doubling from alpha = 1, then
  // its root is found by Newton steps on phi' (phi'' from the pieces' curvatures), each
  // replaced by the bracket's midpoint when it leaves the bracket, until the bracket or
  // phi' vanishes to the working precision.
  T line_search_cone(const T* a, const T* delta) const {
    std::vector<T> e(nr), s(nr);
    for (int i = 0; i < nr; i++) { e[i] = jrow(i, a) - d.aref[i]; s[i] = jrow(i, delta); }
    T dMd = 0.0, dMa = 0.0;
    for (int i = 0; i < n; i++) {
      T t = 0.0;
      for (int k = 0; k < n; k++) t += d.M[i * n + k] * delta[k];
      dMd += delta[i] * t;
      dMa += t * (a[i] - d.qacc_smooth[i]);
    }
    auto dphi = [&](T al, T& d2) {
      T v = dMa + al * dMd;
      d2 = dMd;
      for (int i = 0; i < nr; i++) {
        if (d.in_cone[i]) continue;
        const T ep = e[i] + al * s[i];
        v += s[i] * dsrow(i, ep);
        if (quad(i, ep)) d2 += d.D[i] * s[i] * s[i];
      }
      for (size_t b = 0; b < d.cone_row0.size(); b++) {
        const int r0 = d.cone_row0[b], nd = d.cone_nd[b];
        T eb[6], f[6], Hb[36], c;
        for (int j = 0; j < nd; j++) eb[j] = e[r0 + j] + al * s[r0 + j];
        cone_eval((int)b, eb, c, f, Hb);
        for (int p = 0; p < nd; p++) {
          v -= s[r0 + p] * f[p];
          for (int q = 0; q < nd; q++) d2 += s[r0 + p] * Hb[p * nd + q] * s[r0 + q];
        }
      }
      return v;
    };
    T d2;
    T lo = 0.0, hi = 1.0;
    for (int k = 0; k < 200 && dphi(hi, d2) < 0.0; k++) { lo = hi; hi = 2.0 * hi; }
    T al = lo < 1.0 ? T(1.0) : hi;  // the Newton step length, or the bracket's end
    for (int it = 0; it < 200; it++) {
      const T v = dphi(al, d2);
      if (v == 0.0) return al;
      if (v < 0.0) lo = al; else hi = al;
      T next = al - v / d2;
      if (!(next > lo && next < hi)) next = 0.5 * (lo + hi);
      // converged: the Newton correction (or the bracket) is below the working precision
      if (!(fabs(next - al) > 1e-15 * al) || !(hi - lo > 1e-15 * hi)) return next;
      al = next;
    }
    return al;
  }
  // exact minimiser of phi(alpha) = F(a + alpha delta) over alpha >= 0: phi' is piecewise
  // linear and nondecreasing; walk its breakpoints in increasing order
  T line_search(const T* a, const T* delta) const {
    std::vector<T> e(nr), s(nr), Md(n), da(n);
    for (int i = 0; i < nr; i++) { e[i] = jrow(i, a) - d.aref[i]; s[i] = jrow(i, delta); }
    T dMd = 0.0, dMa = 0.0;
    for (int i = 0; i < n; i++) {
      T t = 0.0;
      for (int k = 0; k < n; k++) t += d.M[i * n + k] * delta[k];
      dMd += delta[i] * t;
      dMa += t * (a[i] - d.qacc_smooth[i]);
    }
    // phi'(alpha) = dMa + alpha dMd + sum_i s_i s_i'(e_i + alpha s_i), linear in alpha
    // between breakpoints: A + alpha Bc with the pieces that hold at `probe`
    auto dphi_lin = [&](T probe, T& A, T& Bc) {
      A = dMa; Bc = dMd;
      for (int i = 0; i < nr; i++) {
        const T ep = e[i] + probe * s[i];
        if (quad(i, ep)) { A += d.D[i] * s[i] * e[i]; Bc += d.D[i] * s[i] * s[i]; }
        else A += s[i] * dsrow(i, ep);  // 0, or the friction bound +-F
      }
    };
    // breakpoints: where a row's e crosses 0 (one-sided) or +-F/D (friction loss)
    std::vector<T> bps;
    for (int i = 0; i < nr; i++)
      if (s[i] != 0.0) {
        const double F = d.fl[i];
        if (std::isinf(F)) continue;  // two-sided rows have no breakpoint
        const int nb = F == 0.0 ? 1 : 2;
        for (int k = 0; k < nb; k++) {
          const T at = F == 0.0 ? T(0.0) : T((k == 0 ? F : -F) / d.D[i]);
          T al = (at - e[i]) / s[i];
          if (al > 0.0) bps.push_back(al);
        }
      }
    std::sort(bps.begin(), bps.end(), [](const T& x, const T& y) { return x < y; });
    T lo = 0.0;
    for (size_t k = 0; k <= bps.size(); k++) {
      // the active set is constant inside (lo, hi); probe it at the interval's middle
      T probe = k < bps.size() ? 0.5 * (lo + bps[k]) : lo + 1.0;
      T A, Bc;
      dphi_lin(probe, A, Bc);
      T root = -A / Bc;
      if (k == bps.size() || root <= bps[k]) return tmax(root, lo);
      lo = bps[k];
    }
    return lo;
  }
  // dense Cholesky H = L L^T in place (lower)
  static bool cholesky(T* H, int n) {
    for (int j = 0; j < n; j++) {
      T s = H[j * n + j];
      for (int k = 0; k < j; k++) s -= H[j * n + k] * H[j * n + k];
      if (!(s > 0.0)) return false;
      T L = sqrt(s);
      H[j * n + j] = L;
      for (int i = j + 1; i < n; i++) {
        T t = H[i * n + j];
        for (int k = 0; k < j; k++) t -= H[i * n + k] * H[j * n + k];
        H[i * n + j] = t / L;
      }
    }
    return true;
  }
  static void chol_solve(const T* L, int n, T* x) {
    for (int i = 0; i < n; i++) {
      T s = x[i];
      for (int k = 0; k < i; k++) s -= L[i * n + k] * x[k];
      x[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; i--) {
      T s = x[i];
      for (int k = i + 1; k < n; k++) s -= L[k * n + i] * x[k];
      x[i] = s / L[i * n + i];
    }
  }
  // mode 0: exactly `iterations` Newton steps; mode 1: iterate to convergence
  void solve(int mode) {
    std::vector<T> a(n), g(n), H(n * n), delta(n);
    // start from the cheaper of the warm start and the unconstrained acceleration
    T cw = cost(d.qacc_ws.data()), c0 = cost(d.qacc_smooth.data());
    a = (cw <= c0) ? d.qacc_ws : d.qacc_smooth;
    const int maxit = mode == 0 ? m.iterations : 200;
    double scale = 1.0;
    for (int i = 0; i < n; i++) scale = std::max(scale, std::fabs(val(d.qfrc_smooth[i])));
    d.newton_iters = 0;
    for (int it = 0; it < maxit && nr > 0; it++) {
      grad_hess(a.data(), g.data(), H.data());
      if (mode == 1) {
        double gmax = 0.0;
        for (int i = 0; i < n; i++) gmax = std::max(gmax, std::fabs(val(g[i])));
        if (gmax <= 1e-13 * scale) break;
      }
      if (!cholesky(H.data(), n)) { d.status |= ST_NODESCENT; break; }
      for (int i = 0; i < n; i++) delta[i] = -g[i];
      chol_solve(H.data(), n, delta.data());
      T slope = 0.0;
      for (int i = 0; i < n; i++) slope += g[i] * delta[i];
      if (!(slope < 0.0)) break;  // zero gradient: already optimal
      T al = d.cone_row0.empty() ? line_search(a.data(), delta.data())
                                 : line_search_cone(a.data(), delta.data());
      for (int i = 0; i < n; i++) a[i] += al * delta[i];
      d.newton_iters++;
    }
    d.qacc = a;
    // Hessian factor at the solution (used for implicit differentiation)
    grad_hess(a.data(), g.data(), H.data());
    if (cholesky(H.data(), n)) d.H = H;
  }
};

// ----------------------------------------------------------------- the full step
template <class T> void forward(const Model& m, Data<T>& d, int mode) {
  d.status = 0;
  kinematics(m, d);
  velocities(m, d);
  crba(m, d);
  rne(m, d, (const T*)nullptr, d.qfrc_bias.data());
  actuation(m, d);
  for (int i = 0; i < m.nv; i++) d.qfrc_smooth[i] = d.qfrc_act[i] + d.qfrc_pass[i] - d.qfrc_bias[i];
  factor_ltdl(m, d.M, d.qLD);
  solve_ltdl(m, d.qLD, d.qfrc_smooth.data(), d.qacc_smooth.data());
  collision(m, d);
  constraint_rows(m, d);
  if (d.nrow == 0) {
    d.qacc = d.qacc_smooth;
  } else {
    Solver<T> s(m, d);
    s.solve(mode);
  }
  // A10: row forces and generalised constraint force
  d.efc_force.assign(d.nrow, 0.0);
  std::fill(d.qfrc_con.begin(), d.qfrc_con.end(), T(0.0));
  for (int r = 0; r < d.nrow; r++) {
    if (d.in_cone[r]) continue;
    T jar = 0.0;
    for (int i = 0; i < m.nv; i++) jar += d.J[r * m.nv + i] * d.qacc[i];
    T f = d.D[r] * (d.aref[r] - jar);
    const double F = d.fl[r];
    if (F == 0.0) d.efc_force[r] = f > 0.0 ? f : T(0.0);
    else d.efc_force[r] = f > F ? T(F) : (f < -F ? T(-F) : f);
  }
  if (!d.cone_row0.empty()) {  // elliptic cone blocks: the projected force of cone_eval
    Solver<T> s(m, d);
    for (size_t b = 0; b < d.cone_row0.size(); b++) {
      const int r0 = d.cone_row0[b], nd = d.cone_nd[b];
      T e[6], c;
      for (int j = 0; j < nd; j++) e[j] = s.jrow(r0 + j, d.qacc.data()) - d.aref[r0 + j];
      s.cone_eval((int)b, e, c, &d.efc_force[r0], nullptr);
    }
  }
  for (int r = 0; r < d.nrow; r++)
    for (int i = 0; i < m.nv; i++) d.qfrc_con[i] += d.J[r * m.nv + i] * d.efc_force[r];
  // Implicit damping: the forces linear in a dof's own velocity (joint damping b_k and
  // the velocity gain kd of a position actuator on it) act at the end-of-step velocity
  // qvel + h a, so the integrator's acceleration solves
  //   (M + h diag(b + kd)) a_int = qfrc_smooth + qfrc_con,
  // with the constraint forces of the solve above (which used M).  Integrator 2 also
  // takes a position actuator's stiffness kp at the end-of-step position q + h qvel'
  // (qvel' = qvel + h a): its force gains -kp h (qvel + h a), so
  //   (M + h diag(b + kd) + h^2 diag(kp)) a_int = qfrc_smooth - h diag(kp) qvel + qfrc_con,
  // which for a linear spring-damper is backward Euler.
  if (m.integrator == 1 || m.integrator == 2) {
    std::vector<T> Mt(d.M), LD(m.nv * m.nv), rhs(m.nv);
    for (int k = 0; k < m.nv; k++) Mt[k * m.nv + k] += m.dt * m.dof_damping[k];
    for (int k = 0; k < m.nv; k++) rhs[k] = d.qfrc_smooth[k] + d.qfrc_con[k];
    for (int a = 0; a < m.nu; a++)
      if (m.act_type[a] == APD) {
        const int k = m.jnt_dofadr[m.act_jnt[a]];
        Mt[k * m.nv + k] += m.dt * m.act_kd[a];
        if (m.integrator == 2) {
          Mt[k * m.nv + k] += m.dt * m.dt * m.act_kp[a];
          rhs[k] -= m.dt * m.act_kp[a] * d.qvel[k];
        }
      }
    factor_ltdl(m, Mt, LD);
    solve_ltdl(m, LD, rhs.data(), d.qacc_int.data());
  } else {
    d.qacc_int = d.qacc;
  }
}

// Position update q <- q (+) h vel: hinge and slide coordinates add h vel; a free
// joint's position adds h v and its orientation turns by the exponential map of the
// body-frame rotation h w.
template <class T> void integrate_pos(const Model& m, std::vector<T>& qpos, const std::vector<T>& vel,
                                      double h) {
  for (int j = 0; j < m.njnt; j++) {
    const int qa = m.jnt_qposadr[j], da = m.jnt_dofadr[j];
    if (m.jnt_type[j] == JFREE) {
      for (int k = 0; k < 3; k++) qpos[qa + k] = qpos[qa + k] + h * vel[da + k];
      T w[3] = {vel[da + 3] * h, vel[da + 4] * h, vel[da + 5] * h};
      T ang = norm3(w);
      T dq[4];
      if (ang > 1e-15) {
        T s = sin(0.5 * ang) / ang;
        dq[0] = cos(0.5 * ang); dq[1] = w[0] * s; dq[2] = w[1] * s; dq[3] = w[2] * s;
      } else {
        dq[0] = 1.0; dq[1] = 0.5 * w[0]; dq[2] = 0.5 * w[1]; dq[3] = 0.5 * w[2];
      }
      T q[4] = {qpos[qa + 3], qpos[qa + 4], qpos[qa + 5], qpos[qa + 6]}, r[4];
      quatmul(q, dq, r);
      T L = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
      for (int k = 0; k < 4; k++) qpos[qa + 3 + k] = r[k] / L;
    } else {
      qpos[qa] = qpos[qa] + h * vel[da];
    }
  }
}

// A11: semi-implicit Euler (velocity first, then positions with the new velocity)
template <class T> void integrate(const Model& m, Data<T>& d) {
  const double h = m.dt;
  for (int i = 0; i < m.nv; i++) d.qvel[i] = d.qvel[i] + h * d.qacc_int[i];
  integrate_pos(m, d.qpos, d.qvel, h);
  d.qacc_ws = d.qacc;
  bool fin = true;
  for (auto& x : d.qpos) fin = fin && isfinite(x);
  for (auto& x : d.qvel) fin = fin && isfinite(x);
  if (!fin) d.status |= ST_NONFINITE;
}

// Integrator 3: classic fourth-order Runge-Kutta on (q, qdot) with the whole forward
// pass (collision, constraint rows and their solve) at every stage, as in MuJoCo's RK4.
// Stage k's state is X_k = (q0 (+) c_k h v_{k-1}, v0 + c_k h a_{k-1}) with c = (0, 1/2,
// 1/2, 1), v_k its velocity and a_k its acceleration; each stage's solve starts from
// the previous stage's solution.  Then q <- q0 (+) h/6 (v1 + 2 v2 + 2 v3 + v4) and
// qdot <- v0 + h/6 (a1 + 2 a2 + 2 a3 + a4).  The reported acceleration, the next warm
// start and the other outputs (contacts, rows) are the first stage's.
template <class T> void step_rk4(const Model& m, Data<T>& d, int mode) {
  const double h = m.dt;
  const std::vector<T> q0 = d.qpos, v0 = d.qvel;
  forward(m, d, mode);
  Data<T> d1 = d;  // the first stage's outputs
  static const double c[4] = {0.0, 0.5, 0.5, 1.0}, b[4] = {1.0, 2.0, 2.0, 1.0};
  std::vector<T> vsum(m.nv), asum(m.nv);
  for (int i = 0; i < m.nv; i++) { vsum[i] = b[0] * v0[i]; asum[i] = b[0] * d.qacc[i]; }
  int status = d.status;
  for (int k = 1; k < 4; k++) {
    std::vector<T> vprev = d.qvel, aprev = d.qacc;
    d.qpos = q0;
    integrate_pos(m, d.qpos, vprev, c[k] * h);
    for (int i = 0; i < m.nv; i++) d.qvel[i] = v0[i] + c[k] * h * aprev[i];
    d.qacc_ws = aprev;
    forward(m, d, mode);
    status |= d.status;
    for (int i = 0; i < m.nv; i++) {
      vsum[i] = vsum[i] + b[k] * d.qvel[i];
      asum[i] = asum[i] + b[k] * d.qacc[i];
    }
  }
  std::vector<T> vel(m.nv);
  for (int i = 0; i < m.nv; i++) vel[i] = vsum[i] / 6.0;
  d = d1;
  d.qpos = q0;
  integrate_pos(m, d.qpos, vel, h);
  for (int i = 0; i < m.nv; i++) d.qvel[i] = v0[i] + h * asum[i] / 6.0;
  d.qacc_ws = d1.qacc;
  d.status = status;
  bool fin = true;
  for (auto& x : d.qpos) fin = fin && isfinite(x);
  for (auto& x : d.qvel) fin = fin && isfinite(x);
  if (!fin) d.status |= ST_NONFINITE;
}

template <class T> void step(const Model& m, Data<T>& d, int mode) {
  if (m.integrator == 3) {
    step_rk4(m, d, mode);
    return;
  }
  forward(m, d, mode);
  integrate(m, d);
}

// ------------------------------------------------------------- model load + derive
static bool load_model(const uint8_t* blob, size_t nbytes, Model& m, std::string& err) {
  Reader r{blob, nbytes};
  int32_t hi[16];
  double hf[16];
  r.read(hi, 16);
  r.read(hf, 16);
  if (!r.ok) { err = "blob too short"; return false; }
  if (hi[0] != 0x4D484A4D || hi[1] != 3) { err = "bad magic/version"; return false; }
  m.nbody = hi[2]; m.njnt = hi[3]; m.ngeom = hi[4]; m.npair = hi[5]; m.nu = hi[6];
  m.nq = hi[7]; m.nv = hi[8]; m.iterations = hi[9]; m.ls_iterations = hi[10];
  m.nconmax = hi[11];
  m.neq = hi[12];
  m.integrator = hi[13];
  m.cone = hi[15];
  const int has_hf = hi[14];
  m.dt = hf[0];
  for (int k = 0; k < 3; k++) m.grav[k] = hf[1 + k];
  m.solref[0] = hf[4]; m.solref[1] = hf[5];
  for (int k = 0; k < 5; k++) m.solimp[k] = hf[6 + k];
  m.tolerance = hf[11];
  if (m.nbody < 1 || m.njnt < 0 || m.ngeom < 0 || m.npair < 0 || m.nu < 0 || m.nconmax < 0 ||
      m.neq < 0 || m.integrator < 0 || m.integrator > 3 || has_hf < 0 || has_hf > 1 ||
      m.cone < 0 || m.cone > 1) {
    err = "negative size"; return false;
  }
  std::vector<int32_t> bi(2 * m.nbody);
  std::vector<double> bf(19 * m.nbody);
  r.read(bi.data(), bi.size()); r.read(bf.data(), bf.size());
  std::vector<int32_t> ji(4 * m.njnt);
  std::vector<double> jf(11 * m.njnt);
  r.read(ji.data(), ji.size()); r.read(jf.data(), jf.size());
  std::vector<int32_t> gi(2 * m.ngeom);
  std::vector<double> gf(11 * m.ngeom);
  r.read(gi.data(), gi.size()); r.read(gf.data(), gf.size());
  std::vector<int32_t> pi(4 * m.npair);
  std::vector<double> pf(3 * m.npair);
  r.read(pi.data(), pi.size()); r.read(pf.data(), pf.size());
  std::vector<int32_t> ai(2 * m.nu);
  std::vector<double> af(7 * m.nu);
  r.read(ai.data(), ai.size()); r.read(af.data(), af.size());
  std::vector<int32_t> ei(4 * m.neq);
  std::vector<double> ef(10 * m.neq);
  r.read(ei.data(), ei.size()); r.read(ef.data(), ef.size());
  if (has_hf) {
    int32_t hd[2];
    r.read(hd, 2);
    r.read(m.hf_size, 3);
    if (!r.ok || hd[0] < 2 || hd[1] < 2 || hd[0] > 4096 || hd[1] > 4096) {
      err = "bad heightfield"; return false;
    }
    m.hf_nrow = hd[0]; m.hf_ncol = hd[1];
    m.hf_data.resize((size_t)m.hf_nrow * m.hf_ncol);
    r.read(m.hf_data.data(), m.hf_data.size());
  }
  m.qpos0.resize(m.nq);
  r.read(m.qpos0.data(), m.nq);
  if (!r.ok || r.off != nbytes) { err = "blob size mismatch"; return false; }
  for (int b = 0; b < m.nbody; b++) {
    m.body_parent.push_back(bi[2 * b]);
    const double* f = &bf[19 * b];
    m.body_pos.insert(m.body_pos.end(), f, f + 3);
    m.body_quat.insert(m.body_quat.end(), f + 3, f + 7);
    m.body_mass.push_back(f[7]);
    m.body_ipos.insert(m.body_ipos.end(), f + 8, f + 11);
    m.body_inertia.insert(m.body_inertia.end(), f + 11, f + 17);
    if (b > 0 && (bi[2 * b] < 0 || bi[2 * b] >= b)) { err = "body order"; return false; }
  }
  for (int j = 0; j < m.njnt; j++) {
    const int* jj = &ji[4 * j];
    m.jnt_type.push_back(jj[0]);
    m.jnt_body.push_back(jj[1]);
    m.jnt_limited.push_back(jj[2] != 0);
    const double* f = &jf[11 * j];
    m.jnt_pos.insert(m.jnt_pos.end(), f, f + 3);
    double ax[3] = {f[3], f[4], f[5]};
    double L = std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
    for (int k = 0; k < 3; k++) m.jnt_axis.push_back(L > 0 ? ax[k] / L : 0.0);
    m.jnt_damping.push_back(f[6]);
    m.jnt_armature.push_back(f[7]);
    m.jnt_range.push_back(f[8]);
    m.jnt_range.push_back(f[9]);
    if (jj[0] < 0 || jj[0] > 2 || jj[1] <= 0 || jj[1] >= m.nbody) {
      err = "bad joint"; return false;
    }
    if (j > 0 && jj[1] < ji[4 * (j - 1) + 1]) { err = "joints not grouped by body"; return false; }
    if (jj[2] != 0) {
      if (jj[0] == JFREE || !(f[8] < f[9])) { err = "bad joint limit"; return false; }
      m.nlimit++;
    }
    if (!(f[10] >= 0.0) || (jj[0] == JFREE && f[10] != 0.0)) {
      err = "bad friction loss"; return false;
    }
    m.jnt_frictionloss.push_back(f[10]);
  }
  for (int g = 0; g < m.ngeom; g++) {
    m.geom_type.push_back(gi[2 * g]);
    m.geom_body.push_back(gi[2 * g + 1]);
    const double* f = &gf[11 * g];
    m.geom_size.insert(m.geom_size.end(), f, f + 3);
    m.geom_pos.insert(m.geom_pos.end(), f + 3, f + 6);
    m.geom_quat.insert(m.geom_quat.end(), f + 6, f + 10);
    m.geom_friction.push_back(f[10]);
  }
  for (int p = 0; p < m.npair; p++) {
    m.pair_g1.push_back(pi[4 * p]);
    m.pair_g2.push_back(pi[4 * p + 1]);
    m.pair_condim.push_back(pi[4 * p + 2]);
    m.pair_mu.push_back(pf[3 * p]);
    m.pair_mu_torsion.push_back(pf[3 * p + 1]);
    m.pair_mu_rolling.push_back(pf[3 * p + 2]);
    if (pi[4 * p] < 0 || pi[4 * p] >= m.ngeom || pi[4 * p + 1] < 0 || pi[4 * p + 1] >= m.ngeom ||
        (pi[4 * p + 2] != 1 && pi[4 * p + 2] != 3 && pi[4 * p + 2] != 4 && pi[4 * p + 2] != 6)) {
      err = "bad pair"; return false;
    }
    int t1 = m.geom_type[pi[4 * p]], t2 = m.geom_type[pi[4 * p + 1]];
    bool ok = t1 <= t2 && !(t1 == GPLANE && t2 == GPLANE) && !(t1 == GBOX && t2 == GBOX);
    if (t2 == GHFIELD) ok = t1 == GSPHERE && m.hf_nrow > 0;
    if (!ok) { err = "unsupported pair"; return false; }
  }
  for (int a = 0; a < m.nu; a++) {
    m.act_type.push_back(ai[2 * a]);
    m.act_jnt.push_back(ai[2 * a + 1]);
    const double* f = &af[7 * a];
    m.act_gear.push_back(f[0]); m.act_kp.push_back(f[1]); m.act_kd.push_back(f[2]);
    m.act_range.push_back(f[3]); m.act_range.push_back(f[4]);
    m.act_qdef.push_back(f[5]);
    if (ai[2 * a + 1] < 0 || ai[2 * a + 1] >= m.njnt) { err = "bad actuator"; return false; }
  }
  for (int e = 0; e < m.neq; e++) {
    const int* q = &ei[4 * e];
    if (q[0] < 0 || q[0] > 1 || q[1] <= 0 || q[1] >= m.nbody || q[2] < 0 || q[2] >= m.nbody ||
        q[1] == q[2]) {
      err = "bad equality"; return false;
    }
    m.eq_type.push_back(q[0]); m.eq_b1.push_back(q[1]); m.eq_b2.push_back(q[2]);
    m.eq_a1.insert(m.eq_a1.end(), &ef[10 * e], &ef[10 * e] + 3);
    m.eq_a2.insert(m.eq_a2.end(), &ef[10 * e] + 3, &ef[10 * e] + 6);
    const double* qr = &ef[10 * e + 6];
    const double qn = std::sqrt(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
    if (q[0] == 1 && !(qn > 0.0)) { err = "bad weld orientation"; return false; }
    double Rq[9];
    const double qu[4] = {qr[0] / qn, qr[1] / qn, qr[2] / qn, qr[3] / qn};
    quat2mat(qu, Rq);
    m.eq_relR.insert(m.eq_relR.end(), Rq, Rq + 9);
    m.neqrow += q[0] == 1 ? 6 : 3;
  }
  // derived addresses
  m.body_jntadr.assign(m.nbody, 0); m.body_jntnum.assign(m.nbody, 0);
  m.body_dofadr.assign(m.nbody, 0); m.body_dofnum.assign(m.nbody, 0);
  int qa = 0, da = 0;
  for (int j = 0; j < m.njnt; j++) {
    m.jnt_qposadr.push_back(qa);
    m.jnt_dofadr.push_back(da);
    int b = m.jnt_body[j];
    if (m.body_jntnum[b] == 0) { m.body_jntadr[b] = j; m.body_dofadr[b] = da; }
    m.body_jntnum[b]++;
    int nd = m.jnt_type[j] == JFREE ? 6 : 1;
    m.body_dofnum[b] += nd;
    for (int k = 0; k < nd; k++) {
      m.dof_body.push_back(b);
      m.dof_jnt.push_back(j);
      m.dof_damping.push_back(m.jnt_damping[j]);
      m.dof_armature.push_back(m.jnt_armature[j]);
      m.dof_frictionloss.push_back(m.jnt_frictionloss[j]);
      if (m.jnt_frictionloss[j] > 0.0) m.nfric++;
    }
    qa += m.jnt_type[j] == JFREE ? 7 : 1;
    da += nd;
    if (m.jnt_type[j] == JFREE && (m.body_parent[b] != 0 || m.body_jntnum[b] != 1)) {
      err = "free joint must be the only joint of a world child"; return false;
    }
  }
  if (qa != m.nq || da != m.nv) { err = "nq/nv mismatch"; return false; }
  // dof parent: previous dof of the same body, else the last dof of the nearest
  // ancestor body that has dofs
  m.dof_parent.assign(m.nv, -1);
  for (int k = 0; k < m.nv; k++) {
    int b = m.dof_body[k];
    if (k > m.body_dofadr[b]) { m.dof_parent[k] = k - 1; continue; }
    for (int p = m.body_parent[b]; p > 0; p = m.body_parent[p])
      if (m.body_dofnum[p] > 0) { m.dof_parent[k] = m.body_dofadr[p] + m.body_dofnum[p] - 1; break; }
  }
  // C8 reading: body translational inverse weight at qpos0,
  //   w(b) = trace(J_com M^-1 J_com^T) / 3
  m.body_invweight.assign(m.nbody, 0.0);
  if (m.nv > 0) {
    Data<double> d;
    d.alloc(m);
    d.qpos = m.qpos0;
    kinematics(m, d);
    crba(m, d);
    factor_ltdl(m, d.M, d.qLD);
    std::vector<double> J(3 * m.nv), x(m.nv);
    for (int b = 1; b < m.nbody; b++) {
      point_jac(m, d, b, &d.xipos[3 * b], J.data());
      double tr = 0.0;
      for (int r = 0; r < 3; r++) {
        solve_ltdl(m, d.qLD, &J[r * m.nv], x.data());
        for (int i = 0; i < m.nv; i++) tr += J[r * m.nv + i] * x[i];
      }
      m.body_invweight[b] = tr / 3.0;
    }
    // joint-limit rows: the dof's own inverse weight (M^-1)_kk at qpos0
    m.dof_invweight.assign(m.nv, 0.0);
    std::vector<double> e(m.nv);
    for (int k = 0; k < m.nv; k++) {
      std::fill(e.begin(), e.end(), 0.0);
      e[k] = 1.0;
      solve_ltdl(m, d.qLD, e.data(), x.data());
      m.dof_invweight[k] = x[k];
    }
  }
  return true;
}

template <class F> void parallel_for(int n, int nthreads, F fn) {
  if (nthreads <= 1 || n <= 1) {
    for (int i = 0; i < n; i++) fn(i);
    return;
  }
  nthreads = std::min(nthreads, n);
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; t++)
    th.emplace_back([&, t]() {
      for (int i = t; i < n; i += nthreads) fn(i);
    });
  for (auto& x : th) x.join();
}

// loss of an adjoint rollout: sum_t (z_t - ztarget)^2 + wctrl * sum_t |u_t|^2 with z_t
// the first free body's height after step t
template <class T>
T rollout_loss(const Model& m, Data<T>& d, int horizon, const T* ctrl_seq, double ztarget,
               double wctrl, int mode, int zidx) {
  T L = 0.0;
  for (int t = 0; t < horizon; t++) {
    for (int a = 0; a < m.nu; a++) {
      d.ctrl[a] = ctrl_seq[t * m.nu + a];
      L += wctrl * d.ctrl[a] * d.ctrl[a];
    }
    step(m, d, mode);
    T z = d.qpos[zidx] - ztarget;
    L += z * z;
  }
  return L;
}

}  // namespace mjo

// =========================================================================== C API
using namespace mjo;

extern "C" {

void* mjo_load(const unsigned char* blob, long nbytes, char* err, int errlen) {
  Model* m = new Model();
  std::string e;
  if (!load_model(blob, (size_t)nbytes, *m, e)) {
    if (err && errlen > 0) { std::strncpy(err, e.c_str(), errlen - 1); err[errlen - 1] = 0; }
    delete m;
    return nullptr;
  }
  return m;
}

void mjo_free(void* h) { delete static_cast<Model*>(h); }

// out[0..14] = nq nv nu nbody njnt ngeom npair nconmax iterations ls_iterations nlimit
// nfric neq neqrow conrows
int mjo_dims(void* h, int* out) {
  Model& m = *static_cast<Model*>(h);
  int conrows = m.npair ? 1 : 4;  // rows of the widest contact
  for (int c : m.pair_condim)  // pyramid edges, or an elliptic cone's frame rows
    conrows = std::max(conrows, (c == 1 || m.cone == 1) ? c : 2 * (c - 1));
  int v[15] = {m.nq, m.nv, m.nu, m.nbody, m.njnt, m.ngeom, m.npair, m.nconmax,
               m.iterations, m.ls_iterations, m.nlimit, m.nfric, m.neq, m.neqrow, conrows};
  std::memcpy(out, v, sizeof(v));
  return 0;
}

int mjo_body_invweight(void* h, double* out) {
  Model& m = *static_cast<Model*>(h);
  for (int b = 0; b < m.nbody; b++) out[b] = m.body_invweight[b];
  return 0;
}

int mjo_dof_invweight(void* h, double* out) {
  Model& m = *static_cast<Model*>(h);
  for (int k = 0; k < m.nv; k++) out[k] = m.dof_invweight[k];
  return 0;
}

// Replace the inverse weights (the A of every row's regulariser).  A model whose
// parameters differ per world keeps those of its nominal model, computed once at qpos0.
int mjo_set_invweight(void* h, const double* body, const double* dof) {
  Model& m = *static_cast<Model*>(h);
  for (int b = 0; b < m.nbody; b++) m.body_invweight[b] = body[b];
  for (int k = 0; k < m.nv; k++) m.dof_invweight[k] = dof[k];
  return 0;
}

int mjo_dof_parent(void* h, int* out) {
  Model& m = *static_cast<Model*>(h);
  for (int k = 0; k < m.nv; k++) out[k] = m.dof_parent[k];
  return 0;
}

static void set_state(const Model& m, Data<double>& d, const double* qpos, const double* qvel,
                      const double* qacc_ws, const double* ctrl) {
  d.alloc(m);
  if (qpos) d.qpos.assign(qpos, qpos + m.nq); else d.qpos = m.qpos0;
  if (qvel) d.qvel.assign(qvel, qvel + m.nv);
  if (qacc_ws) d.qacc_ws.assign(qacc_ws, qacc_ws + m.nv);
  if (ctrl) d.ctrl.assign(ctrl, ctrl + m.nu);
}

static void export_contacts(const Model& m, const Data<double>& d, double* out) {
  int nc = (int)d.con.size();
  for (int c = 0; c < nc && c < m.nconmax; c++) {
    double* o = out + CON_SIZE * c;
    const Contact<double>& k = d.con[c];
    o[0] = k.dist;
    for (int i = 0; i < 3; i++) o[1 + i] = k.pos[i];
    for (int i = 0; i < 9; i++) o[4 + i] = k.frame[i];
    const double* f = &d.efc_force[k.row];
    if (m.cone == 1) {
      // elliptic: the frame rows' forces (normal, tangent 1, tangent 2)
      o[13] = f[0];
      o[14] = k.condim == 1 ? 0.0 : f[1];
      o[15] = k.condim == 1 ? 0.0 : f[2];
    } else {
      // pyramid: the normal force is every edge's (each has unit normal component);
      // tangential forces from the sliding edges
      const int nr = k.condim == 1 ? 1 : 2 * (k.condim - 1);
      o[13] = 0.0;
      for (int e = 0; e < nr; e++) o[13] += f[e];
      o[14] = k.condim == 1 ? 0.0 : val(k.mu) * (f[0] - f[1]);
      o[15] = k.condim == 1 ? 0.0 : val(k.mu) * (f[2] - f[3]);
    }
    // torsional and rolling moments are not exported
    o[16] = k.pair; o[17] = k.sub; o[18] = k.g1; o[19] = k.g2;
  }
}

// Advance nworld worlds by nstep steps.  State arrays are [nworld][n] and updated in
// place; ctrl is [nstep][nworld][nu] (NULL = zero).  Outputs of the last step:
// qacc [nworld][nv], qacc_smooth [nworld][nv], status/ncon [nworld],
// contacts [nworld][nconmax][20].  Any output pointer may be NULL.
int mjo_step(void* h, int nworld, int nstep, double* qpos, double* qvel, double* qacc_ws,
             const double* ctrl, int mode, int nthreads, double* qacc_out,
             double* qacc_smooth_out, int* status, int* ncon, double* contacts) {
  Model& m = *static_cast<Model*>(h);
  parallel_for(nworld, nthreads, [&](int w) {
    Data<double> d;
    set_state(m, d, qpos + (size_t)w * m.nq, qvel + (size_t)w * m.nv,
              qacc_ws ? qacc_ws + (size_t)w * m.nv : nullptr, nullptr);
    int st = 0;
    for (int s = 0; s < nstep; s++) {
      if (ctrl) for (int a = 0; a < m.nu; a++) d.ctrl[a] = ctrl[((size_t)s * nworld + w) * m.nu + a];
      step(m, d, mode);
      st |= d.status;
    }
    std::copy(d.qpos.begin(), d.qpos.end(), qpos + (size_t)w * m.nq);
    std::copy(d.qvel.begin(), d.qvel.end(), qvel + (size_t)w * m.nv);
    if (qacc_ws) std::copy(d.qacc_ws.begin(), d.qacc_ws.end(), qacc_ws + (size_t)w * m.nv);
    if (qacc_out) std::copy(d.qacc.begin(), d.qacc.end(), qacc_out + (size_t)w * m.nv);
    if (qacc_smooth_out)
      std::copy(d.qacc_smooth.begin(), d.qacc_smooth.end(), qacc_smooth_out + (size_t)w * m.nv);
    if (status) status[w] = st;
    if (ncon) ncon[w] = (int)d.con.size();
    if (contacts) export_contacts(m, d, contacts + (size_t)w * m.nconmax * CON_SIZE);
  });
  return 0;
}

// Intermediates of one forward evaluation (no integration) of a single world.
// Output sizes: xpos [nbody*3], xmat [nbody*9], xipos [nbody*3], cdof [nv*6],
// cvel [nbody*6], M [nv*nv], bias [nv], act [nv], pass [nv], qacc_smooth [nv],
// qacc [nv], qfrc_con [nv], ncon, contacts [nconmax*20], nrow, J [nrowmax * nv],
// aref, D, efc_force [nrowmax] with nrowmax = conrows nconmax + nlimit + nfric + neqrow (contact
// rows first, then the violated limits, the friction-loss rows and the equality rows).
// NULL skips an output.
int mjo_forward(void* h, const double* qpos, const double* qvel, const double* qacc_ws,
                const double* ctrl, int mode, double* xpos, double* xmat, double* xipos,
                double* cdof, double* cvel, double* M, double* bias, double* act,
                double* pass, double* qacc_smooth, double* qacc, double* qfrc_con,
                int* ncon, double* contacts, int* nrow, double* J, double* aref, double* D,
                double* efc_force, int* status) {
  Model& m = *static_cast<Model*>(h);
  Data<double> d;
  set_state(m, d, qpos, qvel, qacc_ws, ctrl);
  forward(m, d, mode);
  auto cp = [](const std::vector<double>& v, double* o) {
    if (o) std::copy(v.begin(), v.end(), o);
  };
  cp(d.xpos, xpos); cp(d.xmat, xmat); cp(d.xipos, xipos); cp(d.cdof, cdof); cp(d.cvel, cvel);
  cp(d.M, M); cp(d.qfrc_bias, bias); cp(d.qfrc_act, act); cp(d.qfrc_pass, pass);
  cp(d.qacc_smooth, qacc_smooth); cp(d.qacc, qacc); cp(d.qfrc_con, qfrc_con);
  if (ncon) *ncon = (int)d.con.size();
  if (contacts) export_contacts(m, d, contacts);
  if (nrow) *nrow = d.nrow;
  cp(d.J, J); cp(d.aref, aref); cp(d.D, D); cp(d.efc_force, efc_force);
  if (status) *status = d.status;
  return 0;
}

// the Newton cost F(a) of one world's step (state, ctrl) at the acceleration a
double mjo_cost(void* h, const double* qpos, const double* qvel, const double* ctrl,
                const double* a) {
  Model& m = *static_cast<Model*>(h);
  Data<double> d;
  set_state(m, d, qpos, qvel, nullptr, ctrl);
  forward(m, d, 0);
  Solver<double> s(m, d);
  return s.cost(a);
}

// inverse dynamics tau = M(q) qacc + c(q, qvel) (gravity included)
int mjo_inverse(void* h, const double* qpos, const double* qvel, const double* qacc, double* tau) {
  Model& m = *static_cast<Model*>(h);
  Data<double> d;
  set_state(m, d, qpos, qvel, nullptr, nullptr);
  kinematics(m, d);
  velocities(m, d);
  rne(m, d, qacc, tau);
  return 0;
}

// x = M(q)^{-1} b through the sparse LTDL factors; also returns L (strict lower) + D
int mjo_ltdl_solve(void* h, const double* qpos, const double* b, double* x, double* LD) {
  Model& m = *static_cast<Model*>(h);
  Data<double> d;
  set_state(m, d, qpos, nullptr, nullptr, nullptr);
  kinematics(m, d);
  crba(m, d);
  factor_ltdl(m, d.M, d.qLD);
  solve_ltdl(m, d.qLD, b, x);
  if (LD) std::copy(d.qLD.begin(), d.qLD.end(), LD);
  return 0;
}

// translational Jacobian (3 x nv) of a world point attached to body b
int mjo_point_jac(void* h, const double* qpos, int body, const double* point, double* J) {
  Model& m = *static_cast<Model*>(h);
  Data<double> d;
  set_state(m, d, qpos, nullptr, nullptr, nullptr);
  kinematics(m, d);
  point_jac(m, d, body, point, J);
  return 0;
}

// loss of a rollout for nworld worlds (state [nworld][n], ctrl_seq [horizon][nworld][nu])
int mjo_rollout_loss(void* h, int nworld, int horizon, const double* qpos, const double* qvel,
                     const double* qacc_ws, const double* ctrl_seq, double ztarget,
                     double wctrl, int mode, int zidx, int nthreads, double* loss) {
  Model& m = *static_cast<Model*>(h);
  parallel_for(nworld, nthreads, [&](int w) {
    Data<double> d;
    set_state(m, d, qpos + (size_t)w * m.nq, qvel + (size_t)w * m.nv,
              qacc_ws ? qacc_ws + (size_t)w * m.nv : nullptr, nullptr);
    std::vector<double> u((size_t)horizon * m.nu);
    for (int t = 0; t < horizon; t++)
      for (int a = 0; a < m.nu; a++) u[t * m.nu + a] = ctrl_seq[((size_t)t * nworld + w) * m.nu + a];
    loss[w] = rollout_loss(m, d, horizon, u.data(), ztarget, wctrl, mode, zidx);
  });
  return 0;
}

// directional derivative of the rollout loss along (dqvel [nworld][nv],
// dctrl [horizon][nworld][nu]) by forward-mode dual numbers
int mjo_rollout_jvp(void* h, int nworld, int horizon, const double* qpos, const double* qvel,
                    const double* qacc_ws, const double* ctrl_seq, const double* dqvel,
                    const double* dctrl, double ztarget, double wctrl, int mode, int zidx,
                    int nthreads, double* loss, double* dloss) {
  Model& m = *static_cast<Model*>(h);
  parallel_for(nworld, nthreads, [&](int w) {
    Data<Dual> d;
    d.alloc(m);
    for (int i = 0; i < m.nq; i++) d.qpos[i] = Dual(qpos[(size_t)w * m.nq + i]);
    for (int i = 0; i < m.nv; i++)
      d.qvel[i] = Dual(qvel[(size_t)w * m.nv + i], dqvel[(size_t)w * m.nv + i]);
    if (qacc_ws)
      for (int i = 0; i < m.nv; i++) d.qacc_ws[i] = Dual(qacc_ws[(size_t)w * m.nv + i]);
    std::vector<Dual> u((size_t)horizon * m.nu);
    for (int t = 0; t < horizon; t++)
      for (int a = 0; a < m.nu; a++) {
        size_t idx = ((size_t)t * nworld + w) * m.nu + a;
        u[t * m.nu + a] = Dual(ctrl_seq[idx], dctrl[idx]);
      }
    Dual L = rollout_loss(m, d, horizon, u.data(), ztarget, wctrl, mode, zidx);
    loss[w] = L.v;
    dloss[w] = L.d;
  });
  return 0;
}

// directional derivative of one step's outputs (qpos', qvel') along (dqpos, dqvel, dctrl)
int mjo_step_jvp(void* h, const double* qpos, const double* qvel, const double* qacc_ws,
                 const double* ctrl, const double* dqpos, const double* dqvel,
                 const double* dctrl, int mode, double* qpos_out, double* qvel_out,
                 double* dqpos_out, double* dqvel_out) {
  Model& m = *static_cast<Model*>(h);
  Data<Dual> d;
  d.alloc(m);
  for (int i = 0; i < m.nq; i++) d.qpos[i] = Dual(qpos[i], dqpos ? dqpos[i] : 0.0);
  for (int i = 0; i < m.nv; i++) d.qvel[i] = Dual(qvel[i], dqvel ? dqvel[i] : 0.0);
  if (qacc_ws) for (int i = 0; i < m.nv; i++) d.qacc_ws[i] = Dual(qacc_ws[i]);
  for (int a = 0; a < m.nu; a++) d.ctrl[a] = Dual(ctrl ? ctrl[a] : 0.0, dctrl ? dctrl[a] : 0.0);
  step(m, d, mode);
  for (int i = 0; i < m.nq; i++) { qpos_out[i] = d.qpos[i].v; dqpos_out[i] = d.qpos[i].d; }
  for (int i = 0; i < m.nv; i++) { qvel_out[i] = d.qvel[i].v; dqvel_out[i] = d.qvel[i].d; }
  return 0;
}

}  // extern "C"

extern "C" {
// single world, nstep steps, recording qpos/qvel after every step
// (traj_qpos [nstep][nq], traj_qvel [nstep][nv]); ctrl [nstep][nu] or NULL
int mjo_trajectory(void* h, int nstep, const double* qpos, const double* qvel,
                   const double* qacc_ws, const double* ctrl, int mode, double* traj_qpos,
                   double* traj_qvel, int* status) {
  Model& m = *static_cast<Model*>(h);
  Data<double> d;
  set_state(m, d, qpos, qvel, qacc_ws, nullptr);
  int st = 0;
  for (int s = 0; s < nstep; s++) {
    if (ctrl) for (int a = 0; a < m.nu; a++) d.ctrl[a] = ctrl[(size_t)s * m.nu + a];
    step(m, d, mode);
    st |= d.status;
    std::copy(d.qpos.begin(), d.qpos.end(), traj_qpos + (size_t)s * m.nq);
    std::copy(d.qvel.begin(), d.qvel.end(), traj_qvel + (size_t)s * m.nv);
  }
  if (status) *status = st;
  return 0;
}
}  // extern "C"

extern "C" {
// Set the capsule-box tolerances (the equal-value allowance relative to the segment's
// scale, and the de-duplication distance in t); returns the previous pair in prev[2].
void mjo_set_capsule_box_tolerances(double eq, double dup, double* prev) {
  if (prev) { prev[0] = g_cb_eq; prev[1] = g_cb_dup; }
  g_cb_eq = eq;
  g_cb_dup = dup;
}
// Average floating-point operation count of one step (fixed mode) from each of nworld
// states, counted by the operation-counting scalar: every operation of the dense loops,
// and, when nonzero_out is given, those whose operands are all nonzero (*nonzero_out).
double mjo_count_flops2(void* h, int nworld, const double* qpos, const double* qvel,
                        const double* qacc_ws, const double* ctrl, double* nonzero_out) {
  Model& m = *static_cast<Model*>(h);
  long long total = 0, total_nz = 0;
  for (int w = 0; w < nworld; w++) {
    Data<Cnt> d;
    d.alloc(m);
    for (int i = 0; i < m.nq; i++) d.qpos[i] = qpos[(size_t)w * m.nq + i];
    for (int i = 0; i < m.nv; i++) d.qvel[i] = qvel[(size_t)w * m.nv + i];
    if (qacc_ws) for (int i = 0; i < m.nv; i++) d.qacc_ws[i] = qacc_ws[(size_t)w * m.nv + i];
    if (ctrl) for (int a = 0; a < m.nu; a++) d.ctrl[a] = ctrl[(size_t)w * m.nu + a];
    g_flops = 0;
    g_flops_nz = 0;
    step(m, d, 0);
    total += g_flops;
    total_nz += g_flops_nz;
  }
  if (nonzero_out) *nonzero_out = nworld > 0 ? (double)total_nz / nworld : 0.0;
  return nworld > 0 ? (double)total / nworld : 0.0;
}
double mjo_count_flops(void* h, int nworld, const double* qpos, const double* qvel,
                       const double* qacc_ws, const double* ctrl) {
  return mjo_count_flops2(h, nworld, qpos, qvel, qacc_ws, ctrl, nullptr);
}
}  // extern "C"
