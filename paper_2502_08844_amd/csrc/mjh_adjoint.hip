// Differentiable rollout: checkpointed forward and hand-written reverse sweep.
//
// Forward (rollout_fwd_kernel): every world runs `horizon` steps with the Newton
// solve iterated to convergence (max |g| <= kAdjGtol * max(1, max |qfrc_smooth|), at
// most kAdjIters iterations), stores (qpos, qvel, qacc_ws) every `ckpt` steps and
// accumulates the loss  sum_t (qpos_{t+1}[zidx] - ztarget)^2 + wctrl |u_t|^2.
// Reverse (rollout_bwd_kernel): segments in reverse order; each is recomputed from its
// checkpoint into a per-world tape (Griewank & Walther, checkpointed reverse mode),
// which keeps, for every step of the segment, the on-chip image right after its solve
// (the forward regions of the adjoint layout, a few KB per world-step in HBM). Each
// step's image is then reloaded, not solved again, and its vector-Jacobian product
// taken:
//   * semi-implicit Euler and the exponential-map orientation update, reversed;
//   * the contact solve by implicit differentiation at the Newton solution a*:
//     grad_a F(a*; theta) = 0 gives theta_bar = -(dG/dtheta)^T H^-1 a_bar with
//     G = ID(q, qdot, a*) - tau(q, qdot, u) - sum_active J^T D (aref - J a*), H the
//     Newton Hessian at a*;
//   * reverse sweeps of the recursive Newton-Euler inverse dynamics, of the contact
//     rows (Jacobians, impedance, reference acceleration, contact geometry) and of
//     the forward kinematics.
// Contact geometry is differentiated for plane-sphere and plane-capsule pairs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "mjh_adjoint.h"
#include "mjh_device.h"
#include "mjh_kernels.h"

namespace mjh {

constexpr int kAdjIters = 16;  // Newton iterations cap inside differentiable rollouts
// inside rollouts Newton runs to convergence: max |g| <= kAdjGtol * max(1, max |qfrc_smooth|)
constexpr float kAdjGtol = 1e-5f;
constexpr int kAdjBlock = 64;  // threads per work-group of the rollout kernels

// ------------------------------------------------------------------ small helpers
DEV void skew_mul(const float* w, const float* R, float* out) {  // [w]x R
  for (int j = 0; j < 3; j++) {
    const float r0 = R[j], r1 = R[3 + j], r2 = R[6 + j];
    out[j] = w[1] * r2 - w[2] * r1;
    out[3 + j] = w[2] * r0 - w[0] * r2;
    out[6 + j] = w[0] * r1 - w[1] * r0;
  }
}
DEV void quat_mul4(const float* a, const float* b, float* r) {
  const float w = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  const float x = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  const float y = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  const float z = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
  r[0] = w; r[1] = x; r[2] = y; r[3] = z;
}
// pair (g, mv) of a spatial-inertia product f = I mv: accumulate the cotangent of the
// inertia parameters (m, h, I_O (xx yy zz xy xz yz)) given the cotangent g of f
DEV void inertia_cot(float* ib, const float* g, const float* mv) {
  const float* w = mv;
  const float* v = mv + 3;
  ib[0] += g[3] * v[0] + g[4] * v[1] + g[5] * v[2];
  float a[3], b[3];
  cross3(v, g, a);
  cross3(w, g + 3, b);
  ib[1] += a[0] - b[0]; ib[2] += a[1] - b[1]; ib[3] += a[2] - b[2];
  // symmetric part of g_n w^T, stored as full-matrix entries xx yy zz xy xz yz
  ib[4] += g[0] * w[0]; ib[5] += g[1] * w[1]; ib[6] += g[2] * w[2];
  ib[7] += 0.5f * (g[0] * w[1] + w[0] * g[1]);
  ib[8] += 0.5f * (g[0] * w[2] + w[0] * g[2]);
  ib[9] += 0.5f * (g[1] * w[2] + w[1] * g[2]);
}
// impedance d(r) and its derivative
DEV void impedance_d(const DevModel& m, float r, float& d, float& dd) {
  const float x = fminf(fabsf(r) / m.width, 1.f);
  float y, yp;
  if (x <= m.mid) {
    y = powf(x, m.power) / powf(m.mid, m.power - 1.f);
    yp = m.power * powf(x, m.power - 1.f) / powf(m.mid, m.power - 1.f);
  } else {
    y = 1.f - powf(1.f - x, m.power) / powf(1.f - m.mid, m.power - 1.f);
    yp = m.power * powf(1.f - x, m.power - 1.f) / powf(1.f - m.mid, m.power - 1.f);
  }
  d = m.dmin + y * (m.dmax - m.dmin);
  dd = (x >= 1.f) ? 0.f : (m.dmax - m.dmin) * yp * (r < 0.f ? -1.f : 1.f) / m.width;
}

// subtree force totals (cfrc in place), leaving the body inertias untouched
DEV void accumulate_forces(const DevModel& m, float* W, const Team& t) {
  float* cfrc = W + m.o_cfrc;
  for (int lv = m.nlevel - 1; lv >= 1; lv--) {
    const int e = m.level_start[lv + 1];
    for (int ib = m.level_start[lv] + t.lane; ib < e; ib += t.T) {
      const int b = m.level_body[ib];
      for (int c = m.child_start[b]; c < m.child_start[b + 1]; c++) {
        const int ch = m.child_list[c];
        for (int k = 0; k < 6; k++) cfrc[6 * b + k] += cfrc[6 * ch + k];
      }
    }
    t.sync();
  }
}

// pose of body b's frame before its joints (from the parent's final pose)
DEV void body_base(const DevModel& m, const float* W, int b, float* pos, float* R) {
  const int p = m.body_parent[b];
  const float* xp = W + m.o_xpos + 3 * p;
  const float* Rp = W + m.o_xmat + 9 * p;
  mv3(Rp, m.body_pos + 3 * b, pos);
  pos[0] += xp[0]; pos[1] += xp[1]; pos[2] += xp[2];
  mm3(Rp, m.body_rot + 9 * b, R);
}

// ------------------------------------------------- contact geometry, reversed
// Each takes the cotangents of a forward function's outputs and adds those of its
// inputs, recomputing what it needs (the same branches as the forward code).

// contact_frame: t1 = v / |v|, v = e_ax - n_ax n (ax: the smallest |n_k|), t2 = n x t1.
// Cotangents t1b, t2b are added into nb.
DEV void frame_rev(const float* n, const float* t1, const float* t1b, const float* t2b,
                   float* nb) {
  float a[3], b[3];
  cross3(t1, t2b, a);  // d/dn of (n x t1).g is t1 x g; d/dt1 is g x n
  cross3(t2b, n, b);
  const float tb[3] = {t1b[0] + b[0], t1b[1] + b[1], t1b[2] + b[2]};
  int ax = 0;
  if (fabsf(n[1]) < fabsf(n[ax])) ax = 1;
  if (fabsf(n[2]) < fabsf(n[ax])) ax = 2;
  const float en = n[ax];
  float v[3] = {-en * n[0], -en * n[1], -en * n[2]};
  v[ax] += 1.f;
  const float inv = 1.f / sqrtf(dot3(v, v));
  const float tt = dot3(t1, tb);
  float vb[3];
  for (int k = 0; k < 3; k++) vb[k] = (tb[k] - t1[k] * tt) * inv;
  const float enb = -dot3(n, vb);
  for (int k = 0; k < 3; k++) nb[k] += a[k] - en * vb[k];
  nb[ax] += enb;
}

// sphere_sphere: with d = c2 - c1, L = |d|, n = d / L, dist = L - r1 - r2 and
// pos = c1 + d / 2 + (r1 - r2) n / 2.  Cotangents of pos (xb), n (nb), dist (db).
DEV void sphere_sphere_rev(const float* c1, float r1, const float* c2, float r2,
                           const float* xb, const float* nb, float db, float* c1b,
                           float* c2b) {
  const float d[3] = {c2[0] - c1[0], c2[1] - c1[1], c2[2] - c1[2]};
  const float L = sqrtf(dot3(d, d));
  const bool ok = L > 1e-12f;  // otherwise the forward code fixed n = e_z
  const float n[3] = {ok ? d[0] / L : 0.f, ok ? d[1] / L : 0.f, ok ? d[2] / L : 1.f};
  const float rho = 0.5f * (r1 - r2);
  const float g[3] = {rho * xb[0] + nb[0], rho * xb[1] + nb[1], rho * xb[2] + nb[2]};
  const float gn = dot3(n, g);
  for (int k = 0; k < 3; k++) {
    const float dbar = 0.5f * xb[k] + (ok ? db * n[k] + (g[k] - n[k] * gn) / L : 0.f);
    c1b[k] += xb[k] - dbar;
    c2b[k] += dbar;
  }
}

// nearest point q = a + t u of a segment to x, t = clamp((x - a).u / u.u, 0, 1)
DEV void seg_point_rev(const float* x, const float* a, const float* u, const float* qb,
                       float* xb, float* ab, float* ub) {
  const float uu = dot3(u, u);
  const float ap[3] = {x[0] - a[0], x[1] - a[1], x[2] - a[2]};
  const float t0 = uu < 1e-30f ? 0.f : dot3(ap, u) / uu;
  const float t = fminf(fmaxf(t0, 0.f), 1.f);
  for (int k = 0; k < 3; k++) { ab[k] += qb[k]; ub[k] += t * qb[k]; }
  if (uu >= 1e-30f && t0 > 0.f && t0 < 1.f) {
    const float tb = dot3(qb, u);
    for (int k = 0; k < 3; k++) {
      const float apb = tb * u[k] / uu;
      xb[k] += apb;
      ab[k] -= apb;
      ub[k] += tb * (ap[k] - 2.f * t * u[k]) / uu;
    }
  }
}

// sphere_hfield_tri against a heightfield fixed in the world: the cotangents of pos
// (xb), n (nb) and dist (db) -> of the sphere centre c.  In the field's frame, with
// cl = Rg^T (c - xg), bq the triangle's nearest point and d = cl - bq: pos = (c + r n +
// xg + Rg bq) / 2, n = Rg sg d / |d| and dist = -sg |d| - r (sg = +1 below the
// triangle's plane, -1 above).  bq moves with cl by the projection onto the triangle's
// plane (face), onto the edge's line (edge) or not at all (vertex).
DEV void sphere_hfield_rev(const DevModel& m, const float* xg, const float* Rg, const float* c,
                           float r, int code, const float* xb, const float* nb, float db,
                           float* cb) {
  if (code < 0) return;
  const int cellid = code >> 1, k = code & 1;
  const int i = cellid / m.hf_ncol, j = cellid - i * m.hf_ncol;
  const V3 cl = hfield_local(xg, Rg, c);
  V3 a, b, cc, bn;
  hfield_tri(m, i, j, k, a, b, cc);
  const V3 bq = tri_nearest(a, b, cc, cl, bn);
  const V3 d = v3sub(cl, bq);
  const float L = sqrtf(v3dot(d, d));
  const float nt[3] = {nb[0] + 0.5f * r * xb[0], nb[1] + 0.5f * r * xb[1],
                       nb[2] + 0.5f * r * xb[2]};  // the normal's whole cotangent
  float xl[3], nl[3];
  mtv3(Rg, xb, xl);
  mtv3(Rg, nt, nl);
  for (int q = 0; q < 3; q++) cb[q] += 0.5f * xb[q];
  float dbar[3] = {0.f, 0.f, 0.f};
  if (L > 1e-12f) {  // otherwise the forward code took the triangle's normal: constant
    const float sg = v3dot(bn, d) < 0.f ? 1.f : -1.f;
    const float dh[3] = {d.x / L, d.y / L, d.z / L};
    const float dn = dh[0] * nl[0] + dh[1] * nl[1] + dh[2] * nl[2];
    for (int q = 0; q < 3; q++) dbar[q] = sg * (nl[q] - dh[q] * dn) / L - sg * db * dh[q];
  }
  // d = cl - bq; bq's cotangent is that of pos's Rg bq / 2 minus d's
  float bqb[3], clb[3];
  for (int q = 0; q < 3; q++) { bqb[q] = 0.5f * xl[q] - dbar[q]; clb[q] = dbar[q]; }
  // the region tri_nearest took
  const float hgt = v3dot(v3sub(cl, a), bn) / v3dot(bn, bn);
  const V3 pp = {cl.x - hgt * bn.x, cl.y - hgt * bn.y, cl.z - hgt * bn.z};
  const bool in_a = v3dot(v3cross(v3sub(b, pp), v3sub(cc, pp)), bn) >= 0.f;
  const bool in_b = v3dot(v3cross(v3sub(cc, pp), v3sub(a, pp)), bn) >= 0.f;
  const bool in_c = v3dot(v3cross(v3sub(a, pp), v3sub(b, pp)), bn) >= 0.f;
  if (in_a && in_b && in_c) {
    const float nn = v3dot(bn, bn);
    const float pn = (bqb[0] * bn.x + bqb[1] * bn.y + bqb[2] * bn.z) / nn;
    clb[0] += bqb[0] - pn * bn.x; clb[1] += bqb[1] - pn * bn.y; clb[2] += bqb[2] - pn * bn.z;
  } else {
    // the edge seg_nearest kept: the first strictly nearest of ab, bc, ca
    const V3 s0s[3] = {a, b, cc}, s1s[3] = {b, cc, a};
    float best = INFINITY, tbest = 0.f;
    V3 ubest = {0.f, 0.f, 0.f};
    for (int e = 0; e < 3; e++) {
      const V3 u = v3sub(s1s[e], s0s[e]), w = v3sub(cl, s0s[e]);
      const float tt = fminf(fmaxf(v3dot(w, u) / v3dot(u, u), 0.f), 1.f);
      const V3 x = {s0s[e].x + tt * u.x, s0s[e].y + tt * u.y, s0s[e].z + tt * u.z};
      const V3 dx = v3sub(cl, x);
      const float dd = v3dot(dx, dx);
      if (dd < best) { best = dd; tbest = tt; ubest = u; }
    }
    if (tbest > 0.f && tbest < 1.f) {
      const float uu = v3dot(ubest, ubest);
      const float pu = (bqb[0] * ubest.x + bqb[1] * ubest.y + bqb[2] * ubest.z) / uu;
      clb[0] += pu * ubest.x; clb[1] += pu * ubest.y; clb[2] += pu * ubest.z;
    }
  }
  float cw[3];
  mv3(Rg, clb, cw);  // cl = Rg^T (c - xg)
  for (int q = 0; q < 3; q++) cb[q] += cw[q];
}

// seg_seg: parameters s, t of the closest points p0 + s d1, q0 + t d2; cotangents sb, tb
DEV void seg_seg_rev(const float* p0, const float* d1, const float* q0, const float* d2,
                     float sb, float tb, float* p0b, float* d1b, float* q0b, float* d2b) {
  const float r[3] = {p0[0] - q0[0], p0[1] - q0[1], p0[2] - q0[2]};
  const float a = dot3(d1, d1), e = dot3(d2, d2), f = dot3(d2, r), c = dot3(d1, r),
              b = dot3(d1, d2);
  const float den = a * e - b * b;
  auto inner = [](float x) { return x > 0.f && x < 1.f; };
  float ab_ = 0.f, eb = 0.f, fb = 0.f, cb = 0.f, bb = 0.f;
  if (den > 1e-6f * a * e) {
    const float s1 = (b * f - c * e) / den;
    const float s = fminf(fmaxf(s1, 0.f), 1.f);
    const float t1 = (b * s + f) / e;
    if (t1 < 0.f) {  // t = 0, s = clamp(-c / a)
      if (inner(-c / a)) { cb -= sb / a; ab_ += sb * c / (a * a); }
    } else if (t1 > 1.f) {  // t = 1, s = clamp((b - c) / a)
      const float s2 = (b - c) / a;
      if (inner(s2)) { bb += sb / a; cb -= sb / a; ab_ -= sb * s2 / a; }
    } else {  // t = (b s + f) / e, s = clamp(s1)
      bb += tb * s / e;
      fb += tb / e;
      eb -= tb * t1 / e;
      if (inner(s1)) {
        const float s1b = sb + tb * b / e;
        const float numb = s1b / den, denb = -s1b * s1 / den;
        bb += numb * f - 2.f * denb * b;
        fb += numb * b;
        cb -= numb * e;
        eb += denb * a - numb * c;
        ab_ += denb * e;
      }
    }
  } else {  // near-parallel: s the mean of the two end projections
    const float s0r = -c / a, s1r = (b - c) / a;
    const float s = 0.5f * (fminf(fmaxf(s0r, 0.f), 1.f) + fminf(fmaxf(s1r, 0.f), 1.f));
    const float tr = (b * s + f) / e;
    float sbt = sb;
    if (inner(tr)) { bb += tb * s / e; fb += tb / e; eb -= tb * tr / e; sbt += tb * b / e; }
    if (inner(s0r)) { cb -= 0.5f * sbt / a; ab_ += 0.5f * sbt * c / (a * a); }
    if (inner(s1r)) { bb += 0.5f * sbt / a; cb -= 0.5f * sbt / a; ab_ -= 0.5f * sbt * s1r / a; }
  }
  for (int k = 0; k < 3; k++) {
    const float rb = fb * d2[k] + cb * d1[k];
    d1b[k] += 2.f * ab_ * d1[k] + cb * r[k] + bb * d2[k];
    d2b[k] += 2.f * eb * d2[k] + fb * r[k] + bb * d1[k];
    p0b[k] += rb;
    q0b[k] -= rb;
  }
}

// contact rows: contact c's first row (con_nr c when every contact has con_nr rows,
// else packed in its record), and the contact a row belongs to
DEV int first_row(const DevModel& m, const float* rec, int c) {
  return m.con_nr ? m.con_nr * c : __float_as_int(rec[17]) >> 8;
}
DEV int contact_of_row(const DevModel& m, const float* con, int ncon, int r) {
  if (m.con_nr) return r / m.con_nr;
  int c = 0;
  while (c + 1 < ncon && (__float_as_int(con[kConRec * (c + 1) + 17]) >> 8) <= r) c++;
  return c;
}

// x <- (M + h diag(dof_vgain))^-1 x in place, the implicit integrators' matrix (nv <= T),
// with the dense factor in leaves-first (reversed) order as implicit_damping builds it;
// refactor = false solves with the factor already in o_H.
DEV void mhb_solve(const DevModel& m, float* W, const Team& t, float* x, bool refactor) {
  const int nv = m.nv;
  auto flip = [&]() {
    for (int i = t.lane; i < nv / 2; i += t.T) {
      const float v = x[i];
      x[i] = x[nv - 1 - i];
      x[nv - 1 - i] = v;
    }
    t.sync();
  };
  flip();
  if (refactor) {
    hessian_cholesky(m, W, t, 0, x, x, true, true);
    cholesky_back(m, W, t, x, x);
  } else {
    cholesky_solve(m, W, t, x, x, 1.f);
  }
  flip();
}

// Reverse sweep of the recursive Newton-Euler inverse dynamics: adds to Sbar, cinbar
// (and, unless still, vb) the cotangents of cot^T ID(q, qdot, acc).  still: zero
// velocity and no gravity, so that ID = M(q) acc and the sweep gives the cotangent of
// cot^T M(q) acc.
DEV void rne_reverse(const DevModel& m, float* W, const Team& t, const float* cot,
                     const float* acc, bool still) {
  const int nv = m.nv, nb = m.nbody;
  const float* qv0 = W + m.o_qvel;
  auto qv = [&](int i) { return still ? 0.f : qv0[i]; };
  float* vb = W + m.o_vb;
  const float* cdof = W + m.o_cdof;
  float* Sbar = W + m.o_Sbar;
  float* cinbar = W + m.o_cinbar;
  float* Vbar = W + m.o_Vbar;
  float* Abar = W + m.o_Abar;
  float* Fbar = W + m.o_Fbar;
  float* vup = W + m.o_vup;
  float* aup = W + m.o_aup;
  forward_sweep(m, W, t, acc, nullptr, still);
  accumulate_forces(m, W, t);
  const float* cvel = W + m.o_cvel;
  const float* cacc = W + m.o_cacc;
  const float* cfrc = W + m.o_cfrc;  // subtree totals
  const float* cin = W + m.o_cinert;
  // S_bar = mu_k F_body(k); F_bar(b) = sum_k in b mu_k S_k
  for (int k = t.lane; k < nv; k += t.T) {
    const int b = m.dof_body[k];
    for (int c = 0; c < 6; c++) Sbar[6 * k + c] += cot[k] * cfrc[6 * b + c];
  }
  for (int b = t.lane; b < nb; b += t.T) {
    float f[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int k = m.body_dofadr[b]; k < m.body_dofadr[b] + m.body_dofnum[b]; k++)
      for (int c = 0; c < 6; c++) f[c] += cot[k] * cdof[6 * k + c];
    for (int c = 0; c < 6; c++) Fbar[6 * b + c] = f[c];
  }
  t.sync();
  for (int lv = 1; lv < m.nlevel; lv++) {  // subtree totals: every ancestor's bar adds
    const int e = m.level_start[lv + 1];
    for (int ib = m.level_start[lv] + t.lane; ib < e; ib += t.T) {
      const int b = m.level_body[ib], p = m.body_parent[b];
      if (p > 0)
        for (int c = 0; c < 6; c++) Fbar[6 * b + c] += Fbar[6 * p + c];
    }
    t.sync();
  }
  // f = I A + V x* (I V), reversed (lane per body)
  for (int b = 1 + t.lane; b < nb; b += t.T) {
    const float* I = cin + kCinert * b;
    const float* V = cvel + 6 * b;
    const float* A = cacc + 6 * b;
    const float* fb = Fbar + 6 * b;
    float IV[6], t1[6], t2[6], t3[6];
    inertia_mul(I, fb, Abar + 6 * b);
    inertia_mul(I, V, IV);
    crossf(fb, IV, t1);
    crossm(V, fb, t2);
    inertia_mul(I, t2, t3);
    for (int c = 0; c < 6; c++) Vbar[6 * b + c] = -t1[c] - t3[c];
    float* ib = cinbar + kCinert * b;
    inertia_cot(ib, fb, A);
    for (int c = 0; c < 6; c++) t2[c] = -t2[c];
    inertia_cot(ib, t2, V);
  }
  t.sync();
  // V, A recursions reversed, leaves to root (lane per body; children pass up)
  for (int lv = m.nlevel - 1; lv >= 1; lv--) {
    const int e = m.level_start[lv + 1];
    for (int ib = m.level_start[lv] + t.lane; ib < e; ib += t.T) {
      const int b = m.level_body[ib], p = m.body_parent[b];
      float Vb_[6], Ab_[6];
      for (int c = 0; c < 6; c++) { Vb_[c] = Vbar[6 * b + c]; Ab_[c] = Abar[6 * b + c]; }
      for (int cc = m.child_start[b]; cc < m.child_start[b + 1]; cc++) {
        const int ch = m.child_list[cc];
        for (int c = 0; c < 6; c++) { Vb_[c] += vup[6 * ch + c]; Ab_[c] += aup[6 * ch + c]; }
      }
      // forward velocities inside the body (V after each joint)
      const int j0 = m.body_jntadr[b], nj = m.body_jntnum[b];
      float Vs[4][6];  // V after joint jj (bodies carry at most 4 scalar joints here)
      float V[6];
      for (int c = 0; c < 6; c++) V[c] = cvel[6 * p + c];
      const bool free = nj == 1 && m.jnt_type[j0] == JNT_FREE;
      if (!free) {
        for (int jj = 0; jj < nj && jj < 4; jj++) {
          const int da = m.jnt_dofadr[j0 + jj];
          for (int c = 0; c < 6; c++) { V[c] += cdof[6 * da + c] * qv(da); Vs[jj][c] = V[c]; }
        }
        for (int jj = nj - 1; jj >= 0; jj--) {
          const int da = m.jnt_dofadr[j0 + jj];
          const float* S = cdof + 6 * da;
          // A += Sd v + S a, Sd = V_k x S
          float Sdbar[6], Sd[6], tmp[6];
          crossm(Vs[jj < 4 ? jj : 3], S, Sd);
          for (int c = 0; c < 6; c++) {
            Sdbar[c] = qv(da) * Ab_[c];
            Sbar[6 * da + c] += acc[da] * Ab_[c];
          }
          if (!still) vb[da] += dot6(Sd, Ab_);
          crossf(S, Sdbar, tmp);
          for (int c = 0; c < 6; c++) Vb_[c] += tmp[c];
          crossf(Vs[jj < 4 ? jj : 3], Sdbar, tmp);
          for (int c = 0; c < 6; c++) Sbar[6 * da + c] += -tmp[c] + qv(da) * Vb_[c];
          if (!still) vb[da] += dot6(S, Vb_);
        }
      } else {
        const int da = m.jnt_dofadr[j0];
        for (int i = 0; i < 6; i++)
          for (int c = 0; c < 6; c++) V[c] += cdof[6 * (da + i) + c] * qv(da + i);
        for (int i = 0; i < 6; i++) {
          const float* S = cdof + 6 * (da + i);
          for (int c = 0; c < 6; c++) Sbar[6 * (da + i) + c] += acc[da + i] * Ab_[c];
          if (i >= 3) {
            float Sd[6], Sdbar[6], tmp[6];
            crossm(V, S, Sd);
            for (int c = 0; c < 6; c++) Sdbar[c] = qv(da + i) * Ab_[c];
            if (!still) vb[da + i] += dot6(Sd, Ab_);
            crossf(S, Sdbar, tmp);
            for (int c = 0; c < 6; c++) Vb_[c] += tmp[c];
            crossf(V, Sdbar, tmp);
            for (int c = 0; c < 6; c++) Sbar[6 * (da + i) + c] -= tmp[c];
          }
        }
        for (int i = 0; i < 6; i++) {
          const float* S = cdof + 6 * (da + i);
          for (int c = 0; c < 6; c++) Sbar[6 * (da + i) + c] += qv(da + i) * Vb_[c];
          if (!still) vb[da + i] += dot6(S, Vb_);
        }
      }
      for (int c = 0; c < 6; c++) { vup[6 * b + c] = Vb_[c]; aup[6 * b + c] = Ab_[c]; }
    }
    t.sync();
  }
}

// Directions of edge ed of a pyramid contact (record rec): the row is lin . v + ang . w
// for the relative point velocity v and angular velocity w.  Edges 0-3: n +- mu t_k;
// 4, 5 (condim 4): n and +- mu_t n (spin); 6-9 (condim 6): n and +- mu_r t_k (rolling).
// Returns the frame vector the angular part scales (0: n, 1: t1, 2: t2; -1: none) and
// its factor in sa.
DEV int edge_dirs(const DevModel& m, const float* rec, int ed, float* lin, float* ang,
                  float& sa) {
  const float* n = rec + 4;
  sa = 0.f;
  if (ed < 4) {
    const float sgm = (ed & 1) ? -rec[13] : rec[13];
    const float* tk = rec + 4 + 3 * (1 + (ed >> 1));
    for (int q = 0; q < 3; q++) { lin[q] = n[q] + sgm * tk[q]; ang[q] = 0.f; }
    return -1;
  }
  const int p = __float_as_int(rec[16]);
  const int f = ed < 6 ? 0 : 1 + ((ed - 6) >> 1);
  const float c = ed < 6 ? m.pair_mu_t[p] : m.pair_mu_r[p];
  sa = (ed & 1) ? -c : c;
  for (int q = 0; q < 3; q++) { lin[q] = n[q]; ang[q] = sa * rec[4 + 3 * f + q]; }
  return f;
}

// Reverse of qpos' = q0 (+) ch v (lane per joint), the position update of
// integrate_pos: gq is the cotangent of qpos'; q0b gets q0's (assigned, or added with
// `add`) and vb accumulates v's.  A free joint's rotation is q' = normalize(q0 (x)
// exp(ch w)), w its angular velocity; v is read through vel(dof).
template <class V>
DEV void integrate_pos_rev(const DevModel& m, const Team& t, const float* q0, V vel, float ch,
                           const float* gq, float* q0b, float* vb, bool add) {
  auto put = [&](int i, float x) { q0b[i] = add ? q0b[i] + x : x; };
  for (int j = t.lane; j < m.njnt; j += t.T) {
    const int qa = m.jnt_qposadr[j], da = m.jnt_dofadr[j];
    if (m.jnt_type[j] == JNT_FREE) {
      for (int k = 0; k < 3; k++) {
        put(qa + k, gq[qa + k]);
        vb[da + k] += ch * gq[qa + k];
      }
      float wv[3];
      for (int k = 0; k < 3; k++) wv[k] = ch * vel(da + 3 + k);
      const float th = sqrtf(dot3(wv, wv));
      float sn, cs;
      sincosf(0.5f * th, &sn, &cs);
      // f(th) = sin(th/2)/th and f'(th)/th; series below 0.1 (the closed form cancels)
      float fth, fpt;
      if (th > 0.1f) {
        fth = sn / th;
        fpt = (0.5f * th * cs - sn) / (th * th * th);
      } else {
        const float t2 = th * th;
        fth = 0.5f - t2 / 48.f + t2 * t2 / 3840.f;
        fpt = -1.f / 24.f + t2 / 960.f;
      }
      const float ds0 = -0.5f * fth;
      const float dq[4] = {cs, fth * wv[0], fth * wv[1], fth * wv[2]};
      const float quat[4] = {q0[qa + 3], q0[qa + 4], q0[qa + 5], q0[qa + 6]};
      float r[4];
      quat_mul4(quat, dq, r);
      const float rn = sqrtf(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
      const float qo[4] = {r[0] / rn, r[1] / rn, r[2] / rn, r[3] / rn};
      const float* g4 = gq + qa + 3;
      const float dotq = qo[0] * g4[0] + qo[1] * g4[1] + qo[2] * g4[2] + qo[3] * g4[3];
      float rbar[4];
      for (int k = 0; k < 4; k++) rbar[k] = (g4[k] - qo[k] * dotq) / rn;
      const float dqc[4] = {dq[0], -dq[1], -dq[2], -dq[3]};
      const float qc[4] = {quat[0], -quat[1], -quat[2], -quat[3]};
      float qq[4], dqbar[4];
      quat_mul4(rbar, dqc, qq);
      quat_mul4(qc, rbar, dqbar);
      for (int k = 0; k < 4; k++) put(qa + 3 + k, qq[k]);
      const float wd = wv[0] * dqbar[1] + wv[1] * dqbar[2] + wv[2] * dqbar[3];
      for (int k = 0; k < 3; k++) {
        const float wbar = dqbar[0] * ds0 * wv[k] + fth * dqbar[1 + k] + fpt * wd * wv[k];
        vb[da + 3 + k] += ch * wbar;
      }
    } else {
      put(qa, gq[qa]);
      vb[da] += ch * gq[qa];
    }
  }
}

// ------------------------------------------------------------------ adjoint step
// Inputs in LDS: qpos/qvel (state before the step), qacc (= a*), qbi/vbi (cotangents of
// the state after the step).  Outputs: qb (nq), vb (nv), ub (nu).  With abar_in (one
// stage of a Runge-Kutta step): a*'s cotangent is abar_in, and qb and vb receive the
// solve's cotangents only.  Status bit 4: the Hessian's factor failed.
DEV void adjoint_step(const DevModel& m, float* W, const Team& t, const float* u, int& status,
                      const float* abar_in = nullptr) {
  const int nv = m.nv, nb = m.nbody;
  const float h = m.dt;
  const int ncon = ((const int*)(W + m.o_scal))[SC_NCON];
  const int nrow = ((const int*)(W + m.o_scal))[SC_NROW];
  // contact rows (4 a condim-3 pyramid, 1 a frictionless contact); joint-limit rows
  // follow, then friction loss
  const int nrc = ((const int*)(W + m.o_scal))[SC_NRC];
  const int nrf = nrow - m.nfric - m.neqrow;  // first friction-loss row
  const int nre = nrow - m.neqrow;            // first equality row
  const int nl = nrf - nrc;
  const int* lim = (const int*)(W + m.o_lim);
  const float* fl = W + m.o_fl;
  const float* qpos = W + m.o_qpos;
  const float* qvel = W + m.o_qvel;
  const float* a = W + m.o_qacc;
  const float* qbi = W + m.o_qbi;
  const float* vbi = W + m.o_vbi;
  float* qb = W + m.o_qb;
  float* vb = W + m.o_vb;
  float* ub = W + m.o_ub;
  float* mu = W + m.o_mu;
  float* abar = W + m.o_g;  // scratch of the forward solve, free now
  const float* cdof = W + m.o_cdof;
  float* Sbar = W + m.o_Sbar;
  float* xbar = W + m.o_xbar;
  float* Rbar = W + m.o_Rbar;
  float* cinbar = W + m.o_cinbar;
  float* Vbar = W + m.o_Vbar;
  float* Abar = W + m.o_Abar;
  float* Fbar = W + m.o_Fbar;
  float* vup = W + m.o_vup;
  float* aup = W + m.o_aup;
  float* xup = W + m.o_xup;
  float* Rup = W + m.o_Rup;

  // ---- clear body accumulators
  for (int k = t.lane; k < 3 * nb; k += t.T) xbar[k] = 0.f;
  for (int k = t.lane; k < 9 * nb; k += t.T) Rbar[k] = 0.f;
  for (int k = t.lane; k < kCinert * nb; k += t.T) cinbar[k] = 0.f;
  for (int k = t.lane; k < 6 * nv; k += t.T) Sbar[k] = 0.f;
  for (int k = t.lane; k < m.nu; k += t.T) ub[k] = 0.f;
  // ---- implicit integrators: qvel' = qvel + h a_int, (M + h B) a_int = M a* - c qdot
  // (the converged solve's smooth and row forces sum to M a*; B = diag(dof_vgain), c =
  // dof_hkp for integrator 2, else 0)
  const bool imp = m.implicit != 0;
  const float* M = W + m.o_M;
  float* ai = W + m.o_d;  // a_int, later a* - a_int
  float* y = W + m.o_Md;  // (M + h B)^-1 a_int_bar
  if (imp) {
    for (int i = t.lane; i < nv; i += t.T) {
      float v = m.implicit == 2 ? -m.dof_hkp[i] * qvel[i] : 0.f;
      v += sym_row_dot(M, i, a, nv);
      ai[i] = v;
    }
    t.sync();
    mhb_solve(m, W, t, ai, true);
  }
  const float* av = imp ? ai : a;  // the acceleration of the velocity update
  if (abar_in) {
    // one stage of a Runge-Kutta step: the solve's cotangents alone (the stage loop
    // around this call reverses the stage states and the final combination)
    for (int i = t.lane; i < m.nq; i += t.T) qb[i] = 0.f;
    for (int i = t.lane; i < nv; i += t.T) {
      vb[i] = 0.f;
      abar[i] = abar_in[i];
    }
    t.sync();
  } else {
    // ---- semi-implicit Euler, reversed: qvel' = qvel + h a, qpos' = qpos (+) h qvel'
    for (int i = t.lane; i < nv; i += t.T) vb[i] = vbi[i];
    t.sync();
    integrate_pos_rev(m, t, qpos, [&](int i) { return qvel[i] + h * av[i]; }, h, qbi, qb, vb,
                      false);
    t.sync();
    for (int i = t.lane; i < nv; i += t.T) abar[i] = h * vb[i];
  }
  if (imp) {
    // a_int's cotangent: y = (M + h B)^-1 a_int_bar; then a* gets M y, qdot gets -c y,
    // and M(q) the outer product y (a* - a_int)^T (its sweep below)
    t.sync();
    for (int i = t.lane; i < nv; i += t.T) y[i] = abar[i];
    t.sync();
    mhb_solve(m, W, t, y, false);
    for (int i = t.lane; i < nv; i += t.T) {
      if (m.implicit == 2) vb[i] -= m.dof_hkp[i] * y[i];
      const float v = sym_row_dot(M, i, y, nv);
      abar[i] = v;
      ai[i] = a[i] - ai[i];
    }
    t.sync();
  }
  // ---- implicit differentiation: lambda = H(a*)^-1 a_bar, mu = -lambda
  {
    const float* aref = W + m.o_aref;
    float* e = W + m.o_e;
    const RowBounds rb = pad_rows(m, W, t, nrow);
    rows_times(m, W, t, nrow, rb, a, e);
    for (int r = t.lane; r < nrow; r += t.T) e[r] -= aref[r];
    t.sync();
    if (!hessian_cholesky(m, W, t, rb.nru, nullptr, nullptr, false, false, nullptr, false,
                          rb.nou))
      status |= 4;
    cholesky_solve(m, W, t, abar, mu, -1.f);
  }
  // ---- actuation and passive forces, reversed (lane per dof)
  for (int i = t.lane; i < nv; i += t.T) {
    const float mi = mu[i];
    vb[i] += m.dof_damping[i] * mi;
    const int ac = m.dof_act[i];
    if (ac >= 0) {
      const float c = u ? u[ac] : 0.f;
      const bool inr = c >= m.act_lo[ac] && c <= m.act_hi[ac];
      if (m.act_type[ac] == ACT_MOTOR) {
        ub[ac] = inr ? -m.act_gear[ac] * mi : 0.f;
      } else {
        ub[ac] = inr ? -m.act_kp[ac] * m.act_gear[ac] * mi : 0.f;
        vb[i] += m.act_kd[ac] * mi;
      }
    }
  }
  t.sync();
  for (int i = t.lane; i < nv; i += t.T) {  // PD stiffness acts on qpos (separate pass:
    const int ac = m.dof_act[i];             // qb of a hinge is one word per lane)
    if (ac >= 0 && m.act_type[ac] == ACT_PD) qb[m.act_qadr[ac]] += m.act_kp[ac] * mu[i];
  }
  // ---- inverse dynamics with a*, reversed (implicit integrators: first y^T M(q) (a* - a_int))
  if (imp) rne_reverse(m, W, t, y, ai, true);
  rne_reverse(m, W, t, mu, a, false);
  // ---- contact rows, reversed
  if (nrow > 0) {
    const float* D = W + m.o_D;
    const float* e = W + m.o_e;
    const float* con = W + m.o_con;
    float* rs = W + m.o_rowsc;   // per row: s, x, y, alpha, beta, gamma, rho
    float* cs = W + m.o_consc;   // per contact: kConSc words (below)
    for (int r = t.lane; r < nrow; r += t.T) {
      float sv = 0.f, xv = 0.f, yv = 0.f;
      for (int i = 0; i < nv; i++) {
        const float jr = row_entry(m, W, r, i, ncon);
        sv += jr * mu[i]; xv += jr * qvel[i]; yv += jr * a[i];
      }
      float al = 0.f, be = 0.f, ga = 0.f, rho = 0.f;
      // rows on their quadratic piece; a friction row on a linear piece has the constant
      // slope +-F and carries no cotangent
      if (row_quad(D[r], r < nrf ? 0.f : fl[r], e[r])) {
        float dist = 0.f;  // friction loss: r = 0, not a function of the state
        if (r < nrc) {
          dist = con[kConRec * contact_of_row(m, con, ncon, r)];
        } else if (r < nrf) {
          int dof;
          float sg;
          limit_row(m, W, lim[r - nrc], dof, sg, dist);
        } else if (r >= nre) {  // equality: the residual's component
          const int q = m.eq_row[r - nre] & 0xffff, k = m.eq_row[r - nre] >> 16;
          if (k < 3) {
            float p1[3], p2[3];
            eq_points(m, W, q, p1, p2);
            dist = p1[k] - p2[k];
          } else {
            dist = weld_residual(m, W, q, k - 3);
          }
        }
        float d, dd;
        impedance_d(m, dist, d, dd);
        const float Dv = D[r];
        const float Ahat = d / ((1.f - d) * Dv);
        const float Dp = dd / ((1.f - d) * (1.f - d) * Ahat);
        const float core = m.B * xv + m.K * d * dist + yv;
        al = Dv * core;
        be = m.B * Dv * sv;
        ga = Dv * sv;
        rho = (r < nrf || r >= nre) ? sv * (Dp * core + Dv * m.K * (dd * dist + d)) : 0.f;
      }
      float* o = rs + 7 * r;
      o[0] = sv; o[1] = xv; o[2] = yv; o[3] = al; o[4] = be; o[5] = ga; o[6] = rho;
    }
    t.sync();
    // dofs: qvel cotangent through aref, and the Jacobian's subspace cotangents
    for (int k = t.lane; k < nv; k += t.T) {
      const unsigned long long bit = 1ull << k;
      float vadd = 0.f;
      float sb[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      for (int r = 0; r < nrow; r++) {
        const float* o = rs + 7 * r;
        if (!row_quad(D[r], r < nrf ? 0.f : fl[r], e[r])) continue;
        vadd += o[4] * row_entry(m, W, r, k, ncon);
        if (r >= nre) {  // equality: J_p(b1, p1) - J_p(b2, p2), or J_w(b1) - J_w(b2)
          const int q = m.eq_row[r - nre] & 0xffff, kk = m.eq_row[r - nre] >> 16;
          const bool in1 = (m.body_dofmask[m.eq_body[2 * q]] & bit) != 0;
          const bool in2 = (m.body_dofmask[m.eq_body[2 * q + 1]] & bit) != 0;
          const float w = o[3] * mu[k] + o[4] * qvel[k] + o[5] * a[k];
          if (kk < 3) {
            float p1[3], p2[3];
            eq_points(m, W, q, p1, p2);
            // e_kk . (S_lin + S_ang x p) = S_lin[kk] + S_ang . (p x e_kk)
            const float pe1[3] = {kk == 2 ? p1[1] : (kk == 1 ? -p1[2] : 0.f),
                                  kk == 0 ? p1[2] : (kk == 2 ? -p1[0] : 0.f),
                                  kk == 1 ? p1[0] : (kk == 0 ? -p1[1] : 0.f)};
            const float pe2[3] = {kk == 2 ? p2[1] : (kk == 1 ? -p2[2] : 0.f),
                                  kk == 0 ? p2[2] : (kk == 2 ? -p2[0] : 0.f),
                                  kk == 1 ? p2[0] : (kk == 0 ? -p2[1] : 0.f)};
            const float s1 = in1 ? w : 0.f, s2 = in2 ? w : 0.f;
            for (int c = 0; c < 3; c++) sb[c] += s1 * pe1[c] - s2 * pe2[c];
            sb[3 + kk] += s1 - s2;
          } else {
            sb[kk - 3] += (in1 ? w : 0.f) - (in2 ? w : 0.f);
          }
          continue;
        }
        if (r >= nrc) continue;  // limit and friction rows: constant Jacobians
        const int cr = contact_of_row(m, con, ncon, r);
        const float* rec = con + kConRec * cr;
        const int b1 = __float_as_int(rec[14]), b2 = __float_as_int(rec[15]);
        const bool in2 = (m.body_dofmask[b2] & bit) != 0, in1 = (m.body_dofmask[b1] & bit) != 0;
        if (in1 == in2) continue;
        const float sg = in2 ? 1.f : -1.f;
        const int ed = r - first_row(m, rec, cr);  // (mu = 0: one row, along n)
        float ev[3], ew[3], sa;
        edge_dirs(m, rec, ed, ev, ew, sa);
        const float w = sg * (o[3] * mu[k] + o[4] * qvel[k] + o[5] * a[k]);
        float pe[3];
        cross3(rec + 1, ev, pe);
        for (int c = 0; c < 3; c++) { sb[c] += w * (pe[c] + ew[c]); sb[3 + c] += w * ev[c]; }
      }
      vb[k] += vadd;
      for (int c = 0; c < 6; c++) Sbar[6 * k + c] += sb[c];
    }
    // contacts: cotangents of each contact's point, normal and distance, reversed through
    // its geometry to points fixed on its bodies (record: four points, each a world-frame
    // cotangent and its body-frame position; points 0-1 on body 1, 2-3 on body 2)
    for (int c = t.lane; c < ncon; c += t.T) {
      const float* rec = con + kConRec * c;
      const int b1 = __float_as_int(rec[14]), b2 = __float_as_int(rec[15]);
      const int p = __float_as_int(rec[16]), sub = __float_as_int(rec[17]) & 15;
      const int kind = m.pair_kind[p];
      const bool plane = kind == PK_PLANE_SPHERE || kind == PK_PLANE_CAPSULE || kind == PK_PLANE_BOX;
      float xb[3] = {0.f, 0.f, 0.f}, rb = 0.f;
      float fb[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};  // of n, t1, t2
      const int first = first_row(m, rec, c);
      const int nr = m.con_nr ? m.con_nr : (__float_as_int(rec[17]) >> 4) & 15;
      for (int ed = 0; ed < nr; ed++) {
        const int r = first + ed;
        if (!(e[r] < 0.f)) continue;
        const float* o = rs + 7 * r;
        rb += o[6];
        float ev[3], ew[3], sa;
        const int fa = edge_dirs(m, rec, ed, ev, ew, sa);
        float om[3] = {0.f, 0.f, 0.f}, ln[3] = {0.f, 0.f, 0.f};
        for (int k = 0; k < nv; k++) {
          const unsigned long long bit = 1ull << k;
          const bool in2 = (m.body_dofmask[b2] & bit) != 0, in1 = (m.body_dofmask[b1] & bit) != 0;
          if (in1 == in2) continue;
          const float w = (in2 ? 1.f : -1.f) * (o[3] * mu[k] + o[4] * qvel[k] + o[5] * a[k]);
          for (int q = 0; q < 3; q++) {
            om[q] += cdof[6 * k + q] * w;
            ln[q] += cdof[6 * k + 3 + q] * w;
          }
        }
        float x3[3];
        cross3(ev, om, x3);
        for (int q = 0; q < 3; q++) xb[q] += x3[q];
        if (!plane) {  // the frame moves: the linear direction's cotangent ln + om x pos,
                       // the angular direction's om
          float op[3];
          cross3(om, rec + 1, op);
          const float sgm = (ed & 1) ? -rec[13] : rec[13];
          for (int q = 0; q < 3; q++) {
            const float g = ln[q] + op[q];
            fb[q] += g;
            if (ed < 4) fb[3 + 3 * (ed >> 1) + q] += sgm * g;
            if (fa >= 0) fb[3 * fa + q] += sa * om[q];
          }
        }
      }
      float* o = cs + kConSc * c;
      for (int q = 0; q < 24; q++) o[q] = 0.f;
      o[24] = __int_as_float(b1);
      o[25] = __int_as_float(b2);
      o[26] = 1.f;
      const int g1 = m.pair_g1[p], g2 = m.pair_g2[p];
      // body-frame point of geom g on its axis at offset sh (0: the centre)
      auto local = [&](int k, int g, float sh) {
        const float* L = m.geom_rot + 9 * g;
        for (int q = 0; q < 3; q++) o[6 * k + 3 + q] = m.geom_pos[3 * g + q] + sh * L[3 * q + 2];
      };
      if (plane) {
        // pos = c - n (R + r/2), r = n . (c - p0) - R, c the sphere centre, capsule end
        // or box corner (R = 0)
        const float* n = rec + 4;
        const float nx = dot3(n, xb);
        for (int q = 0; q < 3; q++) o[12 + q] = xb[q] - 0.5f * n[q] * nx + rb * n[q];
        if (kind == PK_PLANE_BOX) {  // corner `sub`: bit k takes +half-size k, else -
          const float* L = m.geom_rot + 9 * g2;
          const float* hs = m.geom_size + 3 * g2;
          const float loc[3] = {(sub & 1) ? hs[0] : -hs[0], (sub & 2) ? hs[1] : -hs[1],
                                (sub & 4) ? hs[2] : -hs[2]};
          for (int q = 0; q < 3; q++)
            o[15 + q] = m.geom_pos[3 * g2 + q] + L[3 * q] * loc[0] + L[3 * q + 1] * loc[1] +
                        L[3 * q + 2] * loc[2];
        } else {
          local(2, g2, kind == PK_PLANE_CAPSULE ? (sub == 0 ? -1.f : 1.f) * m.geom_size[3 * g2 + 1]
                                                : 0.f);
        }
      } else if (kind == PK_SPHERE_SPHERE || kind == PK_SPHERE_CAPSULE ||
                 kind == PK_CAPSULE_CAPSULE) {
        float nb[3] = {fb[0], fb[1], fb[2]};
        frame_rev(rec + 4, rec + 7, fb + 3, fb + 6, nb);
        float x1[3], R1[9], x2[3], R2[9];
        geom_pose(m, W, g1, x1, R1);
        geom_pose(m, W, g2, x2, R2);
        const float r1 = m.geom_size[3 * g1], r2 = m.geom_size[3 * g2];
        const float h1 = m.geom_size[3 * g1 + 1], h2 = m.geom_size[3 * g2 + 1];
        // the capsules' segments: start a, direction u (end a + u)
        float a1[3], u1[3], a2[3], u2[3];
        for (int q = 0; q < 3; q++) {
          a1[q] = x1[q] - h1 * R1[3 * q + 2]; u1[q] = 2.f * h1 * R1[3 * q + 2];
          a2[q] = x2[q] - h2 * R2[3 * q + 2]; u2[q] = 2.f * h2 * R2[3 * q + 2];
        }
        if (kind == PK_SPHERE_SPHERE) {
          sphere_sphere_rev(x1, r1, x2, r2, xb, nb, rb, o, o + 12);
          local(0, g1, 0.f);
          local(2, g2, 0.f);
        } else if (kind == PK_SPHERE_CAPSULE) {
          const float uu = dot3(u2, u2);
          const float ap[3] = {x1[0] - a2[0], x1[1] - a2[1], x1[2] - a2[2]};
          const float tq = uu < 1e-30f ? 0.f : fminf(fmaxf(dot3(ap, u2) / uu, 0.f), 1.f);
          const float qq[3] = {a2[0] + tq * u2[0], a2[1] + tq * u2[1], a2[2] + tq * u2[2]};
          float qb[3] = {0.f, 0.f, 0.f}, ab[3] = {0.f, 0.f, 0.f}, ub[3] = {0.f, 0.f, 0.f};
          sphere_sphere_rev(x1, r1, qq, r2, xb, nb, rb, o, qb);
          seg_point_rev(x1, a2, u2, qb, o, ab, ub);
          for (int q = 0; q < 3; q++) { o[12 + q] = ab[q] - ub[q]; o[18 + q] = ub[q]; }
          local(0, g1, 0.f);
          local(2, g2, -h2);
          local(3, g2, h2);
        } else {
          float sp, tp;
          seg_seg(a1, u1, a2, u2, sp, tp);
          const float pp[3] = {a1[0] + sp * u1[0], a1[1] + sp * u1[1], a1[2] + sp * u1[2]};
          const float qq[3] = {a2[0] + tp * u2[0], a2[1] + tp * u2[1], a2[2] + tp * u2[2]};
          float ppb[3] = {0.f, 0.f, 0.f}, qqb[3] = {0.f, 0.f, 0.f};
          sphere_sphere_rev(pp, r1, qq, r2, xb, nb, rb, ppb, qqb);
          float ab[3], ub[3], bb[3], wb[3];
          for (int q = 0; q < 3; q++) {
            ab[q] = ppb[q]; ub[q] = sp * ppb[q];
            bb[q] = qqb[q]; wb[q] = tp * qqb[q];
          }
          seg_seg_rev(a1, u1, a2, u2, dot3(ppb, u1), dot3(qqb, u2), ab, ub, bb, wb);
          for (int q = 0; q < 3; q++) {
            o[q] = ab[q] - ub[q]; o[6 + q] = ub[q];
            o[12 + q] = bb[q] - wb[q]; o[18 + q] = wb[q];
          }
          local(0, g1, -h1);
          local(1, g1, h1);
          local(2, g2, -h2);
          local(3, g2, h2);
        }
      } else if (kind == PK_SPHERE_HFIELD) {
        float nb[3] = {fb[0], fb[1], fb[2]};
        frame_rev(rec + 4, rec + 7, fb + 3, fb + 6, nb);
        float x1[3], R1[9], x2[3], R2[9];
        geom_pose(m, W, g1, x1, R1);
        geom_pose(m, W, g2, x2, R2);
        const float* cpar = W + m.o_cand + m.ncand;  // the winning triangle per candidate
        const int code = __float_as_int(cpar[m.pair_candadr[p] + (sub & 15)]);
        sphere_hfield_rev(m, x2, R2, x1, m.geom_size[3 * g1], code, xb, nb, rb, o);
        local(0, g1, 0.f);
      } else {
        o[26] = 0.f;  // geometry not differentiated (the rollout refuses such models)
      }
    }
    // equalities (lane per constraint): the anchors' cotangents, from the residual (its
    // distance cotangent) and the translational Jacobians (their dependence on the
    // anchors: p_bar = e_k x sum_dofs w S_ang), and the weld rotation residual's
    // cotangents of the two bodies' rotations: r = (E_ij - E_ji) / 2, E = R1 Q R2^T
    float* eqs = W + m.o_eqsc;
    for (int q = t.lane; q < m.neq; q += t.T) {
      float* o = eqs + kEqSc * q;  // p1_bar [3], p2_bar [3], R1_bar [9], R2_bar [9]
      for (int c = 0; c < kEqSc; c++) o[c] = 0.f;
      const int b1 = m.eq_body[2 * q], b2 = m.eq_body[2 * q + 1];
      const float* R1 = W + m.o_xmat + 9 * b1;
      const float* R2 = W + m.o_xmat + 9 * b2;
      const float* Q = m.eq_relR + 9 * q;
      for (int er = 0; er < m.neqrow; er++) {
        if ((m.eq_row[er] & 0xffff) != q) continue;
        const int kk = m.eq_row[er] >> 16, r = nre + er;
        const float* ro = rs + 7 * r;
        if (kk < 3) {
          float om1[3] = {0.f, 0.f, 0.f}, om2[3] = {0.f, 0.f, 0.f};
          for (int k = 0; k < nv; k++) {
            const unsigned long long bit = 1ull << k;
            const float w = ro[3] * mu[k] + ro[4] * qvel[k] + ro[5] * a[k];
            const bool in1 = (m.body_dofmask[b1] & bit) != 0, in2 = (m.body_dofmask[b2] & bit) != 0;
            for (int c = 0; c < 3; c++) {
              if (in1) om1[c] += w * cdof[6 * k + c];
              if (in2) om2[c] += w * cdof[6 * k + c];
            }
          }
          // d/dp of e . (S_ang x p) = e x S_ang; the residual p1 - p2 adds +-rho e
          const float ek[3] = {kk == 0 ? 1.f : 0.f, kk == 1 ? 1.f : 0.f, kk == 2 ? 1.f : 0.f};
          float x1[3], x2[3];
          cross3(ek, om1, x1);
          cross3(ek, om2, x2);
          for (int c = 0; c < 3; c++) {
            o[c] += x1[c] + ro[6] * ek[c];
            o[3 + c] += -x2[c] - ro[6] * ek[c];
          }
        } else {
          const int k3 = kk - 3;
          const int i = k3 == 0 ? 2 : (k3 == 1 ? 0 : 1), j = k3 == 0 ? 1 : (k3 == 1 ? 2 : 0);
          const float hr = 0.5f * ro[6];
          // dE_ij/dR1[i][a] = (Q R2^T)[a][j], dE_ij/dR2[j][b] = (R1 Q)[i][b]
          for (int aa = 0; aa < 3; aa++) {
            float qj = 0.f, qi = 0.f, ri = 0.f, rj = 0.f;
            for (int bb = 0; bb < 3; bb++) {
              qj += Q[3 * aa + bb] * R2[3 * j + bb];
              qi += Q[3 * aa + bb] * R2[3 * i + bb];
              ri += R1[3 * i + bb] * Q[3 * bb + aa];
              rj += R1[3 * j + bb] * Q[3 * bb + aa];
            }
            o[6 + 3 * i + aa] += hr * qj;
            o[6 + 3 * j + aa] -= hr * qi;
            o[15 + 3 * j + aa] += hr * ri;
            o[15 + 3 * i + aa] -= hr * rj;
          }
        }
      }
    }
    // joint limits: the distance cotangent goes to the joint coordinate, r = +-(q - end)
    for (int k = t.lane; k < nl; k += t.T) {
      int dof;
      float sg, dist;
      limit_row(m, W, lim[k], dof, sg, dist);
      qb[m.lim_qadr[lim[k] & 0xffff]] += sg * rs[7 * (nrc + k) + 6];
    }
    t.sync();
    for (int b = 1 + t.lane; b < nb; b += t.T) {
      for (int q = 0; q < m.neq; q++) {  // anchors p = x_b + R_b l and the weld rotations
        const float* o = eqs + kEqSc * q;
        for (int s2 = 0; s2 < 2; s2++) {
          if (m.eq_body[2 * q + s2] != b) continue;
          const float* pb = o + 3 * s2;
          const float* l = m.eq_anchor + 6 * q + 3 * s2;
          for (int c = 0; c < 3; c++) {
            xbar[3 * b + c] += pb[c];
            for (int k2 = 0; k2 < 3; k2++) Rbar[9 * b + 3 * c + k2] += pb[c] * l[k2];
          }
          for (int c = 0; c < 9; c++) Rbar[9 * b + c] += o[6 + 9 * s2 + c];
        }
      }
      for (int c = 0; c < ncon; c++) {
        const float* o = cs + kConSc * c;
        for (int k = 0; k < 4; k++) {
          if (__float_as_int(o[k < 2 ? 24 : 25]) != b) continue;
          const float* pt = o + 6 * k;  // point = x_b + R_b l: x_b gets pt, R_b gets pt l^T
          for (int q = 0; q < 3; q++) {
            xbar[3 * b + q] += pt[q];
            for (int k2 = 0; k2 < 3; k2++) Rbar[9 * b + 3 * q + k2] += pt[q] * pt[3 + k2];
          }
        }
      }
    }
    int bad = 0;
    for (int c = t.lane; c < ncon; c += t.T) bad |= (cs[kConSc * c + 26] == 0.f);
    if (t.isum(bad)) status |= 8;
  }
  t.sync();
  // ---- body inertias -> body poses (lane per body)
  for (int b = 1 + t.lane; b < nb; b += t.T) {
    const float* xp = W + m.o_xpos + 3 * b;
    const float* R = W + m.o_xmat + 9 * b;
    const float mass = m.body_mass[b];
    const float* ipos = m.body_ipos + 3 * b;
    float c[3];
    mv3(R, ipos, c);
    for (int q = 0; q < 3; q++) c[q] += xp[q];
    const float* ib = cinbar + kCinert * b;
    const float Ib[9] = {ib[4], ib[7], ib[8], ib[7], ib[5], ib[9], ib[8], ib[9], ib[6]};
    const float tr = ib[4] + ib[5] + ib[6];
    float Ic[3];
    mv3(Ib, c, Ic);
    float cb[3];
    for (int q = 0; q < 3; q++) cb[q] = mass * ib[1 + q] + mass * (2.f * tr * c[q] - 2.f * Ic[q]);
    const float* bi = m.body_inertia + 6 * b;
    const float Il[9] = {bi[0], bi[3], bi[4], bi[3], bi[1], bi[5], bi[4], bi[5], bi[2]};
    float T1[9], T2[9];
    mm3(Ib, R, T1);
    mm3(T1, Il, T2);
    for (int q = 0; q < 3; q++) {
      xbar[3 * b + q] += cb[q];
      for (int k = 0; k < 3; k++) Rbar[9 * b + 3 * q + k] += 2.f * T2[3 * q + k] + cb[q] * ipos[k];
    }
  }
  t.sync();
  // ---- forward kinematics, reversed (leaves to root; children pass up)
  for (int lv = m.nlevel - 1; lv >= 1; lv--) {
    const int e = m.level_start[lv + 1];
    for (int ib = m.level_start[lv] + t.lane; ib < e; ib += t.T) {
      const int b = m.level_body[ib];
      float xb[3], Rb[9];
      for (int q = 0; q < 3; q++) xb[q] = xbar[3 * b + q];
      for (int q = 0; q < 9; q++) Rb[q] = Rbar[9 * b + q];
      for (int cc = m.child_start[b]; cc < m.child_start[b + 1]; cc++) {
        const int ch = m.child_list[cc];
        for (int q = 0; q < 3; q++) xb[q] += xup[3 * ch + q];
        for (int q = 0; q < 9; q++) Rb[q] += Rup[9 * ch + q];
      }
      const int j0 = m.body_jntadr[b], nj = m.body_jntnum[b];
      if (nj == 1 && m.jnt_type[j0] == JNT_FREE) {
        const int qa = m.jnt_qposadr[j0], da = m.jnt_dofadr[j0];
        const float* R1 = W + m.o_xmat + 9 * b;
        const float* x1 = W + m.o_xpos + 3 * b;
        for (int q = 0; q < 3; q++) qb[qa + q] += xb[q];
        for (int i = 0; i < 3; i++) {
          const float* Sb = Sbar + 6 * (da + 3 + i);
          const float r[3] = {R1[i], R1[3 + i], R1[6 + i]};
          float t1[3], t2[3];
          cross3(Sb + 3, x1, t1);
          cross3(r, Sb + 3, t2);
          for (int q = 0; q < 3; q++) {
            Rb[3 * q + i] += Sb[q] + t1[q];
            qb[qa + q] += t2[q];
          }
        }
        float qq[4] = {qpos[qa + 3], qpos[qa + 4], qpos[qa + 5], qpos[qa + 6]};
        const float nrm = sqrtf(qq[0] * qq[0] + qq[1] * qq[1] + qq[2] * qq[2] + qq[3] * qq[3]);
        const float w = qq[0] / nrm, x = qq[1] / nrm, y = qq[2] / nrm, z = qq[3] / nrm;
        const float dW[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
        const float dX[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
        const float dY[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
        const float dZ[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
        float qn[4] = {0.f, 0.f, 0.f, 0.f};
        for (int q = 0; q < 9; q++) {
          qn[0] += Rb[q] * dW[q]; qn[1] += Rb[q] * dX[q];
          qn[2] += Rb[q] * dY[q]; qn[3] += Rb[q] * dZ[q];
        }
        const float dot = w * qn[0] + x * qn[1] + y * qn[2] + z * qn[3];
        const float un[4] = {w, x, y, z};
        for (int q = 0; q < 4; q++) qb[qa + 3 + q] += (qn[q] - un[q] * dot) / nrm;
        for (int q = 0; q < 3; q++) xup[3 * b + q] = 0.f;
        for (int q = 0; q < 9; q++) Rup[9 * b + q] = 0.f;
        continue;
      }
      // frames before each joint, recomputed from the parent pose
      float xs[4][3], Rs[4][9];
      float pos[3], R[9];
      body_base(m, W, b, pos, R);
      for (int jj = 0; jj < nj && jj < 4; jj++) {
        const int j = j0 + jj, qa = m.jnt_qposadr[j];
        for (int q = 0; q < 3; q++) xs[jj][q] = pos[q];
        for (int q = 0; q < 9; q++) Rs[jj][q] = R[q];
        float ax[3];
        mv3(R, m.jnt_axis + 3 * j, ax);
        if (m.jnt_type[j] == JNT_SLIDE) {
          for (int q = 0; q < 3; q++) pos[q] += ax[q] * qpos[qa];
        } else {
          float off[3], anc[3], Rj[9];
          mv3(R, m.jnt_pos + 3 * j, off);
          for (int q = 0; q < 3; q++) anc[q] = pos[q] + off[q];
          axis_rot(m.jnt_axis + 3 * j, qpos[qa], Rj);  // R Rot(a, q) = Rot(R a, q) R
          mm3(R, Rj, R);
          mv3(R, m.jnt_pos + 3 * j, off);
          for (int q = 0; q < 3; q++) pos[q] = anc[q] - off[q];
        }
      }
      for (int jj = (nj < 4 ? nj : 4) - 1; jj >= 0; jj--) {
        const int j = j0 + jj, qa = m.jnt_qposadr[j], da = m.jnt_dofadr[j];
        const float* R0 = Rs[jj];
        const float* ev = m.jnt_axis + 3 * j;
        const float* Sb = Sbar + 6 * da;
        float ax[3];
        mv3(R0, ev, ax);
        if (m.jnt_type[j] == JNT_SLIDE) {
          float axb[3];
          for (int q = 0; q < 3; q++) axb[q] = Sb[3 + q] + qpos[qa] * xb[q];
          qb[qa] += dot3(ax, xb);
          for (int q = 0; q < 3; q++)
            for (int k = 0; k < 3; k++) Rb[3 * q + k] += axb[q] * ev[k];
        } else {
          const float* ap = m.jnt_pos + 3 * j;
          float off[3], anc[3], Rj[9];
          mv3(R0, ap, off);
          for (int q = 0; q < 3; q++) anc[q] = xs[jj][q] + off[q];
          axis_rot(ax, qpos[qa], Rj);
          float ancb[3], axb[3], t1[3];
          cross3(ax, Sb + 3, ancb);
          for (int q = 0; q < 3; q++) ancb[q] += xb[q];
          cross3(Sb + 3, anc, t1);
          for (int q = 0; q < 3; q++) axb[q] = Sb[q] + t1[q];
          float R1b[9];
          for (int q = 0; q < 3; q++)
            for (int k = 0; k < 3; k++) R1b[3 * q + k] = Rb[3 * q + k] - xb[q] * ap[k];
          // R1 = Rj R0: Rj_bar = R1b R0^T, R0_bar = Rj^T R1b
          float Rjb[9], R0b[9];
          for (int q = 0; q < 3; q++)
            for (int k = 0; k < 3; k++) {
              float s1 = 0.f, s2 = 0.f;
              for (int l = 0; l < 3; l++) {
                s1 += R1b[3 * q + l] * R0[3 * k + l];
                s2 += Rj[3 * l + q] * R1b[3 * l + k];
              }
              Rjb[3 * q + k] = s1;
              R0b[3 * q + k] = s2;
            }
          float SR[9];
          skew_mul(ax, Rj, SR);
          float qsum = 0.f;
          for (int q = 0; q < 9; q++) qsum += Rjb[q] * SR[q];
          qb[qa] += qsum;
          float sq, cq;
          sincosf(qpos[qa], &sq, &cq);
          const float v2[3] = {Rjb[7] - Rjb[5], Rjb[2] - Rjb[6], Rjb[3] - Rjb[1]};
          for (int q = 0; q < 3; q++) {
            float sa = 0.f;
            for (int k = 0; k < 3; k++) sa += (Rjb[3 * q + k] + Rjb[3 * k + q]) * ax[k];
            axb[q] += sq * v2[q] + (1.f - cq) * sa;
          }
          for (int q = 0; q < 3; q++) xb[q] = ancb[q];
          for (int q = 0; q < 3; q++)
            for (int k = 0; k < 3; k++)
              Rb[3 * q + k] = R0b[3 * q + k] + ancb[q] * ap[k] + axb[q] * ev[k];
        }
      }
      // frame before the joints = parent pose composed with the body offset
      const float* bp = m.body_pos + 3 * b;
      const float* Rl = m.body_rot + 9 * b;
      for (int q = 0; q < 3; q++) xup[3 * b + q] = xb[q];
      for (int q = 0; q < 3; q++)
        for (int k = 0; k < 3; k++) {
          float s = xb[q] * bp[k];
          for (int l = 0; l < 3; l++) s += Rb[3 * q + l] * Rl[3 * k + l];
          Rup[9 * b + 3 * q + k] = s;
        }
    }
    t.sync();
  }
}

// Reverse of one fourth-order Runge-Kutta step (rk4_begin / rk4_accumulate / rk4_combine
// around four solves).  snap: the on-chip image after stage 0's solve, the later stages'
// at multiples of `stride` words after it ([0, words) each); qbi/vbi: the cotangents of
// the step's end state.  Outputs as adjoint_step: qb, vb, ub.  Stage k (0-based) runs at
// q_k = q0 (+) c_k v_{k-1}, v_k = v0 + c_k a_{k-1} (c = h/2, h/2, h for k = 1, 2, 3; q_0 =
// q0, v_0 = v0); the step ends at q0 (+) h (v_0 + 2 v_1 + 2 v_2 + v_3) / 6 and
// v0 + h (a_0 + 2 a_1 + 2 a_2 + a_3) / 6.
DEV void adjoint_step_rk4(const DevModel& m, float* W, const Team& t, const float* u,
                          int& status, const unsigned* snap, size_t stride, int words) {
  const int nq = m.nq, nv = m.nv, nu = m.nu;
  const float h = m.dt;
  float* Qb = W + m.o_rkb;  // q0's cotangent
  float* V0b = Qb + nq;     // v0's
  float* Ab = V0b + nv;     // the current stage's acceleration's
  float* Vc = Ab + nv;      // the current stage's velocity's, through the next stage's position
  float* Wb = Vc + nv;      // the combined velocity's
  float* Ub = Wb + nv;      // the controls'
  const float* qbi = W + m.o_qbi;
  const float* vbi = W + m.o_vbi;
  float* qb = W + m.o_qb;
  float* vb = W + m.o_vb;
  float* ub = W + m.o_ub;
  const float* rk = W + m.o_rk;  // q0, v0, a_0, partial sums (stages 1-3's images)
  auto restore = [&](int k) {
    const unsigned* src = snap + k * stride;
    unsigned* Wu = (unsigned*)W;
    for (int i = t.lane; i < words; i += t.T) Wu[i] = src[i];
    t.sync();
  };
  // the final combination; stage 3's image holds v_0 + 2 v_1 + 2 v_2 and v_3
  restore(3);
  {
    const float* vs = rk + nq + 2 * nv;
    const float* qvel = W + m.o_qvel;
    float* vcomb = W + m.o_tmp;
    for (int i = t.lane; i < nv; i += t.T) {
      vcomb[i] = (vs[i] + qvel[i]) / 6.f;
      V0b[i] = vbi[i];
      Ab[i] = Vc[i] = Wb[i] = 0.f;
    }
    for (int i = t.lane; i < nu; i += t.T) Ub[i] = 0.f;
    t.sync();
    integrate_pos_rev(m, t, rk, [&](int i) { return vcomb[i]; }, h, qbi, Qb, Wb, false);
    t.sync();
  }
  for (int k = 3; k >= 0; k--) {
    if (k < 3) restore(k);
    const float bk = (k == 0 || k == 3) ? 1.f : 2.f;
    for (int i = t.lane; i < nv; i += t.T) Ab[i] += bk * (h / 6.f) * vbi[i];
    t.sync();
    adjoint_step(m, W, t, u, status, Ab);
    t.sync();
    const float ch = (k == 3 ? 1.f : 0.5f) * h;
    for (int i = t.lane; i < nu; i += t.T) Ub[i] += ub[i];
    for (int i = t.lane; i < nv; i += t.T) {
      const float v = vb[i] + Vc[i] + bk / 6.f * Wb[i];  // v_k's whole cotangent
      V0b[i] += v;
      Ab[i] = ch * v;  // a_{k-1}'s, through v_k = v0 + c_k a_{k-1}
      Vc[i] = 0.f;
    }
    t.sync();
    if (k > 0) {  // q_k = q0 (+) c_k v_{k-1}; v_{k-1} is in stage k-1's image
      const unsigned* vprev = snap + (k - 1) * stride + m.o_qvel;
      integrate_pos_rev(m, t, rk, [&](int i) { return __uint_as_float(vprev[i]); }, ch, qb, Qb,
                        Vc, true);
    } else {
      for (int i = t.lane; i < nq; i += t.T) Qb[i] += qb[i];
    }
    t.sync();
  }
  for (int i = t.lane; i < nq; i += t.T) qb[i] = Qb[i];
  for (int i = t.lane; i < nv; i += t.T) vb[i] = V0b[i];
  for (int i = t.lane; i < nu; i += t.T) ub[i] = Ub[i];
  t.sync();
}

// ------------------------------------------------------------------ kernels
struct RolloutArgs {
  DevModel m;
  int nworld, horizon, ckpt, zidx, team, nseg;
  float ztarget, wctrl;
  float* qpos;
  float* qvel;
  float* qacc;
  const float* ctrl;  // [horizon][nworld][nu]
  float* tape_ckpt;   // [nseg][nworld][nq + 2 nv]
  float* tape_seg;    // [ckpt + 1][nworld][nq + 2 nv]
  unsigned* tape_snap;  // [ckpt][stages][nworld][snap_words]: on-chip image after each solve
  int snap_words;       // the forward regions of the adjoint layout, [0, o_qbi)
  float* loss;
  const float* dloss;
  float* grad_qvel0;
  float* grad_ctrl;
  int* status;
};

DEV void store_state(const DevModel& m, const float* W, const Team& t, float* dst) {
  for (int i = t.lane; i < m.nq; i += t.T) dst[i] = W[m.o_qpos + i];
  for (int i = t.lane; i < m.nv; i += t.T) {
    dst[m.nq + i] = W[m.o_qvel + i];
    dst[m.nq + m.nv + i] = W[m.o_qacc + i];
  }
}
DEV void load_state(const DevModel& m, float* W, const Team& t, const float* src) {
  for (int i = t.lane; i < m.nq; i += t.T) W[m.o_qpos + i] = src[i];
  for (int i = t.lane; i < m.nv; i += t.T) {
    W[m.o_qvel + i] = src[m.nq + i];
    W[m.o_qacc + i] = src[m.nq + m.nv + i];
  }
  t.sync();
}

__global__ void __launch_bounds__(kAdjBlock) rollout_fwd_kernel(RolloutArgs A) {
  extern __shared__ float lds[];
  const DevModel& m = A.m;
  load_pair_table(m, (unsigned*)lds);
  const int T = A.team;
  const int team = threadIdx.x / T;
  const int w = blockIdx.x * (blockDim.x / T) + team;
  if (w >= A.nworld) return;
  const Team t{(int)threadIdx.x - team * T, T, (const unsigned char*)lds};
  float* W = lds + table_words(m) + (size_t)team * m.lds_words;
  const int ns = m.nq + 2 * m.nv;
  world_init(m, W, t);
  const float* src0 = nullptr;
  (void)src0;
  for (int i = t.lane; i < m.nq; i += T) W[m.o_qpos + i] = A.qpos[(size_t)w * m.nq + i];
  for (int i = t.lane; i < m.nv; i += T) {
    W[m.o_qvel + i] = A.qvel[(size_t)w * m.nv + i];
    W[m.o_qacc + i] = A.qacc[(size_t)w * m.nv + i];
  }
  t.sync();
  int status = 0;
  float loss = 0.f;
  for (int s = 0; s < A.horizon; s++) {
    if (s % A.ckpt == 0)
      store_state(m, W, t, A.tape_ckpt + ((size_t)(s / A.ckpt) * A.nworld + w) * ns);
    const float* u = A.ctrl + ((size_t)s * A.nworld + w) * m.nu;
    for (int k = 0; k < (m.rk4 ? 4 : 1); k++) {
      if (k > 0) rk4_begin(m, W, t, k);
      world_step(m, W, t, u, status, kAdjIters, kAdjGtol);
      if (m.rk4) rk4_accumulate(m, W, t, k);
    }
    if (m.rk4) rk4_combine(m, W, t, status);
    else integrate(m, W, t, status);
    if (t.lane == 0) {
      const float dz = W[m.o_qpos + A.zidx] - A.ztarget;
      float uu = 0.f;
      for (int k = 0; k < m.nu; k++) uu += u[k] * u[k];
      loss += dz * dz + A.wctrl * uu;
    }
  }
  for (int i = t.lane; i < m.nq; i += T) A.qpos[(size_t)w * m.nq + i] = W[m.o_qpos + i];
  for (int i = t.lane; i < m.nv; i += T) {
    A.qvel[(size_t)w * m.nv + i] = W[m.o_qvel + i];
    A.qacc[(size_t)w * m.nv + i] = W[m.o_qacc + i];
  }
  status = t.ior(status);
  if (t.lane == 0) {
    A.loss[w] = loss;
    if (A.status) A.status[w] = status;
  }
}

__global__ void __launch_bounds__(kAdjBlock) rollout_bwd_kernel(RolloutArgs A) {
  extern __shared__ float lds[];
  const DevModel& m = A.m;
  load_pair_table(m, (unsigned*)lds);
  const int T = A.team;
  const int team = threadIdx.x / T;
  const int w = blockIdx.x * (blockDim.x / T) + team;
  if (w >= A.nworld) return;
  const Team t{(int)threadIdx.x - team * T, T, (const unsigned char*)lds};
  float* W = lds + table_words(m) + (size_t)team * m.lds_words;
  const int ns = m.nq + 2 * m.nv;
  const int nst = m.rk4 ? 4 : 1;  // solves per step
  world_init(m, W, t);
  const float dl = A.dloss[w];
  float* qbi = W + m.o_qbi;
  float* vbi = W + m.o_vbi;
  for (int i = t.lane; i < m.nq; i += T) qbi[i] = 0.f;
  for (int i = t.lane; i < m.nv; i += T) vbi[i] = 0.f;
  t.sync();
  int status = 0;
  auto seg_slot = [&](int k) { return A.tape_seg + ((size_t)k * A.nworld + w) * ns; };
  for (int seg = A.nseg - 1; seg >= 0; seg--) {
    const int s0 = seg * A.ckpt;
    const int len = min(A.ckpt, A.horizon - s0);
    // recompute the segment's states s0 .. s0 + len into the tape, and after each
    // step's solve the on-chip image the reverse step needs (kinematics, mass matrix,
    // rows, solution), so that the reverse sweep does not solve the step again
    load_state(m, W, t, A.tape_ckpt + ((size_t)seg * A.nworld + w) * ns);
    store_state(m, W, t, seg_slot(0));
    for (int k = 0; k < len; k++) {
      const float* u = A.ctrl + ((size_t)(s0 + k) * A.nworld + w) * m.nu;
      for (int st = 0; st < nst; st++) {  // (Runge-Kutta: an image per stage)
        if (st > 0) rk4_begin(m, W, t, st);
        world_step(m, W, t, u, status, kAdjIters, kAdjGtol);
        unsigned* snap = A.tape_snap + (((size_t)k * nst + st) * A.nworld + w) * A.snap_words;
        const unsigned* Wu = (const unsigned*)W;
        for (int i = t.lane; i < A.snap_words; i += T) snap[i] = Wu[i];
        t.sync();
        if (nst > 1) rk4_accumulate(m, W, t, st);
      }
      if (nst > 1) rk4_combine(m, W, t, status);
      else integrate(m, W, t, status);
      store_state(m, W, t, seg_slot(k + 1));
    }
    t.sync();
    for (int k = len - 1; k >= 0; k--) {
      const int s = s0 + k;
      const float* u = A.ctrl + ((size_t)s * A.nworld + w) * m.nu;
      // loss term of the state after step s
      const float znext = seg_slot(k + 1)[A.zidx];
      if (t.lane == 0) qbi[A.zidx] += 2.f * (znext - A.ztarget) * dl;
      const unsigned* snap = A.tape_snap + ((size_t)k * nst * A.nworld + w) * A.snap_words;
      if (nst > 1) {
        adjoint_step_rk4(m, W, t, u, status, snap, (size_t)A.nworld * A.snap_words,
                         A.snap_words);
      } else {
        unsigned* Wu = (unsigned*)W;
        for (int i = t.lane; i < A.snap_words; i += T) Wu[i] = snap[i];
        t.sync();
        adjoint_step(m, W, t, u, status);
      }
      float* gu = A.grad_ctrl + ((size_t)s * A.nworld + w) * m.nu;
      const float* ub = W + m.o_ub;
      for (int i = t.lane; i < m.nu; i += T) gu[i] = ub[i] + 2.f * A.wctrl * u[i] * dl;
      for (int i = t.lane; i < m.nq; i += T) qbi[i] = W[m.o_qb + i];
      for (int i = t.lane; i < m.nv; i += T) vbi[i] = W[m.o_vb + i];
      t.sync();
    }
  }
  for (int i = t.lane; i < m.nv; i += T) A.grad_qvel0[(size_t)w * m.nv + i] = vbi[i];
  status = t.ior(status);
  if (t.lane == 0 && A.status) A.status[w] |= status;
}

// ------------------------------------------------------------------ host side
struct AdjointState {
  RolloutArgs args{};
  float* tape_ckpt = nullptr;
  float* tape_seg = nullptr;
  unsigned* tape_snap = nullptr;
  size_t snap_alloc = 0;  // words
  int* status = nullptr;
  size_t ckpt_words = 0, seg_words = 0, status_words = 0;
  bool have_fwd = false;
  int64_t generation = 0;  // number of forward rollouts so far; the tapes hold the last
};

static int blocks_for(int nworld, int team) {
  const int wpb = kAdjBlock / team;
  return (nworld + wpb - 1) / wpb;
}

mjh_status adjoint_forward(AdjointState** stp, const DevModel& m, int team, int nworld, float* qpos,
                           float* qvel, float* qacc, int horizon, int ckpt, const float* ctrl,
                           int zidx, float ztarget, float wctrl, float* loss, int64_t* generation,
                           hipStream_t stream, std::string& err) {
  if (horizon <= 0 || ckpt <= 0 || (!ctrl && m.nu > 0) || !loss || zidx < 0 || zidx >= m.nq) {
    err = "rollout_fwd: need horizon > 0, ckpt_every > 0, ctrl, loss and 0 <= zidx < nq";
    return MJH_EINVAL;
  }
  if (!qpos || !qvel || !qacc) { err = "rollout_fwd: state not bound"; return MJH_ESTATE; }
  // the reverse sweep differentiates plane-sphere / plane-capsule contact geometry
  team = (team == 16 || team == 32 || team == 64) ? team : 32;
  AdjointState* st = *stp;
  if (!st) {
    st = new (std::nothrow) AdjointState();
    if (!st) { err = "rollout_fwd: out of host memory"; return MJH_ENOMEM; }
    *stp = st;
  }
  const int nseg = (horizon + ckpt - 1) / ckpt;
  const size_t ns = (size_t)m.nq + 2 * m.nv;
  const size_t need_ckpt = (size_t)nseg * nworld * ns;
  const size_t need_seg = (size_t)(std::min(ckpt, horizon) + 1) * nworld * ns;
  if (need_ckpt > st->ckpt_words) {
    if (st->tape_ckpt) (void)hipFree(st->tape_ckpt);
    st->tape_ckpt = nullptr;
    if (hipMalloc(&st->tape_ckpt, need_ckpt * sizeof(float)) != hipSuccess) {
      st->ckpt_words = 0;
      err = "rollout_fwd: out of device memory (checkpoints)";
      return MJH_ENOMEM;
    }
    st->ckpt_words = need_ckpt;
  }
  if (need_seg > st->seg_words) {
    if (st->tape_seg) (void)hipFree(st->tape_seg);
    st->tape_seg = nullptr;
    if (hipMalloc(&st->tape_seg, need_seg * sizeof(float)) != hipSuccess) {
      st->seg_words = 0;
      err = "rollout_fwd: out of device memory (segment tape)";
      return MJH_ENOMEM;
    }
    st->seg_words = need_seg;
  }
  const size_t need_snap =
      (size_t)std::min(ckpt, horizon) * (m.rk4 ? 4 : 1) * nworld * (size_t)m.o_qbi;
  if (need_snap > st->snap_alloc) {
    if (st->tape_snap) (void)hipFree(st->tape_snap);
    st->tape_snap = nullptr;
    if (hipMalloc(&st->tape_snap, need_snap * sizeof(unsigned)) != hipSuccess) {
      st->snap_alloc = 0;
      err = "rollout_fwd: out of device memory (on-chip images of a segment)";
      return MJH_ENOMEM;
    }
    st->snap_alloc = need_snap;
  }
  if ((size_t)nworld > st->status_words) {
    if (st->status) (void)hipFree(st->status);
    st->status = nullptr;
    if (hipMalloc(&st->status, sizeof(int) * (size_t)nworld) != hipSuccess) {
      st->status_words = 0;
      err = "rollout_fwd: out of device memory";
      return MJH_ENOMEM;
    }
    st->status_words = (size_t)nworld;
  }
  RolloutArgs& A = st->args;
  A.m = m;
  A.nworld = nworld; A.horizon = horizon; A.ckpt = ckpt; A.zidx = zidx; A.team = team;
  A.nseg = nseg; A.ztarget = ztarget; A.wctrl = wctrl;
  A.qpos = qpos; A.qvel = qvel; A.qacc = qacc; A.ctrl = ctrl;
  A.tape_ckpt = st->tape_ckpt; A.tape_seg = st->tape_seg; A.loss = loss; A.status = st->status;
  A.tape_snap = st->tape_snap; A.snap_words = m.o_qbi;
  st->have_fwd = false;
  // the tapes are about to be overwritten: an earlier rollout can no longer be reversed
  st->generation++;
  if (generation) *generation = st->generation;
  if (nworld == 0) { st->have_fwd = true; return MJH_OK; }
  const size_t lds =
      ((size_t)table_words(m) + (size_t)(kAdjBlock / team) * m.lds_words) * sizeof(float);
  hipError_t e = hipFuncSetAttribute((const void*)rollout_fwd_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)rollout_bwd_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) { err = std::string("rollout_fwd: ") + hipGetErrorString(e); return MJH_EHIP; }
  hipLaunchKernelGGL(rollout_fwd_kernel, dim3(blocks_for(nworld, team)), dim3(kAdjBlock), lds,
                     stream, A);
  e = hipGetLastError();
  if (e != hipSuccess) { err = std::string("rollout_fwd: ") + hipGetErrorString(e); return MJH_EHIP; }
  st->have_fwd = true;
  return MJH_OK;
}

mjh_status adjoint_backward(AdjointState* st, int64_t generation, const float* dloss,
                            float* grad_qvel0, float* grad_ctrl, hipStream_t stream,
                            std::string& err) {
  if (!st || !st->have_fwd) { err = "rollout_bwd: call rollout_fwd first"; return MJH_ESTATE; }
  if (generation != st->generation) {
    err = "rollout_bwd: the tapes hold rollout " + std::to_string(st->generation) +
          ", not rollout " + std::to_string(generation) + " (a later rollout_fwd replaced it)";
    return MJH_ESTATE;
  }
  if (!dloss || !grad_qvel0 || (!grad_ctrl && st->args.m.nu > 0)) {
    err = "rollout_bwd: NULL argument";
    return MJH_EINVAL;
  }
  RolloutArgs A = st->args;
  A.dloss = dloss;
  A.grad_qvel0 = grad_qvel0;
  A.grad_ctrl = grad_ctrl;
  if (A.nworld == 0) return MJH_OK;
  const size_t lds =
      ((size_t)table_words(A.m) + (size_t)(kAdjBlock / A.team) * A.m.lds_words) * sizeof(float);
  hipLaunchKernelGGL(rollout_bwd_kernel, dim3(blocks_for(A.nworld, A.team)), dim3(kAdjBlock), lds,
                     stream, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) { err = std::string("rollout_bwd: ") + hipGetErrorString(e); return MJH_EHIP; }
  return MJH_OK;
}

// ------------------------------------------------------------------ no-alloc rollouts
// Tapes of mjh_rollout_noalloc: one rollout's checkpoints, segment states and per-step
// on-chip images.  A file-scope device array: every device the library runs on holds its
// own copy from the module's load until the process ends, and every call on that device
// shares it (calls that overlap on one device race).  Host code never passes the array's
// name to a kernel: it is a host-side stand-in, not a device address.  The address comes
// from hipGetSymbolAddress, once per device, in noalloc_scratch_init.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char* g_scratch_ptr[kMaxDevices] = {};

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = static_cast<unsigned char*>(p);
  return hipSuccess;
}

static size_t round256(size_t bytes) { return (bytes + 255) & ~size_t(255); }

size_t noalloc_tape_bytes(const DevModel& m, int nworld, int horizon, int ckpt) {
  const size_t nseg = (size_t)((horizon + ckpt - 1) / ckpt);
  const size_t seglen = (size_t)std::min(ckpt, horizon);
  const size_t ns = (size_t)m.nq + 2 * (size_t)m.nv;
  return round256(nseg * nworld * ns * sizeof(float)) +
         round256((seglen + 1) * nworld * ns * sizeof(float)) +
         round256(seglen * (m.rk4 ? 4 : 1) * nworld * (size_t)m.o_qbi * sizeof(unsigned));
}

mjh_status adjoint_noalloc(int device, const DevModel& m, int team, int nworld, float* qpos,
                           float* qvel, float* qacc, int horizon, int ckpt, const float* ctrl,
                           int zidx, float ztarget, float wctrl, const float* dloss, float* loss,
                           float* grad_qvel0, float* grad_ctrl, hipStream_t stream,
                           std::string& err) {
  if (horizon <= 0 || ckpt <= 0 || (!ctrl && m.nu > 0) || !loss || !dloss || !grad_qvel0 ||
      (!grad_ctrl && m.nu > 0) ||
      zidx < 0 || zidx >= m.nq) {
    err = "rollout_noalloc: need horizon > 0, ckpt_every > 0, ctrl, dloss, loss, gradients "
          "and 0 <= zidx < nq";
    return MJH_EINVAL;
  }
  if (!qpos || !qvel || !qacc) { err = "rollout_noalloc: state not bound"; return MJH_ESTATE; }
  if (nworld < 0) { err = "rollout_noalloc: negative world count"; return MJH_EINVAL; }
  const size_t need = noalloc_tape_bytes(m, nworld, horizon, ckpt);
  if (need > kNoAllocScratchBytes) {
    err = "rollout_noalloc: " + std::to_string(nworld) + " worlds over " +
          std::to_string(horizon) + " steps with a checkpoint every " + std::to_string(ckpt) +
          " need " + std::to_string(need) + " bytes of tape, more than the library's " +
          std::to_string(kNoAllocScratchBytes) + "-byte scratch";
    return MJH_EINVAL;
  }
  unsigned char* base = (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
  if (!base) { err = "rollout_noalloc: device scratch not initialised"; return MJH_ESTATE; }
  if (nworld == 0) return MJH_OK;
  team = (team == 16 || team == 32 || team == 64) ? team : 32;
  RolloutArgs A{};
  A.m = m;
  A.nworld = nworld; A.horizon = horizon; A.ckpt = ckpt; A.zidx = zidx; A.team = team;
  A.nseg = (horizon + ckpt - 1) / ckpt; A.ztarget = ztarget; A.wctrl = wctrl;
  A.qpos = qpos; A.qvel = qvel; A.qacc = qacc; A.ctrl = ctrl;
  const size_t ns = (size_t)m.nq + 2 * (size_t)m.nv;
  const size_t seglen = (size_t)std::min(ckpt, horizon);
  size_t off = 0;
  A.tape_ckpt = reinterpret_cast<float*>(base + off);
  off += round256((size_t)A.nseg * nworld * ns * sizeof(float));
  A.tape_seg = reinterpret_cast<float*>(base + off);
  off += round256((seglen + 1) * nworld * ns * sizeof(float));
  A.tape_snap = reinterpret_cast<unsigned*>(base + off);
  A.snap_words = m.o_qbi;
  A.status = nullptr;  // the rollouts' per-world status is not reported
  A.loss = loss; A.dloss = dloss; A.grad_qvel0 = grad_qvel0; A.grad_ctrl = grad_ctrl;
  const size_t lds =
      ((size_t)table_words(m) + (size_t)(kAdjBlock / team) * m.lds_words) * sizeof(float);
  hipError_t e = hipFuncSetAttribute((const void*)rollout_fwd_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)rollout_bwd_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) { err = std::string("rollout_noalloc: ") + hipGetErrorString(e); return MJH_EHIP; }
  // forward, then reverse: stream order keeps the reverse sweep behind the tapes' writes
  hipLaunchKernelGGL(rollout_fwd_kernel, dim3(blocks_for(nworld, team)), dim3(kAdjBlock), lds,
                     stream, A);
  e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(rollout_bwd_kernel, dim3(blocks_for(nworld, team)), dim3(kAdjBlock), lds,
                       stream, A);
    e = hipGetLastError();
  }
  if (e != hipSuccess) { err = std::string("rollout_noalloc: ") + hipGetErrorString(e); return MJH_EHIP; }
  return MJH_OK;
}

void adjoint_free(AdjointState* st) {
  if (!st) return;
  if (st->tape_ckpt) (void)hipFree(st->tape_ckpt);
  if (st->tape_seg) (void)hipFree(st->tape_seg);
  if (st->tape_snap) (void)hipFree(st->tape_snap);
  if (st->status) (void)hipFree(st->status);
  delete st;
}

}  // namespace mjh
