// Host side of the C ABI: model blob parsing and compilation into device tables,
// world batches, launches, graph capture and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/mjh.h"
#include "mjh_adjoint.h"
#include "mjh_kernels.h"
#include "mjh_model.h"

using namespace mjh;

// ===================================================================== host model
namespace {

struct HostModel {
  // parsed blob (double precision as stored)
  int nbody = 0, njnt = 0, ngeom = 0, npair = 0, nu = 0, nq = 0, nv = 0;
  int iterations = 0, ls_iterations = 0, nconmax = 0, neq = 0, integrator = 0;
  int cone = 0;  // friction cone: 0 pyramidal, 1 elliptic
  int hf_nrow = 0, hf_ncol = 0;
  double hf_size[3] = {0, 0, 0};
  std::vector<double> hf_data;
  std::vector<int> eq_body;        // [neq][2]
  std::vector<double> eq_anchor;   // [neq][6]
  std::vector<int> eq_type;        // [neq] 0 connect, 1 weld
  std::vector<int> pair_condim;    // [npair] 1 frictionless, 3 sliding, 4 + torsion, 6 + rolling
  std::vector<double> pair_mu_t, pair_mu_r;  // [npair] torsional and rolling coefficients
  std::vector<double> eq_relR;     // [neq][9] weld: body2's reference orientation in body1's frame
  int neqrow = 0;                  // 3 rows per connect, 6 per weld
  double dt = 0, grav[3] = {0, 0, 0}, solref[2] = {0, 0}, solimp[5] = {0, 0, 0, 0, 0};
  std::vector<int> body_parent, jnt_type, jnt_body, jnt_limited, geom_type, geom_body,
      pair_g1, pair_g2, act_type, act_jnt;
  std::vector<double> body_pos, body_quat, body_mass, body_ipos, body_inertia, jnt_pos,
      jnt_axis, jnt_damping, jnt_armature, jnt_range, jnt_frictionloss, geom_size, geom_pos,
      geom_quat, pair_mu,
      act_gear, act_kp, act_kd, act_lo, act_hi, act_qdef, qpos0;
};

struct ModelRec {
  HostModel h;
  DevModel dm{};
  DevModel dm_adj{};  // same tables, adjoint on-chip layout
  void* dbuf = nullptr;  // one device allocation for all tables
  size_t dbytes = 0;
  double cost = 0.0;     // relative cost of one world-step (task ordering)
};

class Blob {
 public:
  Blob(const uint8_t* p, size_t n) : p_(p), n_(n) {}
  template <class X> bool read(X* dst, size_t count) {
    const size_t bytes = sizeof(X) * count;
    if (off_ + bytes > n_) return false;
    std::memcpy(dst, p_ + off_, bytes);
    off_ += bytes;
    return true;
  }
  size_t off() const { return off_; }

 private:
  const uint8_t* p_;
  size_t n_, off_ = 0;
};

mjh_status parse_blob(const uint8_t* blob, size_t nbytes, HostModel& m, std::string& err) {
  Blob r(blob, nbytes);
  int32_t hi[16];
  double hf[16];
  if (!r.read(hi, 16) || !r.read(hf, 16)) { err = "model blob: truncated header"; return MJH_EMODEL; }
  if (hi[0] != 0x4D484A4D || hi[1] != 3) { err = "model blob: bad magic or version"; return MJH_EMODEL; }
  m.nbody = hi[2]; m.njnt = hi[3]; m.ngeom = hi[4]; m.npair = hi[5]; m.nu = hi[6];
  m.nq = hi[7]; m.nv = hi[8]; m.iterations = hi[9]; m.ls_iterations = hi[10]; m.nconmax = hi[11];
  m.neq = hi[12];
  m.integrator = hi[13];
  const int has_hf = hi[14];
  m.cone = hi[15];
  if (m.nbody < 1 || m.njnt < 0 || m.ngeom < 0 || m.npair < 0 || m.nu < 0 || m.nq < 0 ||
      m.nv < 0 || m.iterations < 0 || m.nconmax < 0 || m.nbody > 4096 || m.njnt > 4096 ||
      m.ngeom > 4096 || m.npair > 65536 || m.nu > 4096 || m.nconmax > 4096 || m.neq < 0 ||
      m.neq > 1024 || m.integrator < 0 || m.integrator > 3 || has_hf < 0 || has_hf > 1 ||
      m.cone < 0 || m.cone > 1) {
    err = "model blob: size field out of range";
    return MJH_EMODEL;
  }
  m.dt = hf[0];
  for (int k = 0; k < 3; k++) m.grav[k] = hf[1 + k];
  m.solref[0] = hf[4]; m.solref[1] = hf[5];
  for (int k = 0; k < 5; k++) m.solimp[k] = hf[6 + k];
  auto rd = [&](auto& vec, size_t count) {
    vec.resize(count);
    return r.read(vec.data(), count);
  };
  std::vector<int32_t> bi, ji, gi, pi, ai, ei;
  std::vector<double> bf, jf, gf, pf, af, ef;
  bool ok = rd(bi, 2 * m.nbody) && rd(bf, 19 * (size_t)m.nbody) && rd(ji, 4 * m.njnt) &&
            rd(jf, 11 * (size_t)m.njnt) && rd(gi, 2 * m.ngeom) && rd(gf, 11 * (size_t)m.ngeom) &&
            rd(pi, 4 * m.npair) && rd(pf, 3 * (size_t)m.npair) && rd(ai, 2 * m.nu) &&
            rd(af, 7 * (size_t)m.nu) && rd(ei, 4 * (size_t)m.neq) && rd(ef, 10 * (size_t)m.neq);
  if (ok && has_hf) {
    int32_t hd[2];
    ok = r.read(hd, 2) && r.read(m.hf_size, 3);
    if (ok && (hd[0] < 2 || hd[1] < 2 || hd[0] > 4096 || hd[1] > 4096)) {
      err = "model blob: heightfield needs 2..4096 rows and columns";
      return MJH_EMODEL;
    }
    if (ok) {
      m.hf_nrow = hd[0];
      m.hf_ncol = hd[1];
      ok = rd(m.hf_data, (size_t)m.hf_nrow * m.hf_ncol);
    }
  }
  ok = ok && rd(m.qpos0, m.nq);
  if (!ok || r.off() != nbytes) { err = "model blob: size mismatch"; return MJH_EMODEL; }
  for (int b = 0; b < m.nbody; b++) {
    m.body_parent.push_back(bi[2 * b]);
    const double* f = &bf[19 * b];
    m.body_pos.insert(m.body_pos.end(), f, f + 3);
    m.body_quat.insert(m.body_quat.end(), f + 3, f + 7);
    m.body_mass.push_back(f[7]);
    m.body_ipos.insert(m.body_ipos.end(), f + 8, f + 11);
    m.body_inertia.insert(m.body_inertia.end(), f + 11, f + 17);
    if (b == 0 ? bi[0] != -1 : (bi[2 * b] < 0 || bi[2 * b] >= b)) {
      err = "model blob: bodies must follow their parents (body 0 = world)";
      return MJH_EMODEL;
    }
  }
  for (int j = 0; j < m.njnt; j++) {
    const int type = ji[4 * j], body = ji[4 * j + 1], limited = ji[4 * j + 2] != 0;
    if (type < 0 || type > 2 || body <= 0 || body >= m.nbody ||
        (j > 0 && body < ji[4 * (j - 1) + 1])) {
      err = "model blob: bad joint (type/body/order)";
      return MJH_EMODEL;
    }
    const double* f = &jf[11 * j];
    if (limited && (type == JNT_FREE || !(f[8] < f[9]))) {
      err = "model blob: a limit needs a hinge or slide joint and range[0] < range[1]";
      return MJH_EMODEL;
    }
    if (!(f[10] >= 0.0) || (type == JNT_FREE && f[10] != 0.0)) {
      err = "model blob: friction loss needs a hinge or slide joint and a bound >= 0";
      return MJH_EMODEL;
    }
    m.jnt_frictionloss.push_back(f[10]);
    m.jnt_type.push_back(type);
    m.jnt_body.push_back(body);
    m.jnt_limited.push_back(limited);
    m.jnt_range.push_back(f[8]);
    m.jnt_range.push_back(f[9]);
    m.jnt_pos.insert(m.jnt_pos.end(), f, f + 3);
    const double L = std::sqrt(f[3] * f[3] + f[4] * f[4] + f[5] * f[5]);
    if (type != JNT_FREE && !(L > 0)) { err = "model blob: zero joint axis"; return MJH_EMODEL; }
    for (int k = 0; k < 3; k++) m.jnt_axis.push_back(L > 0 ? f[3 + k] / L : 0.0);
    m.jnt_damping.push_back(f[6]);
    m.jnt_armature.push_back(f[7]);
  }
  for (int g = 0; g < m.ngeom; g++) {
    const int type = gi[2 * g], body = gi[2 * g + 1];
    if (type < 0 || type > 4 || body < 0 || body >= m.nbody) { err = "model blob: bad geom"; return MJH_EMODEL; }
    m.geom_type.push_back(type);
    m.geom_body.push_back(body);
    const double* f = &gf[11 * g];
    m.geom_size.insert(m.geom_size.end(), f, f + 3);
    m.geom_pos.insert(m.geom_pos.end(), f + 3, f + 6);
    m.geom_quat.insert(m.geom_quat.end(), f + 6, f + 10);
  }
  for (int p = 0; p < m.npair; p++) {
    const int g1 = pi[4 * p], g2 = pi[4 * p + 1], condim = pi[4 * p + 2];
    if (g1 < 0 || g1 >= m.ngeom || g2 < 0 || g2 >= m.ngeom) { err = "model blob: bad pair"; return MJH_EMODEL; }
    if (condim != 1 && condim != 3 && condim != 4 && condim != 6) {
      err = "pairs take condim 1, 3, 4 or 6"; return MJH_EUNSUPPORTED;
    }
    const int t1 = m.geom_type[g1], t2 = m.geom_type[g2];
    if (t1 > t2) { err = "model blob: pair geoms must be ordered by type"; return MJH_EMODEL; }
    if (t1 == GEOM_PLANE && t2 == GEOM_PLANE) { err = "model blob: plane-plane pair"; return MJH_EMODEL; }
    if (t1 == GEOM_BOX && t2 == GEOM_BOX) { err = "box-box pairs are not supported"; return MJH_EUNSUPPORTED; }
    if (t2 == GEOM_HFIELD && (t1 != GEOM_SPHERE || m.hf_nrow == 0)) {
      err = "heightfields pair with spheres only (and need the model's heightfield)";
      return MJH_EUNSUPPORTED;
    }
    m.pair_g1.push_back(g1);
    m.pair_g2.push_back(g2);
    m.pair_condim.push_back(condim);
    m.pair_mu.push_back(pf[3 * p]);
    m.pair_mu_t.push_back(pf[3 * p + 1]);
    m.pair_mu_r.push_back(pf[3 * p + 2]);
  }
  for (int a = 0; a < m.nu; a++) {
    const int type = ai[2 * a], jnt = ai[2 * a + 1];
    if (type < 0 || type > 1 || jnt < 0 || jnt >= m.njnt) { err = "model blob: bad actuator"; return MJH_EMODEL; }
    if (m.jnt_type[jnt] == JNT_FREE) { err = "actuators on free joints are not supported"; return MJH_EUNSUPPORTED; }
    m.act_type.push_back(type);
    m.act_jnt.push_back(jnt);
    const double* f = &af[7 * a];
    m.act_gear.push_back(f[0]); m.act_kp.push_back(f[1]); m.act_kd.push_back(f[2]);
    m.act_lo.push_back(f[3]); m.act_hi.push_back(f[4]); m.act_qdef.push_back(f[5]);
  }
  for (int e = 0; e < m.neq; e++) {
    const int type = ei[4 * e], b1 = ei[4 * e + 1], b2 = ei[4 * e + 2];
    if (type != 0 && type != 1) { err = "only connect and weld equalities are supported"; return MJH_EUNSUPPORTED; }
    if (b1 <= 0 || b1 >= m.nbody || b2 < 0 || b2 >= m.nbody || b1 == b2) {
      err = "model blob: bad equality bodies"; return MJH_EMODEL;
    }
    m.eq_type.push_back(type);
    m.eq_body.push_back(b1);
    m.eq_body.push_back(b2);
    m.eq_anchor.insert(m.eq_anchor.end(), &ef[10 * e], &ef[10 * e] + 6);
    // the weld's reference orientation: unit quaternion (w, x, y, z) -> rotation matrix
    const double* qr = &ef[10 * e + 6];
    const double qn = std::sqrt(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
    if (type == 1 && !(qn > 0.0)) { err = "model blob: bad weld orientation"; return MJH_EMODEL; }
    const double w = qn > 0 ? qr[0] / qn : 1, x = qn > 0 ? qr[1] / qn : 0;
    const double y = qn > 0 ? qr[2] / qn : 0, z = qn > 0 ? qr[3] / qn : 0;
    const double R[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                         2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                         2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    m.eq_relR.insert(m.eq_relR.end(), R, R + 9);
    m.neqrow += type == 1 ? 6 : 3;
  }
  return MJH_OK;
}

void quat_mat(const double* q, float* R) {
  double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
  double r[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                 2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                 2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
  for (int k = 0; k < 9; k++) R[k] = (float)r[k];
}

int pair_kind_of(int t1, int t2) {
  if (t1 == GEOM_PLANE) return t2 == GEOM_SPHERE ? PK_PLANE_SPHERE : t2 == GEOM_CAPSULE ? PK_PLANE_CAPSULE : PK_PLANE_BOX;
  if (t1 == GEOM_SPHERE)
    return t2 == GEOM_SPHERE ? PK_SPHERE_SPHERE : t2 == GEOM_CAPSULE ? PK_SPHERE_CAPSULE
           : t2 == GEOM_HFIELD ? PK_SPHERE_HFIELD : PK_SPHERE_BOX;
  return t2 == GEOM_CAPSULE ? PK_CAPSULE_CAPSULE : PK_CAPSULE_BOX;
}
int pair_slots(int kind) {
  switch (kind) {
    case PK_PLANE_CAPSULE: return 2;
    case PK_PLANE_BOX: return 8;
    case PK_CAPSULE_BOX: return 4;
    default: return 1;
  }
}

// Derive tree tables and the on-chip layout; pack every table into one host image
// whose device copy DevModel points into.
struct Packer {
  std::vector<uint8_t> bytes;
  std::vector<std::pair<size_t, const void**>> fix;  // offset -> DevModel pointer field
  template <class X> void add(const std::vector<X>& v, const X** field) {
    size_t off = (bytes.size() + 15) & ~size_t(15);
    bytes.resize(off + std::max<size_t>(v.size(), 1) * sizeof(X), 0);
    if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(X));
    fix.push_back({off, reinterpret_cast<const void**>(field)});
  }
};

mjh_status compile_model(const HostModel& h, ModelRec& rec, Packer& pk, std::string& err) {
  DevModel& d = rec.dm;
  d = DevModel{};
  d.nbody = h.nbody; d.njnt = h.njnt; d.nq = h.nq; d.nv = h.nv; d.nu = h.nu;
  d.ngeom = h.ngeom; d.npair = h.npair; d.nconmax = h.nconmax;
  d.iterations = h.iterations;
  d.implicit = (h.integrator == 1 || h.integrator == 2) ? h.integrator : 0;
  d.rk4 = h.integrator == 3;
  d.hf_nrow = h.hf_nrow;
  d.hf_ncol = h.hf_ncol;
  for (int k = 0; k < 3; k++) d.hf_size[k] = (float)h.hf_size[k];
  if (h.nv > kMaxNv) { err = "nv > 64 is not supported"; return MJH_EUNSUPPORTED; }
  // addresses
  std::vector<int> body_jntadr(h.nbody, 0), body_jntnum(h.nbody, 0), body_dofadr(h.nbody, 0),
      body_dofnum(h.nbody, 0), jnt_qposadr, jnt_dofadr, dof_body;
  std::vector<float> dof_armature, dof_damping;
  int qa = 0, da = 0;
  for (int j = 0; j < h.njnt; j++) {
    const int b = h.jnt_body[j];
    if (body_jntnum[b] == 0) { body_jntadr[b] = j; body_dofadr[b] = da; }
    body_jntnum[b]++;
    const int nd = h.jnt_type[j] == JNT_FREE ? 6 : 1;
    if (h.jnt_type[j] == JNT_FREE && h.body_parent[b] != 0) {
      err = "a free joint must attach a child of the world"; return MJH_EUNSUPPORTED;
    }
    body_dofnum[b] += nd;
    jnt_qposadr.push_back(qa);
    jnt_dofadr.push_back(da);
    for (int k = 0; k < nd; k++) {
      dof_body.push_back(b);
      dof_armature.push_back((float)h.jnt_armature[j]);
      dof_damping.push_back((float)h.jnt_damping[j]);
    }
    qa += h.jnt_type[j] == JNT_FREE ? 7 : 1;
    da += nd;
  }
  for (int b = 0; b < h.nbody; b++)
    for (int j = body_jntadr[b]; j < body_jntadr[b] + body_jntnum[b]; j++)
      if (h.jnt_type[j] == JNT_FREE && body_jntnum[b] != 1) {
        err = "a free joint must be its body's only joint"; return MJH_EUNSUPPORTED;
      }
  if (qa != h.nq || da != h.nv) { err = "model blob: nq/nv disagree with the joints"; return MJH_EMODEL; }
  // dof tree
  std::vector<int> dof_parent(h.nv, -1);
  for (int k = 0; k < h.nv; k++) {
    const int b = dof_body[k];
    if (k > body_dofadr[b]) { dof_parent[k] = k - 1; continue; }
    for (int p = h.body_parent[b]; p > 0; p = h.body_parent[p])
      if (body_dofnum[p] > 0) { dof_parent[k] = body_dofadr[p] + body_dofnum[p] - 1; break; }
  }
  std::vector<int> anc_start(h.nv + 1, 0), anc_list, mpair;
  for (int k = 0; k < h.nv; k++) {
    anc_start[k] = (int)anc_list.size();
    for (int i = dof_parent[k]; i >= 0; i = dof_parent[i]) anc_list.push_back(i);
    mpair.push_back((k << 16) | k);
    for (int i = dof_parent[k]; i >= 0; i = dof_parent[i]) mpair.push_back((k << 16) | i);
  }
  anc_start[h.nv] = (int)anc_list.size();
  std::vector<unsigned long long> body_dofmask(h.nbody, 0ull);
  for (int b = 1; b < h.nbody; b++) {
    unsigned long long mk = body_dofmask[h.body_parent[b]];
    for (int k = body_dofadr[b]; k < body_dofadr[b] + body_dofnum[b]; k++) mk |= 1ull << k;
    body_dofmask[b] = mk;
  }
  // tree levels and children
  std::vector<int> level(h.nbody, 0);
  int nlevel = 1;
  for (int b = 1; b < h.nbody; b++) {
    level[b] = level[h.body_parent[b]] + 1;
    nlevel = std::max(nlevel, level[b] + 1);
  }
  std::vector<int> level_start(nlevel + 1, 0), level_body;
  for (int lv = 0; lv < nlevel; lv++) {
    level_start[lv] = (int)level_body.size();
    for (int b = 0; b < h.nbody; b++)
      if (level[b] == lv) level_body.push_back(b);
  }
  level_start[nlevel] = (int)level_body.size();
  std::vector<int> child_start(h.nbody + 1, 0), child_list;
  for (int b = 0; b < h.nbody; b++) {
    child_start[b] = (int)child_list.size();
    for (int c = 1; c < h.nbody; c++)
      if (h.body_parent[c] == b) child_list.push_back(c);
  }
  child_start[h.nbody] = (int)child_list.size();
  // actuators: one per dof at most
  std::vector<int> dof_act(h.nv, -1), act_qadr, act_dadr;
  // implicit gains: h (b + kd) + h^2 kp on the factor's diagonal is h times dof_vgain
  // with dof_vgain = b + kd + h kp; dof_hkp = h kp scales qvel on the right-hand side
  // (integrator 2 only)
  std::vector<float> dof_vgain(dof_damping), dof_hkp(h.nv, 0.f);
  for (int a = 0; a < h.nu; a++) {
    const int j = h.act_jnt[a];
    const int dof = jnt_dofadr[j];
    if (dof_act[dof] >= 0) { err = "two actuators on one dof are not supported"; return MJH_EUNSUPPORTED; }
    dof_act[dof] = a;
    if (h.act_type[a] == ACT_PD) {
      dof_vgain[dof] += (float)h.act_kd[a];
      if (h.integrator == 2) {
        dof_vgain[dof] += (float)(h.dt * h.act_kp[a]);
        dof_hkp[dof] = (float)(h.dt * h.act_kp[a]);
      }
    }
    act_qadr.push_back(jnt_qposadr[j]);
    act_dadr.push_back(dof);
  }
  // joint limits, in joint order
  std::vector<int> lim_qadr, lim_dadr;
  std::vector<float> lim_lo, lim_hi;
  for (int j = 0; j < h.njnt; j++)
    if (h.jnt_limited[j]) {
      lim_qadr.push_back(jnt_qposadr[j]);
      lim_dadr.push_back(jnt_dofadr[j]);
      lim_lo.push_back((float)h.jnt_range[2 * j]);
      lim_hi.push_back((float)h.jnt_range[2 * j + 1]);
    }
  d.nlim = (int)lim_qadr.size();
  // friction loss, in dof order (hinge and slide joints: one dof each)
  std::vector<int> fric_dadr;
  std::vector<float> fric_loss;
  for (int j = 0; j < h.njnt; j++)
    if (h.jnt_frictionloss[j] > 0.0) {
      fric_dadr.push_back(jnt_dofadr[j]);
      fric_loss.push_back((float)h.jnt_frictionloss[j]);
    }
  d.nfric = (int)fric_dadr.size();
  d.neq = h.neq;
  d.neqrow = h.neqrow;
  // a contact's rows: 1 frictionless; 2 (condim - 1) pyramid edges; condim frame rows of
  // an elliptic cone.  con_nr: that count when every pair shares it (contact c's rows
  // are con_nr c ..), else 0 (each contact's first row and count packed in its record)
  d.cone = h.cone;
  auto rows_of = [&](int c) { return (c == 1 || h.cone == 1) ? c : 2 * (c - 1); };
  d.conrows = h.npair ? 1 : 4;
  d.con_nr = h.npair ? rows_of(h.pair_condim[0]) : 4;
  for (int c : h.pair_condim) {
    d.conrows = std::max(d.conrows, rows_of(c));
    if (rows_of(c) != d.con_nr) d.con_nr = 0;
  }
  if (d.con_nr != 3 && d.con_nr != 4) d.con_nr = 0;  // the fast path: 3 and 4 rows
  d.nrowmax = d.conrows * h.nconmax + d.nlim + d.nfric + d.neqrow;
  d.jframe = (!h.cone && d.con_nr == 4) ? 1 : 0;
  // J rows: a frame-row contact keeps 3 of its 4 edge rows' worth
  const int njrow = d.jframe ? 3 * h.nconmax + d.nlim + d.nfric + d.neqrow : d.nrowmax;
  const int nfw = d.jframe ? 5 * h.nconmax + d.nlim + d.nfric + d.neqrow : 0;
  // pairs and candidate slots
  std::vector<int> pair_kind, pair_candadr, cand_pair;
  int ncand = 0;
  for (int p = 0; p < h.npair; p++) {
    const int kind = pair_kind_of(h.geom_type[h.pair_g1[p]], h.geom_type[h.pair_g2[p]]);
    pair_kind.push_back(kind);
    pair_candadr.push_back(ncand);
    for (int k = 0; k < pair_slots(kind); k++) cand_pair.push_back(p);
    ncand += pair_slots(kind);
  }
  d.ncand = ncand;
  d.nlevel = nlevel;
  d.nmpair = (int)mpair.size();
  d.ntri = h.nv * (h.nv + 1) / 2;
  // constants (soft-constraint conventions: time constant at least 2 dt)
  const double tc = std::max(h.solref[0], 2.0 * h.dt), zeta = h.solref[1], dmax = h.solimp[1];
  d.dt = (float)h.dt;
  d.K = (float)(1.0 / (dmax * dmax * tc * tc * zeta * zeta));
  d.B = (float)(2.0 / (dmax * tc));
  d.dmin = (float)h.solimp[0]; d.dmax = (float)h.solimp[1]; d.width = (float)h.solimp[2];
  d.mid = (float)h.solimp[3]; d.power = (float)h.solimp[4];
  for (int k = 0; k < 3; k++) d.grav[k] = (float)h.grav[k];
  // float tables
  auto fv = [](const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); };
  std::vector<float> body_rot(9 * h.nbody), geom_rot(9 * h.ngeom);
  for (int b = 0; b < h.nbody; b++) quat_mat(&h.body_quat[4 * b], &body_rot[9 * b]);
  for (int g = 0; g < h.ngeom; g++) quat_mat(&h.geom_quat[4 * g], &geom_rot[9 * g]);
  std::vector<float> invw(h.nbody, 0.f);
  pk.add(h.body_parent, &d.body_parent);
  pk.add(body_jntadr, &d.body_jntadr);
  pk.add(body_jntnum, &d.body_jntnum);
  pk.add(body_dofadr, &d.body_dofadr);
  pk.add(body_dofnum, &d.body_dofnum);
  pk.add(level_start, &d.level_start);
  pk.add(level_body, &d.level_body);
  pk.add(child_start, &d.child_start);
  pk.add(child_list, &d.child_list);
  pk.add(h.jnt_type, &d.jnt_type);
  pk.add(jnt_qposadr, &d.jnt_qposadr);
  pk.add(jnt_dofadr, &d.jnt_dofadr);
  pk.add(dof_body, &d.dof_body);
  pk.add(dof_act, &d.dof_act);
  pk.add(anc_start, &d.anc_start);
  pk.add(anc_list, &d.anc_list);
  pk.add(mpair, &d.mpair);
  pk.add(body_dofmask, &d.body_dofmask);
  pk.add(h.geom_type, &d.geom_type);
  pk.add(h.geom_body, &d.geom_body);
  pk.add(h.pair_g1, &d.pair_g1);
  pk.add(h.pair_condim, &d.pair_condim);
  std::vector<float> pmut = fv(h.pair_mu_t), pmur = fv(h.pair_mu_r);
  pk.add(pmut, &d.pair_mu_t);
  pk.add(pmur, &d.pair_mu_r);
  pk.add(h.pair_g2, &d.pair_g2);
  pk.add(pair_kind, &d.pair_kind);
  pk.add(pair_candadr, &d.pair_candadr);
  pk.add(cand_pair, &d.cand_pair);
  pk.add(h.act_type, &d.act_type);
  pk.add(act_qadr, &d.act_qadr);
  pk.add(act_dadr, &d.act_dadr);
  pk.add(lim_qadr, &d.lim_qadr);
  pk.add(lim_dadr, &d.lim_dadr);
  pk.add(lim_lo, &d.lim_lo);
  pk.add(lim_hi, &d.lim_hi);
  pk.add(fric_dadr, &d.fric_dadr);
  pk.add(fric_loss, &d.fric_loss);
  pk.add(h.eq_body, &d.eq_body);
  std::vector<float> eq_anchor = fv(h.eq_anchor);
  pk.add(eq_anchor, &d.eq_anchor);
  std::vector<float> eq_relR = fv(h.eq_relR);
  pk.add(eq_relR, &d.eq_relR);
  // each equality row: its equality | component << 16 (0-2 translational, 3-5 rotational)
  std::vector<int> eq_row;
  for (int q = 0; q < h.neq; q++)
    for (int k = 0; k < (h.eq_type[q] == 1 ? 6 : 3); k++) eq_row.push_back(q | (k << 16));
  pk.add(eq_row, &d.eq_row);
  std::vector<float> bpos = fv(h.body_pos), bmass = fv(h.body_mass), bipos = fv(h.body_ipos),
                     binert = fv(h.body_inertia), jpos = fv(h.jnt_pos), jaxis = fv(h.jnt_axis),
                     gsize = fv(h.geom_size), gpos = fv(h.geom_pos), pmu = fv(h.pair_mu),
                     agear = fv(h.act_gear), akp = fv(h.act_kp), akd = fv(h.act_kd),
                     alo = fv(h.act_lo), ahi = fv(h.act_hi), aqd = fv(h.act_qdef),
                     q0 = fv(h.qpos0);
  pk.add(bpos, &d.body_pos);
  pk.add(body_rot, &d.body_rot);
  pk.add(bmass, &d.body_mass);
  pk.add(bipos, &d.body_ipos);
  pk.add(binert, &d.body_inertia);
  pk.add(jpos, &d.jnt_pos);
  pk.add(jaxis, &d.jnt_axis);
  pk.add(dof_armature, &d.dof_armature);
  pk.add(dof_damping, &d.dof_damping);
  pk.add(dof_vgain, &d.dof_vgain);
  pk.add(dof_hkp, &d.dof_hkp);
  pk.add(gsize, &d.geom_size);
  pk.add(gpos, &d.geom_pos);
  pk.add(geom_rot, &d.geom_rot);
  pk.add(pmu, &d.pair_mu);
  pk.add(agear, &d.act_gear);
  pk.add(akp, &d.act_kp);
  pk.add(akd, &d.act_kd);
  pk.add(alo, &d.act_lo);
  pk.add(ahi, &d.act_hi);
  pk.add(aqd, &d.act_qdef);
  pk.add(q0, &d.qpos0);
  std::vector<float> hf = fv(h.hf_data);
  pk.add(hf, &d.hf_data);
  pk.add(invw, const_cast<const float**>(&d.body_invweight));
  std::vector<float> dof_invw(h.nv, 0.f);
  pk.add(dof_invw, const_cast<const float**>(&d.dof_invweight));
  // on-chip layout in 4-byte words, regions packed back to back (every LDS access is a
  // scalar 32-bit one, so no region needs more alignment)
  int off = 0;
  auto take = [&](int words) {
    const int o = off;
    off += words;
    return o;
  };
  const int nb = h.nbody, nv = h.nv, nr = d.nrowmax;
  // persistent across the whole step
  d.o_qpos = take(h.nq);
  d.o_qvel = take(nv);
  d.o_qacc = take(nv);
  d.o_xpos = take(3 * nb);
  d.o_xmat = take(9 * nb);
  d.o_cdof = take(6 * nv);
  d.o_M = take(d.ntri);
  d.o_frc = take(nv);
  d.o_a0 = take(nv);
  d.o_scal = take(SC_COUNT);
  // the sweeps' scratch (velocities, bias accelerations, forces, inertias) is dead once
  // the mass matrix is built; the contact and Newton scratch reuses the same words
  const int shared = off;
  d.o_cvel = take(6 * nb);
  d.o_cacc = take(6 * nb);
  d.o_cfrc = take(6 * nb);
  d.o_cinert = take(kCinert * nb);
  d.o_F = take(6 * nv);
  const int sweep_end = off;
  off = shared;
  d.o_H = take(d.ntri);
  // Newton's vectors are born after the constraint rows, when the body poses and motion
  // subspaces are dead until the next step's kinematics: they live in xmat/cdof past
  // the world body's rotation (constant, set once per launch).
  d.o_Mr = d.o_xmat + 9;
  d.o_g = d.o_Mr + nv;
  d.o_d = d.o_g + nv;
  d.o_Md = d.o_d + nv;
  d.o_tmp = d.o_Md + nv;  // 5 nv words <= 9 (nbody - 1) + 6 nv, always
  // Candidates live from collision to contact selection, while the LTDL factor held in
  // H is already consumed and the Newton Hessian not yet built: they share H's words.
  if (2 * ncand <= d.ntri) d.o_cand = d.o_H;
  else d.o_cand = take(2 * ncand);
  d.o_con = take(kConRec * h.nconmax);
  d.o_lim = take(d.nlim);  // violated limits: joint-limit index | 0x10000 for the upper end
  d.o_J = take(njrow * nv);
  d.o_fw = take(nfw);
  // the reference accelerations are read once, when Newton forms its residuals, before
  // the first Hessian is built: they too share H's words
  d.o_aref = nr <= d.ntri ? d.o_H : take(nr);
  d.o_D = take(nr);
  d.o_e = take(nr);
  d.o_s = take(nr);
  // per-row force bound (0: one-sided row, F: friction loss, +inf: two-sided equality)
  d.o_fl = take(d.nfric + d.neq > 0 ? nr : 0);
  // elliptic cones: the Newton Hessian's rows (a cone's virtual rows, the others' own)
  // and every row's slope ds/de, left behind for the force export and implicit damping
  d.o_Jv = d.cone ? take(nr * nv) : 0;
  d.o_sl = d.cone ? take(nr) : 0;
  d.o_cv = d.cone ? take(h.nconmax * d.conrows * d.conrows) : 0;
  off = std::max(off, sweep_end);
  // fourth-order Runge-Kutta: the step's start (q0, v0), the first stage's acceleration
  // and the weighted sums of the stages' velocities and accelerations, alive across the
  // four forward passes
  d.o_rk = d.rk4 ? take(h.nq + 4 * nv) : 0;
  d.lds_words = off;
  // Table of the packed lower triangle at the head of a work-group's LDS: index
  // p = b (b + 1) / 2 + a -> row b, one byte (nv <= 64), four per word; a is recomputed.
  // One byte rather than two keeps a 64-lane world's work-group small enough for a
  // seventh humanoid world per CU.
  {
    std::vector<uint8_t> entry;
    for (int b = 0; b < h.nv; b++)
      for (int a = 0; a <= b; a++) entry.push_back((uint8_t)b);
    while (entry.size() & 3) entry.push_back(0);
    std::vector<uint32_t> tri_pair(entry.size() / 4);  // little-endian bytes
    for (size_t k = 0; k < tri_pair.size(); k++)
      tri_pair[k] = (uint32_t)entry[4 * k] | ((uint32_t)entry[4 * k + 1] << 8) |
                    ((uint32_t)entry[4 * k + 2] << 16) | ((uint32_t)entry[4 * k + 3] << 24);
    pk.add(tri_pair, &d.tri_pair);
  }
  // adjoint layout: the same tables, every region separate, plus the reverse-sweep
  // scratch (cotangents of dofs, bodies, rows and contacts)
  DevModel& x = rec.dm_adj;
  x = d;
  off = 0;
  x.o_qpos = take(h.nq); x.o_qvel = take(nv); x.o_qacc = take(nv);
  x.o_xpos = take(3 * nb); x.o_xmat = take(9 * nb); x.o_cdof = take(6 * nv);
  x.o_M = take(d.ntri); x.o_frc = take(nv); x.o_a0 = take(nv); x.o_scal = take(SC_COUNT);
  x.o_cvel = take(6 * nb); x.o_cacc = take(6 * nb); x.o_cfrc = take(6 * nb);
  x.o_cinert = take(kCinert * nb); x.o_F = take(6 * nv);
  x.o_H = take(d.ntri); x.o_Mr = take(nv); x.o_g = take(nv); x.o_d = take(nv);
  x.o_Md = take(nv); x.o_tmp = take(nv); x.o_cand = take(2 * ncand);
  x.o_con = take(kConRec * h.nconmax); x.o_lim = take(d.nlim); x.o_J = take(njrow * nv);
  x.o_aref = take(nr);
  x.o_D = take(nr); x.o_e = take(nr); x.o_s = take(nr); x.o_fl = take(d.nfric + d.neq > 0 ? nr : 0);
  x.o_rk = d.rk4 ? take(h.nq + 4 * nv) : 0;  // inside the images a reverse step restores
  x.o_qbi = take(h.nq); x.o_vbi = take(nv); x.o_qb = take(h.nq); x.o_vb = take(nv);
  x.o_Jv = x.o_sl = x.o_cv = 0;  // rollouts take pyramidal cones only
  x.o_ub = take(h.nu); x.o_mu = take(nv); x.o_Sbar = take(6 * nv);
  x.o_xbar = take(3 * nb); x.o_Rbar = take(9 * nb); x.o_cinbar = take(kCinert * nb);
  x.o_Vbar = take(6 * nb); x.o_Abar = take(6 * nb); x.o_Fbar = take(6 * nb);
  x.o_vup = take(6 * nb); x.o_aup = take(6 * nb); x.o_xup = take(3 * nb);
  x.o_Rup = take(9 * nb); x.o_rowsc = take(7 * nr); x.o_consc = take(kConSc * h.nconmax);
  x.o_eqsc = take(kEqSc * h.neq);
  x.o_rkb = d.rk4 ? take(h.nq + 4 * nv + h.nu) : 0;
  x.o_fw = take(nfw);
  x.lds_words = off;
  off = d.lds_words;
  d.lds_words = off;
  rec.cost = (double)nv * nv * (nv + 4.0 * nr) + 50.0 * nb + 30.0 * ncand;
  return MJH_OK;
}

}  // namespace

// ===================================================================== contexts
struct mjh_ctx {
  int device = 0;
  std::string err;
  std::vector<std::unique_ptr<ModelRec>> models;
  size_t lds_limit = 65536;  // dynamic LDS per work-group the device allows
  int num_cu = 0;
};

struct GroupRec {
  int model = 0;
  int nworld = 0;
  float* qpos = nullptr;
  float* qvel = nullptr;
  float* qacc = nullptr;
  int* status = nullptr;
  const float* ctrl = nullptr;
  int ctrl_nstep = 0;
  float* con_out = nullptr;
  int* ncon_out = nullptr;
  int team = 32;
  int block = 128;
};

struct mjh_batch {
  mjh_ctx* ctx = nullptr;
  std::vector<GroupRec> groups;
  DevGroup* d_groups = nullptr;
  DevTask* d_tasks = nullptr;
  int ntask = 0;
  int block = 64;
  int tab_words = 0;
  size_t lds_bytes = 0;
  bool rk4 = false;  // some group integrates by fourth-order Runge-Kutta
  bool cone = false; // some group's model has elliptic cones
  bool dirty = true;       // launch shape or world counts changed: rebuild the tables
  bool ptrs_dirty = false; // only bound pointers changed: rewrite d_groups in place
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int graph_nstep = 0;
  AdjointState* adj = nullptr;
};

#define MJH_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);                    \
      return MJH_EHIP;                                                                 \
    }                                                                                  \
  } while (0)

static mjh_status fail(mjh_ctx* ctx, mjh_status code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

// worlds per work-group for a group's launch shape, bounded by the LDS budget (the
// work-group also holds a triangular pair table of tab_words words)
static int worlds_per_block(const mjh_ctx* ctx, const ModelRec& mr, int team, int block,
                            int tab_words) {
  int wpb = std::max(1, block / team);
  const size_t per = (size_t)mr.dm.lds_words * sizeof(float);
  const size_t tab = (size_t)tab_words * sizeof(float);
  while (wpb > 1 && tab + (size_t)wpb * per > ctx->lds_limit) wpb--;
  return wpb;
}

// the kernel's view of every group: model tables, bound pointers, counts, team
static std::vector<DevGroup> group_table(const mjh_batch* b) {
  const mjh_ctx* ctx = b->ctx;
  std::vector<DevGroup> dg(b->groups.size());
  for (size_t g = 0; g < b->groups.size(); g++) {
    const GroupRec& gr = b->groups[g];
    DevGroup& x = dg[g];
    x.m = ctx->models[gr.model]->dm;
    x.qpos = gr.qpos; x.qvel = gr.qvel; x.qacc = gr.qacc; x.status = gr.status;
    x.ctrl = gr.ctrl; x.con_out = gr.con_out; x.ncon_out = gr.ncon_out;
    x.nworld = gr.nworld; x.ctrl_nstep = gr.ctrl_nstep; x.team = gr.team;
  }
  return dg;
}

// Bring the device group/task tables up to date (synchronous).  A new launch shape or
// world count rebuilds both tables and drops a captured graph.  New bound pointers
// alone are written into the existing group table in place: its device address, which
// a captured graph's kernel node holds, does not change, so the graph replays with the
// new pointers.
static mjh_status sync_tables(mjh_batch* b) {
  mjh_ctx* ctx = b->ctx;
  if (!b->dirty && b->ptrs_dirty && b->d_groups) {
    const std::vector<DevGroup> dg = group_table(b);
    // no launch of this batch may be reading the table while it is rewritten
    MJH_HIP(hipDeviceSynchronize());
    MJH_HIP(hipMemcpy(b->d_groups, dg.data(), dg.size() * sizeof(DevGroup), hipMemcpyHostToDevice));
    b->ptrs_dirty = false;
    return MJH_OK;
  }
  if (!b->dirty && !b->ptrs_dirty) return MJH_OK;
  const std::vector<DevGroup> dg = group_table(b);
  struct Tk { DevTask t; double cost; };
  std::vector<Tk> tasks;
  int block = 0;
  size_t lds = 0;
  int tab_words = 0;
  for (const GroupRec& gr : b->groups)
    if (gr.nworld > 0) tab_words = std::max(tab_words, table_words(ctx->models[gr.model]->dm));
  for (size_t g = 0; g < b->groups.size(); g++) {
    const GroupRec& gr = b->groups[g];
    const ModelRec& mr = *ctx->models[gr.model];
    if (gr.nworld == 0) continue;
    const int wpb = worlds_per_block(ctx, mr, gr.team, gr.block, tab_words);
    const size_t per = (size_t)mr.dm.lds_words * sizeof(float);
    const size_t tab = (size_t)tab_words * sizeof(float);
    if (tab + per > ctx->lds_limit)
      return fail(ctx, MJH_EUNSUPPORTED, "one world's working set exceeds the LDS limit");
    block = std::max(block, wpb * gr.team);
    lds = std::max(lds, tab + (size_t)wpb * per);
    for (int w0 = 0; w0 < gr.nworld; w0 += wpb) {
      Tk t;
      t.t.group = (int)g; t.t.w0 = w0; t.t.nw = std::min(wpb, gr.nworld - w0); t.t.pad_ = 0;
      t.cost = mr.cost * t.t.nw;
      tasks.push_back(t);
    }
  }
  // expensive work-groups first: the dispatcher then fills the device longest-first
  std::stable_sort(tasks.begin(), tasks.end(), [](const Tk& a, const Tk& c) { return a.cost > c.cost; });
  std::vector<DevTask> dt(tasks.size());
  for (size_t i = 0; i < tasks.size(); i++) dt[i] = tasks[i].t;
  if (b->d_groups) { (void)hipFree(b->d_groups); b->d_groups = nullptr; }
  if (b->d_tasks) { (void)hipFree(b->d_tasks); b->d_tasks = nullptr; }
  MJH_HIP(hipMalloc(&b->d_groups, std::max<size_t>(dg.size(), 1) * sizeof(DevGroup)));
  MJH_HIP(hipMalloc(&b->d_tasks, std::max<size_t>(dt.size(), 1) * sizeof(DevTask)));
  if (!dg.empty()) MJH_HIP(hipMemcpy(b->d_groups, dg.data(), dg.size() * sizeof(DevGroup), hipMemcpyHostToDevice));
  if (!dt.empty()) MJH_HIP(hipMemcpy(b->d_tasks, dt.data(), dt.size() * sizeof(DevTask), hipMemcpyHostToDevice));
  b->ntask = (int)dt.size();
  b->tab_words = tab_words;
  b->block = std::max(block, 16);
  b->lds_bytes = lds;
  b->rk4 = false;
  b->cone = false;
  for (const GroupRec& gr : b->groups) {
    if (gr.nworld > 0 && ctx->models[gr.model]->dm.rk4) b->rk4 = true;
    if (gr.nworld > 0 && ctx->models[gr.model]->dm.cone) b->cone = true;
  }
  b->dirty = false;
  b->ptrs_dirty = false;
  if (b->graph_exec) { (void)hipGraphExecDestroy(b->graph_exec); b->graph_exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  return MJH_OK;
}

// ===================================================================== C ABI
extern "C" {

mjh_status mjh_create(int device, mjh_ctx** out) {
  if (!out) return MJH_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return MJH_EINVAL;
  auto* ctx = new (std::nothrow) mjh_ctx();
  if (!ctx) return MJH_ENOMEM;
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess) { delete ctx; return MJH_EHIP; }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete ctx; return MJH_EHIP; }
  int lim = 0;
  if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lim > 0)
    ctx->lds_limit = (size_t)lim;
  ctx->num_cu = prop.multiProcessorCount;
  if (set_step_lds_limit(ctx->lds_limit) != hipSuccess || set_env_lds_limit(ctx->lds_limit) != hipSuccess)
    ctx->lds_limit = 65536;
  // the device address of the no-alloc rollouts' scratch, looked up once per device
  if (noalloc_scratch_init(device) != hipSuccess) { delete ctx; return MJH_EHIP; }
  *out = ctx;
  return MJH_OK;
}

void mjh_destroy(mjh_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  for (auto& m : ctx->models)
    if (m && m->dbuf) (void)hipFree(m->dbuf);
  delete ctx;
}

const char* mjh_last_error(const mjh_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

mjh_status mjh_model_upload(mjh_ctx* ctx, const void* blob, size_t nbytes, int32_t* model_id) {
  if (!ctx) return MJH_EINVAL;
  if (!blob || !model_id) return fail(ctx, MJH_EINVAL, "model_upload: NULL argument");
  ctx->err.clear();
  auto rec = std::make_unique<ModelRec>();
  std::string err;
  mjh_status st = parse_blob(static_cast<const uint8_t*>(blob), nbytes, rec->h, err);
  if (st != MJH_OK) return fail(ctx, st, err);
  Packer pk;
  st = compile_model(rec->h, *rec, pk, err);
  if (st != MJH_OK) return fail(ctx, st, err);
  if ((size_t)(rec->dm.lds_words + table_words(rec->dm)) * 4 > ctx->lds_limit)
    return fail(ctx, MJH_EUNSUPPORTED, "model working set exceeds the device's LDS per work-group");
  MJH_HIP(hipSetDevice(ctx->device));
  MJH_HIP(hipMalloc(&rec->dbuf, pk.bytes.size()));
  rec->dbytes = pk.bytes.size();
  MJH_HIP(hipMemcpy(rec->dbuf, pk.bytes.data(), pk.bytes.size(), hipMemcpyHostToDevice));
  uint8_t* base = static_cast<uint8_t*>(rec->dbuf);
  // every table pointer, in both layouts (the adjoint layout differs only in its
  // on-chip offsets, which compile_model set)
  for (auto& f : pk.fix) {
    const size_t field = reinterpret_cast<const uint8_t*>(f.second) -
                         reinterpret_cast<const uint8_t*>(&rec->dm);
    *f.second = base + f.first;
    *reinterpret_cast<const void**>(reinterpret_cast<uint8_t*>(&rec->dm_adj) + field) =
        base + f.first;
  }
  // translational inverse weights at qpos0, computed on the device
  MJH_HIP(launch_invweight(rec->dm, nullptr));
  MJH_HIP(hipDeviceSynchronize());
  *model_id = (int32_t)ctx->models.size();
  ctx->models.push_back(std::move(rec));
  return MJH_OK;
}

mjh_status mjh_model_info(mjh_ctx* ctx, int32_t model_id, mjh_dims* out) {
  if (!ctx) return MJH_EINVAL;
  if (!out || model_id < 0 || model_id >= (int)ctx->models.size())
    return fail(ctx, MJH_EINVAL, "model_info: bad model id or NULL output");
  const DevModel& d = ctx->models[model_id]->dm;
  out->nq = d.nq; out->nv = d.nv; out->nu = d.nu; out->nbody = d.nbody; out->ngeom = d.ngeom;
  out->npair = d.npair; out->ncand = d.ncand; out->nconmax = d.nconmax;
  out->iterations = d.iterations; out->lds_bytes = d.lds_words * 4; out->timestep = d.dt;
  out->nlimit = d.nlim; out->nrowmax = d.nrowmax; out->nfric = d.nfric; out->neq = d.neq;
  return MJH_OK;
}

mjh_status mjh_model_limit_invweight(mjh_ctx* ctx, int32_t model_id, float* out) {
  if (!ctx) return MJH_EINVAL;
  if (model_id < 0 || model_id >= (int)ctx->models.size() ||
      (!out && ctx->models[model_id]->dm.nlim > 0))
    return fail(ctx, MJH_EINVAL, "model_limit_invweight: bad model id or NULL output");
  const DevModel& d = ctx->models[model_id]->dm;
  if (d.nlim > 0) {
    std::vector<float> all(d.nv);
    MJH_HIP(hipMemcpy(all.data(), d.dof_invweight, d.nv * sizeof(float), hipMemcpyDeviceToHost));
    const ModelRec& rec = *ctx->models[model_id];
    int l = 0, da = 0;
    for (int j = 0; j < rec.h.njnt; j++) {
      if (rec.h.jnt_limited[j]) out[l++] = all[da];
      da += rec.h.jnt_type[j] == JNT_FREE ? 6 : 1;
    }
  }
  return MJH_OK;
}

mjh_status mjh_model_invweight(mjh_ctx* ctx, int32_t model_id, float* out) {
  if (!ctx) return MJH_EINVAL;
  if (!out || model_id < 0 || model_id >= (int)ctx->models.size())
    return fail(ctx, MJH_EINVAL, "model_invweight: bad model id or NULL output");
  const DevModel& d = ctx->models[model_id]->dm;
  MJH_HIP(hipMemcpy(out, d.body_invweight, d.nbody * sizeof(float), hipMemcpyDeviceToHost));
  return MJH_OK;
}

mjh_status mjh_world_alloc(mjh_ctx* ctx, const int32_t* model_ids, const int32_t* counts,
                           int32_t nmodel, mjh_batch** out) {
  if (!ctx) return MJH_EINVAL;
  if (!model_ids || !counts || !out || nmodel <= 0)
    return fail(ctx, MJH_EINVAL, "world_alloc: NULL argument or nmodel <= 0");
  *out = nullptr;
  auto* b = new (std::nothrow) mjh_batch();
  if (!b) return fail(ctx, MJH_ENOMEM, "world_alloc: out of host memory");
  b->ctx = ctx;
  for (int g = 0; g < nmodel; g++) {
    if (model_ids[g] < 0 || model_ids[g] >= (int)ctx->models.size() || counts[g] < 0) {
      delete b;
      return fail(ctx, MJH_EINVAL, "world_alloc: bad model id or negative count");
    }
    GroupRec gr;
    gr.model = model_ids[g];
    gr.nworld = counts[g];
    const DevModel& d = ctx->models[gr.model]->dm;
    // default launch shape: small trees take a quarter or half of a wavefront, large
    // ones a whole one.  A whole-wavefront world is its own work-group, so the LDS of a
    // CU can be filled one world at a time.
    gr.team = d.nv <= 8 ? 16 : (d.nrowmax <= 32 ? 32 : 64);
    gr.block = gr.team == 64 ? 64 : 128;
    b->groups.push_back(gr);
  }
  *out = b;
  return MJH_OK;
}

void mjh_world_free(mjh_batch* b) {
  if (!b) return;
  if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_groups) (void)hipFree(b->d_groups);
  if (b->d_tasks) (void)hipFree(b->d_tasks);
  adjoint_free(b->adj);
  delete b;
}

mjh_status mjh_bind_state(mjh_batch* b, int32_t group, float* qpos, float* qvel, float* qacc_ws,
                          int32_t* status) {
  if (!b) return MJH_EINVAL;
  mjh_ctx* ctx = b->ctx;
  if (group < 0 || group >= (int)b->groups.size())
    return fail(ctx, MJH_EINVAL, "bind_state: bad group");
  GroupRec& g = b->groups[group];
  if (g.nworld > 0 && (!qpos || !qvel || !qacc_ws))
    return fail(ctx, MJH_EINVAL, "bind_state: qpos, qvel and qacc_ws are required");
  g.qpos = qpos; g.qvel = qvel; g.qacc = qacc_ws; g.status = status;
  b->ptrs_dirty = true;
  return sync_tables(b);
}

mjh_status mjh_bind_io(mjh_batch* b, int32_t group, const float* ctrl, int32_t ctrl_nstep,
                       float* contact_out, int32_t* ncon_out) {
  if (!b) return MJH_EINVAL;
  mjh_ctx* ctx = b->ctx;
  if (group < 0 || group >= (int)b->groups.size())
    return fail(ctx, MJH_EINVAL, "bind_io: bad group");
  if (ctrl && ctrl_nstep <= 0) return fail(ctx, MJH_EINVAL, "bind_io: ctrl_nstep must be > 0");
  if (ncon_out && !contact_out) return fail(ctx, MJH_EINVAL, "bind_io: ncon_out needs contact_out");
  GroupRec& g = b->groups[group];
  g.ctrl = ctrl; g.ctrl_nstep = ctrl ? ctrl_nstep : 0;
  g.con_out = contact_out; g.ncon_out = ncon_out;
  b->ptrs_dirty = true;
  return sync_tables(b);
}

static mjh_status check_ready(mjh_batch* b, int32_t nstep) {
  mjh_ctx* ctx = b->ctx;
  if (nstep < 0) return fail(ctx, MJH_EINVAL, "step: nstep < 0");
  for (auto& g : b->groups) {
    if (g.nworld == 0) continue;
    if (!g.qpos || !g.qvel || !g.qacc) return fail(ctx, MJH_ESTATE, "step: state not bound");
    if (g.ctrl && nstep > g.ctrl_nstep)
      return fail(ctx, MJH_EINVAL, "step: nstep exceeds the bound control rows");
  }
  return MJH_OK;
}

mjh_status mjh_step(mjh_batch* b, int32_t nstep, void* stream) {
  if (!b) return MJH_EINVAL;
  mjh_ctx* ctx = b->ctx;
  mjh_status st = check_ready(b, nstep);
  if (st != MJH_OK) return st;
  st = sync_tables(b);
  if (st != MJH_OK) return st;
  if (nstep == 0 || b->ntask == 0) return MJH_OK;
  MJH_HIP(launch_step(b->d_groups, b->d_tasks, b->ntask, nstep, b->block, b->lds_bytes,
                      b->tab_words, b->rk4, b->cone, static_cast<hipStream_t>(stream)));
  return MJH_OK;
}

mjh_status mjh_env_step(mjh_batch* b, int32_t nenv, int32_t nsub, const float* action,
                        const float* command, const float* reset_qpos, const float* reset_qvel,
                        const float* params, const float* obs_noise, float* last_action,
                        float* obs, float* reward, int32_t* done, void* stream) {
  if (!b) return MJH_EINVAL;
  mjh_ctx* ctx = b->ctx;
  if (b->groups.size() != 1) return fail(ctx, MJH_EINVAL, "env_step: single-model batches only");
  if (nenv < 1 || nsub < 1) return fail(ctx, MJH_EINVAL, "env_step: need nenv >= 1 and nsub >= 1");
  const GroupRec& g = b->groups[0];
  const HostModel& h = ctx->models[g.model]->h;
  // the task's layout: a free root, then one position actuator per remaining dof, in order
  bool ok = h.njnt >= 1 && h.jnt_type[0] == JNT_FREE && h.jnt_body[0] == 1 && h.nu == h.nv - 6;
  std::vector<int> dofadr(h.njnt, 0);
  for (int j = 1; j < h.njnt; j++) dofadr[j] = dofadr[j - 1] + (h.jnt_type[j - 1] == JNT_FREE ? 6 : 1);
  for (int k = 0; ok && k < h.nu; k++)
    ok = h.act_type[k] == ACT_PD && dofadr[h.act_jnt[k]] == 6 + k;
  if (!ok)
    return fail(ctx, MJH_EUNSUPPORTED,
                "env_step: needs a free root joint and position actuator k on dof 6 + k");
  if (params && h.integrator != 0)
    return fail(ctx, MJH_EUNSUPPORTED,
                "env_step: per-world parameters with implicit damping are not supported");
  if (h.cone != 0)
    return fail(ctx, MJH_EUNSUPPORTED, "env_step: elliptic cones are not supported");
  if (g.nworld == 0) return MJH_OK;
  if (!action || !command || !reset_qpos || !reset_qvel || !last_action || !obs || !reward ||
      !done)
    return fail(ctx, MJH_EINVAL, "env_step: NULL argument");
  mjh_status st = check_ready(b, 0);
  if (st != MJH_OK) return st;
  st = sync_tables(b);
  if (st != MJH_OK) return st;
  const int teams = std::max(1, b->block / g.team);
  const int ndr = params ? 8 + 2 * h.nu : 0;
  const int ap_words = (teams * (h.nu + ndr) + 3) & ~3;
  const size_t lds = b->lds_bytes + (size_t)ap_words * sizeof(float);
  if (lds > ctx->lds_limit)
    return fail(ctx, MJH_EUNSUPPORTED, "env_step: work-group exceeds the LDS limit");
  EnvArgs E;
  E.nenv = nenv; E.nsub = nsub; E.nobs = 12 + 3 * h.nu;
  E.action = action; E.command = command; E.reset_qpos = reset_qpos; E.reset_qvel = reset_qvel;
  E.last_action = last_action; E.obs = obs; E.reward = reward; E.done = done;
  E.ndr = ndr; E.dr = params; E.noise = obs_noise;
  MJH_HIP(launch_env(b->d_groups, b->d_tasks, b->ntask, E, b->block, lds, b->tab_words, ap_words,
                     b->rk4, static_cast<hipStream_t>(stream)));
  return MJH_OK;
}

mjh_status mjh_graph_capture(mjh_batch* b, int32_t nstep, void* stream) {
  if (!b) return MJH_EINVAL;
  mjh_ctx* ctx = b->ctx;
  if (!stream) return fail(ctx, MJH_EINVAL, "graph_capture: needs a non-default stream");
  mjh_status st = check_ready(b, nstep);
  if (st != MJH_OK) return st;
  st = sync_tables(b);
  if (st != MJH_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (b->graph_exec) { (void)hipGraphExecDestroy(b->graph_exec); b->graph_exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  MJH_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  hipError_t le = launch_step(b->d_groups, b->d_tasks, b->ntask, nstep, b->block, b->lds_bytes,
                              b->tab_words, b->rk4, b->cone, s);
  hipGraph_t g = nullptr;
  hipError_t ce = hipStreamEndCapture(s, &g);
  if (le != hipSuccess || ce != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(ctx, MJH_EHIP, std::string("graph capture failed: ") +
                                   hipGetErrorString(le != hipSuccess ? le : ce));
  }
  b->graph = g;
  MJH_HIP(hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0));
  b->graph_nstep = nstep;
  return MJH_OK;
}

mjh_status mjh_graph_launch(mjh_batch* b, void* stream) {
  if (!b) return MJH_EINVAL;
  mjh_ctx* ctx = b->ctx;
  if (!b->graph_exec) return fail(ctx, MJH_ESTATE, "graph_launch: no captured graph");
  if (b->dirty) return fail(ctx, MJH_ESTATE, "graph_launch: launch shape changed; capture again");
  mjh_status st = check_ready(b, b->graph_nstep);
  if (st != MJH_OK) return st;
  MJH_HIP(hipGraphLaunch(b->graph_exec, static_cast<hipStream_t>(stream)));
  return MJH_OK;
}

mjh_status mjh_set_launch(mjh_batch* b, int32_t group, int32_t team, int32_t block) {
  if (!b) return MJH_EINVAL;
  mjh_ctx* ctx = b->ctx;
  if (group < 0 || group >= (int)b->groups.size())
    return fail(ctx, MJH_EINVAL, "set_launch: bad group");
  if (!(team == 16 || team == 32 || team == 64) || block < team || block > kMaxBlock ||
      block % team != 0)
    return fail(ctx, MJH_EINVAL, "set_launch: team in {16,32,64}, block a multiple of team <= 256");
  b->groups[group].team = team;
  b->groups[group].block = block;
  b->dirty = true;
  return sync_tables(b);
}

mjh_status mjh_get_launch(mjh_batch* b, int32_t group, int32_t* team, int32_t* block) {
  if (!b) return MJH_EINVAL;
  if (group < 0 || group >= (int)b->groups.size() || !team || !block)
    return fail(b->ctx, MJH_EINVAL, "get_launch: bad group or NULL output");
  *team = b->groups[group].team;
  *block = b->groups[group].block;
  return MJH_OK;
}

// Autotune cache key of a group: the model dimensions that set its cost, and its
// world count.  One line of the cache file is "<key> : <team> <block>".
static std::string tune_key(const DevModel& d, int nworld) {
  std::ostringstream k;
  k << d.nq << ' ' << d.nv << ' ' << d.nbody << ' ' << d.npair << ' ' << d.ncand << ' '
    << d.nconmax << ' ' << d.nlim << ' ' << d.nfric << ' ' << d.neq << ' ' << d.conrows << ' '
    << d.implicit << ' ' << d.rk4 << ' ' << d.cone << ' ' << d.iterations << ' ' << nworld;
  return k.str();
}

static bool valid_shape(int team, int block) {
  return (team == 16 || team == 32 || team == 64) && block >= team && block <= kMaxBlock &&
         block % team == 0;
}

// Time every candidate shape per group (other groups keep their shape), keep the
// fastest.  The bound state is saved before and restored after the probes, also when a
// probe fails; groups found in the cache are not probed.
mjh_status mjh_autotune(mjh_batch* b, int32_t nstep_probe, const char* cache_path) {
  if (!b) return MJH_EINVAL;
  mjh_ctx* ctx = b->ctx;
  if (nstep_probe <= 0) return fail(ctx, MJH_EINVAL, "autotune: nstep_probe must be > 0");
  mjh_status st = check_ready(b, nstep_probe);
  if (st != MJH_OK) return st;
  std::map<std::string, std::pair<int, int>> cache;
  if (cache_path) {
    std::ifstream f(cache_path);
    std::string line;
    while (std::getline(f, line)) {
      const size_t c = line.find(':');
      if (c == std::string::npos) continue;
      std::string key = line.substr(0, c);
      while (!key.empty() && key.back() == ' ') key.pop_back();
      std::istringstream is(line.substr(c + 1));
      int t = 0, bl = 0;
      if ((is >> t >> bl) && valid_shape(t, bl)) cache[key] = {t, bl};
    }
  }
  // save state
  struct Saved { std::vector<float> q, v, a; };
  std::vector<Saved> saved(b->groups.size());
  for (size_t g = 0; g < b->groups.size(); g++) {
    GroupRec& gr = b->groups[g];
    const DevModel& d = ctx->models[gr.model]->dm;
    saved[g].q.resize((size_t)gr.nworld * d.nq);
    saved[g].v.resize((size_t)gr.nworld * d.nv);
    saved[g].a.resize((size_t)gr.nworld * d.nv);
    if (gr.nworld == 0) continue;
    MJH_HIP(hipMemcpy(saved[g].q.data(), gr.qpos, saved[g].q.size() * 4, hipMemcpyDeviceToHost));
    MJH_HIP(hipMemcpy(saved[g].v.data(), gr.qvel, saved[g].v.size() * 4, hipMemcpyDeviceToHost));
    MJH_HIP(hipMemcpy(saved[g].a.data(), gr.qacc, saved[g].a.size() * 4, hipMemcpyDeviceToHost));
  }
  std::string herr;  // first failing HIP call of the probes
  auto hip_ok = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && herr.empty()) herr = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipSuccess;
  };
  auto restore = [&]() {
    bool ok = true;
    for (size_t g = 0; g < b->groups.size(); g++) {
      GroupRec& gr = b->groups[g];
      if (gr.nworld == 0) continue;
      ok = ok && hip_ok(hipMemcpy(gr.qpos, saved[g].q.data(), saved[g].q.size() * 4,
                                  hipMemcpyHostToDevice), "autotune: restore qpos");
      ok = ok && hip_ok(hipMemcpy(gr.qvel, saved[g].v.data(), saved[g].v.size() * 4,
                                  hipMemcpyHostToDevice), "autotune: restore qvel");
      ok = ok && hip_ok(hipMemcpy(gr.qacc, saved[g].a.data(), saved[g].a.size() * 4,
                                  hipMemcpyHostToDevice), "autotune: restore qacc_ws");
    }
    return ok;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool ok = hip_ok(hipEventCreate(&e0), "autotune: event") &&
            hip_ok(hipEventCreate(&e1), "autotune: event");
  const int teams[3] = {16, 32, 64};
  const int blocks[3] = {64, 128, 256};
  std::vector<int> counts;
  for (auto& o : b->groups) counts.push_back(o.nworld);
  // each probed group's shapes timed alone, for the combined pass below
  std::vector<std::vector<std::pair<float, std::pair<int, int>>>> solo(b->groups.size());
  auto probe = [&](float& ms) {
    bool good = true;
    for (int rep = 0; good && rep < 2; rep++) {  // the first run warms caches
      good = restore() && hip_ok(hipEventRecord(e0, nullptr), "autotune: event") &&
             hip_ok(launch_step(b->d_groups, b->d_tasks, b->ntask, nstep_probe, b->block,
                                b->lds_bytes, b->tab_words, b->rk4, b->cone, nullptr),
                    "autotune: probe launch") &&
             hip_ok(hipEventRecord(e1, nullptr), "autotune: event") &&
             hip_ok(hipEventSynchronize(e1), "autotune: probe") &&
             hip_ok(hipEventElapsedTime(&ms, e0, e1), "autotune: event");
    }
    return good;
  };
  for (size_t g = 0; ok && g < b->groups.size(); g++) {
    GroupRec& gr = b->groups[g];
    if (gr.nworld == 0) continue;
    const std::string key = tune_key(ctx->models[gr.model]->dm, gr.nworld);
    auto it = cache.find(key);
    if (it != cache.end()) {
      gr.team = it->second.first;
      gr.block = it->second.second;
      b->dirty = true;
      continue;
    }
    // time this group alone: other groups are switched off during its probes
    for (size_t o = 0; o < b->groups.size(); o++)
      if (o != g) b->groups[o].nworld = 0;
    float best = INFINITY;
    int bt = gr.team, bb = gr.block;
    for (int t : teams)
      for (int bl : blocks) {
        if (!ok || bl < t) continue;
        gr.team = t;
        gr.block = bl;
        b->dirty = true;
        st = sync_tables(b);
        if (st != MJH_OK) { ok = false; break; }
        float ms = 0.f;
        ok = probe(ms);
        if (ok) solo[g].push_back({ms, {t, bl}});
        if (ok && ms < best) { best = ms; bt = t; bb = bl; }
      }
    for (size_t o = 0; o < b->groups.size(); o++) b->groups[o].nworld = counts[o];
    gr.team = bt;
    gr.block = bb;
    b->dirty = true;
  }
  for (size_t o = 0; o < b->groups.size(); o++) b->groups[o].nworld = counts[o];
  // A batch of several groups runs as one launch whose block and LDS size are the
  // largest any group needs, so the groups' solo choices can starve each other (a group
  // of small worlds then holds the LDS of the largest group's work-group).  First, for
  // each work-group LDS size L that some group's shape needs, every group takes its
  // fastest solo shape within L (else its smallest): the fastest of these combinations
  // is kept.  Then one pass over the groups tries each of a group's shapes in the
  // combined launch (a group's solo ranking can mislead: alone, a small group may fill
  // the device only with shapes that spread its worlds thinly).
  int nactive = 0;
  for (auto& o : b->groups) nactive += o.nworld > 0;
  if (ok && nactive >= 2) {
    float cur = INFINITY;
    b->dirty = true;
    st = sync_tables(b);
    ok = st == MJH_OK && probe(cur);
    int tab_words = 0;
    for (auto& o : b->groups)
      if (o.nworld > 0) tab_words = std::max(tab_words, table_words(ctx->models[o.model]->dm));
    auto wg_lds = [&](size_t g, int t, int bl) {
      const ModelRec& mr = *ctx->models[b->groups[g].model];
      return (size_t)tab_words * sizeof(float) +
             (size_t)worlds_per_block(ctx, mr, t, bl, tab_words) * mr.dm.lds_words * sizeof(float);
    };
    std::vector<size_t> caps;
    for (size_t g = 0; g < b->groups.size(); g++)
      for (auto& s : solo[g]) caps.push_back(wg_lds(g, s.second.first, s.second.second));
    std::sort(caps.begin(), caps.end());
    caps.erase(std::unique(caps.begin(), caps.end()), caps.end());
    std::vector<std::pair<int, int>> best_shape(b->groups.size());
    for (size_t g = 0; g < b->groups.size(); g++) best_shape[g] = {b->groups[g].team, b->groups[g].block};
    for (size_t ci = 0; ok && ci < caps.size(); ci++) {
      bool same = true;
      for (size_t g = 0; g < b->groups.size(); g++) {
        if (solo[g].empty()) continue;  // not probed (a cached shape): kept as it is
        int pick = -1, small = 0;
        for (size_t k = 0; k < solo[g].size(); k++) {
          const int t = solo[g][k].second.first, bl = solo[g][k].second.second;
          const size_t l = wg_lds(g, t, bl);
          if (l <= caps[ci] && (pick < 0 || solo[g][k].first < solo[g][pick].first)) pick = (int)k;
          const size_t ls = wg_lds(g, solo[g][small].second.first, solo[g][small].second.second);
          if (l < ls || (l == ls && solo[g][k].first < solo[g][small].first)) small = (int)k;
        }
        if (pick < 0) pick = small;
        GroupRec& gr = b->groups[g];
        same = same && gr.team == solo[g][pick].second.first && gr.block == solo[g][pick].second.second;
        gr.team = solo[g][pick].second.first;
        gr.block = solo[g][pick].second.second;
      }
      if (same) continue;
      b->dirty = true;
      st = sync_tables(b);
      if (st != MJH_OK) { ok = false; break; }
      float ms = 0.f;
      ok = probe(ms);
      if (ok && ms < cur) {
        cur = ms;
        for (size_t g = 0; g < b->groups.size(); g++) best_shape[g] = {b->groups[g].team, b->groups[g].block};
      }
    }
    for (size_t g = 0; g < b->groups.size(); g++) {
      b->groups[g].team = best_shape[g].first;
      b->groups[g].block = best_shape[g].second;
    }
    b->dirty = true;
    for (size_t g = 0; ok && g < b->groups.size(); g++) {
      std::sort(solo[g].begin(), solo[g].end());
      GroupRec& gr = b->groups[g];
      for (size_t k = 0; ok && k < solo[g].size(); k++) {
        const int t = solo[g][k].second.first, bl = solo[g][k].second.second;
        if (t == gr.team && bl == gr.block) continue;
        const int t0 = gr.team, b0 = gr.block;
        gr.team = t;
        gr.block = bl;
        b->dirty = true;
        st = sync_tables(b);
        if (st != MJH_OK) { ok = false; break; }
        float ms = 0.f;
        ok = probe(ms);
        if (ok && ms < cur) {
          cur = ms;
        } else {
          gr.team = t0;
          gr.block = b0;
          b->dirty = true;
        }
      }
    }
  }
  for (size_t g = 0; ok && g < b->groups.size(); g++)
    if (b->groups[g].nworld > 0)
      cache[tune_key(ctx->models[b->groups[g].model]->dm, b->groups[g].nworld)] =
          {b->groups[g].team, b->groups[g].block};
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  const bool restored = restore();
  if (st == MJH_OK && !(ok && restored)) st = MJH_EHIP;
  const mjh_status ts = sync_tables(b);
  if (st == MJH_EHIP && !herr.empty()) ctx->err = herr;
  if (st == MJH_OK) st = ts;
  if (st == MJH_OK && cache_path) {
    std::ofstream f(cache_path);
    for (auto& kv : cache) f << kv.first << " : " << kv.second.first << ' ' << kv.second.second << '\n';
    if (!f) return fail(ctx, MJH_EINVAL, std::string("autotune: cannot write ") + cache_path);
  }
  return st;
}

}  // extern "C"

// The models the rollouts' reverse sweep covers: the contact geometry below with pyramid
// contacts of any dimension, connect and weld equalities, no elliptic cones, semi-implicit Euler or the implicit
// integrators (not RK4), bodies of at most four joints.
static mjh_status rollout_model_check(mjh_ctx* ctx, const ModelRec& mr) {
  // the reverse sweep covers the contact geometry of planes, spheres and capsules against
  // spheres and capsules, of planes against boxes, and of spheres against a heightfield
  // fixed in the world; and
  // bodies of at most four scalar joints
  for (int p = 0; p < mr.h.npair; p++) {
    const int g1 = mr.h.pair_g1[p], g2 = mr.h.pair_g2[p];
    const int t1 = mr.h.geom_type[g1], t2 = mr.h.geom_type[g2];
    const bool round2 = t2 == GEOM_SPHERE || t2 == GEOM_CAPSULE;
    const bool field = t1 == GEOM_SPHERE && t2 == GEOM_HFIELD && mr.h.geom_body[g2] == 0;
    const bool plane_box = t1 == GEOM_PLANE && t2 == GEOM_BOX;
    if (!field && !plane_box &&
        !(round2 && (t1 == GEOM_PLANE || t1 == GEOM_SPHERE || t1 == GEOM_CAPSULE)))
      return fail(ctx, MJH_EUNSUPPORTED,
                  "rollout: only contacts of planes, spheres and capsules with spheres and "
                  "capsules, of planes with boxes and of spheres with a fixed heightfield are "
                  "differentiated");
  }
  for (int p = 0; p < mr.h.npair; p++)
    if (mr.h.pair_condim[p] != 1 && mr.h.pair_condim[p] != 3 && mr.h.pair_condim[p] != 4 &&
        mr.h.pair_condim[p] != 6)
      return fail(ctx, MJH_EUNSUPPORTED, "rollout: contact dimension not differentiated");
  if (mr.h.cone != 0)
    return fail(ctx, MJH_EUNSUPPORTED, "rollout: elliptic cones are not differentiated");
  {
    std::vector<int> nj(mr.h.nbody, 0);
    for (int j = 0; j < mr.h.njnt; j++) nj[mr.h.jnt_body[j]]++;
    for (int b = 0; b < mr.h.nbody; b++)
      if (nj[b] > 4) return fail(ctx, MJH_EUNSUPPORTED, "rollout: a body has more than 4 joints");
  }
  return MJH_OK;
}

extern "C" {

mjh_status mjh_rollout_fwd(mjh_batch* b, int32_t horizon, int32_t ckpt_every, const float* ctrl,
                           int32_t zidx, float ztarget, float wctrl, float* loss,
                           int64_t* generation, void* stream) {
  if (!b) return MJH_EINVAL;
  mjh_ctx* ctx = b->ctx;
  if (b->groups.size() != 1) return fail(ctx, MJH_EINVAL, "rollout: single-model batches only");
  GroupRec& g = b->groups[0];
  const ModelRec& mr = *ctx->models[g.model];
  mjh_status st = rollout_model_check(ctx, mr);
  if (st != MJH_OK) return st;
  if ((mr.h.integrator == 1 || mr.h.integrator == 2) && mr.dm.nv > g.team)
    return fail(ctx, MJH_EUNSUPPORTED,
                "rollout: implicit integrators are differentiated for worlds of at most one "
                "dof per lane of their team");
  std::string err;
  st = adjoint_forward(&b->adj, mr.dm_adj, g.team, g.nworld, g.qpos, g.qvel, g.qacc, horizon,
                       ckpt_every, ctrl, zidx, ztarget, wctrl, loss, generation,
                       static_cast<hipStream_t>(stream), err);
  if (st != MJH_OK) return fail(ctx, st, err);
  return MJH_OK;
}

mjh_status mjh_rollout_bwd(mjh_batch* b, int64_t generation, const float* dloss,
                           float* grad_qvel0, float* grad_ctrl, void* stream) {
  if (!b) return MJH_EINVAL;
  mjh_ctx* ctx = b->ctx;
  std::string err;
  mjh_status st = adjoint_backward(b->adj, generation, dloss, grad_qvel0, grad_ctrl,
                                   static_cast<hipStream_t>(stream), err);
  if (st != MJH_OK) return fail(ctx, st, err);
  return MJH_OK;
}

mjh_status mjh_rollout_noalloc(mjh_batch* b, int32_t horizon, int32_t ckpt_every,
                               const float* ctrl, int32_t zidx, float ztarget, float wctrl,
                               const float* dloss, float* loss, float* grad_qvel0,
                               float* grad_ctrl, void* stream) {
  if (!b) return MJH_EINVAL;
  mjh_ctx* ctx = b->ctx;
  if (b->groups.size() != 1) return fail(ctx, MJH_EINVAL, "rollout: single-model batches only");
  GroupRec& g = b->groups[0];
  const ModelRec& mr = *ctx->models[g.model];
  mjh_status st = rollout_model_check(ctx, mr);
  if (st != MJH_OK) return st;
  std::string err;
  st = adjoint_noalloc(ctx->device, mr.dm_adj, g.team, g.nworld, g.qpos, g.qvel, g.qacc, horizon,
                       ckpt_every, ctrl, zidx, ztarget, wctrl, dloss, loss, grad_qvel0,
                       grad_ctrl, static_cast<hipStream_t>(stream), err);
  if (st != MJH_OK) return fail(ctx, st, err);
  return MJH_OK;
}

}  // extern "C"
