// Device-side model description and per-world on-chip layout.
//
// A model is uploaded once as a single device allocation of FP32 and int32 tables;
// DevModel holds the sizes, the derived constants and pointers into that allocation.
// Every kernel reads model tables through these pointers (they are identical for all
// worlds of a model, so they stay resident in L2 / the scalar cache).
#pragma once
#include <cstdint>

namespace mjh {

enum JointType : int { JNT_FREE = 0, JNT_SLIDE = 1, JNT_HINGE = 2 };
enum GeomType : int { GEOM_PLANE = 0, GEOM_SPHERE = 1, GEOM_CAPSULE = 2, GEOM_BOX = 3,
                      GEOM_HFIELD = 4 };
enum ActType : int { ACT_MOTOR = 0, ACT_PD = 1 };
// pair kinds (type(geom1) <= type(geom2)) and their candidate contact slots
enum PairKind : int {
  PK_PLANE_SPHERE = 0,   // 1 candidate
  PK_PLANE_CAPSULE = 1,  // 2: the two segment ends
  PK_PLANE_BOX = 2,      // 8 corners, at most 4 kept
  PK_SPHERE_SPHERE = 3,  // 1
  PK_SPHERE_CAPSULE = 4, // 1
  PK_SPHERE_BOX = 5,     // 1
  PK_CAPSULE_CAPSULE = 6,// 1
  PK_CAPSULE_BOX = 7,    // 4: ends + ends of the minimiser interval, at most 2 kept
  PK_SPHERE_HFIELD = 8   // 1: nearest point of the heightfield's triangles
};

constexpr int kMaxNv = 64;      // ancestor masks are 64-bit
constexpr int kConRec = 18;     // on-chip contact record (floats)
constexpr int kConOut = 20;     // exported contact record (MJH_CON_SIZE)
constexpr int kCinert = 10;     // spatial inertia: m, m c (3), I at origin (6)
constexpr int kEqSc = 24;       // adjoint scratch per equality: two anchors' and two
                                // rotations' cotangents
constexpr int kConSc = 28;      // adjoint scratch per contact: four (cotangent, body point)
                                // pairs, the two bodies, a flag

struct DevModel {
  // ---- sizes
  int nbody, njnt, nq, nv, nu, ngeom, npair, ncand, nconmax, nlim, nfric, neq, nrowmax;
  int neqrow;  // equality rows: 3 per connect, 6 per weld
  int conrows;   // rows of the widest contact (nrowmax = conrows nconmax + ...)
  int con_nr;    // rows of every contact when all pairs have the same count (4: pyramid,
                 // 3: elliptic cone, both condim 3; contact c's rows are con_nr c ..),
                 // else 0 (first row and count packed in the contact record)
  int cone;      // friction cone: 0 pyramidal (edge rows), 1 elliptic (frame rows)
  int jframe;    // 1: every contact is a condim-3 pyramid whose Jacobian is stored as its
                 // three frame rows (normal, t1, t2); its four edge rows J_n +- mu J_tk
                 // are formed where they are used.  Contact c's frames are J rows 3c ..
                 // 3c + 2, its edges rows 4c .. 4c + 3 of the per-row arrays, and a
                 // non-contact row r >= 4 ncon is J row r - ncon.
  int iterations, nlevel, nmpair, ntri;
  int implicit;  // 1: joint damping and PD velocity gains integrated implicitly;
                 // 2: also the PD position gains
  int rk4;       // 1: fourth-order Runge-Kutta (forward pass at four stages)
  int hf_nrow, hf_ncol;  // heightfield grid (0 without one)
  float hf_size[3];      // half extents x, y and the height scale
  // ---- constants
  float dt, K, B;                       // soft-constraint stiffness/damping
  float dmin, dmax, width, mid, power;  // impedance (solimp)
  float grav[3];
  // ---- int tables
  const int* body_parent;
  const int* body_jntadr;
  const int* body_jntnum;
  const int* body_dofadr;
  const int* body_dofnum;
  const int* level_start;   // [nlevel + 1] into level_body
  const int* level_body;    // bodies sorted by tree depth (level 0 = world)
  const int* child_start;   // [nbody + 1] CSR of children
  const int* child_list;
  const int* jnt_type;
  const int* jnt_qposadr;
  const int* jnt_dofadr;
  const int* dof_body;
  const int* dof_act;       // actuator driving the dof, or -1
  const int* anc_start;     // [nv + 1] strict dof ancestors, nearest first
  const int* anc_list;
  const int* mpair;         // [nmpair] (i << 16) | j, j ancestor-or-self of i
  const unsigned long long* body_dofmask;  // dofs on the path body -> root
  const unsigned* tri_pair;  // [(ntri + 3) / 4] row b of packed index p = b (b + 1) / 2 + a,
                             // one byte each, four per word (p % 4 == 0: low byte)
  const int* geom_type;
  const int* geom_body;
  const int* pair_g1;
  const int* pair_g2;
  const int* pair_kind;
  const int* pair_candadr;  // first candidate slot of each pair
  const int* cand_pair;     // [ncand] owning pair
  const int* act_type;
  const int* act_qadr;
  const int* act_dadr;
  const int* lim_qadr;      // [nlim] qpos address of each limited joint (joint order)
  const int* lim_dadr;      // [nlim] its dof
  const int* fric_dadr;     // [nfric] dofs with friction loss (dof order)
  const int* eq_body;       // [neq][2] equalities: body1, body2 (0 = world)
  const int* eq_row;        // [neqrow] equality | component << 16 (3-5: a weld's rotation)
  // ---- float tables
  const float* body_pos;      // [nbody][3] in parent frame
  const float* body_rot;      // [nbody][9] in parent frame
  const float* body_mass;
  const float* body_ipos;     // [nbody][3]
  const float* body_inertia;  // [nbody][6] xx yy zz xy xz yz (body frame, about COM)
  const float* jnt_pos;       // [njnt][3]
  const float* jnt_axis;      // [njnt][3] unit
  const float* dof_armature;
  const float* dof_damping;
  const float* dof_vgain;     // [nv] damping + velocity gains of PD actuators on the dof
                              // (+ h kp with implicit position gains)
  const float* dof_hkp;       // [nv] h kp of a PD actuator on the dof (implicit position
                              // gains only, else 0)
  const float* geom_size;     // [ngeom][3]
  const float* geom_pos;      // [ngeom][3]
  const float* geom_rot;      // [ngeom][9]
  const float* pair_mu;
  const int* pair_condim;     // [npair] 1 frictionless (1 row); 3 sliding (4 rows); 4 and
                              // torsion (6); 6 and rolling (10)
  const float* pair_mu_t;     // [npair] torsional friction coefficient (condim >= 4)
  const float* pair_mu_r;     // [npair] rolling friction coefficient (condim 6)
  const float* act_gear;
  const float* act_kp;
  const float* act_kd;
  const float* act_lo;
  const float* act_hi;
  const float* act_qdef;
  const float* qpos0;
  const float* hf_data;       // [hf_nrow][hf_ncol] elevations in [0, 1]
  const float* lim_lo;        // [nlim] range of each limited joint
  const float* lim_hi;
  const float* fric_loss;     // [nfric] friction-loss bound of each such dof
  const float* eq_anchor;     // [neq][6] the held point in body1's and in body2's frame
  const float* eq_relR;       // [neq][9] weld: body2's reference orientation in body1's frame
  float* body_invweight;      // filled on the device at upload
  float* dof_invweight;       // [nv] (M^-1)_kk at qpos0 (limit and friction rows), likewise
  // ---- per-world on-chip layout (offsets in 4-byte words)
  int lds_words;
  int o_qpos, o_qvel, o_qacc;
  int o_xpos, o_xmat, o_cvel, o_cacc, o_cfrc, o_cinert, o_cdof, o_F;
  int o_M, o_H;
  int o_frc, o_a0, o_Mr, o_g, o_d, o_Md, o_tmp;
  int o_cand, o_con, o_lim, o_J, o_aref, o_D, o_e, o_s, o_fl, o_scal;
  int o_fw;  // jframe only: per-frame staging of products and weights, and each
             // contact's five Hessian coefficients (5 nconmax + non-contact rows words)
  int o_rk;  // Runge-Kutta block (rk4 only): q0 [nq], v0, a1, vsum, asum [nv each]
  int o_Jv, o_sl;  // elliptic cones only: Hessian rows [nrowmax][nv], row slopes [nrowmax]
  int o_cv;        // elliptic cones only: each contact's virtual-row map [nconmax][conrows^2]
  // adjoint layout only (no aliasing between the sweep and contact scratch there)
  int o_qbi, o_vbi, o_qb, o_vb, o_ub, o_mu, o_Sbar, o_xbar, o_Rbar, o_cinbar;
  int o_Vbar, o_Abar, o_Fbar, o_vup, o_aup, o_xup, o_Rup, o_rowsc, o_consc, o_eqsc;
  int o_rkb;  // rk4 only: a step's cotangent sums [nq + 4 nv + nu] across its stages
};

// scalar slots inside o_scal: the contact count, the row count (the contacts' rows, then
// one per violated joint limit, one per friction-loss dof and the equality rows) and the
// contacts' rows alone
enum ScalSlot : int {
  SC_NCON = 0, SC_NROW = 1, SC_NRC = 2, SC_COUNT = 4
};

// one group of worlds of the same model inside a batch, as the kernel sees it
struct DevGroup {
  DevModel m;
  float* qpos;
  float* qvel;
  float* qacc;
  int* status;
  const float* ctrl;
  float* con_out;
  int* ncon_out;
  int nworld;
  int ctrl_nstep;
  int team;       // lanes per world
  int pad_;
};

// a work item: one work-group advances worlds [w0, w0 + nw) of group g
struct DevTask {
  int group, w0, nw, pad_;
};

}  // namespace mjh
