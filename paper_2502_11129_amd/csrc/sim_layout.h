// Internal layout of the packed model and state in the device workspace,
// shared by the host library (packing, launches) and the HIP kernels.
#pragma once
#include <stdint.h>

namespace simk {

constexpr int kGroup = 16;       // lanes cooperating on one variant (one DPP row)
constexpr int kVarPerWave = 4;   // 64-lane wave = 4 variants
constexpr int kMaxBodies = 32;   // body capacity of the largest bin (2 slots of 16)
constexpr int kQStride = 32;     // floats of q per variant (nq <= 29)
constexpr int kVStride = 32;     // floats of v per variant (nv <= 28)

// Body record: 24 words per body, bin stride = body capacity.
enum BodyWord {
  BW_HALF = 0,      // 3 half extents
  BW_MASS = 3,
  BW_AP = 4,        // anchor in the parent frame (3)
  BW_AC = 7,        // anchor in the child frame (3)
  BW_RQ = 10,       // rest quaternion w,x,y,z (4)
  BW_AXIS = 14,     // hinge axis, child frame (3)
  BW_CPG = 17,      // A, omega, phi (3)
  BW_PARENT = 20,   // int
  BW_DEPTH = 21,    // int
  BW_CHILDREN = 22, // uint bitmask over variant-local bodies
  BW_ANCESTORS = 23,// uint bitmask: ancestors-or-self
  BW_WORDS = 24
};

// Per-variant integer header.  HW_NV counts every DoF (the ball's too),
// HW_NVR the robot's only; the robot's q entries are HW_NQR.
enum HdrWord { HW_NB = 0, HW_NH, HW_NV, HW_R0, HW_MAXDEPTH, HW_USER, HW_NVR, HW_NQR, HW_WORDS };
// Per-variant float header: mu, fixed root pose (p[3], q[4]), ball radius and mass.
enum HdrfWord { HF_MU = 0, HF_ROOTP = 1, HF_ROOTQ = 4, HF_BALLR = 8, HF_BALLM = 9, HF_WORDS = 10 };

// Contact list entry (floats): plane-only kernels keep x, y, z and the
// ancestor mask of the body; ball and self-collision kernels add the normal,
// the depth, the kind (0 box corner - plane, 1 ball - plane, 2 ball - box,
// 3 box corner - box) and a second ancestor mask: a contact's rows act on
// (velocity of the CL_ANC body's point) - (velocity of the CL_MINUS body's
// point) + (the ball's, for kinds 1 and 2).
enum ListWord { CL_X = 0, CL_ANC = 3, CL_N = 4, CL_DEPTH = 7, CL_KIND = 8, CL_MINUS = 9 };
constexpr int kListWords = 4;
constexpr int kListWordsBall = 12;
// self-collision contacts a variant may have; beyond it the variant freezes
constexpr int kMaxSelfContacts = 256;

// Overflow scratch per contact (contacts that do not fit in registers).
constexpr int kOvfScal = 12;     // per-contact solver scalars

struct ModelParams {
  float kp, kd, tau_max, k_contact, b_contact, dt;
  float g[3];
  int K;
};

// Arguments of one bin's rollout kernel: device pointers into the workspace.
struct BinArgs {
  int n;                        // variants in this bin
  const int* hdr;               // [n][HW_WORDS]
  const float* hdrf;            // [n][HF_WORDS]
  const float* body;            // [n][nbc][BW_WORDS]
  const int* lvl;               // [n][lvl_stride]: bodies in depth order, then level start offsets
  int lvl_stride;
  const float* q0;              // [n][kQStride]
  const float* v0;              // [n][kVStride]
  float* q;                     // [n][kQStride]
  float* v;                     // [n][kVStride]
  long long* k;                 // [n]
  unsigned* status;             // [n]
  float* xy0;                   // [n][2]  core xy at k = 0
  float* fit;                   // [n]     fitness
  unsigned long long* cnt;      // [n][2]  contact rows, clamp rows
  float* ovf;                   // [n][ovf_stride]
  long long ovf_stride;         // floats per variant
  int n_steps;
  int reset;                    // 1: start from q0, v0 at k = 0
};

// All bins of a population in one launch: workgroups [block_start[i],
// block_start[i + 1]) run bin i with the kernel family kind[i] (an index into
// the multi-bin family list); bins are placed in decreasing cost order, so the
// most expensive workgroups are dispatched first.
constexpr int kMaxMultiBins = 8;
struct MultiArgs {
  int nbins;
  int kind[kMaxMultiBins];
  int block_start[kMaxMultiBins + 1];
  BinArgs bin[kMaxMultiBins];
};

// Overflow scratch layout per variant (floats):
//   list  [max_contacts][list_words]   contact list entries (ListWord)
//   scal  [max_contacts][kOvfScal]
//   rows  [max_contacts][6][nvc]  J_n, J_x, J_y, W_n, W_x, W_y
inline long long ovf_floats(int max_contacts, int nvc, int list_words) {
  return (long long)max_contacts * (list_words + kOvfScal + 6 * nvc);
}
// Largest contact count of a variant: 8 corners per box, plus for a ball one
// plane contact and one per box, plus the self-collision allowance.
constexpr int max_contacts(int nbc, bool ball, bool self = false) {
  return 8 * nbc + (ball ? 1 + nbc : 0) + (self ? kMaxSelfContacts : 0);
}

}  // namespace simk
