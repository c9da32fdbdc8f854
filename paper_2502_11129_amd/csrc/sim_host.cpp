// Host side of the C ABI in include/sim.h: validation, packing of variants
// into DoF bins, workspace layout, launches, state transfer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "sim.h"
#include "launch.h"
#include "sim_layout.h"

using namespace simk;

namespace {

constexpr int kNvCaps[] = {8, 12, 16, 20, 24, 28};
constexpr int kMaxNv = 28;
constexpr int kMaxBodiesPerVariant = 32;
constexpr int kStepsPerLaunch = 1000;  // long runs are split so each launch stays short

std::string g_create_error;

struct Bin {
  int nvc = 0, sb = 0, ncr = 0;
  launch_fn fn = nullptr;
  std::vector<int> users;  // user index of each packed variant
  // packed host copies (uploaded by sim_bind)
  std::vector<int> hdr;
  std::vector<float> hdrf, body, q0, v0;
  // device offsets (bytes from the workspace base)
  size_t o_hdr, o_hdrf, o_body, o_q0, o_v0, o_q, o_v, o_k, o_status, o_xy0, o_fit, o_cnt, o_ovf;
  long long ovf_stride = 0;
  BinArgs args{};
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct sim_handle {
  int n = 0;
  int root_type = 0;
  ModelParams params{};
  sim_options opts{};
  std::vector<int> nq, nv, q_off, v_off;
  std::vector<Bin> bins;
  std::vector<int> bin_of, slot_of;  // user variant -> (bin, packed index)
  size_t ws_bytes = 0;
  char* ws = nullptr;
  bool bound = false;
  bool device_error = false;
  std::string err;
  // graph of a rollout of graph_T steps (replayed when use_graph != 0)
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int graph_T = -1;
  hipStream_t cap_stream = nullptr;
};

namespace {

int fail(sim_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg; else g_create_error = msg;
  return code;
}

int dev_check(sim_handle* h, hipError_t e, const char* what) {
  if (e == hipSuccess) return SIM_OK;
  h->device_error = true;
  h->err = std::string(what) + ": " + hipGetErrorString(e);
  return SIM_E_DEVICE;
}

bool finite_all(const float* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

const KernelVariant* find_variant(int nvc, int sb, int ncr) {
  for (int i = 0; i < kNumKernelVariants; ++i) {
    const KernelVariant& k = kKernelVariants[i];
    if (k.nvc == nvc && k.sb == sb && (ncr <= 0 || k.ncr == ncr)) return &k;
  }
  return nullptr;
}

// Launch every bin's kernel for n_steps (reset on the first chunk if asked).
int launch_all(sim_handle* h, int n_steps, bool reset, hipStream_t st) {
  int done = 0;
  bool first = true;
  while (first || done < n_steps) {
    const int chunk = std::min(kStepsPerLaunch, n_steps - done);
    for (Bin& b : h->bins) {
      BinArgs a = b.args;
      a.n_steps = chunk;
      a.reset = (reset && first) ? 1 : 0;
      hipError_t e = b.fn(a, h->params, st);
      if (e != hipSuccess) return dev_check(h, e, "kernel launch");
    }
    done += chunk;
    first = false;
  }
  return SIM_OK;
}

}  // namespace

extern "C" {

int sim_create(const sim_model_desc* d, const sim_options* opts, sim_handle** out) {
  if (out) *out = nullptr;
  if (!d || !out) return fail(nullptr, SIM_E_INVALID, "null descriptor or output pointer");
  std::unique_ptr<sim_handle> h(new sim_handle());
  sim_handle* hp = h.get();
  auto bad = [&](const std::string& m) {
    g_create_error = m;
    return SIM_E_INVALID;
  };
  if (d->n_variants < 1) return bad("n_variants must be >= 1");
  if (d->root_type != SIM_ROOT_FREE && d->root_type != SIM_ROOT_FIXED) return bad("root_type must be FREE or FIXED");
  if (!d->body_offset || !d->parent || !d->half_ext || !d->mass || !d->anchor_parent || !d->anchor_child ||
      !d->rest_quat || !d->axis || !d->cpg || !d->mu || !d->q0 || !d->v0)
    return bad("a required model array is NULL");
  if (d->root_type == SIM_ROOT_FIXED && !d->root_pose) return bad("FIXED roots need root_pose");
  if (!(d->dt > 0.f) || !std::isfinite(d->dt)) return bad("dt must be > 0");
  if (d->pgs_iters < 1) return bad("pgs_iters must be >= 1");
  const float prm[] = {d->kp, d->kd, d->tau_max, d->k_contact, d->b_contact, d->gravity[0], d->gravity[1], d->gravity[2]};
  if (!finite_all(prm, 8)) return bad("non-finite model constant");
  if (d->kp < 0 || d->kd < 0 || d->tau_max < 0 || d->k_contact < 0 || d->b_contact < 0)
    return bad("gains, torque limit and contact constants must be >= 0");
  if (opts) hp->opts = *opts;
  const int n = d->n_variants;
  hp->n = n;
  hp->root_type = d->root_type;
  hp->params = ModelParams{d->kp, d->kd, d->tau_max, d->k_contact, d->b_contact, d->dt,
                           {d->gravity[0], d->gravity[1], d->gravity[2]}, d->pgs_iters};
  const int r0 = d->root_type == SIM_ROOT_FREE ? 6 : 0;
  if (d->body_offset[0] != 0) return bad("body_offset[0] must be 0");
  hp->nq.resize(n); hp->nv.resize(n); hp->q_off.resize(n + 1); hp->v_off.resize(n + 1);
  hp->q_off[0] = hp->v_off[0] = 0;
  for (int i = 0; i < n; ++i) {
    const int nb = d->body_offset[i + 1] - d->body_offset[i];
    if (nb < 1 || nb > kMaxBodiesPerVariant) return bad("variant " + std::to_string(i) + ": 1..32 bodies required");
    const int nh = nb - 1;
    hp->nv[i] = r0 + nh;
    hp->nq[i] = (r0 ? 7 : 0) + nh;
    if (hp->nv[i] < 1 || hp->nv[i] > kMaxNv)
      return bad("variant " + std::to_string(i) + ": degrees of freedom must be in 1..28");
    hp->q_off[i + 1] = hp->q_off[i] + hp->nq[i];
    hp->v_off[i + 1] = hp->v_off[i] + hp->nv[i];
  }
  // per-body checks and derived topology
  struct VInfo { int nb, maxdepth; std::vector<int> depth; std::vector<unsigned> children, anc; };
  std::vector<VInfo> info(n);
  for (int i = 0; i < n; ++i) {
    const int b0 = d->body_offset[i], nb = d->body_offset[i + 1] - b0;
    VInfo& vi = info[i];
    vi.nb = nb;
    vi.depth.assign(nb, 0);
    vi.children.assign(nb, 0u);
    vi.anc.assign(nb, 0u);
    vi.maxdepth = 0;
    for (int b = 0; b < nb; ++b) {
      const int g = b0 + b, p = d->parent[g];
      const std::string where = "variant " + std::to_string(i) + " body " + std::to_string(b);
      if (b == 0 && p != -1) return bad(where + ": the core must have parent -1");
      if (b > 0 && (p < 0 || p >= b)) return bad(where + ": parent must satisfy 0 <= parent < child");
      for (int k = 0; k < 3; ++k)
        if (!(d->half_ext[3 * g + k] > 0.f) || !std::isfinite(d->half_ext[3 * g + k])) return bad(where + ": half extents must be > 0");
      if (!(d->mass[g] > 0.f) || !std::isfinite(d->mass[g])) return bad(where + ": mass must be > 0");
      const float* ax = d->axis + 3 * g;
      const float* rq = d->rest_quat + 4 * g;
      if (!finite_all(ax, 3) || !finite_all(rq, 4) || !finite_all(d->anchor_parent + 3 * g, 3) ||
          !finite_all(d->anchor_child + 3 * g, 3) || !finite_all(d->cpg + 3 * g, 3))
        return bad(where + ": non-finite geometry or CPG");
      const float an = std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
      const float qn = std::sqrt(rq[0] * rq[0] + rq[1] * rq[1] + rq[2] * rq[2] + rq[3] * rq[3]);
      if (b > 0 && std::fabs(an - 1.f) > 1e-5f) return bad(where + ": hinge axis must be a unit vector");
      if (std::fabs(qn - 1.f) > 1e-5f) return bad(where + ": rest quaternion must be a unit quaternion");
      if (b > 0) {
        vi.depth[b] = vi.depth[p] + 1;
        vi.children[p] |= 1u << b;
      }
      vi.maxdepth = std::max(vi.maxdepth, vi.depth[b]);
      for (int j = b; j >= 0; j = (j == 0 ? -1 : d->parent[b0 + j])) vi.anc[b] |= 1u << j;
    }
    if (!(d->mu[i] >= 0.f) || !std::isfinite(d->mu[i])) return bad("variant " + std::to_string(i) + ": mu must be >= 0");
    if (!finite_all(d->q0 + hp->q_off[i], hp->nq[i]) || !finite_all(d->v0 + hp->v_off[i], hp->nv[i]))
      return bad("variant " + std::to_string(i) + ": non-finite initial state");
    const float* q = (r0 ? d->q0 + hp->q_off[i] + 3 : d->root_pose + 7 * i + 3);
    const float qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (std::fabs(qn - 1.f) > 1e-5f) return bad("variant " + std::to_string(i) + ": root quaternion must be a unit quaternion");
  }
  // bins: smallest DoF capacity, body slots from the body count
  const int want_ncr = hp->opts.contacts_in_registers;
  std::vector<std::pair<int, int>> keys(n);
  for (int i = 0; i < n; ++i) {
    int nvc = 0;
    for (int c : kNvCaps)
      if (hp->nv[i] <= c) { nvc = c; break; }
    const int sb_need = info[i].nb > 16 ? 2 : 1;
    // smallest compiled (nv capacity, body slots) that holds the variant
    int sb = 0;
    for (; nvc <= kMaxNv; nvc += 4) {
      if (find_variant(nvc, sb_need, want_ncr)) { sb = sb_need; break; }
      if (sb_need == 1 && find_variant(nvc, 2, want_ncr)) { sb = 2; break; }
    }
    if (!sb)
      return bad("no compiled kernel for nv=" + std::to_string(hp->nv[i]) + " bodies=" + std::to_string(info[i].nb) +
                 " contacts_in_registers=" + std::to_string(want_ncr));
    keys[i] = {nvc, sb};
  }
  std::vector<std::pair<int, int>> uk = keys;
  std::sort(uk.begin(), uk.end());
  uk.erase(std::unique(uk.begin(), uk.end()), uk.end());
  hp->bin_of.assign(n, -1);
  hp->slot_of.assign(n, -1);
  for (auto& kk : uk) {
    Bin b;
    b.nvc = kk.first;
    b.sb = kk.second;
    const KernelVariant* kv = find_variant(b.nvc, b.sb, want_ncr);
    b.ncr = kv->ncr;
    b.fn = kv->fn;
    for (int i = 0; i < n; ++i)
      if (keys[i] == kk) b.users.push_back(i);
    // within a bin, neighbours in a wave should share nv and tree depth
    std::stable_sort(b.users.begin(), b.users.end(), [&](int x, int y) {
      if (hp->nv[x] != hp->nv[y]) return hp->nv[x] > hp->nv[y];
      return info[x].maxdepth > info[y].maxdepth;
    });
    hp->bins.push_back(std::move(b));
  }
  // pack
  for (size_t bi = 0; bi < hp->bins.size(); ++bi) {
    Bin& b = hp->bins[bi];
    const int nbc = 16 * b.sb;
    const int m = (int)b.users.size();
    b.hdr.assign((size_t)m * HW_WORDS, 0);
    b.hdrf.assign((size_t)m * HF_WORDS, 0.f);
    b.body.assign((size_t)m * nbc * BW_WORDS, 0.f);
    b.q0.assign((size_t)m * kQStride, 0.f);
    b.v0.assign((size_t)m * kVStride, 0.f);
    for (int s = 0; s < m; ++s) {
      const int i = b.users[s];
      hp->bin_of[i] = (int)bi;
      hp->slot_of[i] = s;
      const VInfo& vi = info[i];
      int* hd = &b.hdr[(size_t)s * HW_WORDS];
      hd[HW_NB] = vi.nb; hd[HW_NH] = vi.nb - 1; hd[HW_NV] = hp->nv[i]; hd[HW_R0] = r0;
      hd[HW_MAXDEPTH] = vi.maxdepth; hd[HW_USER] = i;
      float* hf = &b.hdrf[(size_t)s * HF_WORDS];
      hf[HF_MU] = d->mu[i];
      if (!r0) {
        for (int k = 0; k < 3; ++k) hf[HF_ROOTP + k] = d->root_pose[7 * i + k];
        for (int k = 0; k < 4; ++k) hf[HF_ROOTQ + k] = d->root_pose[7 * i + 3 + k];
      }
      const int b0 = d->body_offset[i];
      for (int bb = 0; bb < vi.nb; ++bb) {
        const int g = b0 + bb;
        float* rec = &b.body[((size_t)s * nbc + bb) * BW_WORDS];
        for (int k = 0; k < 3; ++k) {
          rec[BW_HALF + k] = d->half_ext[3 * g + k];
          rec[BW_AP + k] = d->anchor_parent[3 * g + k];
          rec[BW_AC + k] = d->anchor_child[3 * g + k];
          rec[BW_AXIS + k] = d->axis[3 * g + k];
          rec[BW_CPG + k] = d->cpg[3 * g + k];
        }
        for (int k = 0; k < 4; ++k) rec[BW_RQ + k] = d->rest_quat[4 * g + k];
        rec[BW_MASS] = d->mass[g];
        int par = d->parent[g], dep = vi.depth[bb];
        unsigned ch = vi.children[bb], an = vi.anc[bb];
        std::memcpy(&rec[BW_PARENT], &par, 4);
        std::memcpy(&rec[BW_DEPTH], &dep, 4);
        std::memcpy(&rec[BW_CHILDREN], &ch, 4);
        std::memcpy(&rec[BW_ANCESTORS], &an, 4);
      }
      std::copy(d->q0 + hp->q_off[i], d->q0 + hp->q_off[i + 1], &b.q0[(size_t)s * kQStride]);
      std::copy(d->v0 + hp->v_off[i], d->v0 + hp->v_off[i + 1], &b.v0[(size_t)s * kVStride]);
    }
  }
  // workspace layout
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  for (Bin& b : hp->bins) {
    const size_t m = b.users.size();
    b.ovf_stride = ovf_floats(8 * 16 * b.sb, b.nvc);
    b.o_hdr = take(m * HW_WORDS * 4);
    b.o_hdrf = take(m * HF_WORDS * 4);
    b.o_body = take(m * 16 * b.sb * BW_WORDS * 4);
    b.o_q0 = take(m * kQStride * 4);
    b.o_v0 = take(m * kVStride * 4);
    b.o_q = take(m * kQStride * 4);
    b.o_v = take(m * kVStride * 4);
    b.o_k = take(m * 8);
    b.o_status = take(m * 4);
    b.o_xy0 = take(m * 8);
    b.o_fit = take(m * 4);
    b.o_cnt = take(m * 16);
    b.o_ovf = take(m * (size_t)b.ovf_stride * 4);
  }
  hp->ws_bytes = off;
  *out = h.release();
  return SIM_OK;
}

int sim_workspace_bytes(const sim_handle* h, size_t* bytes) {
  if (!h || !bytes) return SIM_E_INVALID;
  *bytes = h->ws_bytes;
  return SIM_OK;
}

int sim_bind(sim_handle* h, void* ws, size_t bytes, void* stream) {
  if (!h) return SIM_E_INVALID;
  if (!ws) return fail(h, SIM_E_INVALID, "workspace pointer is NULL");
  if (bytes < h->ws_bytes) return fail(h, SIM_E_NOMEM, "workspace smaller than sim_workspace_bytes()");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(h, SIM_E_INVALID, "workspace must be 256-byte aligned");
  if (h->device_error) return SIM_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  h->ws = (char*)ws;
  for (Bin& b : h->bins) {
    char* base = h->ws;
    const size_t m = b.users.size();
    int rc;
    if ((rc = dev_check(h, hipMemcpyAsync(base + b.o_hdr, b.hdr.data(), m * HW_WORDS * 4, hipMemcpyHostToDevice, st), "upload"))) return rc;
    if ((rc = dev_check(h, hipMemcpyAsync(base + b.o_hdrf, b.hdrf.data(), m * HF_WORDS * 4, hipMemcpyHostToDevice, st), "upload"))) return rc;
    if ((rc = dev_check(h, hipMemcpyAsync(base + b.o_body, b.body.data(), b.body.size() * 4, hipMemcpyHostToDevice, st), "upload"))) return rc;
    if ((rc = dev_check(h, hipMemcpyAsync(base + b.o_q0, b.q0.data(), b.q0.size() * 4, hipMemcpyHostToDevice, st), "upload"))) return rc;
    if ((rc = dev_check(h, hipMemcpyAsync(base + b.o_v0, b.v0.data(), b.v0.size() * 4, hipMemcpyHostToDevice, st), "upload"))) return rc;
    BinArgs& a = b.args;
    a.n = (int)m;
    a.hdr = (const int*)(base + b.o_hdr);
    a.hdrf = (const float*)(base + b.o_hdrf);
    a.body = (const float*)(base + b.o_body);
    a.q0 = (const float*)(base + b.o_q0);
    a.v0 = (const float*)(base + b.o_v0);
    a.q = (float*)(base + b.o_q);
    a.v = (float*)(base + b.o_v);
    a.k = (long long*)(base + b.o_k);
    a.status = (unsigned*)(base + b.o_status);
    a.xy0 = (float*)(base + b.o_xy0);
    a.fit = (float*)(base + b.o_fit);
    a.cnt = (unsigned long long*)(base + b.o_cnt);
    a.ovf = (float*)(base + b.o_ovf);
    a.ovf_stride = b.ovf_stride;
  }
  // pageable host buffers: make the uploads complete before returning
  int rc = dev_check(h, hipStreamSynchronize(st), "upload sync");
  if (rc) return rc;
  h->bound = true;
  // initial state: a zero-step rollout copies (q0, v0) and clears counters
  rc = launch_all(h, 0, true, st);
  if (rc) return rc;
  return dev_check(h, hipStreamSynchronize(st), "initial state");
}

int sim_step_batch(sim_handle* h, int32_t n_steps, void* stream) {
  if (!h) return SIM_E_INVALID;
  if (!h->bound) return fail(h, SIM_E_STATE, "sim_bind has not been called");
  if (h->device_error) return SIM_E_DEVICE;
  if (n_steps < 0) return fail(h, SIM_E_INVALID, "n_steps must be >= 0");
  if (n_steps == 0) return SIM_OK;
  return launch_all(h, n_steps, false, (hipStream_t)stream);
}

int sim_rollout(sim_handle* h, int32_t T, void* stream) {
  if (!h) return SIM_E_INVALID;
  if (!h->bound) return fail(h, SIM_E_STATE, "sim_bind has not been called");
  if (h->device_error) return SIM_E_DEVICE;
  if (T < 0) return fail(h, SIM_E_INVALID, "T must be >= 0");
  hipStream_t st = (hipStream_t)stream;
  if (!h->opts.use_graph) return launch_all(h, T, true, st);
  if (h->graph_T != T) {
    if (h->graph_exec) { hipGraphExecDestroy(h->graph_exec); h->graph_exec = nullptr; }
    if (h->graph) { hipGraphDestroy(h->graph); h->graph = nullptr; }
    if (!h->cap_stream) {
      int rc = dev_check(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking), "stream create");
      if (rc) return rc;
    }
    int rc = dev_check(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    if (rc) return rc;
    rc = launch_all(h, T, true, h->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (rc) return rc;
    if ((rc = dev_check(h, e, "end capture"))) return rc;
    h->graph = g;
    if ((rc = dev_check(h, hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0), "graph instantiate"))) return rc;
    h->graph_T = T;
  }
  return dev_check(h, hipGraphLaunch(h->graph_exec, st), "graph launch");
}

int sim_fitness(const sim_handle* hc, float* out, int where, void* stream) {
  sim_handle* h = const_cast<sim_handle*>(hc);
  if (!h || !out) return SIM_E_INVALID;
  if (!h->bound) return fail(h, SIM_E_STATE, "sim_bind has not been called");
  if (h->device_error) return SIM_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  if (where == SIM_HOST) {
    for (Bin& b : h->bins) {
      std::vector<float> tmp(b.users.size());
      int rc = dev_check(h, hipMemcpyAsync(tmp.data(), h->ws + b.o_fit, tmp.size() * 4, hipMemcpyDeviceToHost, st), "fitness copy");
      if (rc) return rc;
      if ((rc = dev_check(h, hipStreamSynchronize(st), "fitness sync"))) return rc;
      for (size_t s = 0; s < tmp.size(); ++s) out[b.users[s]] = tmp[s];
    }
    return SIM_OK;
  }
  if (where == SIM_DEVICE) {
    // user-order scatter: one contiguous run per maximal block of consecutive user indices
    for (Bin& b : h->bins) {
      size_t s = 0;
      while (s < b.users.size()) {
        size_t e = s + 1;
        while (e < b.users.size() && b.users[e] == b.users[e - 1] + 1) ++e;
        int rc = dev_check(h, hipMemcpyAsync(out + b.users[s], h->ws + b.o_fit + s * 4, (e - s) * 4,
                                             hipMemcpyDeviceToDevice, st), "fitness scatter");
        if (rc) return rc;
        s = e;
      }
    }
    return SIM_OK;
  }
  return fail(h, SIM_E_INVALID, "where must be SIM_HOST or SIM_DEVICE");
}

int sim_get_state(const sim_handle* hc, float* q, float* v, int64_t* k, int where, void* stream) {
  sim_handle* h = const_cast<sim_handle*>(hc);
  if (!h) return SIM_E_INVALID;
  if (!h->bound) return fail(h, SIM_E_STATE, "sim_bind has not been called");
  if (where != SIM_HOST) return fail(h, SIM_E_INVALID, "state transfer supports where=SIM_HOST only");
  if (h->device_error) return SIM_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  const int r0 = h->root_type == SIM_ROOT_FREE ? 6 : 0;
  for (Bin& b : h->bins) {
    const size_t m = b.users.size();
    std::vector<float> qq(m * kQStride), vv(m * kVStride);
    std::vector<long long> kk(m);
    int rc;
    if ((rc = dev_check(h, hipMemcpyAsync(qq.data(), h->ws + b.o_q, qq.size() * 4, hipMemcpyDeviceToHost, st), "state copy"))) return rc;
    if ((rc = dev_check(h, hipMemcpyAsync(vv.data(), h->ws + b.o_v, vv.size() * 4, hipMemcpyDeviceToHost, st), "state copy"))) return rc;
    if ((rc = dev_check(h, hipMemcpyAsync(kk.data(), h->ws + b.o_k, kk.size() * 8, hipMemcpyDeviceToHost, st), "state copy"))) return rc;
    if ((rc = dev_check(h, hipStreamSynchronize(st), "state sync"))) return rc;
    for (size_t s = 0; s < m; ++s) {
      const int i = b.users[s];
      if (q) std::copy(&qq[s * kQStride], &qq[s * kQStride] + h->nq[i], q + h->q_off[i]);
      if (v) std::copy(&vv[s * kVStride], &vv[s * kVStride] + h->nv[i], v + h->v_off[i]);
      if (k) k[i] = kk[s];
    }
  }
  (void)r0;
  return SIM_OK;
}

int sim_set_state(sim_handle* h, const float* q, const float* v, const int64_t* k, int where, void* stream) {
  if (!h || !q || !v) return SIM_E_INVALID;
  if (!h->bound) return fail(h, SIM_E_STATE, "sim_bind has not been called");
  if (where != SIM_HOST) return fail(h, SIM_E_INVALID, "state transfer supports where=SIM_HOST only");
  if (h->device_error) return SIM_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  for (Bin& b : h->bins) {
    const size_t m = b.users.size();
    std::vector<float> qq(m * kQStride, 0.f), vv(m * kVStride, 0.f);
    std::vector<long long> kk(m, 0);
    std::vector<unsigned> zero(m, 0u);
    if (!k) {
      int rc = dev_check(h, hipMemcpyAsync(kk.data(), h->ws + b.o_k, m * 8, hipMemcpyDeviceToHost, st), "state copy");
      if (rc) return rc;
      if ((rc = dev_check(h, hipStreamSynchronize(st), "state sync"))) return rc;
    }
    for (size_t s = 0; s < m; ++s) {
      const int i = b.users[s];
      std::copy(q + h->q_off[i], q + h->q_off[i + 1], &qq[s * kQStride]);
      std::copy(v + h->v_off[i], v + h->v_off[i + 1], &vv[s * kVStride]);
      if (k) kk[s] = k[i];
    }
    int rc;
    if ((rc = dev_check(h, hipMemcpyAsync(h->ws + b.o_q, qq.data(), qq.size() * 4, hipMemcpyHostToDevice, st), "state upload"))) return rc;
    if ((rc = dev_check(h, hipMemcpyAsync(h->ws + b.o_v, vv.data(), vv.size() * 4, hipMemcpyHostToDevice, st), "state upload"))) return rc;
    if ((rc = dev_check(h, hipMemcpyAsync(h->ws + b.o_k, kk.data(), m * 8, hipMemcpyHostToDevice, st), "state upload"))) return rc;
    if ((rc = dev_check(h, hipMemcpyAsync(h->ws + b.o_status, zero.data(), m * 4, hipMemcpyHostToDevice, st), "state upload"))) return rc;
    if ((rc = dev_check(h, hipStreamSynchronize(st), "state upload sync"))) return rc;
  }
  return SIM_OK;
}

int sim_counters(const sim_handle* hc, uint64_t* rows_contact, uint64_t* rows_clamp, uint32_t* status, int where,
                 void* stream) {
  sim_handle* h = const_cast<sim_handle*>(hc);
  if (!h) return SIM_E_INVALID;
  if (!h->bound) return fail(h, SIM_E_STATE, "sim_bind has not been called");
  if (where != SIM_HOST) return fail(h, SIM_E_INVALID, "counters support where=SIM_HOST only");
  if (h->device_error) return SIM_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  for (Bin& b : h->bins) {
    const size_t m = b.users.size();
    std::vector<unsigned long long> cc(2 * m);
    std::vector<unsigned> ss(m);
    int rc;
    if ((rc = dev_check(h, hipMemcpyAsync(cc.data(), h->ws + b.o_cnt, cc.size() * 8, hipMemcpyDeviceToHost, st), "counter copy"))) return rc;
    if ((rc = dev_check(h, hipMemcpyAsync(ss.data(), h->ws + b.o_status, m * 4, hipMemcpyDeviceToHost, st), "counter copy"))) return rc;
    if ((rc = dev_check(h, hipStreamSynchronize(st), "counter sync"))) return rc;
    for (size_t s = 0; s < m; ++s) {
      const int i = b.users[s];
      if (rows_contact) rows_contact[i] = cc[2 * s];
      if (rows_clamp) rows_clamp[i] = cc[2 * s + 1];
      if (status) status[i] = ss[s];
    }
  }
  return SIM_OK;
}

int sim_bins(const sim_handle* h, int32_t* n_bins, int32_t* info, int32_t max_bins) {
  if (!h || !n_bins) return SIM_E_INVALID;
  *n_bins = (int32_t)h->bins.size();
  for (int i = 0; i < (int)h->bins.size() && i < max_bins && info; ++i) {
    info[4 * i] = h->bins[i].nvc;
    info[4 * i + 1] = 16 * h->bins[i].sb;
    info[4 * i + 2] = h->bins[i].ncr;
    info[4 * i + 3] = (int32_t)h->bins[i].users.size();
  }
  return SIM_OK;
}

void sim_destroy(sim_handle* h) {
  if (!h) return;
  if (h->graph_exec) hipGraphExecDestroy(h->graph_exec);
  if (h->graph) hipGraphDestroy(h->graph);
  if (h->cap_stream) hipStreamDestroy(h->cap_stream);
  delete h;
}

const char* sim_last_error(const sim_handle* h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

}  // extern "C"
