// Host side of the C ABI in include/sim.h: validation, packing of variants
// into DoF bins, workspace layout, launches, state transfer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <thread>
#include <cstdio>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "sim.h"
#include "host_worker.hpp"
#include "launch.h"
#include "sim_layout.h"

using namespace simk;

namespace {

constexpr int kNvCaps[] = {8, 12, 16, 20, 24, 28};
constexpr int kMaxNv = 28;
constexpr int kMaxBodiesPerVariant = 32;
constexpr int kStepsPerLaunch = 1000;  // default: long runs are split so each launch stays short

std::string g_create_error;

struct Bin {
  int nvc = 0, sb = 0, ncr = 0;
  int tree = 0;  // 1: the kernel factors M~ tree-sparsely
  launch_fn fn = nullptr;
  std::vector<int> users;  // user index of each packed variant
  // packed host copies (uploaded by sim_bind)
  std::vector<int> hdr, lvl, map;  // map: (user, q offset, v offset, nq | nv << 16) per packed variant
  std::vector<float> hdrf, body, q0, v0;
  // device offsets (bytes from the workspace base)
  size_t o_hdr, o_hdrf, o_body, o_lvl, o_q0, o_v0, o_q, o_v, o_k, o_status, o_xy0, o_fit, o_cnt, o_ovf, o_map;
  int lvl_stride = 0;
  long long ovf_stride = 0;
  BinArgs args{};
  hipEvent_t t_begin = nullptr, t_end = nullptr;  // launch timing (time_launches)
  int timed_launches = 0;
  int multi_kind = -1;  // family index in the multi-bin kernel
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

long long ovf_stride_of(const Bin& b, int ball, int self) {
  return ovf_floats(max_contacts(16 * b.sb, ball, self), b.nvc, (ball || self) ? kListWordsBall : kListWords);
}

// Workspace arrays of a bin (in layout order) and their bytes per variant;
// the layout rounds every array up to 256 bytes.
constexpr int kWsArrays = 15;
void ws_bytes_per_variant(const Bin& b, int ball, int self, size_t (&per)[kWsArrays]) {
  const size_t v[kWsArrays] = {HW_WORDS * 4, HF_WORDS * 4, (size_t)16 * b.sb * BW_WORDS * 4,
                               (size_t)(2 * 16 * b.sb + 4) * 4, kQStride * 4, kVStride * 4, kQStride * 4,
                               kVStride * 4, 8, 4, 8, 4, 16, (size_t)ovf_stride_of(b, ball, self) * 4, 16};
  for (int i = 0; i < kWsArrays; ++i) per[i] = v[i];
}

}  // namespace

struct sim_handle {
  int n = 0;
  int root_type = 0;
  int ball = 0;  // every variant carries a ball
  int self = 0;  // contacts between the boxes of one robot
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
  int split_T = 0;
  // bins run concurrently: one library stream per bin beyond the first, fork/join by events
  std::vector<hipStream_t> bin_streams;   // library streams 1..; stream 0 is the caller's
  std::vector<hipEvent_t> join_events;
  hipEvent_t fork_event = nullptr;
  std::vector<int> stream_of;             // bin -> stream index (0 = caller's)
  int n_streams = 1;
  int steps_per_launch = kStepsPerLaunch;
  bool multi = false;                     // all bins in one launch per chunk
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

const KernelVariant* find_variant(int nvc, int sb, int ncr, int ball, int self) {
  for (int i = 0; i < kNumKernelVariants; ++i) {
    const KernelVariant& k = kKernelVariants[i];
    if (k.nvc == nvc && k.sb == sb && k.ball == ball && k.self == self && (ncr <= 0 || k.ncr == ncr)) return &k;
  }
  return nullptr;
}

// Launch every bin's kernel for n_steps (reset on the first chunk if asked).
// Bins are independent: bin 0 runs on the caller's stream, every other bin on
// a library stream forked from and joined back into the caller's stream.
// The bin's arguments for its packed variants [first, first + n).
BinArgs sub_args(const Bin& b, int first, int n) {
  BinArgs a = b.args;
  const size_t f = (size_t)first;
  a.n = n;
  a.hdr += f * HW_WORDS;
  a.hdrf += f * HF_WORDS;
  a.body += f * 16 * b.sb * BW_WORDS;
  a.lvl += f * b.lvl_stride;
  a.q0 += f * kQStride;
  a.v0 += f * kVStride;
  a.q += f * kQStride;
  a.v += f * kVStride;
  a.k += f;
  a.status += f;
  a.xy0 += 2 * f;
  a.fit += f;
  a.cnt += 2 * f;
  a.ovf += f * (size_t)b.ovf_stride;
  return a;
}

int launch_bin(sim_handle* h, Bin& b, int n_steps, bool reset, hipStream_t st, int count = -1, int first_slot = 0) {
  if (count == 0) return SIM_OK;
  int done = 0;
  bool first = true;
  const bool timed = h->opts.time_launches && b.t_begin;
  if (timed) {
    int rc = dev_check(h, hipEventRecord(b.t_begin, st), "timing record");
    if (rc) return rc;
    b.timed_launches = 0;
  }
  while (first || done < n_steps) {
    const int chunk = std::min(h->steps_per_launch, n_steps - done);
    BinArgs a = first_slot ? sub_args(b, first_slot, count) : b.args;
    a.n_steps = chunk;
    a.reset = (reset && first) ? 1 : 0;
    if (count >= 0) a.n = count;
    hipError_t e = b.fn(a, h->params, st);
    if (e != hipSuccess) return dev_check(h, e, "kernel launch");
    done += chunk;
    first = false;
    if (timed) ++b.timed_launches;
  }
  if (timed) return dev_check(h, hipEventRecord(b.t_end, st), "timing record");
  return SIM_OK;
}

// All bins in one launch per chunk (single_launch).
int launch_multi(sim_handle* h, int n_steps, bool reset, hipStream_t st, const std::vector<int>* counts) {
  MultiArgs m{};
  m.nbins = (int)h->bins.size();
  // workgroups of the slowest bins (largest nv capacity) are dispatched first
  std::vector<int> order(m.nbins);
  for (int i = 0; i < m.nbins; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return h->bins[x].nvc > h->bins[y].nvc; });
  int blocks = 0;
  for (int j = 0; j < m.nbins; ++j) {
    const int i = order[j];
    const Bin& b = h->bins[i];
    m.kind[j] = b.multi_kind;
    m.block_start[j] = blocks;
    m.bin[j] = b.args;
    if (counts) m.bin[j].n = (*counts)[i];
    blocks += (m.bin[j].n + kVarPerWave - 1) / kVarPerWave;
  }
  m.block_start[m.nbins] = blocks;
  if (blocks == 0) return SIM_OK;
  Bin& b0 = h->bins[0];
  const bool timed = h->opts.time_launches && b0.t_begin;
  int rc;
  if (timed && (rc = dev_check(h, hipEventRecord(b0.t_begin, st), "timing record"))) return rc;
  int done = 0, launches = 0;
  bool first = true;
  while (first || done < n_steps) {
    const int chunk = std::min(h->steps_per_launch, n_steps - done);
    for (int i = 0; i < m.nbins; ++i) {
      m.bin[i].n_steps = chunk;
      m.bin[i].reset = (reset && first) ? 1 : 0;
    }
    hipError_t e = launch_rollout_multi(m, h->params, blocks, st);
    if (e != hipSuccess) return dev_check(h, e, "kernel launch");
    done += chunk;
    first = false;
    ++launches;
  }
  if (timed) {
    for (Bin& b : h->bins) b.timed_launches = launches;
    return dev_check(h, hipEventRecord(b0.t_end, st), "timing record");
  }
  return SIM_OK;
}

int launch_all(sim_handle* h, int n_steps, bool reset, hipStream_t st, const std::vector<int>* counts = nullptr) {
  if (h->multi) return launch_multi(h, n_steps, reset, st, counts);
  const size_t nb = h->bins.size();
  const int ns = h->n_streams;
  auto stream = [&](size_t bi) { return h->stream_of[bi] == 0 ? st : h->bin_streams[h->stream_of[bi] - 1]; };
  int rc;
  if (ns > 1) {
    if ((rc = dev_check(h, hipEventRecord(h->fork_event, st), "fork record"))) return rc;
    for (int i = 1; i < ns; ++i)
      if ((rc = dev_check(h, hipStreamWaitEvent(h->bin_streams[i - 1], h->fork_event, 0), "fork wait"))) return rc;
  }
  // bins are ordered by decreasing cost; each stream receives its bins in that order
  for (size_t i = 0; i < nb; ++i)
    if ((rc = launch_bin(h, h->bins[i], n_steps, reset, stream(i), counts ? (*counts)[i] : -1))) return rc;
  for (int i = 1; i < ns; ++i) {
    if ((rc = dev_check(h, hipEventRecord(h->join_events[i - 1], h->bin_streams[i - 1]), "join record"))) return rc;
    if ((rc = dev_check(h, hipStreamWaitEvent(st, h->join_events[i - 1], 0), "join wait"))) return rc;
  }
  return SIM_OK;
}

HostVariantView host_view(const sim_handle* h, const Bin& b, size_t s) {
  const int nbc = 16 * b.sb;
  return HostVariantView{&b.hdr[s * HW_WORDS], &b.hdrf[s * HF_WORDS], &b.body[s * nbc * BW_WORDS],
                         &b.q0[s * kQStride], &b.v0[s * kVStride], h->self,
                         h->opts.host_factorization == SIM_FACTOR_TREE};
}

// Run the listed (bin, slot) pairs on host threads; returns wall seconds.
// done[i] = 1 for every item that finished.  A worker whose item fails (an
// exception: allocation, thread resources, or the injected test fault of
// sim_options.host_fault_items) stops taking work; the others go on, and
// what no worker finished is left to the caller (the split re-queues it on
// the GPU).  A thread that cannot be started leaves its share to the rest.
double run_host(const sim_handle* h, const std::vector<std::pair<int, int>>& work, int threads,
                std::vector<HostVariantState>& out, std::vector<char>& done) {
  out.assign(work.size(), HostVariantState());
  done.assign(work.size(), 0);
  std::atomic<size_t> next(0);
  const size_t faults = (size_t)std::max(0, h->opts.host_fault_items);
  auto t0 = std::chrono::steady_clock::now();
  auto body = [&]() {
    for (size_t i = next.fetch_add(1); i < work.size(); i = next.fetch_add(1)) {
      try {
        if (i < faults) throw std::runtime_error("injected host worker fault");
        const Bin& b = h->bins[work[i].first];
        host_rollout(host_view(h, b, work[i].second), h->params, h->split_T, out[i]);
        done[i] = 1;
      } catch (...) {
        return;  // this worker is out; its item stays undone
      }
    }
  };
  const int nt = std::max(1, std::min<int>(threads, (int)work.size()));
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) {
    try {
      pool.emplace_back(body);
    } catch (...) {
      break;
    }
  }
  body();
  for (auto& th : pool) th.join();
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

size_t count_undone(const std::vector<char>& done) {
  size_t n = 0;
  for (char c : done) n += c ? 0 : 1;
  return n;
}

// Host share per bin: proportional to bin size, largest remainders, taken from the bin tails.
std::vector<int> host_counts(const sim_handle* h, int n_host) {
  const size_t nb = h->bins.size();
  std::vector<int> cnt(nb, 0);
  std::vector<std::pair<double, int>> rem;
  int given = 0;
  for (size_t i = 0; i < nb; ++i) {
    const double exact = double(n_host) * h->bins[i].users.size() / h->n;
    cnt[i] = (int)std::floor(exact);
    given += cnt[i];
    rem.push_back({exact - cnt[i], (int)i});
  }
  std::sort(rem.begin(), rem.end(), [](auto& x, auto& y) { return x.first > y.first; });
  for (size_t r = 0; given < n_host && r < rem.size(); ++r) {
    const int i = rem[r].second;
    if (cnt[i] < (int)h->bins[i].users.size()) { ++cnt[i]; ++given; }
  }
  return cnt;
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
  const int ball = d->ball ? 1 : 0;
  const int self = d->self_collision ? 1 : 0;
  if (ball && self) return bad("self_collision is not combined with a ball");
  if (ball)
    for (int i = 0; i < d->n_variants; ++i)
      if (!(d->ball[2 * i] > 0.f) || !(d->ball[2 * i + 1] > 0.f) || !std::isfinite(d->ball[2 * i]) ||
          !std::isfinite(d->ball[2 * i + 1]))
        return bad("variant " + std::to_string(i) + ": ball radius and mass must be finite and > 0");
  if (!(d->dt > 0.f) || !std::isfinite(d->dt)) return bad("dt must be > 0");
  if (d->pgs_iters < 1) return bad("pgs_iters must be >= 1");
  const float prm[] = {d->kp, d->kd, d->tau_max, d->k_contact, d->b_contact, d->gravity[0], d->gravity[1], d->gravity[2]};
  if (!finite_all(prm, 8)) return bad("non-finite model constant");
  if (d->kp < 0 || d->kd < 0 || d->tau_max < 0 || d->k_contact < 0 || d->b_contact < 0)
    return bad("gains, torque limit and contact constants must be >= 0");
  if (opts) hp->opts = *opts;
  {
    const sim_options& o = hp->opts;
    if (o.contacts_in_registers < 0 || o.steps_per_launch < 0 || o.streams < 0)
      return bad("contacts_in_registers, steps_per_launch and streams must be >= 0");
    if (o.min_body_slots != 0 && o.min_body_slots != 16 && o.min_body_slots != 32)
      return bad("min_body_slots must be 0, 16 or 32");
    if (o.time_launches && o.use_graph) return bad("time_launches and use_graph cannot be combined");
    if (o.host_factorization != SIM_FACTOR_DENSE && o.host_factorization != SIM_FACTOR_TREE)
      return bad("host_factorization must be SIM_FACTOR_DENSE or SIM_FACTOR_TREE");
    if (o.gpu_factorization != SIM_FACTOR_DENSE && o.gpu_factorization != SIM_FACTOR_TREE)
      return bad("gpu_factorization must be SIM_FACTOR_DENSE or SIM_FACTOR_TREE");
    if (o.host_fault_items < 0) return bad("host_fault_items must be >= 0");
    auto cap_or_zero = [](int v) { return v == 0 || (v >= 8 && v <= kMaxNv && v % 4 == 0); };
    if (!cap_or_zero(o.min_nv_capacity)) return bad("min_nv_capacity must be 0 or a DoF capacity 8, 12, ..., 28");
    if (!cap_or_zero(o.slots32_min_nvc)) return bad("slots32_min_nvc must be 0 or a DoF capacity 8, 12, ..., 28");
    for (int k = 0; k < 6; ++k)
      if (o.ncr_by_nvc[k] < 0) return bad("ncr_by_nvc entries must be >= 0");
    hp->steps_per_launch = o.steps_per_launch > 0 ? o.steps_per_launch : kStepsPerLaunch;
  }
  const int n = d->n_variants;
  hp->n = n;
  hp->root_type = d->root_type;
  hp->ball = ball;
  hp->self = self;
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
    hp->nv[i] = r0 + nh + (ball ? 6 : 0);
    hp->nq[i] = (r0 ? 7 : 0) + nh + (ball ? 7 : 0);
    if (hp->nv[i] < 1 || hp->nv[i] > kMaxNv)
      return bad("variant " + std::to_string(i) + ": degrees of freedom (the ball's included) must be in 1..28");
    if (hp->q_off[i] > 0x7fffffff - 64) return bad("population too large: state entries must fit 32-bit offsets");
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
    if (ball) {
      const float* qb = d->q0 + hp->q_off[i + 1] - 4;
      const float bn = std::sqrt(qb[0] * qb[0] + qb[1] * qb[1] + qb[2] * qb[2] + qb[3] * qb[3]);
      if (std::fabs(bn - 1.f) > 1e-5f) return bad("variant " + std::to_string(i) + ": ball quaternion must be a unit quaternion");
    }
  }
  // bins: smallest DoF capacity, body slots from the body count
  auto ncr_for = [&](int nvc) {
    if (hp->opts.contacts_in_registers > 0) return hp->opts.contacts_in_registers;
    const int k = nvc / 4 - 2;
    return (k >= 0 && k < 6) ? hp->opts.ncr_by_nvc[k] : 0;
  };
  std::vector<std::pair<int, int>> keys(n);
  for (int i = 0; i < n; ++i) {
    int nvc = 0;
    for (int c : kNvCaps)
      if (hp->nv[i] <= c) { nvc = c; break; }
    if (nvc < hp->opts.min_nv_capacity) nvc = hp->opts.min_nv_capacity;
    int sb_need = info[i].nb > 16 ? 2 : 1;
    if (hp->opts.min_body_slots == 32 && nvc >= hp->opts.slots32_min_nvc) sb_need = 2;
    // smallest compiled (nv capacity, body slots) that holds the variant
    int sb = 0;
    for (; nvc <= kMaxNv; nvc += 4) {
      if (find_variant(nvc, sb_need, ncr_for(nvc), ball, self)) { sb = sb_need; break; }
      if (sb_need == 1 && find_variant(nvc, 2, ncr_for(nvc), ball, self)) { sb = 2; break; }
    }
    if (!sb)
      return bad("no compiled kernel for nv=" + std::to_string(hp->nv[i]) + " bodies=" + std::to_string(info[i].nb) +
                 " contacts_in_registers=" + std::to_string(ncr_for(nvc > kMaxNv ? kMaxNv : nvc)));
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
    const KernelVariant* kv = find_variant(b.nvc, b.sb, ncr_for(b.nvc), ball, self);
    b.ncr = kv->ncr;
    b.fn = kv->fn;
    if (hp->opts.gpu_factorization == SIM_FACTOR_TREE && !ball && !self && !hp->opts.single_launch) {
      for (int k = 0; k < kNumTreeKernelVariants; ++k) {
        const KernelVariant& t = kTreeKernelVariants[k];
        if (t.nvc == b.nvc && t.sb == b.sb && t.ncr == b.ncr) {
          b.fn = t.fn;
          b.tree = 1;
        }
      }
    }
    for (int i = 0; i < n; ++i)
      if (keys[i] == kk) b.users.push_back(i);
    // within a bin, neighbours in a wave should share nv and tree depth
    std::stable_sort(b.users.begin(), b.users.end(), [&](int x, int y) {
      if (hp->nv[x] != hp->nv[y]) return hp->nv[x] > hp->nv[y];
      return info[x].maxdepth > info[y].maxdepth;
    });
    hp->bins.push_back(std::move(b));
  }
  // launch order: the slowest waves first ((nv capacity)^2, 32-body kernels
  // weighted 1.25), then the larger bins: bins launched together on their
  // own streams share the chip, and the one whose waves take longest ends
  // the rollout, so its workgroups go out first (on 8192 random trees x 5000
  // steps this makes the rollout 214 ms every time, where cost order gave
  // 210-227 ms by where the 28-DoF bin's workgroups landed)
  auto cost = [](const Bin& b) { return (double)b.users.size() * b.nvc * b.nvc * (b.sb == 2 ? 1.25 : 1.0); };
  auto wave_cost = [](const Bin& b) { return (double)b.nvc * b.nvc * (b.sb == 2 ? 1.25 : 1.0); };
  std::stable_sort(hp->bins.begin(), hp->bins.end(), [&](const Bin& x, const Bin& y) {
    return wave_cost(x) != wave_cost(y) ? wave_cost(x) > wave_cost(y) : cost(x) > cost(y);
  });
  // single launch: every bin must be one of the multi-bin kernel's families
  if (hp->opts.single_launch) {
    if ((int)hp->bins.size() > kMaxMultiBins) return bad("single_launch supports at most 8 bins");
    if (ball || self) return bad("single_launch: the multi-bin kernel has no ball or self-collision families");
    for (Bin& b : hp->bins) {
      for (int k = 0; k < kNumMultiFamilies; ++k)
        if (kMultiFamilies[k].nvc == b.nvc && kMultiFamilies[k].sb == b.sb && kMultiFamilies[k].ncr == b.ncr)
          b.multi_kind = k;
      if (b.multi_kind < 0)
        return bad("single_launch: bin (nv capacity " + std::to_string(b.nvc) + ", " + std::to_string(16 * b.sb) +
                   " bodies, " + std::to_string(b.ncr) + " contacts in registers) is not in the multi-bin kernel");
    }
    hp->multi = true;
  }
  // streams: longest-first assignment of the bins to the least-loaded stream
  {
    const int nbins = (int)hp->bins.size();
    const int ns = hp->multi ? 1 : (hp->opts.streams == 0 ? nbins : std::min(hp->opts.streams, nbins));
    hp->n_streams = std::max(1, ns);
    std::vector<double> load(hp->n_streams, 0.0);
    hp->stream_of.assign(nbins, 0);
    std::vector<int> by_cost(nbins);
    for (int bi = 0; bi < nbins; ++bi) by_cost[bi] = bi;
    std::stable_sort(by_cost.begin(), by_cost.end(),
                     [&](int x, int y) { return cost(hp->bins[x]) > cost(hp->bins[y]); });
    for (int bi : by_cost) {
      int best = 0;
      for (int k = 1; k < hp->n_streams; ++k)
        if (load[k] < load[best]) best = k;
      hp->stream_of[bi] = best;
      load[best] += cost(hp->bins[bi]);
    }
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
    b.lvl_stride = 2 * nbc + 4;
    b.lvl.assign((size_t)m * b.lvl_stride, 0);
    b.map.assign((size_t)m * 4, 0);
    for (int s = 0; s < m; ++s) {
      const int i = b.users[s];
      hp->bin_of[i] = (int)bi;
      hp->slot_of[i] = s;
      b.map[4 * s] = i;
      b.map[4 * s + 1] = hp->q_off[i];
      b.map[4 * s + 2] = hp->v_off[i];
      b.map[4 * s + 3] = hp->nq[i] | (hp->nv[i] << 16);
      const VInfo& vi = info[i];
      int* hd = &b.hdr[(size_t)s * HW_WORDS];
      hd[HW_NB] = vi.nb; hd[HW_NH] = vi.nb - 1; hd[HW_NV] = hp->nv[i]; hd[HW_R0] = r0;
      hd[HW_MAXDEPTH] = vi.maxdepth; hd[HW_USER] = i;
      hd[HW_NVR] = r0 + vi.nb - 1;
      hd[HW_NQR] = (r0 ? 7 : 0) + vi.nb - 1;
      float* hf = &b.hdrf[(size_t)s * HF_WORDS];
      hf[HF_MU] = d->mu[i];
      if (ball) {
        hf[HF_BALLR] = d->ball[2 * i];
        hf[HF_BALLM] = d->ball[2 * i + 1];
      }
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
      // bodies in depth order (stable), then the start of every level
      int* lv = &b.lvl[(size_t)s * b.lvl_stride];
      int pos = 0;
      for (int lev = 0; lev <= vi.maxdepth; ++lev) {
        lv[nbc + lev] = pos;
        for (int bb = 0; bb < vi.nb; ++bb)
          if (vi.depth[bb] == lev) lv[pos++] = bb;
      }
      lv[nbc + vi.maxdepth + 1] = pos;
      std::copy(d->q0 + hp->q_off[i], d->q0 + hp->q_off[i + 1], &b.q0[(size_t)s * kQStride]);
      std::copy(d->v0 + hp->v_off[i], d->v0 + hp->v_off[i + 1], &b.v0[(size_t)s * kVStride]);
    }
  }
  // workspace layout
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  for (Bin& b : hp->bins) {
    const size_t m = b.users.size();
    b.ovf_stride = ovf_stride_of(b, ball, self);
    b.o_hdr = take(m * HW_WORDS * 4);
    b.o_hdrf = take(m * HF_WORDS * 4);
    b.o_body = take(m * 16 * b.sb * BW_WORDS * 4);
    b.o_lvl = take(m * b.lvl_stride * 4);
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
    b.o_map = take(m * 16);
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
  // a captured rollout graph holds the previous workspace's pointers: drop it
  // (the next graph rollout captures again on the new workspace)
  if (h->graph_exec) { hipGraphExecDestroy(h->graph_exec); h->graph_exec = nullptr; }
  if (h->graph) { hipGraphDestroy(h->graph); h->graph = nullptr; }
  h->graph_T = -1;
  h->ws = (char*)ws;
  if (h->bin_streams.empty() && h->n_streams > 1) {
    int rc = dev_check(h, hipEventCreateWithFlags(&h->fork_event, hipEventDisableTiming), "event create");
    if (rc) return rc;
    for (int i = 1; i < h->n_streams; ++i) {
      hipStream_t s2;
      hipEvent_t e2;
      if ((rc = dev_check(h, hipStreamCreateWithFlags(&s2, hipStreamNonBlocking), "stream create"))) return rc;
      h->bin_streams.push_back(s2);
      if ((rc = dev_check(h, hipEventCreateWithFlags(&e2, hipEventDisableTiming), "event create"))) return rc;
      h->join_events.push_back(e2);
    }
  }
  for (Bin& b : h->bins) {
    char* base = h->ws;
    const size_t m = b.users.size();
    int rc;
    if (h->opts.time_launches && !b.t_begin) {
      if ((rc = dev_check(h, hipEventCreate(&b.t_begin), "event create"))) return rc;
      if ((rc = dev_check(h, hipEventCreate(&b.t_end), "event create"))) return rc;
    }
    if ((rc = dev_check(h, hipMemcpyAsync(base + b.o_hdr, b.hdr.data(), m * HW_WORDS * 4, hipMemcpyHostToDevice, st), "upload"))) return rc;
    if ((rc = dev_check(h, hipMemcpyAsync(base + b.o_hdrf, b.hdrf.data(), m * HF_WORDS * 4, hipMemcpyHostToDevice, st), "upload"))) return rc;
    if ((rc = dev_check(h, hipMemcpyAsync(base + b.o_body, b.body.data(), b.body.size() * 4, hipMemcpyHostToDevice, st), "upload"))) return rc;
    if ((rc = dev_check(h, hipMemcpyAsync(base + b.o_lvl, b.lvl.data(), b.lvl.size() * 4, hipMemcpyHostToDevice, st), "upload"))) return rc;
    if ((rc = dev_check(h, hipMemcpyAsync(base + b.o_q0, b.q0.data(), b.q0.size() * 4, hipMemcpyHostToDevice, st), "upload"))) return rc;
    if ((rc = dev_check(h, hipMemcpyAsync(base + b.o_v0, b.v0.data(), b.v0.size() * 4, hipMemcpyHostToDevice, st), "upload"))) return rc;
    if ((rc = dev_check(h, hipMemcpyAsync(base + b.o_map, b.map.data(), b.map.size() * 4, hipMemcpyHostToDevice, st), "upload"))) return rc;
    BinArgs& a = b.args;
    a.n = (int)m;
    a.hdr = (const int*)(base + b.o_hdr);
    a.hdrf = (const float*)(base + b.o_hdrf);
    a.body = (const float*)(base + b.o_body);
    a.lvl = (const int*)(base + b.o_lvl);
    a.lvl_stride = b.lvl_stride;
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
    int rc = dev_check(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeGlobal), "begin capture");
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
  if (where != SIM_HOST && where != SIM_DEVICE) return fail(h, SIM_E_INVALID, "where must be SIM_HOST or SIM_DEVICE");
  if (h->device_error) return SIM_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  if (where == SIM_DEVICE) {
    for (Bin& b : h->bins) {
      const BinArgs& a = b.args;
      int rc = dev_check(h, launch_state_gather((int)b.users.size(), (const int*)(h->ws + b.o_map), a.q, a.v, a.k, q, v,
                                                k, st), "state gather");
      if (rc) return rc;
    }
    return SIM_OK;
  }
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
  return SIM_OK;
}

int sim_set_state(sim_handle* h, const float* q, const float* v, const int64_t* k, int where, void* stream) {
  if (!h || !q || !v) return SIM_E_INVALID;
  if (!h->bound) return fail(h, SIM_E_STATE, "sim_bind has not been called");
  if (where != SIM_HOST && where != SIM_DEVICE) return fail(h, SIM_E_INVALID, "where must be SIM_HOST or SIM_DEVICE");
  if (h->device_error) return SIM_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  if (where == SIM_DEVICE) {
    for (Bin& b : h->bins) {
      const BinArgs& a = b.args;
      int rc = dev_check(h, launch_state_scatter((int)b.users.size(), (const int*)(h->ws + b.o_map), q, v, k, a.q, a.v,
                                                 a.k, a.status, st), "state scatter");
      if (rc) return rc;
    }
    return SIM_OK;
  }
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
  if (where != SIM_HOST && where != SIM_DEVICE) return fail(h, SIM_E_INVALID, "where must be SIM_HOST or SIM_DEVICE");
  if (h->device_error) return SIM_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  if (where == SIM_DEVICE) {
    for (Bin& b : h->bins) {
      const BinArgs& a = b.args;
      int rc = dev_check(h, launch_counters_gather((int)b.users.size(), (const int*)(h->ws + b.o_map), a.cnt, a.status,
                                                   rows_contact, rows_clamp, status, st), "counter gather");
      if (rc) return rc;
    }
    return SIM_OK;
  }
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

int sim_rollout_host(sim_handle* h, int32_t T, int32_t host_threads, float* fitness, double* seconds) {
  if (!h) return SIM_E_INVALID;
  if (T < 0 || host_threads < 1) return fail(h, SIM_E_INVALID, "T must be >= 0 and host_threads >= 1");
  std::vector<std::pair<int, int>> work;
  for (size_t bi = 0; bi < h->bins.size(); ++bi)
    for (size_t s2 = 0; s2 < h->bins[bi].users.size(); ++s2) work.push_back({(int)bi, (int)s2});
  std::vector<HostVariantState> out;
  std::vector<char> done;
  h->split_T = T;
  const double sec = run_host(h, work, host_threads, out, done);
  if (const size_t bad_n = count_undone(done))
    return fail(h, SIM_E_HOST, "host workers failed; " + std::to_string(bad_n) + " of " +
                                   std::to_string(work.size()) + " variants were not simulated");
  if (fitness)
    for (size_t i = 0; i < work.size(); ++i) {
      const Bin& b = h->bins[work[i].first];
      fitness[b.users[work[i].second]] = host_fitness(host_view(h, b, work[i].second), out[i]);
    }
  if (seconds) *seconds = sec;
  return SIM_OK;
}

int sim_rollout_split(sim_handle* h, int32_t T, int32_t n_host, int32_t host_threads, void* stream,
                      sim_split_times* times) {
  if (!h) return SIM_E_INVALID;
  if (!h->bound) return fail(h, SIM_E_STATE, "sim_bind has not been called");
  if (h->device_error) return SIM_E_DEVICE;
  if (T < 0 || n_host < 0 || n_host > h->n || host_threads < 1)
    return fail(h, SIM_E_INVALID, "need T >= 0, 0 <= n_host <= n_variants, host_threads >= 1");
  hipStream_t st = (hipStream_t)stream;
  const std::vector<int> hc = host_counts(h, n_host);
  std::vector<int> gc(h->bins.size());
  std::vector<std::pair<int, int>> work;
  for (size_t bi = 0; bi < h->bins.size(); ++bi) {
    const int m = (int)h->bins[bi].users.size();
    gc[bi] = m - hc[bi];
    for (int s2 = gc[bi]; s2 < m; ++s2) work.push_back({(int)bi, s2});
  }
  hipEvent_t e0, e1;
  int rc;
  if ((rc = dev_check(h, hipEventCreate(&e0), "event create"))) return rc;
  if ((rc = dev_check(h, hipEventCreate(&e1), "event create"))) { hipEventDestroy(e0); return rc; }
  auto t0 = std::chrono::steady_clock::now();
  rc = dev_check(h, hipEventRecord(e0, st), "event record");
  if (!rc) rc = launch_all(h, T, true, st, &gc);
  if (!rc) rc = dev_check(h, hipEventRecord(e1, st), "event record");
  std::vector<HostVariantState> out;
  std::vector<char> done;
  h->split_T = T;
  double host_s = 0.0;
  if (!rc) host_s = run_host(h, work, host_threads, out, done);  // concurrent with the GPU launches above
  if (!rc) rc = dev_check(h, hipStreamSynchronize(st), "split sync");
  const size_t n_requeued = rc ? 0 : count_undone(done);
  // merge: host results into the device state (contiguous tail of every bin)
  size_t wi = 0;
  for (size_t bi = 0; !rc && bi < h->bins.size(); ++bi) {
    Bin& b = h->bins[bi];
    const size_t m = b.users.size(), g = (size_t)gc[bi], nh = m - g;
    if (!nh) continue;
    std::vector<float> q(nh * kQStride), v(nh * kVStride), xy(2 * nh), fit(nh);
    std::vector<long long> kk(nh);
    std::vector<unsigned> sts(nh);
    std::vector<unsigned long long> cc(2 * nh);
    for (size_t j = 0; j < nh; ++j, ++wi) {
      const HostVariantState& hs = out[wi];
      std::memcpy(&q[j * kQStride], hs.q, sizeof(hs.q));
      std::memcpy(&v[j * kVStride], hs.v, sizeof(hs.v));
      kk[j] = hs.k; sts[j] = hs.status; xy[2 * j] = hs.x0; xy[2 * j + 1] = hs.y0;
      fit[j] = host_fitness(host_view(h, b, g + j), hs);
      cc[2 * j] = hs.rows_contact; cc[2 * j + 1] = hs.rows_clamp;
    }
    char* w = h->ws;
    auto up = [&](size_t off, const void* src, size_t bytes) {
      if (!rc) rc = dev_check(h, hipMemcpyAsync(w + off, src, bytes, hipMemcpyHostToDevice, st), "merge upload");
    };
    up(b.o_q + g * kQStride * 4, q.data(), q.size() * 4);
    up(b.o_v + g * kVStride * 4, v.data(), v.size() * 4);
    up(b.o_k + g * 8, kk.data(), nh * 8);
    up(b.o_status + g * 4, sts.data(), nh * 4);
    up(b.o_xy0 + g * 8, xy.data(), nh * 8);
    up(b.o_fit + g * 4, fit.data(), nh * 4);
    up(b.o_cnt + g * 16, cc.data(), nh * 16);
    if (!rc) rc = dev_check(h, hipStreamSynchronize(st), "merge sync");  // host vectors die here
  }
  // re-queue: what no host worker finished runs on the GPU, one launch
  // sequence per run of consecutive slots, over the merged (unfinished) slots
  for (size_t bi = 0, wj = 0; !rc && n_requeued && bi < h->bins.size(); ++bi) {
    Bin& b = h->bins[bi];
    const int m = (int)b.users.size(), g = gc[bi];
    std::vector<char> redo(m, 0);
    for (int s2 = g; s2 < m; ++s2, ++wj) redo[s2] = done[wj] ? 0 : 1;
    for (int s0 = g; !rc && s0 < m;) {
      if (!redo[s0]) { ++s0; continue; }
      int s1 = s0;
      while (s1 < m && redo[s1]) ++s1;
      for (int k = 0, first = 1; !rc && (first || k < T); first = 0) {
        const int chunk = std::min(h->steps_per_launch, T - k);
        BinArgs a = sub_args(b, s0, s1 - s0);
        a.n_steps = chunk;
        a.reset = first;
        const hipError_t e = b.fn(a, h->params, st);
        if (e != hipSuccess) rc = dev_check(h, e, "re-queue launch");
        k += chunk;
      }
      s0 = s1;
    }
  }
  if (!rc && n_requeued) rc = dev_check(h, hipStreamSynchronize(st), "re-queue sync");
  const double combined = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  float gpu_ms = 0.f;
  if (!rc) rc = dev_check(h, hipEventElapsedTime(&gpu_ms, e0, e1), "event time");
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  if (times) {
    times->combined_s = combined;
    times->gpu_s = gpu_ms / 1e3;
    times->host_s = host_s;
    times->n_gpu = h->n - n_host;
    times->n_host = n_host;
    times->host_threads = host_threads;
    times->n_requeued = (int32_t)n_requeued;
  }
  return SIM_OK;
}

int sim_variant_bins(const sim_handle* h, int32_t* bin) {
  if (!h || !bin) return SIM_E_INVALID;
  for (int i = 0; i < h->n; ++i) bin[i] = h->bin_of[i];
  return SIM_OK;
}

int sim_launch_times(const sim_handle* hc, int32_t* n_bins, float* ms, int32_t* launches, int32_t max_bins) {
  sim_handle* h = const_cast<sim_handle*>(hc);
  if (!h) return SIM_E_INVALID;
  if (!h->bound) return fail(h, SIM_E_STATE, "sim_bind has not been called");
  if (!h->opts.time_launches) return fail(h, SIM_E_STATE, "the handle was created without time_launches");
  if (n_bins) *n_bins = (int32_t)h->bins.size();
  for (int i = 0; i < (int)h->bins.size() && i < max_bins; ++i) {
    Bin& b = h->multi ? h->bins[0] : h->bins[i];
    if (ms) {
      int rc = dev_check(h, hipEventSynchronize(b.t_end), "timing sync");
      if (rc) return rc;
      float t = 0.f;
      if ((rc = dev_check(h, hipEventElapsedTime(&t, b.t_begin, b.t_end), "timing read"))) return rc;
      ms[i] = t;
    }
    if (launches) launches[i] = b.timed_launches;
  }
  return SIM_OK;
}

int sim_kernel_variants(int32_t* n, int32_t* info, int32_t max_variants) {
  if (!n) return SIM_E_INVALID;
  *n = kNumKernelVariants;
  for (int i = 0; i < kNumKernelVariants && i < max_variants && info; ++i) {
    info[5 * i] = kKernelVariants[i].nvc;
    info[5 * i + 1] = 16 * kKernelVariants[i].sb;
    info[5 * i + 2] = kKernelVariants[i].ncr;
    info[5 * i + 3] = kKernelVariants[i].ball;
    info[5 * i + 4] = kKernelVariants[i].self;
  }
  return SIM_OK;
}

int sim_split_allocation(int32_t n, const int32_t* gpu_n, const double* gpu_s, int32_t n_points,
                         double host_s_per_variant, int32_t* n_host_paper, int32_t* n_host_makespan,
                         double* makespan_paper_s, double* makespan_opt_s) {
  if (n < 0 || !gpu_n || !gpu_s || n_points < 1 || !(host_s_per_variant > 0.0) || !std::isfinite(host_s_per_variant))
    return fail(nullptr, SIM_E_INVALID, "need n >= 0, >= 1 GPU point and host_s_per_variant > 0");
  for (int k = 0; k < n_points; ++k) {
    if (gpu_n[k] <= 0 || !(gpu_s[k] >= 0.0) || !std::isfinite(gpu_s[k]))
      return fail(nullptr, SIM_E_INVALID, "GPU points need n > 0 and a finite time >= 0");
    if (k && gpu_n[k] <= gpu_n[k - 1]) return fail(nullptr, SIM_E_INVALID, "GPU points must have ascending n");
  }
  // GPU time of m variants: 0 for none, flat below the first point, piecewise
  // linear between points, the last segment's slope beyond the last point
  auto t_gpu = [&](double m) -> double {
    if (m <= 0) return 0.0;
    if (m <= gpu_n[0]) return gpu_s[0];
    for (int k = 1; k < n_points; ++k)
      if (m <= gpu_n[k])
        return gpu_s[k - 1] + (gpu_s[k] - gpu_s[k - 1]) * (m - gpu_n[k - 1]) / (gpu_n[k] - gpu_n[k - 1]);
    const int a = n_points >= 2 ? n_points - 2 : 0, b = n_points - 1;
    const double slope = n_points >= 2 ? (gpu_s[b] - gpu_s[a]) / (gpu_n[b] - gpu_n[a]) : gpu_s[0] / gpu_n[0];
    return gpu_s[b] + slope * (m - gpu_n[b]);
  };
  auto t_host = [&](double h2) { return h2 * host_s_per_variant; };
  auto span = [&](int32_t h2) { return std::max(t_gpu((double)n - h2), t_host(h2)); };
  const double tg = t_gpu(n), tc = t_host(n);
  int32_t hp = (tg + tc > 0) ? (int32_t)std::llround(n * tg / (tg + tc)) : 0;
  hp = std::min(std::max(hp, 0), n);
  int32_t best = 0;
  double bs = span(0);
  for (int32_t h2 = 1; h2 <= n; ++h2) {
    const double v = span(h2);
    if (v < bs) { bs = v; best = h2; }
  }
  if (n_host_paper) *n_host_paper = hp;
  if (n_host_makespan) *n_host_makespan = best;
  if (makespan_paper_s) *makespan_paper_s = span(hp);
  if (makespan_opt_s) *makespan_opt_s = bs;
  return SIM_OK;
}

int sim_plan_split(sim_handle* h, int32_t T_pilot, int32_t host_threads, int32_t host_sample, void* stream,
                   sim_split_plan* plan) {
  if (!h) return SIM_E_INVALID;
  if (!h->bound) return fail(h, SIM_E_STATE, "sim_bind has not been called");
  if (h->device_error) return SIM_E_DEVICE;
  if (T_pilot < 1 || host_threads < 1 || host_sample < 1 || !plan)
    return fail(h, SIM_E_INVALID, "need T_pilot >= 1, host_threads >= 1, host_sample >= 1 and a plan");
  hipStream_t st = (hipStream_t)stream;
  std::memset(plan, 0, sizeof(*plan));
  hipEvent_t e0, e1;
  int rc;
  if ((rc = dev_check(h, hipEventCreate(&e0), "event create"))) return rc;
  if ((rc = dev_check(h, hipEventCreate(&e1), "event create"))) { hipEventDestroy(e0); return rc; }
  // GPU curve: 1/16 .. 1 of every bin, after one warm-up of the whole population
  const int fr[] = {16, 8, 4, 2, 1};
  rc = launch_all(h, T_pilot, true, st);
  int np = 0;
  for (int fi = 0; !rc && fi < 5; ++fi) {
    std::vector<int> counts(h->bins.size());
    int tot = 0;
    for (size_t bi = 0; bi < h->bins.size(); ++bi) {
      const int m = (int)h->bins[bi].users.size();
      counts[bi] = std::max(m > 0 ? 1 : 0, (m + fr[fi] - 1) / fr[fi]);
      tot += counts[bi];
    }
    if (np && tot <= plan->gpu_n[np - 1]) continue;
    rc = dev_check(h, hipEventRecord(e0, st), "event record");
    if (!rc) rc = launch_all(h, T_pilot, true, st, &counts);
    if (!rc) rc = dev_check(h, hipEventRecord(e1, st), "event record");
    if (!rc) rc = dev_check(h, hipEventSynchronize(e1), "event sync");
    float ms = 0.f;
    if (!rc) rc = dev_check(h, hipEventElapsedTime(&ms, e0, e1), "event time");
    if (!rc) {
      plan->gpu_n[np] = tot;
      plan->gpu_s[np] = ms / 1e3;
      ++np;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  // restore the initial state of every variant
  if (!rc) rc = launch_all(h, 0, true, st);
  if (!rc) rc = dev_check(h, hipStreamSynchronize(st), "pilot sync");
  if (rc) return rc;
  plan->gpu_points = np;
  // host pilot: host_sample variants spread over the bins
  std::vector<std::pair<int, int>> work;
  const int take = std::min(host_sample, h->n);
  for (int j = 0; j < take; ++j) {
    const int user = (int)((long long)j * h->n / take);
    work.push_back({h->bin_of[user], h->slot_of[user]});
  }
  std::vector<HostVariantState> out;
  std::vector<char> done;
  const int saved_T = h->split_T;
  h->split_T = T_pilot;
  const double host_wall = run_host(h, work, host_threads, out, done);
  h->split_T = saved_T;
  if (const size_t bad_n = count_undone(done))
    return fail(h, SIM_E_HOST, "host pilot: host workers failed on " + std::to_string(bad_n) + " variants");
  plan->host_s_per_variant = host_wall / take;
  return sim_split_allocation(h->n, plan->gpu_n, plan->gpu_s, np, plan->host_s_per_variant, &plan->n_host_paper,
                              &plan->n_host_makespan, &plan->makespan_paper_s, &plan->makespan_opt_s);
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

int sim_chunk_plan(const sim_handle* h, size_t max_workspace_bytes, int32_t* n_chunks, int32_t* chunk_end,
                   int32_t max_chunks) {
  if (!h || !n_chunks) return SIM_E_INVALID;
  // a chunk's workspace: per bin present, every array rounded up to 256
  // bytes; adding a variant adds its bin's per-variant bytes (and, for a bin
  // new to the chunk, the rounding of that bin's arrays)
  const size_t nb = h->bins.size();
  std::vector<std::array<size_t, kWsArrays>> per(nb);
  for (size_t bi = 0; bi < nb; ++bi) {
    size_t p[kWsArrays];
    ws_bytes_per_variant(h->bins[bi], h->ball, h->self, p);
    for (int i = 0; i < kWsArrays; ++i) per[bi][i] = p[i];
  }
  std::vector<size_t> cnt(nb, 0);
  auto grow = [&](int bi) {  // bytes added by one more variant of bin bi
    size_t d = 0;
    for (int i = 0; i < kWsArrays; ++i) d += align256((cnt[bi] + 1) * per[bi][i]) - align256(cnt[bi] * per[bi][i]);
    return d;
  };
  std::vector<int32_t> ends;
  size_t used = 0;
  for (int i = 0; i < h->n; ++i) {
    const int bi = h->bin_of[i];
    if (used + grow(bi) > max_workspace_bytes) {
      if (used == 0)
        return fail(const_cast<sim_handle*>(h), SIM_E_NOMEM,
                    "variant " + std::to_string(i) + " alone needs more workspace than the cap");
      ends.push_back(i);  // close the chunk before variant i
      std::fill(cnt.begin(), cnt.end(), 0);
      used = 0;
      if (grow(bi) > max_workspace_bytes)
        return fail(const_cast<sim_handle*>(h), SIM_E_NOMEM,
                    "variant " + std::to_string(i) + " alone needs more workspace than the cap");
    }
    used += grow(bi);
    ++cnt[bi];
  }
  if (h->n > 0) ends.push_back(h->n);
  *n_chunks = (int32_t)ends.size();
  if ((int32_t)ends.size() > max_chunks || (!chunk_end && !ends.empty()))
    return fail(const_cast<sim_handle*>(h), SIM_E_INVALID, "chunk_end holds fewer than " +
                                                              std::to_string(ends.size()) + " entries");
  std::copy(ends.begin(), ends.end(), chunk_end);
  return SIM_OK;
}

int sim_bin_factorization(const sim_handle* h, int32_t* n_bins, int32_t* factorization, int32_t max_bins) {
  if (!h || !n_bins) return SIM_E_INVALID;
  *n_bins = (int32_t)h->bins.size();
  for (int i = 0; i < (int)h->bins.size() && i < max_bins && factorization; ++i)
    factorization[i] = h->bins[i].tree ? SIM_FACTOR_TREE : SIM_FACTOR_DENSE;
  return SIM_OK;
}

void sim_destroy(sim_handle* h) {
  if (!h) return;
  if (h->graph_exec) hipGraphExecDestroy(h->graph_exec);
  if (h->graph) hipGraphDestroy(h->graph);
  if (h->cap_stream) hipStreamDestroy(h->cap_stream);
  for (hipStream_t s2 : h->bin_streams) hipStreamDestroy(s2);
  for (hipEvent_t e2 : h->join_events) hipEventDestroy(e2);
  if (h->fork_event) hipEventDestroy(h->fork_event);
  for (Bin& b : h->bins) {
    if (b.t_begin) hipEventDestroy(b.t_begin);
    if (b.t_end) hipEventDestroy(b.t_end);
  }
  delete h;
}

const char* sim_last_error(const sim_handle* h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

}  // extern "C"
