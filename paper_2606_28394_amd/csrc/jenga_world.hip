// Host side of the C ABI (include/jenga.h): world bookkeeping, packing towers
// into on-chip packs, host <-> device transfers, launches and queries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "../../include/jenga.h"
#include "jenga_device.h"

namespace {

thread_local std::string g_err;

int32_t fail(int32_t code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(JG_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  hipError_t ensure(size_t count) {
    if (count <= n && p) return hipSuccess;
    if (p) {
      const hipError_t f = hipFree(p);
      p = nullptr;
      n = 0;
      if (f != hipSuccess) return f;
    }
    size_t c = count ? count : 1;
    hipError_t e = hipMalloc((void**)&p, c * sizeof(T));
    if (e == hipSuccess) n = c;
    return e;
  }
  hipError_t release() {
    const hipError_t e = p ? hipFree(p) : hipSuccess;
    p = nullptr;
    n = 0;
    return e;
  }
};

struct PushRow {
  int body;
  double force[3];
  int start, steps;
  double withdraw;
  double x0[3];
  int move;        // JG_MOVE_* (episode counts)
};

}  // namespace

int32_t jg::set_error(int32_t code, const std::string& msg) { return fail(code, msg); }

struct jg_world {
  jg_params prm;
  int max_towers = 0, max_bodies = 0;
  hipStream_t stream = nullptr;
  // host mirror, indexed by body id
  std::vector<double> he, mass, x, q, v, w;
  std::vector<uint8_t> active;
  std::vector<int> body_tower;
  std::vector<std::vector<int>> tower_bodies;
  std::vector<double> mu;
  std::vector<PushRow> pushes;
  // state flags
  bool layout_dirty = true;   // bodies, towers or pushes changed
  bool host_dirty = true;     // host mirror newer than the device
  bool device_newer = false;  // device newer than the host mirror
  bool clear_warm = true;     // forget the previous step's impulses before the next launch
  bool views_out = false;     // jg_device_views was called: device memory may be newer at any time
  uint32_t err_reported = 0;  // device error bits already returned by a syncing call
  // layout (internal order)
  std::vector<int> int_of_body, body_of_int;
  std::vector<int> tower_order;      // internal tower slot -> tower id
  std::vector<int> tower_slot;       // tower id -> internal slot
  std::vector<int> pack_body0, pack_tower0, pack_push0, pack_slot0;
  struct PackClass {
    int first = 0, count = 0, per_cu = 0, nbp = 1, pc = 16, tpc = 1, ppc = 1;
    size_t lds = 0;
    bool global = false;     // packs keep their state in device memory (islands too large for LDS)
    bool hot_bodies = false; // global packs: the serial walks' body arrays in LDS
    bool lat = false;        // one tower per workgroup of four waves (small batches)
    int64_t gwords = 0;      // words of one pack's device region
  };
  std::vector<PackClass> classes;   // launch classes, in pack order
  // launch classes run concurrently: one auxiliary stream per class after the first, forked from
  // and joined back into the world's stream with events (all at the default priority)
  std::vector<hipStream_t> aux;
  std::vector<hipEvent_t> aux_done;
  hipEvent_t fork = nullptr;
  std::vector<int> push_order;       // internal push row -> pushes index
  std::vector<int> pack_of_tower;    // tower id -> pack
  int n_packs = 0;
  // device buffers
  DevBuf<float> d_x, d_q, d_v, d_w, d_he, d_mass;
  DevBuf<uint32_t> d_flags;
  DevBuf<int32_t> d_body_tower, d_pack_body0, d_pack_tower0, d_pack_push0, d_pack_slot0, d_tower_body0;
  DevBuf<int64_t> d_pack_goff;
  DevBuf<float> d_gmem;           // per-pack device regions (lever arms, impulses; global packs: all)
  DevBuf<float> d_tower_mu;
  DevBuf<int32_t> d_push_body, d_push_start, d_push_steps;
  DevBuf<float> d_push_force, d_push_withdraw, d_push_x0;
  DevBuf<uint32_t> d_tower_count;
  DevBuf<float> d_tower_res;
  DevBuf<uint32_t> d_pack_error;
  DevBuf<uint32_t> d_err_flag;      // error bits raised by launches since the host last read them
  DevBuf<uint32_t> d_tower_frozen;  // [tower slot] frozen (non-finite state) flags
  // episodes (jg_begin_episodes): per tower slot kEpisodeWords words, reference positions
  DevBuf<uint32_t> d_ep_state;
  DevBuf<float> d_ep_x0;
  bool ep_on = false;
  DevBuf<uint32_t> d_out_ab, d_out_meta;
  DevBuf<float> d_out_geo, d_out_pts;
  DevBuf<int32_t> d_out_count, d_out_tower;
  DevBuf<uint32_t> d_prev_key;
  DevBuf<float> d_prev_data;
  DevBuf<int32_t> d_prev_count;
  DevBuf<unsigned long long> d_phase_cycles;
  // learned warm start and feature records
  DevBuf<float> d_mlp_params;
  DevBuf<uint8_t> d_mlp_packed;
  bool mlp_set = false;
  DevBuf<float> d_feat;
  DevBuf<uint32_t> d_tower_fallback;
  // statistics (per tower id)
  std::vector<int64_t> st_cand, st_man, st_pts, st_ci, st_fb;
  std::vector<int32_t> st_col;
  std::vector<uint32_t> st_err;
  std::vector<double> st_rms, st_max;
  std::vector<uint32_t> pack_err_acc;
  int64_t step = 0;
  int64_t launched_points_iters = 0;
  bool stats_pending = false;
  int last_launch_steps = 0;
  // graphs of the launch (use_graph): one kernel node per launch class, no edges between them
  struct StepGraph {
    int n_steps = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipGraphNode_t> nodes;
    std::vector<jg::StepArgs> args;   // as last set; step0 is rewritten on every replay
    std::vector<size_t> lds;
    std::vector<const void*> func;
    std::vector<unsigned> block;
  };
  std::vector<StepGraph> graphs;    // most recently built last
  // towers stepped by the whole GPU (at least mega_bodies bodies): after every pack in internal
  // order, each with its own scratch
  struct Mega {
    int tower = -1, g0 = 0, nb = 0, tslot = 0, p0 = 0, np = 0;
    int ncell_cap = 0, cand_cap = 0, nparts = 0, grid = 0;
    DevBuf<float> body, md, red, out_geo, out_pts;
    DevBuf<uint32_t> ubody, cand, out_meta, err;
    DevBuf<int32_t> cells, man, part, ired, scal, out_a, out_b, out_count;
    hipError_t release() {
      hipError_t first = hipSuccess;
      for (hipError_t e : {body.release(), md.release(), red.release(), out_geo.release(), out_pts.release(),
                           ubody.release(), cand.release(), out_meta.release(), err.release(), cells.release(),
                           man.release(), part.release(), ired.release(), scal.release(), out_a.release(),
                           out_b.release(), out_count.release()})
        if (first == hipSuccess) first = e;
      return first;
    }
  };
  std::vector<Mega> megas;
  std::vector<int> mega_of_tower;   // tower id -> index in megas (-1: in a pack)
};

namespace {

hipError_t destroy_graph(jg_world::StepGraph& g) {
  hipError_t first = hipSuccess;
  if (g.exec) { first = hipGraphExecDestroy(g.exec); g.exec = nullptr; }
  if (g.graph) {
    hipError_t e = hipGraphDestroy(g.graph);
    if (first == hipSuccess) first = e;
    g.graph = nullptr;
  }
  return first;
}

int32_t check_world(jg_world* w) {
  if (!w) return fail(JG_EINVAL, "null world");
  return JG_OK;
}

int32_t set_device(jg_world* w) {
  HIP_TRY(hipSetDevice(w->prm.device));
  return JG_OK;
}

// device -> host mirror
int32_t download_state(jg_world* w) {
  if (!w->device_newer && !(w->views_out && !w->layout_dirty && !w->host_dirty)) return JG_OK;
  const int n = (int)w->body_of_int.size();
  const int cap = w->max_bodies;
  std::vector<float> buf((size_t)4 * cap);
  std::vector<uint32_t> fl(cap);
  HIP_TRY(hipStreamSynchronize(w->stream));
  auto get = [&](DevBuf<float>& d, int comps, std::vector<double>& dst) -> int32_t {
    HIP_TRY(hipMemcpy(buf.data(), d.p, sizeof(float) * comps * cap, hipMemcpyDeviceToHost));
    for (int k = 0; k < comps; ++k)
      for (int i = 0; i < n; ++i) dst[(size_t)comps * w->body_of_int[i] + k] = buf[(size_t)k * cap + i];
    return JG_OK;
  };
  int32_t r;
  if ((r = get(w->d_x, 3, w->x))) return r;
  if ((r = get(w->d_q, 4, w->q))) return r;
  if ((r = get(w->d_v, 3, w->v))) return r;
  if ((r = get(w->d_w, 3, w->w))) return r;
  HIP_TRY(hipMemcpy(fl.data(), w->d_flags.p, sizeof(uint32_t) * cap, hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i) w->active[w->body_of_int[i]] = (fl[i] & jg::kActive) ? 1 : 0;
  if (!w->pushes.empty()) {
    std::vector<float> x0(3 * w->push_order.size());
    HIP_TRY(hipMemcpy(x0.data(), w->d_push_x0.p, sizeof(float) * x0.size(), hipMemcpyDeviceToHost));
    for (size_t r2 = 0; r2 < w->push_order.size(); ++r2)
      for (int k = 0; k < 3; ++k) w->pushes[w->push_order[r2]].x0[k] = x0[3 * r2 + k];
  }
  w->device_newer = false;
  return JG_OK;
}

// Pack towers into workgroups (first fit, largest first).  A pack holds whole towers and at
// most `target` bodies, where `target` is the largest pack whose LDS fits as many workgroups on
// a CU as the step kernel's registers allow: eight (two waves per SIMD) for the plain variant,
// four for the variant with contact features (learned warm start, feature records); or one
// tower per pack when the batch has no more towers than the GPU holds such workgroups.  A tower
// larger than the target gets a pack of its own.  Packs are then grouped into launch
// classes of equal workgroups-per-CU, each launched with the LDS its largest pack needs.
int32_t build_layout(jg_world* w) {
  const int T = (int)w->tower_bodies.size();
  std::vector<int> order, mega_towers;
  int max_tower = 1;
  for (int t = 0; t < T; ++t) {
    const int n = (int)w->tower_bodies[t].size();
    if (n == 0) continue;
    if (w->prm.mega_bodies > 0 && n >= w->prm.mega_bodies) {
      mega_towers.push_back(t);
      continue;
    }
    order.push_back(t);
    max_tower = std::max(max_tower, n);
  }
  if (max_tower > 65534) return fail(JG_ECAPACITY, "a tower has more bodies than one pack can index (65534)");
  if (!mega_towers.empty() && (w->prm.warm_start != 0 || w->prm.use_graph || w->prm.record_features))
    return fail(JG_EINVAL, "towers of mega_bodies bodies or more are stepped with warm_start 0, without graphs "
                           "or feature records");
  for (auto& m : w->megas) HIP_TRY(m.release());
  w->megas.clear();
  w->mega_of_tower.assign(T, -1);
  // manifold slots per body: 3.5 in shared packs (sized for LDS); a batch stepped one tower per
  // workgroup (below) has LDS to spare and gets 6, room for a sinking or collapsing tower's pairs
  float mpb = w->prm.manifolds_per_body > 0.f ? w->prm.manifolds_per_body : 3.5f;
  const int mode = w->prm.warm_start == 2 ? 2 : ((w->prm.warm_start == 1 || w->prm.record_features) ? 1 : 0);
  auto pc_of = [&](int nb) { return std::max(16, (int)std::ceil(mpb * nb)); };
  auto lds_of = [&](int nb, int towers, int pushes) -> size_t {
    return (size_t)jg::lds_words(nb, pc_of(nb), std::max(1, towers), std::max(1, pushes), mode) * 4;
  };
  // an on-chip pack holds at most kRegBodies bodies (the register broadphase); larger islands
  // are kept in device memory, one tower each
  int target = w->prm.pack_bodies > 0 ? std::min(w->prm.pack_bodies, jg::kRegBodies) : 0;
  bool lat = false;
  if (target <= 0) {
    const bool wide = w->prm.warm_start == 2 || w->prm.record_features;
    const size_t budget = wide ? 40 * 1024 : 20 * 1024;
    target = 8;
    while (lds_of(target + 1, 4, 8) <= budget) ++target;
    // A batch with no more towers than the GPU holds workgroups at once gets one tower per pack:
    // sharing a pack would only run towers one after another that could run side by side
    // (the 450-tower removal batch steps 11 % faster so).
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, w->prm.device) == hipSuccess && cus > 0 &&
        (int64_t)order.size() <= (int64_t)cus * (wide ? 4 : 8)) {
      target = 1;
      if (!(w->prm.manifolds_per_body > 0.f)) mpb = 6.0f;
      // at most two towers per CU: each gets a workgroup of four waves (two per CU at two waves
      // per SIMD), which share its manifolds, sweeps and residual
      lat = w->prm.small_batch >= 0 && !wide && (int64_t)order.size() <= 2 * (int64_t)cus;
    }
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return w->tower_bodies[a].size() > w->tower_bodies[b].size();
  });
  struct Bin { int bodies = 0, cap = 0; std::vector<int> towers; bool global = false; };
  std::vector<Bin> bins;
  std::vector<int> tower_pushes(T, 0);
  for (const auto& pr : w->pushes) ++tower_pushes[w->body_tower[pr.body]];
  for (int t : order) {
    const int n = (int)w->tower_bodies[t].size();
    // an island beyond the LDS path (register broadphase windows, or LDS) is a global pack
    if (n > jg::kRegBodies || lds_of(n, 1, tower_pushes[t]) > 160 * 1024 || w->prm.pack_bodies < 0) {
      Bin b;
      b.bodies = n; b.cap = n; b.towers.push_back(t); b.global = true;
      bins.push_back(b);
      continue;
    }
    bool placed = false;
    for (auto& b : bins)
      if (!b.global && b.bodies + n <= b.cap && (int)b.towers.size() < 255) {
        b.towers.push_back(t); b.bodies += n; placed = true; break;
      }
    if (!placed) { Bin b; b.bodies = n; b.cap = std::max(target, n); b.towers.push_back(t); bins.push_back(b); }
  }
  std::stable_sort(bins.begin(), bins.end(), [](const Bin& a, const Bin& b) { return a.bodies > b.bodies; });
  // group packs by how many fit a CU (their LDS), largest LDS first, so that each launch class
  // is one contiguous range: a handful of classes, not one per change of push count
  {
    std::vector<int> key(bins.size());
    for (size_t b = 0; b < bins.size(); ++b) {
      int pushes = 0;
      for (int t : bins[b].towers) pushes += tower_pushes[t];
      key[b] = bins[b].global ? (1 << 30)   // global packs last, one class of their own
                              : (int)((160 * 1024) / std::max<size_t>(1, lds_of(bins[b].bodies, (int)bins[b].towers.size(), pushes)));
    }
    std::vector<size_t> idx(bins.size());
    for (size_t b = 0; b < idx.size(); ++b) idx[b] = b;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return key[a] < key[b]; });
    std::vector<Bin> sorted;
    sorted.reserve(bins.size());
    for (size_t b : idx) sorted.push_back(std::move(bins[b]));
    bins.swap(sorted);
  }
  // internal order
  const int N = (int)w->he.size() / 3;
  w->int_of_body.assign(N, -1);
  w->body_of_int.clear();
  w->tower_order.clear();
  w->tower_slot.assign(T, -1);
  w->pack_of_tower.assign(T, -1);
  w->pack_body0.assign(1, 0);
  w->pack_tower0.assign(1, 0);
  w->pack_push0.assign(1, 0);
  w->pack_slot0.assign(1, 0);
  w->push_order.clear();
  w->classes.clear();
  std::vector<std::vector<int>> push_of_body(N);
  for (size_t r = 0; r < w->pushes.size(); ++r) push_of_body[w->pushes[r].body].push_back((int)r);
  for (size_t b = 0; b < bins.size(); ++b) {
    int pushes = 0;
    for (int t : bins[b].towers) {
      w->tower_slot[t] = (int)w->tower_order.size();
      w->tower_order.push_back(t);
      w->pack_of_tower[t] = (int)b;
      for (int id : w->tower_bodies[t]) {
        w->int_of_body[id] = (int)w->body_of_int.size();
        w->body_of_int.push_back(id);
      }
    }
    for (int t : bins[b].towers)
      for (int id : w->tower_bodies[t])
        for (int r : push_of_body[id]) { w->push_order.push_back(r); ++pushes; }
    w->pack_body0.push_back((int)w->body_of_int.size());
    w->pack_tower0.push_back((int)w->tower_order.size());
    w->pack_push0.push_back((int)w->push_order.size());
    // launch class: packs that fit the same number of workgroups per CU (global packs: one class)
    const size_t lds = lds_of(bins[b].bodies, (int)bins[b].towers.size(), pushes);
    const int per_cu = bins[b].global ? 0 : (int)((160 * 1024) / lds);
    if (!bins[b].global && per_cu == 0)
      return fail(JG_ECAPACITY, "a pack needs " + std::to_string(lds) + " bytes of LDS (max 163840); "
                                "use smaller towers or fewer manifolds per body");
    if (w->classes.empty() || w->classes.back().per_cu != per_cu || w->classes.back().global != bins[b].global) {
      jg_world::PackClass c;
      c.first = (int)b;
      c.per_cu = per_cu;
      c.global = bins[b].global;
      c.lat = lat && !bins[b].global;
      w->classes.push_back(c);
    }
    jg_world::PackClass& c = w->classes.back();
    c.count += 1;
    c.nbp = std::max(c.nbp, bins[b].bodies);
    c.tpc = std::max(c.tpc, (int)bins[b].towers.size());
    c.ppc = std::max(c.ppc, std::max(1, pushes));
  }
  // towers stepped by the whole GPU: their bodies, slots and push rows after every pack's
  for (int t : mega_towers) {
    jg_world::Mega m;
    m.tower = t;
    m.tslot = (int)w->tower_order.size();
    w->tower_slot[t] = m.tslot;
    w->tower_order.push_back(t);
    m.g0 = (int)w->body_of_int.size();
    for (int id : w->tower_bodies[t]) {
      w->int_of_body[id] = (int)w->body_of_int.size();
      w->body_of_int.push_back(id);
    }
    m.nb = (int)w->body_of_int.size() - m.g0;
    m.p0 = (int)w->push_order.size();
    for (int id : w->tower_bodies[t])
      for (int r : push_of_body[id]) w->push_order.push_back(r);
    m.np = (int)w->push_order.size() - m.p0;
    w->mega_of_tower[t] = (int)w->megas.size();
    w->megas.push_back(m);
  }
  // neighbouring classes whose LDS would fit more workgroups per CU than the kernel's registers
  // allow run at the same occupancy: one launch holds them all (with the largest pack's LDS, as
  // long as that still fits the register-bound count), so that they share one launch tail
  {
    const int reg_cap = lat ? 2 : ((w->prm.warm_start == 2 || w->prm.record_features) ? 4 : 8);
    for (size_t k = 1; k < w->classes.size();) {
      jg_world::PackClass& into = w->classes[k - 1];
      const jg_world::PackClass& from = w->classes[k];
      const bool same = !into.global && !from.global && into.lat == from.lat && into.per_cu >= reg_cap &&
                        from.per_cu >= reg_cap;
      const int nbp = std::max(into.nbp, from.nbp), tpc = std::max(into.tpc, from.tpc),
                ppc = std::max(into.ppc, from.ppc);
      if (same && (int)((160 * 1024) / lds_of(nbp, tpc, ppc)) >= reg_cap) {
        into.count += from.count;
        into.nbp = nbp;
        into.tpc = tpc;
        into.ppc = ppc;
        w->classes.erase(w->classes.begin() + (long)k);
      } else {
        ++k;
      }
    }
  }
  // at most four classes (the hardware queues a process gets by default): fold the smallest class
  // into its neighbour with the larger LDS (its packs then run at that neighbour's occupancy)
  auto lds_classes = [&]() {
    size_t n = 0;
    for (const auto& c : w->classes) n += c.global ? 0 : 1;
    return n;
  };
  while (lds_classes() > 4) {
    size_t k = 1;
    for (size_t i = 2; i < w->classes.size(); ++i)
      if (!w->classes[i].global && w->classes[i].count < w->classes[k].count) k = i;
    jg_world::PackClass& into = w->classes[k - 1];
    const jg_world::PackClass& from = w->classes[k];
    into.count += from.count;
    into.nbp = std::max(into.nbp, from.nbp);
    into.tpc = std::max(into.tpc, from.tpc);
    into.ppc = std::max(into.ppc, from.ppc);
    w->classes.erase(w->classes.begin() + (long)k);
  }
  // class capacities; every pack of a class gets the class's contact slots
  std::vector<int64_t> goff;
  int64_t gtotal = 0;
  for (auto& c : w->classes) {
    c.pc = pc_of(c.nbp);
    if (c.global) {
      // small arrays in LDS always; the serial walks' body arrays too when they fit
      c.hot_bodies = jg::hot_words(c.nbp, c.tpc, c.ppc, true) * 4 <= 160 * 1024;
      c.lds = (size_t)jg::hot_words(c.nbp, c.tpc, c.ppc, c.hot_bodies) * 4;
      if (c.lds > 160 * 1024)
        return fail(JG_ECAPACITY, "a pack kept in device memory needs " + std::to_string(c.lds) +
                                  " bytes of LDS for its towers and pushes (max 163840)");
      // (with the network, every wave of the island has its own staging rows)
      c.gwords = ((int64_t)jg::kManPackWords * c.pc + jg::lds_words(c.nbp, c.pc, c.tpc, c.ppc, mode) +
                  (mode == 2 ? (int64_t)(jg::kLearnedIslandWaves - 1) * jg::kStageWords : 0) +
                  jg::window_words(c.nbp) + 2 * (int64_t)jg::kCandPerBody * c.nbp + 3) & ~(int64_t)3;
      for (int k = 0; k < c.count; ++k) { goff.push_back(gtotal); gtotal += c.gwords; }
    } else {
      c.lds = (size_t)jg::lds_words(c.nbp, c.pc, c.tpc, c.ppc, mode) * 4;
      if (c.lds > 160 * 1024)
        return fail(JG_ECAPACITY, "a launch class needs " + std::to_string(c.lds) + " bytes of LDS (max 163840)");
      c.gwords = ((int64_t)jg::kManPackWords * c.pc + 3) & ~(int64_t)3;
      for (int k = 0; k < c.count; ++k) { goff.push_back(gtotal); gtotal += c.gwords; }
    }
    for (int k = 0; k < c.count; ++k) w->pack_slot0.push_back(w->pack_slot0.back() + c.pc);
  }
  w->n_packs = (int)bins.size();
  // device buffers sized by the layout
  const size_t np = (size_t)std::max(1, w->n_packs);
  const size_t nt = (size_t)std::max(1, T);
  const size_t npush = std::max<size_t>(1, w->push_order.size());
  HIP_TRY(w->d_pack_body0.ensure(np + 1));
  HIP_TRY(w->d_pack_tower0.ensure(np + 1));
  HIP_TRY(w->d_pack_push0.ensure(np + 1));
  HIP_TRY(w->d_pack_slot0.ensure(np + 1));
  HIP_TRY(w->d_pack_goff.ensure(np));
  HIP_TRY(w->d_gmem.ensure((size_t)std::max<int64_t>(4, gtotal)));
  HIP_TRY(w->d_tower_body0.ensure(nt + 1));
  HIP_TRY(w->d_tower_mu.ensure(nt));
  HIP_TRY(w->d_tower_count.ensure(4 * nt));
  HIP_TRY(w->d_tower_res.ensure(2 * nt));
  HIP_TRY(w->d_pack_error.ensure(np));
  HIP_TRY(w->d_tower_frozen.ensure(nt));
  HIP_TRY(w->d_push_body.ensure(npush));
  HIP_TRY(w->d_push_start.ensure(npush));
  HIP_TRY(w->d_push_steps.ensure(npush));
  HIP_TRY(w->d_push_force.ensure(3 * npush));
  HIP_TRY(w->d_push_withdraw.ensure(npush));
  HIP_TRY(w->d_push_x0.ensure(3 * npush));
  const size_t slots = std::max<size_t>(1, (size_t)w->pack_slot0.back());
  HIP_TRY(w->d_out_ab.ensure(slots));
  HIP_TRY(w->d_out_meta.ensure(slots));
  HIP_TRY(w->d_out_geo.ensure(8 * slots));
  HIP_TRY(w->d_out_pts.ensure(24 * slots));
  HIP_TRY(w->d_out_count.ensure(np));
  HIP_TRY(w->d_out_tower.ensure(slots));
  HIP_TRY(w->d_prev_key.ensure(slots));
  HIP_TRY(w->d_prev_data.ensure(16 * slots));
  HIP_TRY(w->d_prev_count.ensure(np));
  HIP_TRY(w->d_tower_fallback.ensure(2 * nt));
  HIP_TRY(hipMemsetAsync(w->d_tower_fallback.p, 0, sizeof(uint32_t) * 2 * nt, w->stream));
  if (w->prm.record_features) HIP_TRY(w->d_feat.ensure((size_t)4 * jg::kFeatRecord * slots));
  HIP_TRY(hipMemsetAsync(w->d_tower_count.p, 0, sizeof(uint32_t) * 4 * nt, w->stream));
  HIP_TRY(hipMemsetAsync(w->d_tower_res.p, 0, sizeof(float) * 2 * nt, w->stream));
  HIP_TRY(hipMemsetAsync(w->d_pack_error.p, 0, sizeof(uint32_t) * np, w->stream));
  HIP_TRY(hipMemsetAsync(w->d_out_count.p, 0, sizeof(int32_t) * np, w->stream));
  HIP_TRY(hipMemsetAsync(w->d_prev_count.p, 0, sizeof(int32_t) * np, w->stream));
  std::vector<int32_t> tb0(T + 1, 0);
  for (int s = 0; s < (int)w->tower_order.size(); ++s)
    tb0[s + 1] = tb0[s] + (int)w->tower_bodies[w->tower_order[s]].size();
  HIP_TRY(hipMemcpy(w->d_pack_body0.p, w->pack_body0.data(), sizeof(int32_t) * w->pack_body0.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w->d_pack_tower0.p, w->pack_tower0.data(), sizeof(int32_t) * w->pack_tower0.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w->d_pack_push0.p, w->pack_push0.data(), sizeof(int32_t) * w->pack_push0.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w->d_pack_slot0.p, w->pack_slot0.data(), sizeof(int32_t) * w->pack_slot0.size(), hipMemcpyHostToDevice));
  if (!goff.empty())
    HIP_TRY(hipMemcpy(w->d_pack_goff.p, goff.data(), sizeof(int64_t) * goff.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w->d_tower_body0.p, tb0.data(), sizeof(int32_t) * (w->tower_order.size() + 1), hipMemcpyHostToDevice));
  std::vector<int32_t> btw(w->max_bodies, 0);
  for (int s = 0; s < (int)w->tower_order.size(); ++s)
    for (int k = tb0[s]; k < tb0[s + 1]; ++k) btw[k] = s;
  HIP_TRY(hipMemcpy(w->d_body_tower.p, btw.data(), sizeof(int32_t) * w->max_bodies, hipMemcpyHostToDevice));
  // scratch of the towers stepped by the whole GPU
  if (!w->megas.empty()) {
    for (auto& m : w->megas) {
      if (int e = jg::mega_blocks(m.nb, &m.grid))
        return fail(JG_EDEVICE, std::string("sizing the grid-wide launch: ") + hipGetErrorString((hipError_t)e));
      const size_t G = (size_t)m.grid;
      const size_t nb = (size_t)m.nb;
      m.ncell_cap = (int)std::min<size_t>(2 * nb + 64, (size_t)1 << 30);
      const double cc = std::ceil((double)w->prm.mega_cand_per_body * (double)nb);
      if (cc > 2.0e9) return fail(JG_ECAPACITY, "candidate capacity of a large island beyond 2e9");
      m.cand_cap = std::max(64, (int)cc);
      m.nparts = (int)((nb + (size_t)w->prm.colour_partition - 1) / (size_t)w->prm.colour_partition);
      const size_t C = (size_t)m.cand_cap;
      HIP_TRY(m.body.ensure(jg::kMegaBodyWords * nb));
      HIP_TRY(m.ubody.ensure(jg::kMegaBodyU32 * nb));
      HIP_TRY(m.cells.ensure(2 * ((size_t)m.ncell_cap + 1)));
      HIP_TRY(m.cand.ensure(3 * C));
      HIP_TRY(m.man.ensure(7 * C));
      HIP_TRY(m.md.ensure((size_t)(jg::kManDevWords + jg::kManBiasWords) * C));
      HIP_TRY(m.part.ensure(2 * (size_t)m.nparts + 1));
      HIP_TRY(m.red.ensure(2 * G + 2));
      HIP_TRY(m.ired.ensure(G + 1));
      HIP_TRY(m.scal.ensure(jg::kMegaScal));
      HIP_TRY(m.out_a.ensure(C));
      HIP_TRY(m.out_b.ensure(C));
      HIP_TRY(m.out_meta.ensure(C));
      HIP_TRY(m.out_geo.ensure(8 * C));
      HIP_TRY(m.out_pts.ensure(24 * C));
      HIP_TRY(m.out_count.ensure(1));
      HIP_TRY(m.err.ensure(1));
      HIP_TRY(hipMemsetAsync(m.out_count.p, 0, sizeof(int32_t), w->stream));
      HIP_TRY(hipMemsetAsync(m.err.p, 0, sizeof(uint32_t), w->stream));
    }
  }
  w->layout_dirty = false;
  w->clear_warm = true;
  w->ep_on = false;   // the episode state is per tower slot of the old layout
  return JG_OK;
}

// host mirror -> device (state, statics, towers, pushes)
int32_t upload_all(jg_world* w) {
  const int n = (int)w->body_of_int.size();
  const int cap = w->max_bodies;
  std::vector<float> buf((size_t)4 * cap, 0.f);
  auto put = [&](DevBuf<float>& d, int comps, const std::vector<double>& src) -> int32_t {
    std::fill(buf.begin(), buf.end(), 0.f);
    for (int k = 0; k < comps; ++k)
      for (int i = 0; i < n; ++i) buf[(size_t)k * cap + i] = (float)src[(size_t)comps * w->body_of_int[i] + k];
    HIP_TRY(hipMemcpy(d.p, buf.data(), sizeof(float) * comps * cap, hipMemcpyHostToDevice));
    return JG_OK;
  };
  int32_t r;
  if ((r = put(w->d_x, 3, w->x))) return r;
  if ((r = put(w->d_q, 4, w->q))) return r;
  if ((r = put(w->d_v, 3, w->v))) return r;
  if ((r = put(w->d_w, 3, w->w))) return r;
  if ((r = put(w->d_he, 3, w->he))) return r;
  std::vector<float> ms(cap, 0.f);
  std::vector<uint32_t> fl(cap, 0u);
  for (int i = 0; i < n; ++i) {
    const int id = w->body_of_int[i];
    ms[i] = (float)w->mass[id];
    fl[i] = (w->active[id] ? jg::kActive : 0u) | (w->mass[id] > 0.0 ? jg::kDynamic : 0u);
  }
  HIP_TRY(hipMemcpy(w->d_mass.p, ms.data(), sizeof(float) * cap, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(w->d_flags.p, fl.data(), sizeof(uint32_t) * cap, hipMemcpyHostToDevice));
  std::vector<float> mu(std::max<size_t>(1, w->tower_order.size()));
  for (size_t s = 0; s < w->tower_order.size(); ++s) mu[s] = (float)w->mu[w->tower_order[s]];
  HIP_TRY(hipMemcpy(w->d_tower_mu.p, mu.data(), sizeof(float) * mu.size(), hipMemcpyHostToDevice));
  // the host's state replaces the device's: no tower is frozen until a step finds it non-finite
  HIP_TRY(hipMemset(w->d_tower_frozen.p, 0, sizeof(uint32_t) * mu.size()));
  const size_t P = w->push_order.size();
  if (P) {
    std::vector<int32_t> pb(P), ps(P), pn(P);
    std::vector<float> pf(3 * P), pw(P), px(3 * P);
    for (size_t r2 = 0; r2 < P; ++r2) {
      const PushRow& pr = w->pushes[w->push_order[r2]];
      pb[r2] = w->int_of_body[pr.body];
      ps[r2] = pr.start;
      pn[r2] = pr.steps;
      pw[r2] = (float)pr.withdraw;
      for (int k = 0; k < 3; ++k) { pf[3 * r2 + k] = (float)pr.force[k]; px[3 * r2 + k] = (float)pr.x0[k]; }
    }
    HIP_TRY(hipMemcpy(w->d_push_body.p, pb.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(w->d_push_start.p, ps.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(w->d_push_steps.p, pn.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(w->d_push_force.p, pf.data(), sizeof(float) * 3 * P, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(w->d_push_withdraw.p, pw.data(), sizeof(float) * P, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(w->d_push_x0.p, px.data(), sizeof(float) * 3 * P, hipMemcpyHostToDevice));
  }
  w->host_dirty = false;
  return JG_OK;
}

// fold device counters into the host statistics and clear them
int32_t collect_stats(jg_world* w) {
  if (!w->stats_pending) return JG_OK;
  const int T = (int)w->tower_order.size();
  if (T == 0) { w->stats_pending = false; return JG_OK; }
  HIP_TRY(hipStreamSynchronize(w->stream));
  std::vector<uint32_t> cnt(4 * T);
  std::vector<float> res(2 * T);
  std::vector<uint32_t> perr(w->n_packs);
  std::vector<uint32_t> fb(2 * T, 0u);
  const bool learned = w->prm.warm_start == 2;
  if (learned)
    HIP_TRY(hipMemcpy(fb.data(), w->d_tower_fallback.p, sizeof(uint32_t) * 2 * T, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(cnt.data(), w->d_tower_count.p, sizeof(uint32_t) * 4 * T, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(res.data(), w->d_tower_res.p, sizeof(float) * 2 * T, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(perr.data(), w->d_pack_error.p, sizeof(uint32_t) * w->n_packs, hipMemcpyDeviceToHost));
  for (int s = 0; s < T; ++s) {
    const int t = w->tower_order[s];
    w->st_cand[t] += cnt[4 * s];
    w->st_man[t] += cnt[4 * s + 1];
    w->st_pts[t] += cnt[4 * s + 2];
    w->st_ci[t] += (int64_t)cnt[4 * s + 2] * (learned ? w->prm.mlp_iters : w->prm.iters) +
                   (int64_t)fb[2 * s + 1] * w->prm.iters;
    w->st_fb[t] += fb[2 * s];
    w->st_col[t] = (int32_t)cnt[4 * s + 3];
    w->st_rms[t] = res[2 * s];
    w->st_max[t] = res[2 * s + 1];
    if (w->pack_of_tower[t] >= 0) w->st_err[t] |= perr[w->pack_of_tower[t]];
  }
  for (auto& m : w->megas) {
    uint32_t e = 0;
    HIP_TRY(hipMemcpy(&e, m.err.p, sizeof(e), hipMemcpyDeviceToHost));
    w->st_err[m.tower] |= e;
  }
  for (int k = 0; k < 4 * T; k += 4) { cnt[k] = cnt[k + 1] = cnt[k + 2] = 0; }
  HIP_TRY(hipMemcpy(w->d_tower_count.p, cnt.data(), sizeof(uint32_t) * 4 * T, hipMemcpyHostToDevice));
  if (learned) HIP_TRY(hipMemset(w->d_tower_fallback.p, 0, sizeof(uint32_t) * 2 * T));
  w->stats_pending = false;
  return JG_OK;
}

// Error bits that launches raised since the last syncing call (the stream has been waited
// for): JG_ENAN when a state was non-finite, JG_ECAPACITY for a capacity bit, else JG_OK.  Each
// bit raised by a launch is returned once.
int32_t report_device_errors(jg_world* w) {
  uint32_t bits = 0;
  HIP_TRY(hipStreamSynchronize(w->stream));
  HIP_TRY(hipMemcpy(&bits, w->d_err_flag.p, sizeof(bits), hipMemcpyDeviceToHost));
  if (!bits) return JG_OK;
  HIP_TRY(hipMemset(w->d_err_flag.p, 0, sizeof(uint32_t)));
  w->err_reported |= bits;
  std::string what;
  if (bits & JG_ERR_CANDIDATES) what += " JG_ERR_CANDIDATES (an island body had more than 16 candidates)";
  if (bits & JG_ERR_MANIFOLDS) what += " JG_ERR_MANIFOLDS (colliding pairs beyond a pack's capacity were dropped)";
  if (bits & JG_ERR_COLOURS) what += " JG_ERR_COLOURS (manifolds beyond 64 colours were dropped)";
  if (bits & JG_ERR_NAN) what += " JG_ERR_NAN (a tower's state was non-finite: it is frozen)";
  return fail((bits & JG_ERR_NAN) ? JG_ENAN : JG_ECAPACITY, "device error bits since the last syncing call:" + what);
}

// The launch as a HIP graph: one kernel node per launch class and no edges, so the classes may
// run side by side as on the forked streams of the direct launch.  A graph is kept per step
// count and reused while every argument but the first step's index is unchanged (the same
// layout, buffers and parameters); a replay rewrites that index in each node.  Graphs hold
// kernel nodes only.
int32_t launch_graph(jg_world* w, std::vector<jg::StepArgs>& cls, int n_steps) {
  const size_t nc = cls.size();
  auto matches = [&](const jg_world::StepGraph& g) {
    if (g.n_steps != n_steps || g.args.size() != nc) return false;
    for (size_t k = 0; k < nc; ++k) {
      jg::StepArgs x = cls[k];
      x.step0 = g.args[k].step0;
      if (std::memcmp(&x, &g.args[k], sizeof(x)) != 0 || g.lds[k] != w->classes[k].lds) return false;
    }
    return true;
  };
  size_t gi = w->graphs.size();
  for (size_t i = 0; i < w->graphs.size(); ++i)
    if (w->graphs[i].n_steps == n_steps) { gi = i; break; }
  const bool stale = gi < w->graphs.size() && !matches(w->graphs[gi]);
  if (stale || (gi == w->graphs.size() && w->graphs.size() >= 8))
    HIP_TRY(hipStreamSynchronize(w->stream));   // no launch of a graph in flight when it is destroyed
  if (stale) {
    // the layout, a buffer or a parameter changed since it was built
    hipError_t e = destroy_graph(w->graphs[gi]);
    w->graphs.erase(w->graphs.begin() + gi);
    gi = w->graphs.size();
    if (e != hipSuccess) return fail(JG_EDEVICE, std::string("destroying a stale graph: ") + hipGetErrorString(e));
  }
  if (gi == w->graphs.size()) {
    if (w->graphs.size() >= 8) {
      hipError_t e = destroy_graph(w->graphs.front());
      w->graphs.erase(w->graphs.begin());
      if (e != hipSuccess) return fail(JG_EDEVICE, std::string("destroying a graph: ") + hipGetErrorString(e));
    }
    jg_world::StepGraph g;
    g.n_steps = n_steps;
    g.args = cls;
    g.nodes.resize(nc);
    g.lds.resize(nc);
    g.func.resize(nc);
    g.block.resize(nc);
    hipError_t e = hipGraphCreate(&g.graph, 0);
    for (size_t k = 0; k < nc && e == hipSuccess; ++k) {
      g.lds[k] = w->classes[k].lds;
      if (int r = jg::step_launch_config(g.args[k], &g.func[k], &g.block[k])) { e = (hipError_t)r; break; }
      void* kp[1] = {&g.args[k]};
      hipKernelNodeParams p;
      std::memset(&p, 0, sizeof(p));
      p.func = const_cast<void*>(g.func[k]);
      p.gridDim = dim3(g.args[k].n_packs);
      p.blockDim = dim3(g.block[k]);
      p.sharedMemBytes = (unsigned)g.lds[k];
      p.kernelParams = kp;
      p.extra = nullptr;
      e = hipGraphAddKernelNode(&g.nodes[k], g.graph, nullptr, 0, &p);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)destroy_graph(g);   // the build error is the one reported
      return fail(JG_EDEVICE, std::string("building the step graph: ") + hipGetErrorString(e));
    }
    w->graphs.push_back(std::move(g));
    gi = w->graphs.size() - 1;
  }
  jg_world::StepGraph& g = w->graphs[gi];
  for (size_t k = 0; k < nc; ++k) {
    g.args[k].step0 = cls[k].step0;
    void* kp[1] = {&g.args[k]};
    hipKernelNodeParams p;
    std::memset(&p, 0, sizeof(p));
    p.func = const_cast<void*>(g.func[k]);
    p.gridDim = dim3(g.args[k].n_packs);
    p.blockDim = dim3(g.block[k]);
    p.sharedMemBytes = (unsigned)g.lds[k];
    p.kernelParams = kp;
    p.extra = nullptr;
    HIP_TRY(hipGraphExecKernelNodeSetParams(g.exec, g.nodes[k], &p));
  }
  HIP_TRY(hipGraphLaunch(g.exec, w->stream));
  return JG_OK;
}

}  // namespace

extern "C" {

void jg_default_params(jg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->gravity[0] = 0.0; p->gravity[1] = 0.0; p->gravity[2] = -9.81;
  p->dt = 1.0 / 240.0;
  p->restitution = 0.10;
  p->beta = 0.35;
  p->slop = 4e-4;
  p->margin = 2e-3;
  p->n_sub = 1;
  p->iters = 20;
  p->warm_start = 0;
  p->device = 0;
  p->stream = nullptr;
  p->pack_bodies = 0;
  p->manifolds_per_body = 0.f;
  p->mlp_iters = 8;
  p->fallback_tau = 1e30;
  p->record_features = 0;
  p->use_graph = 0;
  p->collapse_fd = 0.5;
  p->collapse_ek = 5e-5;
  p->collapse_theta = 30.0;
  p->rest_ek = 1e-7;
  p->support_eps = 2e-3;
  p->rest_steps = 400;
  p->friction_cone = 0;
  p->restitution_bias = 0;
  p->manifold_mode = 0;
  p->mega_bodies = 16384;
  p->colour_partition = 1024;
  p->mega_cand_per_body = 16.f;
  p->small_batch = 0;
  p->precision = JG_FP32;
}

const char* jg_last_error(void) { return g_err.c_str(); }

int32_t jg_create_world(const jg_params* p, int32_t max_towers, int32_t max_bodies, jg_world** out) {
  if (!out) return fail(JG_EINVAL, "null output handle");
  *out = nullptr;
  if (!p) return fail(JG_EINVAL, "null params");
  if (max_towers <= 0 || max_bodies <= 0) return fail(JG_EINVAL, "max_towers and max_bodies must be positive");
  if (p->iters < 0 || p->n_sub < 1 || !(p->dt > 0.0)) return fail(JG_EINVAL, "bad iters, n_sub or dt");
  if (p->warm_start < 0 || p->warm_start > 2) return fail(JG_EINVAL, "warm_start must be 0, 1 or 2");
  if (p->mlp_iters < 0) return fail(JG_EINVAL, "mlp_iters must not be negative");
  if (p->rest_steps < 0 || !(p->collapse_fd >= 0.0) || !(p->support_eps >= 0.0))
    return fail(JG_EINVAL, "bad episode parameters");
  if (p->friction_cone < 0 || p->friction_cone > 1 || p->restitution_bias < 0 || p->restitution_bias > 1 ||
      p->manifold_mode < 0 || p->manifold_mode > 1)
    return fail(JG_EINVAL, "friction_cone, restitution_bias and manifold_mode are 0 or 1");
  if (p->mega_bodies < 0 || p->colour_partition < 1 || !(p->mega_cand_per_body >= 1.f))
    return fail(JG_EINVAL, "mega_bodies >= 0, colour_partition >= 1 and mega_cand_per_body >= 1");
  if (p->precision == JG_FP64) return fail(JG_EINVAL, "FP64 stepping is not built: the step kernels compute in FP32");
  if (p->precision != JG_FP32) return fail(JG_EINVAL, "precision is JG_FP32 or JG_FP64");
  jg_world* w = new (std::nothrow) jg_world();
  if (!w) return fail(JG_ENOMEM, "host allocation failed");
  w->prm = *p;
  w->max_towers = max_towers;
  w->max_bodies = max_bodies;
  w->stream = (hipStream_t)p->stream;
  int32_t r = set_device(w);
  if (r) { delete w; return r; }
  const size_t cap = (size_t)max_bodies;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = w->d_x.ensure(3 * cap);
  if (e == hipSuccess) e = w->d_q.ensure(4 * cap);
  if (e == hipSuccess) e = w->d_v.ensure(3 * cap);
  if (e == hipSuccess) e = w->d_w.ensure(3 * cap);
  if (e == hipSuccess) e = w->d_he.ensure(3 * cap);
  if (e == hipSuccess) e = w->d_mass.ensure(cap);
  if (e == hipSuccess) e = w->d_flags.ensure(cap);
  if (e == hipSuccess) e = w->d_body_tower.ensure(cap);
  if (e == hipSuccess) e = w->d_phase_cycles.ensure(jg::kPhases);
  if (e == hipSuccess) e = hipMemset(w->d_phase_cycles.p, 0, sizeof(unsigned long long) * jg::kPhases);
  if (e == hipSuccess) e = w->d_err_flag.ensure(1);
  if (e == hipSuccess) e = hipMemset(w->d_err_flag.p, 0, sizeof(uint32_t));
  if (e != hipSuccess) {
    jg_destroy_world(w);
    return fail(JG_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
  }
  *out = w;
  return JG_OK;
}

int32_t jg_destroy_world(jg_world* w) {
  if (!w) return JG_OK;
  // tear everything down even if a call fails; report the first failure
  hipError_t first = hipSuccess;
  auto note = [&](hipError_t e) { if (first == hipSuccess && e != hipSuccess) first = e; };
  note(hipSetDevice(w->prm.device));
  note(hipStreamSynchronize(w->stream));
  for (hipStream_t s : w->aux) note(hipStreamSynchronize(s));
  for (auto& g : w->graphs) note(destroy_graph(g));
  note(w->d_x.release()); note(w->d_q.release()); note(w->d_v.release()); note(w->d_w.release());
  note(w->d_he.release()); note(w->d_mass.release()); note(w->d_flags.release()); note(w->d_body_tower.release());
  note(w->d_pack_body0.release()); note(w->d_pack_tower0.release()); note(w->d_pack_push0.release());
  note(w->d_pack_slot0.release()); note(w->d_tower_body0.release());
  note(w->d_pack_goff.release()); note(w->d_gmem.release());
  note(w->d_tower_mu.release()); note(w->d_push_body.release()); note(w->d_push_start.release());
  note(w->d_push_steps.release()); note(w->d_push_force.release()); note(w->d_push_withdraw.release());
  note(w->d_push_x0.release());
  note(w->d_tower_count.release()); note(w->d_tower_res.release()); note(w->d_pack_error.release());
  note(w->d_err_flag.release()); note(w->d_tower_frozen.release());
  note(w->d_ep_state.release()); note(w->d_ep_x0.release());
  note(w->d_out_ab.release()); note(w->d_out_meta.release()); note(w->d_out_geo.release());
  note(w->d_out_pts.release()); note(w->d_out_count.release()); note(w->d_out_tower.release());
  note(w->d_prev_key.release()); note(w->d_prev_data.release()); note(w->d_prev_count.release());
  note(w->d_phase_cycles.release());
  note(w->d_mlp_params.release()); note(w->d_mlp_packed.release()); note(w->d_feat.release());
  note(w->d_tower_fallback.release());
  for (auto& m : w->megas) note(m.release());
  for (hipStream_t s : w->aux) note(hipStreamDestroy(s));
  for (hipEvent_t e : w->aux_done) note(hipEventDestroy(e));
  if (w->fork) note(hipEventDestroy(w->fork));
  delete w;
  if (first != hipSuccess) return fail(JG_EDEVICE, std::string("releasing the world: ") + hipGetErrorString(first));
  return JG_OK;
}

int32_t jg_add_boxes(jg_world* w, int32_t tower, int32_t n, const double* half_extents, const double* mass,
                     const double* pos, const double* quat, const double* linvel, const double* angvel,
                     int32_t* body_ids_out) {
  if (int32_t r = check_world(w)) return r;
  if (n < 0) return fail(JG_EINVAL, "negative body count");
  if (tower < 0 || tower >= w->max_towers) return fail(JG_EINVAL, "tower index out of range");
  if (tower > (int)w->tower_bodies.size()) return fail(JG_EINVAL, "towers must be numbered densely by first use");
  if (n == 0) return JG_OK;
  if (!half_extents || !mass || !pos || !quat) return fail(JG_EINVAL, "null geometry array");
  const int N = (int)w->mass.size();
  if (N + n > w->max_bodies) return fail(JG_ECAPACITY, "max_bodies exceeded");
  for (int i = 0; i < n; ++i) {
    for (int k = 0; k < 3; ++k)
      if (!(half_extents[3 * i + k] > 0.0)) return fail(JG_EINVAL, "half extents must be positive");
    if (!(mass[i] >= 0.0)) return fail(JG_EINVAL, "mass must be >= 0");
    double qq = 0.0;
    for (int k = 0; k < 4; ++k) qq += quat[4 * i + k] * quat[4 * i + k];
    if (!(qq > 0.0) || !std::isfinite(qq)) return fail(JG_EINVAL, "quaternion must be non-zero and finite");
  }
  if (int32_t r = download_state(w)) return r;
  if (tower == (int)w->tower_bodies.size()) {
    w->tower_bodies.emplace_back();
    w->mu.push_back(0.4);
    w->st_cand.push_back(0); w->st_man.push_back(0); w->st_pts.push_back(0); w->st_ci.push_back(0);
    w->st_fb.push_back(0);
    w->st_col.push_back(0); w->st_err.push_back(0); w->st_rms.push_back(0.0); w->st_max.push_back(0.0);
  }
  for (int i = 0; i < n; ++i) {
    const int id = N + i;
    for (int k = 0; k < 3; ++k) {
      w->he.push_back(half_extents[3 * i + k]);
      w->x.push_back(pos[3 * i + k]);
      w->v.push_back(linvel ? linvel[3 * i + k] : 0.0);
      w->w.push_back(angvel ? angvel[3 * i + k] : 0.0);
    }
    double qq = 0.0;
    for (int k = 0; k < 4; ++k) qq += quat[4 * i + k] * quat[4 * i + k];
    const double il = 1.0 / std::sqrt(qq);
    for (int k = 0; k < 4; ++k) w->q.push_back(quat[4 * i + k] * il);
    w->mass.push_back(mass[i]);
    w->active.push_back(1);
    w->body_tower.push_back(tower);
    w->tower_bodies[tower].push_back(id);
    if (body_ids_out) body_ids_out[i] = id;
  }
  w->layout_dirty = true;
  w->host_dirty = true;
  return JG_OK;
}

int32_t jg_set_friction(jg_world* w, int32_t tower, double mu) {
  if (int32_t r = check_world(w)) return r;
  if (!(mu >= 0.0) || !std::isfinite(mu)) return fail(JG_EINVAL, "friction must be finite and >= 0");
  if (tower < -1 || tower >= (int)w->tower_bodies.size()) return fail(JG_EINVAL, "tower index out of range");
  if (int32_t r = download_state(w)) return r;
  if (tower == -1) std::fill(w->mu.begin(), w->mu.end(), mu);
  else w->mu[tower] = mu;
  w->host_dirty = true;
  return JG_OK;
}

int32_t jg_set_push(jg_world* w, int32_t body, const double force[3], int32_t start_step, int32_t n_steps,
                    double withdraw, int32_t move) {
  if (int32_t r = check_world(w)) return r;
  if (body < 0 || body >= (int)w->mass.size()) return fail(JG_EINVAL, "body index out of range");
  if (!force || n_steps < 0 || !(withdraw >= 0.0)) return fail(JG_EINVAL, "bad push arguments");
  if (move < JG_MOVE_NONE || move > JG_MOVE_SIDE_X) return fail(JG_EINVAL, "unknown move type");
  if (int32_t r = download_state(w)) return r;
  PushRow pr;
  pr.body = body;
  for (int k = 0; k < 3; ++k) { pr.force[k] = force[k]; pr.x0[k] = w->x[3 * body + k]; }
  pr.start = start_step;
  pr.steps = n_steps;
  pr.withdraw = withdraw;
  pr.move = move;
  w->pushes.push_back(pr);
  w->layout_dirty = true;
  w->host_dirty = true;
  return JG_OK;
}

int32_t jg_set_active(jg_world* w, int32_t body, int32_t active) {
  if (int32_t r = check_world(w)) return r;
  if (body < 0 || body >= (int)w->mass.size()) return fail(JG_EINVAL, "body index out of range");
  if (int32_t r = download_state(w)) return r;
  w->active[body] = active ? 1 : 0;
  if (!active) for (int k = 0; k < 3; ++k) { w->v[3 * body + k] = 0.0; w->w[3 * body + k] = 0.0; }
  w->host_dirty = true;
  return JG_OK;
}

int32_t jg_commit(jg_world* w) {
  if (int32_t r = check_world(w)) return r;
  if (int32_t r = set_device(w)) return r;
  if (w->layout_dirty || w->host_dirty) {
    if (int32_t r = download_state(w)) return r;
    if (int32_t r = collect_stats(w)) return r;
    if (w->layout_dirty)
      if (int32_t r = build_layout(w)) return r;
    if (int32_t r = upload_all(w)) return r;
  }
  if (w->clear_warm) {
    if (w->n_packs > 0) HIP_TRY(hipMemset(w->d_prev_count.p, 0, sizeof(int32_t) * w->n_packs));
    w->clear_warm = false;
  }
  // one auxiliary stream (and its join event) per launch class after the first
  const size_t nc = w->classes.size();
  while (w->aux.size() + 1 < nc) {
    hipStream_t st;
    hipEvent_t ev;
    HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    w->aux.push_back(st);
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    w->aux_done.push_back(ev);
  }
  if (nc > 1 && !w->fork) HIP_TRY(hipEventCreateWithFlags(&w->fork, hipEventDisableTiming));
  // the copies and fills above ran on the null stream and the world's: both are done before
  // the first launch
  HIP_TRY(hipStreamSynchronize(nullptr));
  HIP_TRY(hipStreamSynchronize(w->stream));
  return JG_OK;
}

int32_t jg_step_batch(jg_world* w, int32_t n_steps) {
  if (int32_t r = check_world(w)) return r;
  if (n_steps < 0) return fail(JG_EINVAL, "negative step count");
  if (w->layout_dirty || w->host_dirty || w->clear_warm)
    return fail(JG_ESTATE, "host-side changes are not on the device yet: call jg_commit first");
  if (int32_t r = set_device(w)) return r;
  if (n_steps == 0) return JG_OK;
  if (w->prm.warm_start == 2 && !w->mlp_set) return fail(JG_ESTATE, "warm_start 2 needs jg_set_mlp first");
  if (w->n_packs == 0 && w->megas.empty()) { w->step += n_steps; return JG_OK; }
  jg::StepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.x = w->d_x.p; a.q = w->d_q.p; a.v = w->d_v.p; a.w = w->d_w.p;
  a.he = w->d_he.p; a.mass = w->d_mass.p; a.flags = w->d_flags.p;
  a.body_tower = w->d_body_tower.p; a.cap = w->max_bodies;
  a.pack_body0 = w->d_pack_body0.p; a.pack_tower0 = w->d_pack_tower0.p; a.pack_push0 = w->d_pack_push0.p;
  a.pack_slot0 = w->d_pack_slot0.p;
  a.tower_body0 = w->d_tower_body0.p; a.tower_mu = w->d_tower_mu.p;
  a.push_body = w->d_push_body.p; a.push_start = w->d_push_start.p; a.push_steps = w->d_push_steps.p;
  a.push_force = w->d_push_force.p; a.push_withdraw = w->d_push_withdraw.p; a.push_x0 = w->d_push_x0.p;
  a.tower_count = w->d_tower_count.p; a.tower_res = w->d_tower_res.p; a.pack_error = w->d_pack_error.p;
  a.err_flag = w->d_err_flag.p; a.tower_frozen = w->d_tower_frozen.p;
  a.ep_state = w->ep_on ? w->d_ep_state.p : nullptr;
  a.ep_x0 = w->d_ep_x0.p;
  a.ep_fd = (float)w->prm.collapse_fd;
  a.ep_ek_collapse = (float)w->prm.collapse_ek;
  a.ep_cos_theta = (float)std::cos(w->prm.collapse_theta * 3.14159265358979323846 / 180.0);
  a.ep_ek_rest = (float)w->prm.rest_ek;
  a.ep_eps = (float)w->prm.support_eps;
  a.ep_rest_steps = w->prm.rest_steps;
  a.out_ab = w->d_out_ab.p; a.out_meta = w->d_out_meta.p; a.out_geo = w->d_out_geo.p; a.out_pts = w->d_out_pts.p;
  a.out_count = w->d_out_count.p; a.out_tower = w->d_out_tower.p;
  a.prev_key = w->d_prev_key.p; a.prev_data = w->d_prev_data.p; a.prev_count = w->d_prev_count.p;
  a.phase_cycles = w->d_phase_cycles.p;
  for (int k = 0; k < 3; ++k) a.g[k] = (float)w->prm.gravity[k];
  a.dt = (float)(w->prm.dt / w->prm.n_sub);
  a.restitution = (float)w->prm.restitution;
  a.beta = (float)w->prm.beta;
  a.slop = (float)w->prm.slop;
  a.margin = (float)w->prm.margin;
  a.iters = w->prm.iters;
  a.n_sub = w->prm.n_sub;
  a.friction_cone = w->prm.friction_cone;
  a.restitution_bias = w->prm.restitution_bias;
  a.manifold_mode = w->prm.manifold_mode;
  a.n_steps = n_steps;
  a.warm_start = w->prm.warm_start;
  a.step0 = w->step;
  a.mlp = w->mlp_set ? (const void*)w->d_mlp_packed.p : nullptr;
  a.feat_out = w->prm.record_features ? w->d_feat.p : nullptr;
  a.tower_fallback = w->d_tower_fallback.p;
  a.mlp_iters = w->prm.mlp_iters;
  a.fallback_tau = (float)std::min(w->prm.fallback_tau, 3.0e38);
  const size_t nc = w->classes.size();
  std::vector<jg::StepArgs> cls(nc, a);
  for (size_t k = 0; k < nc; ++k) {
    const auto& c = w->classes[k];
    cls[k].pack_first = c.first;
    cls[k].n_packs = c.count;
    cls[k].nbp = c.nbp; cls[k].pc = c.pc; cls[k].tpc = c.tpc; cls[k].ppc = c.ppc;
    cls[k].gmem = w->d_gmem.p;
    cls[k].in_gmem = c.global ? 1 : 0;
    cls[k].hot_bodies = c.hot_bodies ? 1 : 0;
    cls[k].lat = c.lat ? 1 : 0;
    cls[k].pack_goff = w->d_pack_goff.p;
  }
  if (w->prm.use_graph) {
    if (int32_t r = launch_graph(w, cls, n_steps)) return r;
  } else {
    // Classes are independent (disjoint packs, towers and bodies): run them side by side, so a
    // small batch fills the GPU and one class's tail overlaps the others.
    if (nc > 1) HIP_TRY(hipEventRecord(w->fork, w->stream));
    for (size_t k = 0; k < nc; ++k) {
      hipStream_t s = k == 0 ? w->stream : w->aux[k - 1];
      if (k > 0) HIP_TRY(hipStreamWaitEvent(s, w->fork, 0));
      if (int e = jg::launch_step(cls[k], w->classes[k].lds, s))
        return fail(JG_EDEVICE, std::string("step kernel launch: ") + hipGetErrorString((hipError_t)e));
      if (k > 0) HIP_TRY(hipEventRecord(w->aux_done[k - 1], s));
    }
    for (size_t k = 1; k < nc; ++k) HIP_TRY(hipStreamWaitEvent(w->stream, w->aux_done[k - 1], 0));
  }
  // towers stepped by the whole GPU, one cooperative launch each (after the packs on the stream)
  for (auto& m : w->megas) {
    jg::MegaArgs g;
    std::memset(&g, 0, sizeof(g));
    g.x = w->d_x.p; g.q = w->d_q.p; g.v = w->d_v.p; g.w = w->d_w.p;
    g.he = w->d_he.p; g.mass = w->d_mass.p; g.flags = w->d_flags.p;
    g.cap = w->max_bodies; g.g0 = m.g0; g.nb = m.nb; g.tslot = m.tslot;
    g.mu = (float)w->mu[m.tower];
    g.push_body = w->d_push_body.p; g.push_start = w->d_push_start.p; g.push_steps = w->d_push_steps.p;
    g.push_force = w->d_push_force.p; g.push_withdraw = w->d_push_withdraw.p; g.push_x0 = w->d_push_x0.p;
    g.p0 = m.p0; g.np = m.np;
    g.tower_count = w->d_tower_count.p; g.tower_res = w->d_tower_res.p; g.tower_frozen = w->d_tower_frozen.p;
    g.err_flag = w->d_err_flag.p; g.island_err = m.err.p;
    for (int k = 0; k < 3; ++k) g.g[k] = a.g[k];
    g.dt = a.dt; g.restitution = a.restitution; g.beta = a.beta; g.slop = a.slop; g.margin = a.margin;
    g.iters = a.iters; g.n_sub = a.n_sub; g.n_steps = n_steps;
    g.friction_cone = a.friction_cone; g.restitution_bias = a.restitution_bias; g.manifold_mode = a.manifold_mode;
    g.partition = w->prm.colour_partition;
    g.step0 = w->step;
    g.body = m.body.p; g.ubody = m.ubody.p; g.cells = m.cells.p; g.ncell_cap = m.ncell_cap;
    g.cand = m.cand.p; g.cand_cap = m.cand_cap; g.man = m.man.p; g.md = m.md.p;
    g.mtb = m.md.p + (size_t)jg::kManDevWords * m.cand_cap;
    g.part = m.part.p; g.nparts = m.nparts; g.red = m.red.p; g.ired = m.ired.p; g.scal = m.scal.p;
    g.out_a = m.out_a.p; g.out_b = m.out_b.p; g.out_meta = m.out_meta.p; g.out_geo = m.out_geo.p;
    g.out_pts = m.out_pts.p; g.out_count = m.out_count.p;
    if (int e = jg::launch_mega(g, m.grid, w->stream))
      return fail(JG_EDEVICE, std::string("grid-wide island launch: ") + hipGetErrorString((hipError_t)e));
  }
  w->step += n_steps;
  w->device_newer = true;
  w->stats_pending = true;
  w->last_launch_steps = n_steps;
  return JG_OK;
}

int32_t jg_query_state(jg_world* w, int32_t first_body, int32_t n, double* pos, double* quat, double* linvel,
                       double* angvel) {
  if (int32_t r = check_world(w)) return r;
  if (first_body < 0 || n < 0 || first_body + n > (int)w->mass.size()) return fail(JG_EINVAL, "body range out of range");
  if (int32_t r = set_device(w)) return r;
  if (int32_t r = download_state(w)) return r;
  for (int i = 0; i < n; ++i) {
    const int id = first_body + i;
    for (int k = 0; k < 3; ++k) {
      if (pos) pos[3 * i + k] = w->x[3 * id + k];
      if (linvel) linvel[3 * i + k] = w->v[3 * id + k];
      if (angvel) angvel[3 * i + k] = w->w[3 * id + k];
    }
    if (quat) for (int k = 0; k < 4; ++k) quat[4 * i + k] = w->q[4 * id + k];
  }
  return report_device_errors(w);
}

int32_t jg_set_state(jg_world* w, int32_t first_body, int32_t n, const double* pos, const double* quat,
                     const double* linvel, const double* angvel) {
  if (int32_t r = check_world(w)) return r;
  if (first_body < 0 || n < 0 || first_body + n > (int)w->mass.size()) return fail(JG_EINVAL, "body range out of range");
  if (int32_t r = set_device(w)) return r;
  if (int32_t r = download_state(w)) return r;
  for (int i = 0; i < n; ++i) {
    const int id = first_body + i;
    for (int k = 0; k < 3; ++k) {
      if (pos) w->x[3 * id + k] = pos[3 * i + k];
      if (linvel) w->v[3 * id + k] = linvel[3 * i + k];
      if (angvel) w->w[3 * id + k] = angvel[3 * i + k];
    }
    if (quat) {
      double qq = 0.0;
      for (int k = 0; k < 4; ++k) qq += quat[4 * i + k] * quat[4 * i + k];
      if (!(qq > 0.0)) return fail(JG_EINVAL, "zero quaternion");
      const double il = 1.0 / std::sqrt(qq);
      for (int k = 0; k < 4; ++k) w->q[4 * id + k] = quat[4 * i + k] * il;
    }
  }
  w->host_dirty = true;
  w->clear_warm = true;
  return JG_OK;
}

int32_t jg_query_active(jg_world* w, int32_t first_body, int32_t n, uint8_t* active) {
  if (int32_t r = check_world(w)) return r;
  if (!active || first_body < 0 || n < 0 || first_body + n > (int)w->mass.size())
    return fail(JG_EINVAL, "bad body range or null output");
  if (int32_t r = set_device(w)) return r;
  if (int32_t r = download_state(w)) return r;
  for (int i = 0; i < n; ++i) active[i] = w->active[first_body + i];
  return report_device_errors(w);
}

int32_t jg_query_contacts(jg_world* w, int32_t tower, jg_contact* out, int32_t capacity, int32_t* n_out) {
  if (int32_t r = check_world(w)) return r;
  if (!n_out || capacity < 0 || (capacity > 0 && !out)) return fail(JG_EINVAL, "bad output buffer");
  if (tower < 0 || tower >= (int)w->tower_bodies.size()) return fail(JG_EINVAL, "tower index out of range");
  *n_out = 0;
  if (w->layout_dirty || (w->n_packs == 0 && w->megas.empty())) return JG_OK;
  if (int32_t r = set_device(w)) return r;
  HIP_TRY(hipStreamSynchronize(w->stream));
  if (w->mega_of_tower[tower] >= 0) {
    // a tower stepped by the whole GPU: its pairs in canonical order, 32-bit indices
    const auto& m = w->megas[w->mega_of_tower[tower]];
    int32_t cnt = 0;
    HIP_TRY(hipMemcpy(&cnt, m.out_count.p, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (cnt <= 0) return report_device_errors(w);
    std::vector<int32_t> ia(cnt), ib(cnt);
    std::vector<uint32_t> meta(cnt);
    std::vector<float> geo(8 * (size_t)cnt), pts(24 * (size_t)cnt);
    HIP_TRY(hipMemcpy(ia.data(), m.out_a.p, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ib.data(), m.out_b.p, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(meta.data(), m.out_meta.p, sizeof(uint32_t) * cnt, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(geo.data(), m.out_geo.p, sizeof(float) * 8 * cnt, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(pts.data(), m.out_pts.p, sizeof(float) * 24 * cnt, hipMemcpyDeviceToHost));
    int total = 0, order = 0;
    for (int k = 0; k < cnt; ++k) {
      const int npts = (int)(meta[k] & 15u);
      if (npts == 0) continue;
      for (int q = 0; q < npts; ++q) {
        if (total < capacity) {
          jg_contact& c = out[total];
          c.tower = tower;
          c.body_a = w->body_of_int[m.g0 + ia[k]];
          c.body_b = ib[k] < 0 ? -1 : w->body_of_int[m.g0 + ib[k]];
          c.slot = (int)((meta[k] >> (12 + 4 * q)) & 15u);
          c.colour = (int)((meta[k] >> 4) & 255u);
          c.order = order;
          for (int j = 0; j < 3; ++j) {
            c.point[j] = pts[24 * (size_t)k + 6 * q + j];
            c.normal[j] = geo[8 * (size_t)k + j];
            c.t1[j] = geo[8 * (size_t)k + 3 + j];
          }
          c.depth = geo[8 * (size_t)k + 6];
          c.lambda_n = pts[24 * (size_t)k + 6 * q + 3];
          c.lambda_t1 = pts[24 * (size_t)k + 6 * q + 4];
          c.lambda_t2 = pts[24 * (size_t)k + 6 * q + 5];
        }
        ++total;
      }
      ++order;
    }
    *n_out = total;
    return report_device_errors(w);
  }
  const int pk = w->pack_of_tower[tower];
  if (pk < 0) return JG_OK;
  int32_t cnt = 0;
  HIP_TRY(hipMemcpy(&cnt, w->d_out_count.p + pk, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (cnt <= 0) return JG_OK;
  const size_t base = (size_t)w->pack_slot0[pk];
  std::vector<uint32_t> ab(cnt), meta(cnt);
  std::vector<int32_t> tw(cnt);
  std::vector<float> geo(8 * (size_t)cnt), pts(24 * (size_t)cnt);
  HIP_TRY(hipMemcpy(ab.data(), w->d_out_ab.p + base, sizeof(uint32_t) * cnt, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(meta.data(), w->d_out_meta.p + base, sizeof(uint32_t) * cnt, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(tw.data(), w->d_out_tower.p + base, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(geo.data(), w->d_out_geo.p + 8 * base, sizeof(float) * 8 * cnt, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(pts.data(), w->d_out_pts.p + 24 * base, sizeof(float) * 24 * cnt, hipMemcpyDeviceToHost));
  const int local = w->tower_slot[tower] - w->pack_tower0[pk];
  const int b0 = w->pack_body0[pk];
  int total = 0, order = 0;
  for (int m = 0; m < cnt; ++m) {
    if (tw[m] != local) continue;
    const int a = (int)(ab[m] >> 16), b = (int)(ab[m] & 0xffffu);
    const int npts = (int)(meta[m] & 15u);
    const int colour = (int)((meta[m] >> 4) & 255u);
    for (int q = 0; q < npts; ++q) {
      if (total < capacity) {
        jg_contact& c = out[total];
        c.tower = tower;
        c.body_a = w->body_of_int[b0 + a];
        c.body_b = (b == 0xffff) ? -1 : w->body_of_int[b0 + b];
        c.slot = (int)((meta[m] >> (12 + 4 * q)) & 15u);
        c.colour = colour;
        c.order = order;
        for (int k = 0; k < 3; ++k) {
          c.point[k] = pts[24 * (size_t)m + 6 * q + k];
          c.normal[k] = geo[8 * (size_t)m + k];
          c.t1[k] = geo[8 * (size_t)m + 3 + k];
        }
        c.depth = geo[8 * (size_t)m + 6];
        c.lambda_n = pts[24 * (size_t)m + 6 * q + 3];
        c.lambda_t1 = pts[24 * (size_t)m + 6 * q + 4];
        c.lambda_t2 = pts[24 * (size_t)m + 6 * q + 5];
      }
      ++total;
    }
    ++order;
  }
  *n_out = total;
  return report_device_errors(w);
}

int32_t jg_query_stats(jg_world* w, int32_t tower, jg_stats* out) {
  if (int32_t r = check_world(w)) return r;
  if (!out) return fail(JG_EINVAL, "null output");
  if (tower < -1 || tower >= (int)w->tower_bodies.size()) return fail(JG_EINVAL, "tower index out of range");
  if (int32_t r = set_device(w)) return r;
  if (int32_t r = collect_stats(w)) return r;
  std::memset(out, 0, sizeof(*out));
  out->steps = w->step;
  auto add = [&](int t) {
    out->candidates += w->st_cand[t];
    out->manifolds += w->st_man[t];
    out->points += w->st_pts[t];
    out->contact_iters += w->st_ci[t];
    out->colours = std::max(out->colours, w->st_col[t]);
    out->error_word |= w->st_err[t];
    out->residual_rms = std::max(out->residual_rms, w->st_rms[t]);
    out->residual_max = std::max(out->residual_max, w->st_max[t]);
    out->fallbacks += w->st_fb[t];
  };
  if (tower >= 0) add(tower);
  else for (int t = 0; t < (int)w->tower_bodies.size(); ++t) add(t);
  return report_device_errors(w);
}

int32_t jg_query_features(jg_world* w, int32_t tower, float* out, int32_t capacity, int32_t* n_out) {
  if (int32_t r = check_world(w)) return r;
  if (!n_out || capacity < 0 || (capacity > 0 && !out)) return fail(JG_EINVAL, "bad output buffer");
  if (tower < -1 || tower >= (int)w->tower_bodies.size()) return fail(JG_EINVAL, "tower index out of range");
  if (!w->prm.record_features) return fail(JG_ESTATE, "the world was created without record_features");
  *n_out = 0;
  if (w->layout_dirty || w->n_packs == 0) return JG_OK;
  if (int32_t r = set_device(w)) return r;
  HIP_TRY(hipStreamSynchronize(w->stream));
  const int p0 = tower >= 0 ? w->pack_of_tower[tower] : 0;
  const int p1 = tower >= 0 ? p0 + 1 : w->n_packs;
  if (p0 < 0) return JG_OK;
  std::vector<int32_t> cnt(p1 - p0);
  HIP_TRY(hipMemcpy(cnt.data(), w->d_out_count.p + p0, sizeof(int32_t) * (p1 - p0), hipMemcpyDeviceToHost));
  const size_t s0 = (size_t)w->pack_slot0[p0], s1 = (size_t)w->pack_slot0[p1];
  std::vector<uint32_t> meta(s1 - s0);
  std::vector<int32_t> tw(s1 - s0);
  std::vector<float> rec((s1 - s0) * 4 * jg::kFeatRecord);
  HIP_TRY(hipMemcpy(meta.data(), w->d_out_meta.p + s0, sizeof(uint32_t) * (s1 - s0), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(tw.data(), w->d_out_tower.p + s0, sizeof(int32_t) * (s1 - s0), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(rec.data(), w->d_feat.p + s0 * 4 * jg::kFeatRecord, sizeof(float) * rec.size(),
                    hipMemcpyDeviceToHost));
  const int local = tower >= 0 ? w->tower_slot[tower] - w->pack_tower0[p0] : -1;
  int total = 0;
  for (int pk = p0; pk < p1; ++pk) {
    const size_t base = (size_t)w->pack_slot0[pk] - s0;
    for (int m = 0; m < cnt[pk - p0]; ++m) {
      if (tower >= 0 && tw[base + m] != local) continue;
      const int npts = (int)(meta[base + m] & 15u);
      for (int q = 0; q < npts; ++q) {
        if (total < capacity)
          std::memcpy(out + (size_t)total * jg::kFeatRecord, &rec[((base + m) * 4 + q) * jg::kFeatRecord],
                      sizeof(float) * jg::kFeatRecord);
        ++total;
      }
    }
  }
  *n_out = total;
  return report_device_errors(w);
}

int32_t jg_set_mlp(jg_world* w, const float* params) {
  if (int32_t r = check_world(w)) return r;
  if (!params) return fail(JG_EINVAL, "null parameters");
  if (int32_t r = set_device(w)) return r;
  size_t bytes = 0;
  if (int32_t r = jg_mlp_packed_bytes(&bytes)) return r;
  HIP_TRY(w->d_mlp_params.ensure(JG_MLP_PARAMS));
  HIP_TRY(w->d_mlp_packed.ensure(bytes));
  HIP_TRY(hipMemcpyAsync(w->d_mlp_params.p, params, sizeof(float) * JG_MLP_PARAMS, hipMemcpyHostToDevice, w->stream));
  if (int32_t r = jg_mlp_pack(w->d_mlp_params.p, w->d_mlp_packed.p, w->stream)) return r;
  HIP_TRY(hipStreamSynchronize(w->stream));
  w->mlp_set = true;
  return JG_OK;
}

int32_t jg_world_size(jg_world* w, int32_t* n_towers, int32_t* n_bodies) {
  if (int32_t r = check_world(w)) return r;
  if (n_towers) *n_towers = (int32_t)w->tower_bodies.size();
  if (n_bodies) *n_bodies = (int32_t)w->mass.size();
  return JG_OK;
}

int32_t jg_query_phase_cycles(jg_world* w, uint64_t* cycles, int32_t n) {
  if (int32_t r = check_world(w)) return r;
  if (!cycles || n < 0) return fail(JG_EINVAL, "bad output buffer");
  if (int32_t r = set_device(w)) return r;
  HIP_TRY(hipStreamSynchronize(w->stream));
  unsigned long long c[jg::kPhases];
  HIP_TRY(hipMemcpy(c, w->d_phase_cycles.p, sizeof(c), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(w->d_phase_cycles.p, 0, sizeof(c)));
  for (int k = 0; k < n; ++k) cycles[k] = k < jg::kPhases ? (uint64_t)c[k] : 0u;
  return report_device_errors(w);
}

int32_t jg_sync(jg_world* w) {
  if (int32_t r = check_world(w)) return r;
  if (int32_t r = set_device(w)) return r;
  HIP_TRY(hipStreamSynchronize(w->stream));
  return report_device_errors(w);
}

int32_t jg_device_views(jg_world* w, void** x, void** q, void** v, void** angvel, int32_t* stride) {
  if (int32_t r = check_world(w)) return r;
  if (w->layout_dirty || w->host_dirty || w->clear_warm)
    return fail(JG_ESTATE, "host-side changes are not on the device yet: call jg_commit first");
  if (x) *x = w->d_x.p;
  if (q) *q = w->d_q.p;
  if (v) *v = w->d_v.p;
  if (angvel) *angvel = w->d_w.p;
  if (stride) *stride = w->max_bodies;
  w->views_out = true;
  return JG_OK;
}

int32_t jg_begin_episodes(jg_world* w) {
  if (int32_t r = check_world(w)) return r;
  if (w->layout_dirty || w->host_dirty || w->clear_warm)
    return fail(JG_ESTATE, "host-side changes are not on the device yet: call jg_commit first");
  if (int32_t r = set_device(w)) return r;
  const size_t nt = std::max<size_t>(1, w->tower_order.size());
  HIP_TRY(w->d_ep_state.ensure(nt * jg::kEpisodeWords));
  HIP_TRY(w->d_ep_x0.ensure((size_t)3 * w->max_bodies));
  std::vector<uint32_t> init(nt * jg::kEpisodeWords, 0u);
  const float qnan = std::numeric_limits<float>::quiet_NaN();
  uint32_t nan_bits;
  std::memcpy(&nan_bits, &qnan, sizeof(nan_bits));
  for (size_t t = 0; t < nt; ++t) {
    init[t * jg::kEpisodeWords + jg::kEpCollapseStep] = (uint32_t)-1;
    init[t * jg::kEpisodeWords + jg::kEpRestStep] = (uint32_t)-1;
    init[t * jg::kEpisodeWords + jg::kEpImbalance] = nan_bits;
  }
  HIP_TRY(hipMemcpyAsync(w->d_ep_x0.p, w->d_x.p, sizeof(float) * 3 * w->max_bodies, hipMemcpyDeviceToDevice,
                         w->stream));
  HIP_TRY(hipMemcpyAsync(w->d_ep_state.p, init.data(), sizeof(uint32_t) * init.size(), hipMemcpyHostToDevice,
                         w->stream));
  HIP_TRY(hipStreamSynchronize(w->stream));
  w->ep_on = true;
  return JG_OK;
}

int32_t jg_query_episode(jg_world* w, int32_t tower, jg_episode* out) {
  if (int32_t r = check_world(w)) return r;
  if (!out) return fail(JG_EINVAL, "null output");
  if (tower < 0 || tower >= (int)w->tower_bodies.size()) return fail(JG_EINVAL, "tower index out of range");
  if (!w->ep_on) return fail(JG_ESTATE, "no episodes: call jg_begin_episodes first");
  if (int32_t r = set_device(w)) return r;
  if (int32_t r = download_state(w)) return r;   // the active flags of withdrawn blocks
  uint32_t st[jg::kEpisodeWords];
  HIP_TRY(hipMemcpy(st, w->d_ep_state.p + (size_t)w->tower_slot[tower] * jg::kEpisodeWords, sizeof(st),
                    hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof(*out));
  auto f = [&](int k) { float v; std::memcpy(&v, &st[k], sizeof(v)); return v; };
  out->collapsed = (st[jg::kEpFlags] & jg::kEpCollapsed) ? 1 : 0;
  out->done = (st[jg::kEpFlags] & jg::kEpDone) ? 1 : 0;
  out->collapse_step = (int32_t)st[jg::kEpCollapseStep];
  out->rest_step = (int32_t)st[jg::kEpRestStep];
  out->support_vertices = (int32_t)st[jg::kEpSupport];
  out->ek = f(jg::kEpEk);
  out->dx_max = f(jg::kEpDx);
  out->theta_max = f(jg::kEpTheta);
  out->margin = f(jg::kEpMargin);
  out->imbalance = f(jg::kEpImbalance);
  out->com[0] = f(jg::kEpComX);
  out->com[1] = f(jg::kEpComY);
  // the moves started by the collapse step (or by the last step taken)
  const int64_t last = out->collapsed ? (int64_t)out->collapse_step : w->step - 1;
  for (const PushRow& pr : w->pushes) {
    if (pr.move == JG_MOVE_NONE || w->body_tower[pr.body] != tower || (int64_t)pr.start > last) continue;
    ++out->rounds;
    if (pr.move == JG_MOVE_SIDE_X) ++out->torque_moves;
    if (!w->active[pr.body]) ++out->removed;
  }
  return report_device_errors(w);
}

int32_t jg_body_slots(jg_world* w, int32_t first_body, int32_t n, int32_t* slots) {
  if (int32_t r = check_world(w)) return r;
  if (!slots || first_body < 0 || n < 0 || first_body + n > (int)w->mass.size())
    return fail(JG_EINVAL, "bad body range or null output");
  if (w->layout_dirty) return fail(JG_ESTATE, "the layout changed since the last jg_commit");
  for (int i = 0; i < n; ++i) slots[i] = w->int_of_body[first_body + i];
  return JG_OK;
}

}  // extern "C"
