// C ABI of libfock.so (declared in include/fock.h).
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <new>
#include <string>

#include "fock_internal.hpp"

namespace fock {

namespace {
thread_local std::string g_last_error;
}

fock_status set_error(fock_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

void clear_error() { g_last_error.clear(); }

fock_status validate_desc(const fock_desc& d, int idx);
fock_status build_plan(const fock_desc* descs, int n_inst, fock_precision prec, void* stream, const fock_tuning* tune,
                       Plan** out);
hipError_t launch_zero_outputs(const Plan& p, int inst, void* out);

hipEvent_t Profiler::next(hipStream_t s) {
  if (used == pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    pool.push_back(e);
  }
  hipEvent_t e = pool[used++];
  if (hipEventRecord(e, s) != hipSuccess) (void)hipGetLastError();
  return e;
}

void Profiler::begin(int kind, hipStream_t s) {
  if (!on) return;
  const size_t a = used;
  if (next(s)) spans[kind].push_back({a, a});
}

void Profiler::end(int kind, hipStream_t s) {
  if (!on || spans[kind].empty()) return;
  const size_t b = used;
  if (next(s)) spans[kind].back().second = b;
}

void Profiler::release() {
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  pool.clear();
  used = 0;
  for (auto& v : spans) v.clear();
}

// ---- call records (FOCK_LOG) ----------------------------------------------
namespace {

hipEvent_t log_event(CallLog& L) {
  if (!L.pool.empty()) {
    hipEvent_t e = L.pool.back();
    L.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void log_open(Plan* p) {
  const char* path = std::getenv("FOCK_LOG");
  if (!path || !*path) return;
  CallLog& L = p->log;
  L.serial = p->serial;
  if (std::strcmp(path, "stderr") == 0) {
    L.f = stderr;
  } else {
    L.f = std::fopen(path, "a");
    L.own = L.f != nullptr;
  }
}

// Write the pending records (waiting for their events) and recycle the events.
void log_flush(const Plan* p, CallLog& L) {
  for (CallLog::Rec& r : L.pending) {
    double ms = -1.0;
    if (r.e0 && r.e1) {
      float t = 0.0f;
      if (hipEventSynchronize(r.e1) == hipSuccess && hipEventElapsedTime(&t, r.e0, r.e1) == hipSuccess) ms = t;
      (void)hipGetLastError();
    }
    std::fprintf(L.f,
                 "{\"plan\": %llu, \"call\": \"%s\", \"status\": %d, \"graph\": %d, \"enqueue_us\": %.1f, "
                 "\"device_ms\": %.4f, \"instances\": %zu, \"ordered_pairs\": %lld, \"apply_fft_pairs\": %lld, "
                 "\"apply_launches\": %lld}\n",
                 static_cast<unsigned long long>(L.serial), r.call, r.status, r.graph ? 1 : 0, r.enqueue_us, ms,
                 p->inst.size(), static_cast<long long>(p->ordered_pairs), static_cast<long long>(p->apply_fft_pairs),
                 static_cast<long long>(p->apply_launches));
    CallLog::Total* tot = nullptr;
    for (auto& kv : L.totals)
      if (kv.first == r.call) tot = &kv.second;
    if (!tot) {
      L.totals.emplace_back(r.call, CallLog::Total{});
      tot = &L.totals.back().second;
    }
    tot->calls += 1;
    if (ms > 0.0) tot->device_ms += ms;
    if (r.e0) L.pool.push_back(r.e0);
    if (r.e1) L.pool.push_back(r.e1);
  }
  L.pending.clear();
  std::fflush(L.f);
}

// Run one API call's body `f`, recorded when the plan logs.
template <typename F>
fock_status logged(Plan* p, const char* name, F&& f) {
  CallLog& L = p->log;
  if (!L.on()) return f();
  const auto t0 = std::chrono::steady_clock::now();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (p->uploaded && (e0 = log_event(L)) != nullptr && hipEventRecord(e0, p->stream) != hipSuccess) {
    (void)hipGetLastError();
    L.pool.push_back(e0);
    e0 = nullptr;
  }
  const fock_status st = f();
  if (e0 && (e1 = log_event(L)) != nullptr && hipEventRecord(e1, p->stream) != hipSuccess) {
    (void)hipGetLastError();
    L.pool.push_back(e1);
    e1 = nullptr;
  }
  const double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  L.pending.push_back(CallLog::Rec{name, static_cast<int>(st), us, p->use_graph, e0, e1});
  if (L.pending.size() >= 1024) log_flush(p, L);
  return st;
}

}  // namespace

Plan::~Plan() {
  if (log.on()) {
    log_flush(this, log);
    for (const auto& kv : log.totals)
      std::fprintf(log.f,
                   "{\"plan\": %llu, \"summary\": \"%s\", \"calls\": %lld, \"device_ms\": %.4f, "
                   "\"ordered_pairs_per_s\": %.1f}\n",
                   static_cast<unsigned long long>(log.serial), kv.first.c_str(),
                   static_cast<long long>(kv.second.calls), kv.second.device_ms,
                   kv.second.device_ms > 0.0 ? kv.second.calls * static_cast<double>(ordered_pairs) /
                                                   (kv.second.device_ms * 1e-3)
                                             : 0.0);
    std::fflush(log.f);
    for (hipEvent_t e : log.pool) (void)hipEventDestroy(e);
    if (log.own) std::fclose(log.f);
  }
  prof.release();
  release_graphs();
}

namespace {

fock_status device_ok() {
  int n = 0;
  const hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n < 1) {
    (void)hipGetLastError();
    return set_error(FOCK_ERR_DEVICE, "no usable GPU (hipGetDeviceCount)");
  }
  return FOCK_OK;
}

fock_status check_ready(const Plan* p) {
  if (!p) return set_error(FOCK_ERR_ARG, "plan is NULL");
  if (!p->uploaded || !p->ws) return set_error(FOCK_ERR_STATE, "no workspace attached (call fock_set_workspace)");
  return FOCK_OK;
}

fock_status check_ptrs(const Plan* p, const void* const* a, const char* what) {
  if (!a) return set_error(FOCK_ERR_ARG, std::string(what) + " array is NULL");
  for (size_t i = 0; i < p->inst.size(); ++i)
    if (!a[i]) return set_error(FOCK_ERR_ARG, std::string(what) + "[" + std::to_string(i) + "] is NULL");
  return FOCK_OK;
}

fock_status hip_fail(hipError_t e, const char* where) {
  (void)hipGetLastError();  // do not leave a sticky error for the caller's next HIP call
  return set_error(FOCK_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

bool has_empty_k(const Instance& in) {
  for (const auto& v : in.kpartners)
    if (v.empty()) return true;
  return false;
}

// apply and backward share the batch loop; they differ in the output factor.
// with_energy: the whole-pair kernels also write their energy partials.
fock_status run_apply(Plan* p, const void* const* psi, const double* const* occ, void* const* out,
                      const double* gscale, double hscale, bool backward, bool with_energy = false) {
  double* eblk = with_energy ? reinterpret_cast<double*>(p->ws + p->eblk_off) : nullptr;
  for (size_t i = 0; i < p->inst.size(); ++i) {
    if (has_empty_k(p->inst[i])) {
      const hipError_t e = launch_zero_outputs(*p, static_cast<int>(i), out[i]);
      if (e != hipSuccess) return hip_fail(e, "zero outputs");
    }
  }
  for (const FusedGroup& g : p->fused_groups) {
    const hipError_t e = launch_fused_apply(*p, g, psi[g.inst], occ[g.inst], out[g.inst],
                                            gscale ? gscale + g.inst : nullptr, hscale, backward,
                                            eblk ? eblk + g.eblk0 : nullptr);
    if (e != hipSuccess) return hip_fail(e, "whole-pair apply launch");
  }
  for (const FusedRounds& r : p->fused_rounds) {
    const hipError_t e = launch_fused_rounds(*p, r, psi[r.inst], occ[r.inst], out[r.inst],
                                             gscale ? gscale + r.inst : nullptr, hscale, backward,
                                             eblk ? eblk + r.eblk0 : nullptr);
    if (e != hipSuccess) return hip_fail(e, "whole-pair round launch");
  }
  for (const Batch& b : p->apply_batches) {
    const hipError_t e = launch_apply_batch(*p, b, psi[b.inst], occ[b.inst], out[b.inst], with_energy,
                                            gscale ? gscale + b.inst : nullptr, hscale, backward);
    if (e != hipSuccess) return hip_fail(e, "apply batch launch");
  }
  return FOCK_OK;
}

// band overlaps M of every instance with a non-null vmat entry (vmat may be null)
fock_status run_overlaps(Plan* p, const void* const* psi, void* const* vx_psi, void* const* vmat) {
  if (!vmat) return FOCK_OK;
  for (size_t i = 0; i < p->inst.size(); ++i) {
    if (!vmat[i]) continue;
    const hipError_t e = launch_overlap(*p, static_cast<int>(i), psi[i], vx_psi[i], vmat[i]);
    if (e != hipSuccess) return hip_fail(e, "overlap launch");
  }
  return FOCK_OK;
}

// E_x of every instance into ex[i].  after_apply: every instance takes its
// energy from the partials the apply just wrote (per block of the whole-pair
// kernel, or per apply batch of the three-pass paths).
fock_status run_energy(Plan* p, const void* const* psi, const double* const* occ, double* ex, bool after_apply) {
  for (const Batch& b : p->energy_batches) {
    const bool fused = p->inst[b.inst].fused;
    if (after_apply && (fused || batch_apply_energy(*p, b.inst))) continue;
    hipError_t e;
    if (fused) {
      e = launch_fused_energy(*p, b, psi[b.inst]);
      if (e == hipSuccess) e = launch_energy_reduce(*p, b, occ[b.inst], 1);
    } else {
      e = launch_energy_batch(*p, b, psi[b.inst], occ[b.inst]);
    }
    if (e != hipSuccess) return hip_fail(e, "energy batch launch");
  }
  for (size_t i = 0; i < p->inst.size(); ++i) {
    const int ii = static_cast<int>(i);
    const hipError_t e = !after_apply             ? launch_energy_finish(*p, ii, ex + i)
                         : p->inst[i].fused       ? launch_eblk_finish(*p, ii, ex + i)
                         : batch_apply_energy(*p, ii) ? launch_aslot_finish(*p, ii, ex + i)
                                                  : launch_energy_finish(*p, ii, ex + i);
    if (e != hipSuccess) return hip_fail(e, "energy finish launch");
  }
  return FOCK_OK;
}

// Argument checks of the apply-with-energy calls (after check_ready).
fock_status check_apply_energy_args(const Plan* p, const void* const* psi, const double* const* occ,
                                    void* const* vx_psi, const double* ex) {
  fock_status s;
  if ((s = check_ptrs(p, psi, "psi")) != FOCK_OK) return s;
  if ((s = check_ptrs(p, reinterpret_cast<const void* const*>(occ), "occ")) != FOCK_OK) return s;
  if ((s = check_ptrs(p, reinterpret_cast<const void* const*>(vx_psi), "vx_psi")) != FOCK_OK) return s;
  if (!ex) return set_error(FOCK_ERR_ARG, "ex is NULL");
  for (size_t i = 0; i < p->inst.size(); ++i)
    if (vx_psi[i] == psi[i]) return set_error(FOCK_ERR_ARG, "vx_psi aliases psi");
  return FOCK_OK;
}

// The launches of fock_apply_energy on the plan's current workspace.
fock_status run_apply_energy(Plan* p, const void* const* psi, const double* const* occ, void* const* vx_psi,
                             void* const* vmat, double* ex) {
  fock_status st = run_apply(p, psi, occ, vx_psi, nullptr, 1.0, false, true);
  if (st != FOCK_OK) return st;
  if ((st = run_overlaps(p, psi, vx_psi, vmat)) != FOCK_OK) return st;
  return run_energy(p, psi, occ, ex, true);
}

// ---- library-owned workspace of fock_apply_energy_static -----------------
// One array per device, kept until the process ends.  Host code never uses
// the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kStaticWorkspaceBytes = static_cast<size_t>(FOCK_STATIC_WORKSPACE_BYTES);
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

constexpr int kMaxDevices = 64;
struct StaticSlot {
  unsigned char* ptr = nullptr;  // device address of `scratch` on this device
  uint64_t owner = 0;            // serial of the plan whose tables it holds (0: none)
};
std::mutex g_static_mu;
StaticSlot g_static[kMaxDevices];

// The current device's array (its address looked up on first use) and its
// slot; FOCK_ERR_DEVICE if the device or the lookup fails.
fock_status static_workspace(StaticSlot** slot) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return set_error(FOCK_ERR_DEVICE, "device index beyond the static workspace table");
  std::lock_guard<std::mutex> lock(g_static_mu);
  StaticSlot& s = g_static[dev];
  if (!s.ptr) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "static workspace lookup");
    s.ptr = static_cast<unsigned char*>(ptr);
  }
  *slot = &s;
  return FOCK_OK;
}

// Run `enqueue` eagerly, or replay (recording first if needed) the graph of
// its launches for this argument set.
template <typename F>
fock_status with_graph(Plan* p, GraphCache& cache, std::vector<uintptr_t> key, F&& enqueue) {
  if (!p->use_graph) return enqueue();
  if (cache.exec && cache.key == key) {
    const hipError_t e = hipGraphLaunch(cache.exec, p->stream);
    return e == hipSuccess ? FOCK_OK : hip_fail(e, "graph launch");
  }
  cache.release();
  const bool prof_on = p->prof.on;
  p->prof.on = false;  // no event nodes in the graph
  hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    p->prof.on = prof_on;
    return hip_fail(e, "begin capture");
  }
  const fock_status st = enqueue();
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(p->stream, &graph);
  p->prof.on = prof_on;
  if (st != FOCK_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(e, "end capture");
  e = hipGraphInstantiate(&cache.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    cache.exec = nullptr;
    return hip_fail(e, "graph instantiate");
  }
  cache.key = std::move(key);
  e = hipGraphLaunch(cache.exec, p->stream);
  return e == hipSuccess ? FOCK_OK : hip_fail(e, "graph launch");
}

std::vector<uintptr_t> ptr_key(const Plan* p, std::initializer_list<const void* const*> arrays,
                               std::initializer_list<uintptr_t> extra) {
  std::vector<uintptr_t> k;
  for (const void* const* a : arrays)
    for (size_t i = 0; i < p->inst.size(); ++i) k.push_back(a ? reinterpret_cast<uintptr_t>(a[i]) : 0);
  for (uintptr_t x : extra) k.push_back(x);
  return k;
}

}  // namespace
}  // namespace fock

using namespace fock;

namespace {

fock_status check_sphere(const Plan* p, const int32_t* const* gidx, const int32_t* const* npw,
                         const int32_t* npw_max) {
  if (!gidx || !npw || !npw_max) return set_error(FOCK_ERR_ARG, "gidx, npw or npw_max is NULL");
  for (size_t i = 0; i < p->inst.size(); ++i) {
    if (!gidx[i] || !npw[i]) return set_error(FOCK_ERR_ARG, "gidx or npw of instance " + std::to_string(i) + " is NULL");
    if (npw_max[i] < 1) return set_error(FOCK_ERR_ARG, "npw_max of instance " + std::to_string(i) + " < 1");
  }
  return FOCK_OK;
}

fock_status run_pw_to_grid(Plan* p, const void* const* coef, const int32_t* const* gidx, const int32_t* const* npw,
                           const int32_t* npw_max, void* const* psi) {
  for (size_t i = 0; i < p->inst.size(); ++i) {
    const hipError_t e = launch_pw_to_grid(*p, static_cast<int>(i), coef[i], gidx[i], npw[i], npw_max[i], psi[i]);
    if (e != hipSuccess) return hip_fail(e, "sphere-to-grid launch");
  }
  return FOCK_OK;
}

fock_status run_grid_to_pw(Plan* p, void* const* f, const int32_t* const* gidx, const int32_t* const* npw,
                           const int32_t* npw_max, void* const* coef) {
  for (size_t i = 0; i < p->inst.size(); ++i) {
    const hipError_t e = launch_grid_to_pw(*p, static_cast<int>(i), f[i], gidx[i], npw[i], npw_max[i], coef[i]);
    if (e != hipSuccess) return hip_fail(e, "grid-to-sphere launch");
  }
  return FOCK_OK;
}

}  // namespace

extern "C" {

fock_status fock_plan(const fock_desc* descs, int32_t n_inst, fock_precision prec, void* hip_stream,
                      fock_plan_t* out) {
  return fock_plan_tuned(descs, n_inst, prec, hip_stream, nullptr, out);
}

fock_status fock_plan_tuned(const fock_desc* descs, int32_t n_inst, fock_precision prec, void* hip_stream,
                            const fock_tuning* tuning, fock_plan_t* out) {
  clear_error();
  if (!out) return set_error(FOCK_ERR_ARG, "out is NULL");
  if (!descs) return set_error(FOCK_ERR_ARG, "descs is NULL");
  if (n_inst < 1) return set_error(FOCK_ERR_ARG, "n_inst < 1");
  if (prec != FOCK_C128 && prec != FOCK_C64 && prec != FOCK_MIXED && prec != FOCK_MIXED_INV)
    return set_error(FOCK_ERR_ARG, "unknown precision");
  for (int i = 0; i < n_inst; ++i) {
    const fock_status s = validate_desc(descs[i], i);
    if (s != FOCK_OK) return s;
  }
  try {
    Plan* p = nullptr;
    if (tuning && (tuning->acc_workgroups < 0 || tuning->tbuf_mb < 0 || tuning->fused_split < 0 ||
                   tuning->fused_split > 4 || tuning->fused_rounds < 0 || tuning->fused_rounds > 1))
      return set_error(FOCK_ERR_ARG, "tuning knob out of range");
    const fock_status s = build_plan(descs, n_inst, prec, hip_stream, tuning, &p);
    if (s != FOCK_OK) return s;
    log_open(p);
    *out = reinterpret_cast<fock_plan_t>(p);
    return FOCK_OK;
  } catch (const std::bad_alloc&) {
    return set_error(FOCK_ERR_NOMEM, "host allocation failed while planning");
  } catch (...) {
    return set_error(FOCK_ERR_ARG, "planning failed");
  }
}

fock_status fock_workspace_size(fock_plan_t plan, size_t* bytes) {
  clear_error();
  if (!plan || !bytes) return set_error(FOCK_ERR_ARG, "NULL argument");
  *bytes = reinterpret_cast<Plan*>(plan)->total_bytes;
  return FOCK_OK;
}

fock_status fock_set_workspace(fock_plan_t plan, void* dev_ptr, size_t bytes) {
  clear_error();
  if (!plan || !dev_ptr) return set_error(FOCK_ERR_ARG, "NULL argument");
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (reinterpret_cast<uintptr_t>(dev_ptr) % 256 != 0) return set_error(FOCK_ERR_ARG, "workspace not 256-byte aligned");
  if (bytes < p->total_bytes)
    return set_error(FOCK_ERR_NOMEM, "workspace of " + std::to_string(bytes) + " bytes < required " +
                                         std::to_string(p->total_bytes));
  fock_status s = device_ok();
  if (s != FOCK_OK) return s;
  hipError_t e = prepare_kernels(p->prec, &p->max_lds);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return hip_fail(e, "device query");
  }
  if (p->lds_needed > p->max_lds)
    return set_error(FOCK_ERR_UNSUPPORTED, "grid needs " + std::to_string(p->lds_needed) +
                                               " bytes of LDS per workgroup; the device allows " +
                                               std::to_string(p->max_lds));
  // recorded graphs hold the old workspace's addresses as kernel arguments
  p->release_graphs();
  p->ws = static_cast<unsigned char*>(dev_ptr);
  p->ws_bytes = bytes;
  e = hipMemcpyAsync(p->ws, p->host_image.data(), p->const_bytes, hipMemcpyHostToDevice, p->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p->ws = nullptr;
    return hip_fail(e, "table upload");
  }
  p->uploaded = true;
  return FOCK_OK;
}

fock_status fock_set_stream(fock_plan_t plan, void* hip_stream) {
  clear_error();
  if (!plan) return set_error(FOCK_ERR_ARG, "plan is NULL");
  Plan* p = reinterpret_cast<Plan*>(plan);
  p->stream = static_cast<hipStream_t>(hip_stream);
  if (p->use_graph && p->stream == nullptr) {
    p->use_graph = false;
    p->release_graphs();
  }
  return FOCK_OK;
}

fock_status fock_apply(fock_plan_t plan, const void* const* psi, const double* const* occ, void* const* vx_psi,
                       void* const* vmat) {
  clear_error();
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return set_error(FOCK_ERR_ARG, "plan is NULL");
  return logged(p, "fock_apply", [&]() -> fock_status {
    fock_status s = check_ready(p);
    if (s != FOCK_OK) return s;
    if ((s = check_ptrs(p, psi, "psi")) != FOCK_OK) return s;
    if ((s = check_ptrs(p, reinterpret_cast<const void* const*>(occ), "occ")) != FOCK_OK) return s;
    if ((s = check_ptrs(p, reinterpret_cast<const void* const*>(vx_psi), "vx_psi")) != FOCK_OK) return s;
    for (size_t i = 0; i < p->inst.size(); ++i)
      if (vx_psi[i] == psi[i]) return set_error(FOCK_ERR_ARG, "vx_psi aliases psi");
    auto enqueue = [&]() -> fock_status {
      fock_status st = run_apply(p, psi, occ, vx_psi, nullptr, 1.0, false);
      if (st != FOCK_OK) return st;
      return run_overlaps(p, psi, vx_psi, vmat);
    };
    return with_graph(p, p->g_apply,
                      ptr_key(p, {psi, reinterpret_cast<const void* const*>(occ), reinterpret_cast<const void* const*>(vx_psi),
                                  reinterpret_cast<const void* const*>(vmat)},
                              {reinterpret_cast<uintptr_t>(vmat)}),
                      enqueue);
  });
}

fock_status fock_energy(fock_plan_t plan, const void* const* psi, const double* const* occ, double* ex) {
  clear_error();
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return set_error(FOCK_ERR_ARG, "plan is NULL");
  return logged(p, "fock_energy", [&]() -> fock_status {
    fock_status s = check_ready(p);
    if (s != FOCK_OK) return s;
    if ((s = check_ptrs(p, psi, "psi")) != FOCK_OK) return s;
    if ((s = check_ptrs(p, reinterpret_cast<const void* const*>(occ), "occ")) != FOCK_OK) return s;
    if (!ex) return set_error(FOCK_ERR_ARG, "ex is NULL");
    return with_graph(p, p->g_energy, ptr_key(p, {psi, reinterpret_cast<const void* const*>(occ)},
                                              {reinterpret_cast<uintptr_t>(ex)}),
                      [&]() { return run_energy(p, psi, occ, ex, false); });
  });
}

fock_status fock_apply_energy(fock_plan_t plan, const void* const* psi, const double* const* occ,
                              void* const* vx_psi, void* const* vmat, double* ex) {
  clear_error();
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return set_error(FOCK_ERR_ARG, "plan is NULL");
  return logged(p, "fock_apply_energy", [&]() -> fock_status {
    fock_status s = check_ready(p);
    if (s != FOCK_OK) return s;
    if ((s = check_apply_energy_args(p, psi, occ, vx_psi, ex)) != FOCK_OK) return s;
    auto enqueue = [&]() -> fock_status { return run_apply_energy(p, psi, occ, vx_psi, vmat, ex); };
    return with_graph(p, p->g_apply_energy,
                      ptr_key(p, {psi, reinterpret_cast<const void* const*>(occ), reinterpret_cast<const void* const*>(vx_psi),
                                  reinterpret_cast<const void* const*>(vmat)},
                              {reinterpret_cast<uintptr_t>(vmat), reinterpret_cast<uintptr_t>(ex)}),
                      enqueue);
  });
}

fock_status fock_apply_energy_static(fock_plan_t plan, const void* const* psi, const double* const* occ,
                                     void* const* vx_psi, void* const* vmat, double* ex) {
  clear_error();
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return set_error(FOCK_ERR_ARG, "plan is NULL");
  if (p->total_bytes > kStaticWorkspaceBytes)
    return set_error(FOCK_ERR_NOMEM, "plan needs " + std::to_string(p->total_bytes) +
                                         " bytes of workspace; the static workspace holds " +
                                         std::to_string(kStaticWorkspaceBytes));
  fock_status s = check_apply_energy_args(p, psi, occ, vx_psi, ex);
  if (s != FOCK_OK) return s;
  if ((s = device_ok()) != FOCK_OK) return s;
  size_t max_lds = 0;
  hipError_t e = prepare_kernels(p->prec, &max_lds);
  if (e != hipSuccess) return hip_fail(e, "device query");
  if (p->lds_needed > max_lds)
    return set_error(FOCK_ERR_UNSUPPORTED, "grid needs " + std::to_string(p->lds_needed) +
                                               " bytes of LDS per workgroup; the device allows " +
                                               std::to_string(max_lds));
  StaticSlot* slot = nullptr;
  if ((s = static_workspace(&slot)) != FOCK_OK) return s;
  // tables into the array unless this plan's are still there (the last call on
  // this device was this plan's)
  if (slot->owner != p->serial) {
    e = hipMemcpyAsync(slot->ptr, p->host_image.data(), p->const_bytes, hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) {
      slot->owner = 0;
      return hip_fail(e, "table upload");
    }
    slot->owner = p->serial;
  }
  // run eagerly on the array, without event timing (events would be created);
  // the plan's own workspace is restored afterwards
  unsigned char* const ws = p->ws;
  const size_t ws_bytes = p->ws_bytes;
  const bool prof_on = p->prof.on;
  p->ws = slot->ptr;
  p->ws_bytes = kStaticWorkspaceBytes;
  p->prof.on = false;
  s = run_apply_energy(p, psi, occ, vx_psi, vmat, ex);
  p->ws = ws;
  p->ws_bytes = ws_bytes;
  p->prof.on = prof_on;
  return s;
}

fock_status fock_energy_backward(fock_plan_t plan, const void* const* psi, const double* const* occ,
                                 const double* grad_ex, double scale, void* const* grad_psi) {
  clear_error();
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return set_error(FOCK_ERR_ARG, "plan is NULL");
  return logged(p, "fock_energy_backward", [&]() -> fock_status {
    for (size_t i = 0; i < p->inst.size(); ++i)
      if (!p->inst[i].symmetric)
        return set_error(FOCK_ERR_UNSUPPORTED, "instance " + std::to_string(i) +
                                                   ": the gradient needs a k-pair list closed under swapping (k, k') -> (k', k)");
    fock_status s = check_ready(p);
    if (s != FOCK_OK) return s;
    if ((s = check_ptrs(p, psi, "psi")) != FOCK_OK) return s;
    if ((s = check_ptrs(p, reinterpret_cast<const void* const*>(occ), "occ")) != FOCK_OK) return s;
    if ((s = check_ptrs(p, reinterpret_cast<const void* const*>(grad_psi), "grad_psi")) != FOCK_OK) return s;
    if (!grad_ex) return set_error(FOCK_ERR_ARG, "grad_ex is NULL");
    if (!std::isfinite(scale)) return set_error(FOCK_ERR_ARG, "scale not finite");
    for (size_t i = 0; i < p->inst.size(); ++i)
      if (grad_psi[i] == psi[i]) return set_error(FOCK_ERR_ARG, "grad_psi aliases psi");
    uint64_t sbits;
    static_assert(sizeof(sbits) == sizeof(scale), "double is 64-bit");
    std::memcpy(&sbits, &scale, sizeof(sbits));
    return with_graph(p, p->g_backward,
                      ptr_key(p, {psi, reinterpret_cast<const void* const*>(occ), reinterpret_cast<const void* const*>(grad_psi)},
                              {reinterpret_cast<uintptr_t>(grad_ex), static_cast<uintptr_t>(sbits)}),
                      [&]() { return run_apply(p, psi, occ, grad_psi, grad_ex, scale, true); });
  });
}

fock_status fock_set_graph(fock_plan_t plan, int enable) {
  clear_error();
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return set_error(FOCK_ERR_ARG, "plan is NULL");
  if (enable && p->stream == nullptr)
    return set_error(FOCK_ERR_STATE, "graph replay needs a stream other than the legacy default stream");
  p->use_graph = enable != 0;
  if (!p->use_graph) {
    p->release_graphs();
  }
  return FOCK_OK;
}

fock_status fock_pw_to_grid(fock_plan_t plan, const void* const* coef, const int32_t* const* gidx,
                            const int32_t* const* npw, const int32_t* npw_max, void* const* psi) {
  clear_error();
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return set_error(FOCK_ERR_ARG, "plan is NULL");
  return logged(p, "fock_pw_to_grid", [&]() -> fock_status {
    fock_status s = check_ready(p);
    if (s != FOCK_OK) return s;
    if ((s = check_ptrs(p, coef, "coef")) != FOCK_OK) return s;
    if ((s = check_ptrs(p, reinterpret_cast<const void* const*>(psi), "psi")) != FOCK_OK) return s;
    if ((s = check_sphere(p, gidx, npw, npw_max)) != FOCK_OK) return s;
    return run_pw_to_grid(p, coef, gidx, npw, npw_max, psi);
  });
}

fock_status fock_grid_to_pw(fock_plan_t plan, void* const* f, const int32_t* const* gidx, const int32_t* const* npw,
                            const int32_t* npw_max, void* const* coef_out) {
  clear_error();
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return set_error(FOCK_ERR_ARG, "plan is NULL");
  return logged(p, "fock_grid_to_pw", [&]() -> fock_status {
    fock_status s = check_ready(p);
    if (s != FOCK_OK) return s;
    if ((s = check_ptrs(p, reinterpret_cast<const void* const*>(f), "f")) != FOCK_OK) return s;
    if ((s = check_ptrs(p, reinterpret_cast<const void* const*>(coef_out), "coef_out")) != FOCK_OK) return s;
    if ((s = check_sphere(p, gidx, npw, npw_max)) != FOCK_OK) return s;
    return run_grid_to_pw(p, f, gidx, npw, npw_max, coef_out);
  });
}

fock_status fock_apply_pw(fock_plan_t plan, const void* const* coef, const int32_t* const* gidx,
                          const int32_t* const* npw, const int32_t* npw_max, const double* const* occ,
                          void* const* psi_work, void* const* vx_work, void* const* vx_coef) {
  clear_error();
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return set_error(FOCK_ERR_ARG, "plan is NULL");
  return logged(p, "fock_apply_pw", [&]() -> fock_status {
    fock_status s = check_ready(p);
    if (s != FOCK_OK) return s;
    if ((s = check_ptrs(p, coef, "coef")) != FOCK_OK) return s;
    if ((s = check_ptrs(p, reinterpret_cast<const void* const*>(occ), "occ")) != FOCK_OK) return s;
    if ((s = check_ptrs(p, reinterpret_cast<const void* const*>(psi_work), "psi_work")) != FOCK_OK) return s;
    if ((s = check_ptrs(p, reinterpret_cast<const void* const*>(vx_work), "vx_work")) != FOCK_OK) return s;
    if ((s = check_ptrs(p, reinterpret_cast<const void* const*>(vx_coef), "vx_coef")) != FOCK_OK) return s;
    if ((s = check_sphere(p, gidx, npw, npw_max)) != FOCK_OK) return s;
    for (size_t i = 0; i < p->inst.size(); ++i)
      if (psi_work[i] == vx_work[i]) return set_error(FOCK_ERR_ARG, "psi_work aliases vx_work");
    if ((s = run_pw_to_grid(p, coef, gidx, npw, npw_max, psi_work)) != FOCK_OK) return s;
    if ((s = run_apply(p, psi_work, occ, vx_work, nullptr, 1.0, false)) != FOCK_OK) return s;
    return run_grid_to_pw(p, vx_work, gidx, npw, npw_max, vx_coef);
  });
}

fock_status fock_dft3(fock_plan_t plan, int32_t inst, int32_t sign, int64_t count, void* data, int64_t stride) {
  clear_error();
  Plan* p = reinterpret_cast<Plan*>(plan);
  if (!p) return set_error(FOCK_ERR_ARG, "plan is NULL");
  return logged(p, "fock_dft3", [&]() -> fock_status {
    fock_status s = check_ready(p);
    if (s != FOCK_OK) return s;
    if (inst < 0 || static_cast<size_t>(inst) >= p->inst.size()) return set_error(FOCK_ERR_ARG, "instance out of range");
    if (sign != -1 && sign != 1) return set_error(FOCK_ERR_ARG, "sign must be -1 or +1");
    if (count < 0) return set_error(FOCK_ERR_ARG, "count < 0");
    if (count == 0) return FOCK_OK;
    if (!data) return set_error(FOCK_ERR_ARG, "data is NULL");
    if (stride < p->inst[inst].npts) return set_error(FOCK_ERR_ARG, "stride smaller than the grid");
    const hipError_t e = launch_dft3(*p, inst, sign, count, data, stride);
    return e == hipSuccess ? FOCK_OK : hip_fail(e, "3-D DFT launch");
  });
}

fock_status fock_plan_stats(fock_plan_t plan, int64_t* ordered_pairs, int64_t* apply_fft_pairs,
                            int64_t* energy_fft_pairs, int64_t* apply_launches) {
  clear_error();
  if (!plan) return set_error(FOCK_ERR_ARG, "plan is NULL");
  const Plan* p = reinterpret_cast<const Plan*>(plan);
  if (ordered_pairs) *ordered_pairs = p->ordered_pairs;
  if (apply_fft_pairs) *apply_fft_pairs = p->apply_fft_pairs;
  if (energy_fft_pairs) *energy_fft_pairs = p->energy_fft_pairs;
  if (apply_launches) *apply_launches = p->apply_launches;
  return FOCK_OK;
}

fock_status fock_profile_enable(fock_plan_t plan, int enable) {
  clear_error();
  if (!plan) return set_error(FOCK_ERR_ARG, "plan is NULL");
  reinterpret_cast<Plan*>(plan)->prof.on = enable != 0;
  return FOCK_OK;
}

fock_status fock_profile_read(fock_plan_t plan, int kind, double* total_ms, int64_t* launches) {
  clear_error();
  if (!plan || !total_ms || !launches) return set_error(FOCK_ERR_ARG, "NULL argument");
  if (kind < 0 || kind >= FOCK_K_COUNT) return set_error(FOCK_ERR_ARG, "unknown kernel kind");
  Profiler& pr = reinterpret_cast<Plan*>(plan)->prof;
  double ms = 0.0;
  int64_t n = 0;
  for (const auto& sp : pr.spans[kind]) {
    if (sp.second == sp.first) continue;
    hipError_t e = hipEventSynchronize(pr.pool[sp.second]);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, pr.pool[sp.first], pr.pool[sp.second]);
    if (e != hipSuccess) return hip_fail(e, "profile read");
    ms += t;
    ++n;
  }
  pr.spans[kind].clear();
  bool any = false;
  for (const auto& v : pr.spans) any = any || !v.empty();
  if (!any) pr.used = 0;  // every recorded event has been read: recycle the pool
  *total_ms = ms;
  *launches = n;
  return FOCK_OK;
}

fock_status fock_destroy(fock_plan_t plan) {
  clear_error();
  delete reinterpret_cast<Plan*>(plan);
  return FOCK_OK;
}

const char* fock_status_string(fock_status s) {
  switch (s) {
    case FOCK_OK: return "FOCK_OK";
    case FOCK_ERR_ARG: return "FOCK_ERR_ARG: invalid argument";
    case FOCK_ERR_UNSUPPORTED: return "FOCK_ERR_UNSUPPORTED: unsupported size or option";
    case FOCK_ERR_NOMEM: return "FOCK_ERR_NOMEM: out of memory or workspace too small";
    case FOCK_ERR_DEVICE: return "FOCK_ERR_DEVICE: GPU unavailable or HIP error";
    case FOCK_ERR_STATE: return "FOCK_ERR_STATE: call out of order";
    default: break;
  }
  return "unknown fock_status";
}

const char* fock_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
