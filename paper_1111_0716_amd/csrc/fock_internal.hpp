// Internal plan representation shared by the host planner, the C ABI and
// the kernel launchers of libfock.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/fock.h"

namespace fock {

// One ordered pair of an energy batch: output (k, n), partner (k', m), table
// q and multiplicity (2 when the swapped pair is folded in, else 1).
struct PairRef {
  int32_t k, n, kp, m, q, mult;
};

// A batch of band pairs.
//   apply:  outputs o0..o0+nO-1 (global band index k*nbands + n, all with the
//           same partner list) times partners (k', m) stored as int2 at
//           part_off; every output block is covered by consecutive batches,
//           the first of which writes its outputs (the rest add).
//           mirror: the pairs are unordered (outputs and partners are two
//           disjoint orbital blocks); a second accumulate pass gives the
//           partners their share, conj(W_ab) = W_ba (first_mirror: it writes
//           them rather than adds), and the pair energies count twice.
//           tri: outputs and partners are the same block (nO == nP), and the
//           batch holds its unordered pairs o <= p (npairs = nO (nO + 1) / 2,
//           row-major over the upper triangle); the accumulate pass takes
//           conj(W) from the slot (p, o) for p < o, and pairs o != p count
//           twice in the energy.
//   energy: an explicit PairRef list at pair_off; its partial sum goes to slot.
struct Batch {
  int32_t inst = 0;
  int32_t o0 = 0, nO = 0;
  size_t part_off = 0;  // bytes into the workspace
  int32_t nP = 0;
  int32_t first = 0;
  int32_t mirror = 0;
  int32_t first_mirror = 0;
  int32_t tri = 0;
  size_t pair_off = 0;  // bytes into the workspace
  int32_t npairs = 0;   // pairs in the batch (apply: nO*nP)
  int32_t slot = 0;
  int32_t per_wg = 1;   // energy on the whole-pair path: pairs per workgroup
  int32_t eslot = -1;   // apply batch of the register-line path: its energy sum slot
};

// Outputs o0..o0+nout-1 of one instance on the whole-pair path, all sharing
// the partner list (int2 (k', m)) at part_off.
struct FusedGroup {
  int32_t inst = 0;
  int32_t o0 = 0, nout = 0;
  size_t part_off = 0;
  int32_t npart = 0;
  int32_t nsplit = 1;  // partner slices per output (slices > 0 sum into partial buffers)
  int32_t eblk0 = 0;   // first of its nout * nsplit energy partials (apply with energy)
};

// The unordered band pairs (a, b), a <= b, of one instance on the whole-pair
// path, as int2 at pairs_off, cut into rounds of pairwise disjoint pairs
// (round i: pairs round_start[i] .. round_start[i + 1] - 1).  With energy,
// pair j writes energy partial eblk0 + j; the partials sum into slot eslot.
struct FusedRounds {
  int32_t inst = 0;
  size_t pairs_off = 0;
  std::vector<int32_t> round_start;
  int32_t npairs = 0;
  int32_t eblk0 = 0;
  int32_t eslot = -1;
};

struct Instance {
  double lattice[9];
  int grid[3];
  int nk;
  std::vector<double> kfrac, kweight;
  std::vector<std::vector<int>> kpartners;  // k -> list of k'
  bool symmetric = true;                     // (k, k') listed iff (k', k) listed
  bool fused = false;                        // whole-pair path (cubic grid that fits one CU)
  bool reg = false;                          // three-pass path with register-line kernels (N1 x L x L)
  bool slab = false;                         // cubic FP32 register-line path with the slab pencil (pair buffer [j1][c2][c3])
  int rounds = -1;                           // whole-pair path by unordered pairs: its FusedRounds
  int nbands;
  int64_t band_stride;
  double mu;
  int64_t npts;
  double omega;
  int nq = 0;
  std::vector<int> qmap;  // [nk*nk] -> table index or -1
  // workspace offsets (bytes)
  size_t vtab_off = 0, kw_off = 0, qmap_off = 0;
  int first_ebatch = 0, n_ebatches = 0;
  int first_eblk = 0, n_eblk = 0;  // whole-pair apply-with-energy partials of this instance
  int first_aslot = 0, n_aslot = 0;  // register-line apply-with-energy sum slots
};

// Event-based per-kernel timing (see fock_profile_enable).
struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;  // reusable events
  size_t used = 0;
  std::vector<std::pair<size_t, size_t>> spans[FOCK_K_COUNT];  // (start, stop) pool indices
  hipEvent_t next(hipStream_t s);
  void begin(int kind, hipStream_t s);
  void end(int kind, hipStream_t s);
  void release();
};

// Call records of a plan (FOCK_LOG): one JSON line per API call with its
// status, host enqueue time and device time (events around the call on the
// plan stream), written when the plan is destroyed or the pending records
// pass a bound, followed at destruction by a per-call summary.
struct CallLog {
  struct Rec {
    const char* call;
    int status;
    double enqueue_us;
    bool graph;
    hipEvent_t e0, e1;  // null when no device work could be enqueued
  };
  FILE* f = nullptr;
  bool own = false;  // f was opened here (not stderr)
  uint64_t serial = 0;
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  struct Total {
    int64_t calls = 0;
    double device_ms = 0.0;
  };
  std::vector<std::pair<std::string, Total>> totals;  // per call name, first-use order
  bool on() const { return f != nullptr; }
};

// A captured launch sequence and the arguments it was captured with.
struct GraphCache {
  std::vector<uintptr_t> key;
  hipGraphExec_t exec = nullptr;
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    key.clear();
  }
};

struct Plan {
  uint64_t serial = 0;  // distinct for every plan of the process (never reused)
  fock_precision prec;
  size_t csize;  // sizeof(complex element) of orbitals and outputs
  // orbitals, outputs and overlaps are complex128 (FOCK_C128 and FOCK_MIXED)
  bool io64() const { return prec != FOCK_C64; }
  hipStream_t stream = nullptr;
  std::vector<Instance> inst;
  std::vector<Batch> apply_batches, energy_batches;
  std::vector<FusedGroup> fused_groups;
  std::vector<FusedRounds> fused_rounds;
  // workspace layout (bytes)
  size_t tw_off = 0;                  // twiddle tables
  size_t const_bytes = 0;             // uploaded prefix
  size_t tbuf_off = 0, tbuf_bytes = 0;
  size_t tbuf64_off = 0;  // FOCK_MIXED: FP64 pair buffer beside the FP32 one at tbuf_off
  size_t epart_off = 0, epart_bytes = 0;
  size_t ebsum_off = 0, ebsum_bytes = 0;
  size_t partial_off = 0, partial_bytes = 0;
  size_t ovl_off = 0, ovl_bytes = 0;  // overlap split-K partials
  size_t eblk_off = 0, eblk_bytes = 0;  // per-block energy partials of the whole-pair apply
  size_t total_bytes = 0;
  std::vector<unsigned char> host_image;  // constant prefix, uploaded by set_workspace
  unsigned char* ws = nullptr;            // device workspace (caller-owned)
  size_t ws_bytes = 0;
  bool uploaded = false;
  int64_t ordered_pairs = 0, apply_fft_pairs = 0, energy_fft_pairs = 0, apply_launches = 0;
  int max_pairs_per_batch = 0;
  size_t max_lds = 0;      // per-block LDS limit of the device
  size_t lds_needed = 0;   // largest dynamic LDS of any launch (+ static)
  mutable Profiler prof;
  CallLog log;
  bool use_graph = false;
  GraphCache g_apply, g_apply_energy, g_energy, g_backward;
  void release_graphs() {
    g_apply.release();
    g_apply_energy.release();
    g_energy.release();
    g_backward.release();
  }
  ~Plan();
};

// status helpers (thread-local last error)
fock_status set_error(fock_status s, const std::string& msg);
void clear_error();

// kernel launchers (kernels.hip); return hipSuccess or the launch error
hipError_t prepare_kernels(fock_precision prec, size_t* max_lds);
hipError_t launch_apply_batch(const Plan& p, const Batch& b, const void* psi, const double* occ, void* vx, bool energy,
                              const double* gscale, double hscale, bool backward);
hipError_t launch_energy_batch(const Plan& p, const Batch& b, const void* psi, const double* occ);
hipError_t launch_energy_finish(const Plan& p, int inst, double* ex);
// E_x of a whole-pair instance from the per-block partials of an apply with energy
hipError_t launch_eblk_finish(const Plan& p, int inst, double* ex);
hipError_t launch_zero_outputs(const Plan& p, int inst, void* out);
hipError_t launch_zero_all_bands(const Plan& p, int inst, void* out);
void prepare_dft_kernels(fock_precision prec, int lim);
bool reg_dft_supported(fock_precision prec, const int grid[3]);
void prepare_reg_dft_kernels(fock_precision prec, int lim);
hipError_t launch_reg_dft3(const Plan& p, int inst, int sign, int count, void* data, long long stride);
hipError_t launch_dft3(const Plan& p, int inst, int sign, long long count, void* data, long long stride);
hipError_t launch_pw_to_grid(const Plan& p, int inst, const void* coef, const int* gidx, const int* npw, int npw_max,
                             void* psi);
hipError_t launch_grid_to_pw(const Plan& p, int inst, void* f, const int* gidx, const int* npw, int npw_max,
                             void* coef);
hipError_t launch_energy_reduce(const Plan& p, const Batch& b, const double* occ, int n2);
// whole-pair path (pair_fused.hip)
bool fused_supported(fock_precision prec, const int grid[3]);
size_t fused_lds_bytes(fock_precision prec, int L);
int fused_threads(fock_precision prec, int L);
size_t overlap_scratch_bytes(const Instance& in);
void prepare_fused_kernels(fock_precision prec, int lim);
bool reg_supported(fock_precision prec, const int grid[3]);
// grids where the register-line path can run its pencil pass over slabs of
// fixed c2 (and the accumulate over independent lines)
bool reg_slab_supported(fock_precision prec, const int grid[3]);
// where it is taken without FOCK_SLAB=1 (measured per size)
bool reg_slab_default(fock_precision prec, const int grid[3]);
size_t reg_lds_bytes(fock_precision prec, int L);
void prepare_reg_kernels(fock_precision prec, int lim);
// energy: the pencil pass also writes the batch's weighted pair energies to
// its slot (b.eslot); only where batch_apply_energy(inst)
hipError_t launch_reg_apply_batch(const Plan& p, const Batch& b, const void* psi, const double* occ, void* out,
                                  const double* gscale, double hscale, bool backward, bool energy);
// the instance's apply batches take its energy (the three-pass paths)
bool batch_apply_energy(const Plan& p, int inst);
// ebsum[slot] = mult * fixed-order sum of the first n energy partials (epart)
hipError_t launch_sum_slot(const Plan& p, long long n, int slot, double mult);
// E_x of a three-pass instance from its apply-with-energy slots
hipError_t launch_aslot_finish(const Plan& p, int inst, double* ex);
hipError_t launch_reg_energy_batch(const Plan& p, const Batch& b, const void* psi, const double* occ);
// eblk: if not null, the apply also writes per-block energy partials there
hipError_t launch_fused_apply(const Plan& p, const FusedGroup& g, const void* psi, const double* occ, void* out,
                              const double* gscale, double hscale, bool backward, double* eblk);
hipError_t launch_fused_energy(const Plan& p, const Batch& b, const void* psi);
// whole-pair path by unordered pairs (FP32 32^3): the grids it serves, and
// its rounds (outputs zeroed first); eblk: this instance's energy partials or null
bool fused_rounds_supported(fock_precision prec, const int grid[3]);
hipError_t launch_fused_rounds(const Plan& p, const FusedRounds& r, const void* psi, const double* occ, void* out,
                               const double* gscale, double hscale, bool backward, double* eblk);
// ebsum[slot] = fixed-order sum of n partials at part (FP64)
hipError_t launch_sum_partials(const Plan& p, const double* part, long long n, int slot);
hipError_t launch_overlap(const Plan& p, int inst, const void* psi, const void* vx, void* vmat);

}  // namespace fock
