// Host planner of libfock.so: descriptor validation, FP64 kernel tables,
// twiddle tables, the batched band-pair schedule and the workspace layout.
// Host work only; nothing here touches the device.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <memory>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "fft_lds.hpp"
#include "fock_internal.hpp"

namespace fock {

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool finite_all(const double* p, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

double det3(const double* a) {
  return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) + a[2] * (a[3] * a[7] - a[4] * a[6]);
}

// b_i rows with a_i . b_j = 2 pi delta_ij, i.e. B = 2 pi A^{-T}
void reciprocal(const double* a, double b[3][3]) {
  const double d = det3(a);
  const double two_pi = 6.283185307179586476925286766559;
  // inverse of A (rows a_i), then transpose
  double inv[3][3];
  inv[0][0] = (a[4] * a[8] - a[5] * a[7]) / d;
  inv[0][1] = (a[2] * a[7] - a[1] * a[8]) / d;
  inv[0][2] = (a[1] * a[5] - a[2] * a[4]) / d;
  inv[1][0] = (a[5] * a[6] - a[3] * a[8]) / d;
  inv[1][1] = (a[0] * a[8] - a[2] * a[6]) / d;
  inv[1][2] = (a[2] * a[3] - a[0] * a[5]) / d;
  inv[2][0] = (a[3] * a[7] - a[4] * a[6]) / d;
  inv[2][1] = (a[1] * a[6] - a[0] * a[7]) / d;
  inv[2][2] = (a[0] * a[4] - a[1] * a[3]) / d;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) b[i][j] = two_pi * inv[j][i];
}

// Screened kernel of HSE06: 4 pi/K^2 (1 - exp(-K^2/(4 mu^2))), K -> 0 limit pi/mu^2.
inline double screened(double k2, double mu) {
  if (k2 == 0.0) return M_PI / (mu * mu);
  return -4.0 * M_PI / k2 * std::expm1(-k2 / (4.0 * mu * mu));
}

// v_q on every class of the grid divided by N, Nyquist classes averaged over
// their +-N/2 aliases (all combinations when several axes sit at Nyquist).
void build_kernel_table(const Instance& in, const double q[3], std::vector<double>& out) {
  double b[3][3];
  reciprocal(in.lattice, b);
  // per axis and class: the Cartesian vectors (g + q_i) b_i of its representatives
  std::vector<std::vector<std::array<double, 3>>> reps[3];
  for (int ax = 0; ax < 3; ++ax) {
    const int n = in.grid[ax];
    reps[ax].resize(n);
    for (int c = 0; c < n; ++c) {
      std::vector<double> gs;
      if (2 * c == n) {
        gs = {static_cast<double>(c), static_cast<double>(c - n)};
      } else if (2 * c < n) {
        gs = {static_cast<double>(c)};
      } else {
        gs = {static_cast<double>(c - n)};
      }
      for (double g : gs) {
        const double x = g + q[ax];
        reps[ax][c].push_back({x * b[ax][0], x * b[ax][1], x * b[ax][2]});
      }
    }
  }
  const int n1 = in.grid[0], n2 = in.grid[1], n3 = in.grid[2];
  const double inv_n = 1.0 / static_cast<double>(in.npts);
  out.assign(in.npts, 0.0);
  for (int c1 = 0; c1 < n1; ++c1)
    for (int c2 = 0; c2 < n2; ++c2)
      for (int c3 = 0; c3 < n3; ++c3) {
        double sum = 0.0;
        int cnt = 0;
        for (const auto& r1 : reps[0][c1])
          for (const auto& r2 : reps[1][c2])
            for (const auto& r3 : reps[2][c3]) {
              const double kx = r1[0] + r2[0] + r3[0];
              const double ky = r1[1] + r2[1] + r3[1];
              const double kz = r1[2] + r2[2] + r3[2];
              sum += screened(kx * kx + ky * ky + kz * kz, in.mu);
              ++cnt;
            }
        out[(static_cast<size_t>(c1) * n2 + c2) * n3 + c3] = sum / cnt * inv_n;
      }
}

// every k' is a partner of every k, in order (the full k-pair set)
bool full_kset(const Instance& in) {
  for (int k = 0; k < in.nk; ++k) {
    if (static_cast<int>(in.kpartners[k].size()) != in.nk) return false;
    for (int kp = 0; kp < in.nk; ++kp)
      if (in.kpartners[k][kp] != kp) return false;
  }
  return true;
}

// The unordered pairs (a, b), a <= b, of the listed k-pairs (orbital a =
// k nbands + n), in rounds of at most `cap` pairwise disjoint pairs.  Source
// order: the n - 1 perfect matchings of the circle method on the orbitals
// (a dummy orbital makes the count even), then the self pairs; each pair goes
// first-fit into the oldest of a few open rounds that has room and neither of
// its orbitals, so nearly every round is full.  pairs: (a, b) flattened;
// starts: first pair of every round and the total at the end.
void build_rounds(const Instance& in, int cap, std::vector<int32_t>& pairs, std::vector<int32_t>& starts) {
  const int nb = in.nbands, O = in.nk * nb, n = O + (O & 1);
  std::vector<char> listed(static_cast<size_t>(in.nk) * in.nk, 0);
  for (int k = 0; k < in.nk; ++k)
    for (int kp : in.kpartners[k]) listed[static_cast<size_t>(k) * in.nk + kp] = 1;
  struct Round {
    std::vector<int32_t> p;
    std::vector<char> used;
  };
  constexpr size_t kWindow = 8;
  std::vector<Round> open;  // oldest first
  auto close_oldest = [&]() {
    starts.push_back(static_cast<int32_t>(pairs.size() / 2));
    pairs.insert(pairs.end(), open.front().p.begin(), open.front().p.end());
    open.erase(open.begin());
  };
  auto place = [&](int a, int b) {
    if (a > b) std::swap(a, b);
    if (!listed[static_cast<size_t>(a / nb) * in.nk + b / nb]) return;
    for (Round& r : open)
      if (static_cast<int>(r.p.size() / 2) < cap && !r.used[a] && !r.used[b]) {
        r.p.push_back(a);
        r.p.push_back(b);
        r.used[a] = r.used[b] = 1;
        return;
      }
    if (open.size() == kWindow) close_oldest();
    open.push_back(Round{{a, b}, std::vector<char>(O, 0)});
    open.back().used[a] = open.back().used[b] = 1;
  };
  for (int r = 0; r + 1 < n; ++r) {
    if (n - 1 < O) place(r, n - 1);  // the fixed vertex (absent when it is the dummy)
    for (int i = 1; i < n / 2; ++i) place((r + i) % (n - 1), (r - i + (n - 1)) % (n - 1));
  }
  for (int a = 0; a < O; ++a) place(a, a);
  while (!open.empty()) close_oldest();
  starts.push_back(static_cast<int32_t>(pairs.size() / 2));
}

// The schedule's contract, checked on the host: every listed unordered pair
// exactly once, no orbital twice within a round.
bool rounds_valid(const Instance& in, const std::vector<int32_t>& pairs, const std::vector<int32_t>& starts) {
  const int nb = in.nbands, O = in.nk * nb;
  std::vector<char> listed(static_cast<size_t>(in.nk) * in.nk, 0);
  for (int k = 0; k < in.nk; ++k)
    for (int kp : in.kpartners[k]) listed[static_cast<size_t>(k) * in.nk + kp] = 1;
  std::vector<char> seen(static_cast<size_t>(O) * O, 0);
  std::vector<int32_t> last_round(O, -1);
  for (size_t r = 0; r + 1 < starts.size(); ++r) {
    for (int32_t j = starts[r]; j < starts[r + 1]; ++j) {
      const int a = pairs[2 * j], b = pairs[2 * j + 1];
      if (a < 0 || b >= O || a > b) return false;
      if (last_round[a] == static_cast<int32_t>(r) || last_round[b] == static_cast<int32_t>(r)) return false;
      last_round[a] = last_round[b] = static_cast<int32_t>(r);
      char& s = seen[static_cast<size_t>(a) * O + b];
      if (s) return false;
      s = 1;
    }
  }
  for (int a = 0; a < O; ++a)
    for (int b = a; b < O; ++b)
      if (seen[static_cast<size_t>(a) * O + b] != listed[static_cast<size_t>(a / nb) * in.nk + b / nb]) return false;
  return true;
}

size_t env_mb(const char* name, size_t dflt) {
  const char* s = std::getenv(name);
  if (!s || !*s) return dflt;
  const long long v = std::atoll(s);
  return v > 0 ? static_cast<size_t>(v) : dflt;
}

}  // namespace

fock_status validate_desc(const fock_desc& d, int idx) {
  const std::string at = "instance " + std::to_string(idx) + ": ";
  if (!finite_all(d.lattice, 9)) return set_error(FOCK_ERR_ARG, at + "lattice not finite");
  double nrm = 1.0;
  for (int i = 0; i < 3; ++i)
    nrm *= std::sqrt(d.lattice[3 * i] * d.lattice[3 * i] + d.lattice[3 * i + 1] * d.lattice[3 * i + 1] +
                     d.lattice[3 * i + 2] * d.lattice[3 * i + 2]);
  if (!(nrm > 0.0) || std::fabs(det3(d.lattice)) <= 1e-12 * nrm) return set_error(FOCK_ERR_ARG, at + "singular lattice");
  for (int i = 0; i < 3; ++i) {
    if (d.grid[i] < 2) return set_error(FOCK_ERR_ARG, at + "grid axis < 2");
    if (d.grid[i] > kNMax || !smooth235(d.grid[i]))
      return set_error(FOCK_ERR_UNSUPPORTED,
                       at + "grid axis " + std::to_string(d.grid[i]) + " is not a {2,3,5}-smooth length <= 72");
  }
  if (d.nk < 1) return set_error(FOCK_ERR_ARG, at + "nk < 1");
  if (!d.kfrac) return set_error(FOCK_ERR_ARG, at + "kfrac is NULL");
  if (!finite_all(d.kfrac, 3 * d.nk)) return set_error(FOCK_ERR_ARG, at + "kfrac not finite");
  if (d.kweight) {
    for (int i = 0; i < d.nk; ++i)
      if (!std::isfinite(d.kweight[i]) || d.kweight[i] < 0.0) return set_error(FOCK_ERR_ARG, at + "bad k weight");
  }
  if (d.npairs < 0) return set_error(FOCK_ERR_ARG, at + "npairs < 0");
  if (d.npairs > 0) {
    if (!d.kpairs) return set_error(FOCK_ERR_ARG, at + "kpairs is NULL");
    for (int i = 0; i < 2 * d.npairs; ++i)
      if (d.kpairs[i] < 0 || d.kpairs[i] >= d.nk) return set_error(FOCK_ERR_ARG, at + "k-pair index out of range");
  }
  if (d.nbands < 1) return set_error(FOCK_ERR_ARG, at + "nbands < 1");
  const int64_t npts = static_cast<int64_t>(d.grid[0]) * d.grid[1] * d.grid[2];
  if (d.band_stride < npts) return set_error(FOCK_ERR_ARG, at + "band_stride < N1*N2*N3");
  if (!std::isfinite(d.mu) || !(d.mu > 0.0)) return set_error(FOCK_ERR_ARG, at + "mu must be finite and > 0");
  return FOCK_OK;
}

fock_status build_plan(const fock_desc* descs, int n_inst, fock_precision prec, void* stream, const fock_tuning* tune,
                       Plan** out) {
  const fock_tuning tn = tune ? *tune : fock_tuning{0, 0, 0, 0, 0, 0};
  static std::atomic<uint64_t> next_serial{1};
  auto p = std::make_unique<Plan>();
  p->serial = next_serial.fetch_add(1);
  p->prec = prec;
  p->csize = prec == FOCK_C64 ? 8 : 16;
  const size_t rsize = prec == FOCK_C64 ? 4 : 8;  // kernel tables: FP64 unless the whole path is FP32
  p->stream = static_cast<hipStream_t>(stream);
  p->inst.resize(n_inst);

  // ---- instances, transfers and kernel tables (FP64) ----
  std::vector<std::vector<std::vector<double>>> tables(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    const fock_desc& d = descs[i];
    Instance& in = p->inst[i];
    std::memcpy(in.lattice, d.lattice, sizeof(in.lattice));
    for (int a = 0; a < 3; ++a) in.grid[a] = d.grid[a];
    in.nk = d.nk;
    in.kfrac.assign(d.kfrac, d.kfrac + 3 * d.nk);
    in.kweight.resize(d.nk);
    for (int k = 0; k < d.nk; ++k) in.kweight[k] = d.kweight ? d.kweight[k] : 1.0 / d.nk;
    in.kpartners.assign(d.nk, {});
    if (d.npairs == 0) {
      for (int k = 0; k < d.nk; ++k)
        for (int kp = 0; kp < d.nk; ++kp) in.kpartners[k].push_back(kp);
    } else {
      for (int e = 0; e < d.npairs; ++e) in.kpartners[d.kpairs[2 * e]].push_back(d.kpairs[2 * e + 1]);
    }
    std::vector<char> listed(static_cast<size_t>(d.nk) * d.nk, 0);
    for (int k = 0; k < d.nk; ++k)
      for (int kp : in.kpartners[k]) {
        if (listed[static_cast<size_t>(k) * d.nk + kp])
          return set_error(FOCK_ERR_ARG, "instance " + std::to_string(i) + ": duplicate k-pair");
        listed[static_cast<size_t>(k) * d.nk + kp] = 1;
      }
    in.symmetric = true;
    for (int k = 0; k < d.nk; ++k)
      for (int kp = 0; kp < d.nk; ++kp)
        if (listed[static_cast<size_t>(k) * d.nk + kp] != listed[static_cast<size_t>(kp) * d.nk + k])
          in.symmetric = false;
    in.nbands = d.nbands;
    in.band_stride = d.band_stride;
    in.mu = d.mu;
    in.npts = static_cast<int64_t>(d.grid[0]) * d.grid[1] * d.grid[2];
    in.omega = std::fabs(det3(d.lattice));
    // distinct transfers q = k - k' (FP64 differences, compared bit for bit)
    in.qmap.assign(static_cast<size_t>(d.nk) * d.nk, -1);
    std::map<std::array<double, 3>, int> qidx;
    for (int k = 0; k < d.nk; ++k)
      for (int kp : in.kpartners[k]) {
        std::array<double, 3> q = {in.kfrac[3 * k] - in.kfrac[3 * kp], in.kfrac[3 * k + 1] - in.kfrac[3 * kp + 1],
                                   in.kfrac[3 * k + 2] - in.kfrac[3 * kp + 2]};
        auto it = qidx.find(q);
        int id;
        if (it == qidx.end()) {
          id = static_cast<int>(qidx.size());
          qidx.emplace(q, id);
          tables[i].emplace_back();
          build_kernel_table(in, q.data(), tables[i].back());
        } else {
          id = it->second;
        }
        in.qmap[static_cast<size_t>(k) * d.nk + kp] = id;
      }
    in.nq = static_cast<int>(qidx.size());
  }
  const char* nofused = std::getenv("FOCK_NO_FUSED");
  const bool no_fused = tn.no_fused != 0 || (nofused && *nofused && *nofused != '0');
  const char* noreg = std::getenv("FOCK_NO_REG");
  const bool no_reg = noreg && *noreg && *noreg != '0';
  const char* nosym = std::getenv("FOCK_NO_PAIR_SYMMETRY");
  const bool no_sym = tn.no_pair_symmetry != 0 || (nosym && *nosym && *nosym != '0');
  // FOCK_SLAB=0 keeps every grid on the plane-wise accumulate, FOCK_SLAB=1 puts
  // every supported cubic grid on the slab path (measurement switch)
  const char* slab_env = std::getenv("FOCK_SLAB");
  const int slab_force = slab_env && *slab_env ? (*slab_env != '0' ? 1 : 0) : -1;
  const char* rounds_env = std::getenv("FOCK_FUSED_ROUNDS");
  const bool use_rounds = tn.fused_rounds != 0 || (rounds_env && *rounds_env && *rounds_env != '0');
  for (auto& in : p->inst) {
    // The 32^3 FP32 whole-pair kernel read-modify-writes its output per
    // partner; with the full k-pair set the three-pass path with pair
    // symmetry moves fewer bytes per ordered pair and is faster (alpha boron
    // 416 against 606 ms per step), so it takes those instances.
    const bool sym_three_pass = !no_sym && !use_rounds && fused_rounds_supported(prec, in.grid) && full_kset(in) &&
                                reg_supported(prec, in.grid) && !no_reg;
    const bool mixed = prec == FOCK_MIXED || prec == FOCK_MIXED_INV;
    in.fused = !mixed && fused_supported(prec, in.grid) && !no_fused && !sym_three_pass;
    in.reg = !in.fused && reg_supported(prec, in.grid) && !no_reg;
    in.slab = in.reg && (slab_force < 0 ? reg_slab_default(prec, in.grid)
                                        : slab_force == 1 && reg_slab_supported(prec, in.grid));
    if (mixed && !in.reg)
      return set_error(FOCK_ERR_UNSUPPORTED, "mixed precision needs a grid N1 x L x L with N1 and L in {24, 32, 36, 40, 48, 50, 54, 60, 64, 72}");
  }

  // ---- batch shapes ----
  // pair-buffer budget: 4 GiB, 8 GiB in FP64, whose pairs are twice the
  // bytes (the same block shapes; alpha boron FP64 1.02 s per step against
  // 1.06 s at 4 GiB)
  const size_t tbuf_default = prec == FOCK_C128 ? 8192 : 4096;
  const size_t tbuf_target =
      (tn.tbuf_mb > 0 ? static_cast<size_t>(tn.tbuf_mb) : env_mb("FOCK_TBUF_MB", tbuf_default)) << 20;
  const int acc_wgs = tn.acc_workgroups > 0 ? tn.acc_workgroups : 2048;

  // ---- workspace layout: constant prefix ----
  size_t off = 0;
  p->tw_off = off;
  off = align_up(off + static_cast<size_t>(kTwiddleTotal) * p->csize);
  for (auto& in : p->inst) {
    in.vtab_off = off;
    off = align_up(off + static_cast<size_t>(in.nq) * in.npts * rsize);
    in.qmap_off = off;
    off = align_up(off + in.qmap.size() * sizeof(int32_t));
    in.kw_off = off;
    off = align_up(off + in.kweight.size() * sizeof(double));
  }
  // partner lists per group of consecutive k sharing one partner list; apply batches
  struct Group {
    int inst, k0, k1;  // k in [k0, k1)
    size_t off;
    std::vector<int32_t> parts;  // (k', m) pairs
  };
  std::vector<Group> groups;
  for (int i = 0; i < n_inst; ++i) {
    const Instance& in = p->inst[i];
    int k = 0;
    while (k < in.nk) {
      int k1 = k + 1;
      while (k1 < in.nk && in.kpartners[k1] == in.kpartners[k]) ++k1;
      Group g{i, k, k1, 0, {}};
      for (int kp : in.kpartners[k])
        for (int m = 0; m < in.nbands; ++m) {
          g.parts.push_back(kp);
          g.parts.push_back(m);
        }
      g.off = off;
      off = align_up(off + g.parts.size() * sizeof(int32_t));
      groups.push_back(std::move(g));
      k = k1;
    }
  }
  size_t max_pairs_elems = 0;  // max over batches of npairs * npts
  size_t max_partial = 0;      // bytes of partial sums of the whole-pair path
  const int n_cus = static_cast<int>(env_mb("FOCK_CUS", 256));
  // whole-pair path by unordered pairs (the grids whose output is
  // read-modify-written per pair anyway), on request: rounds of two
  // workgroups per CU
  std::vector<std::vector<int32_t>> round_pairs;
  for (int i = 0; i < n_inst; ++i) {
    Instance& in = p->inst[i];
    if (!(use_rounds && in.fused && in.symmetric && fused_rounds_supported(prec, in.grid))) continue;
    FusedRounds r;
    r.inst = i;
    std::vector<int32_t> pl;
    build_rounds(in, static_cast<int>(env_mb("FOCK_ROUND_PAIRS", 2 * static_cast<size_t>(n_cus))), pl, r.round_start);
    if (!rounds_valid(in, pl, r.round_start))
      return set_error(FOCK_ERR_UNSUPPORTED, "instance " + std::to_string(i) + ": internal error in the pair rounds");
    r.npairs = static_cast<int32_t>(pl.size() / 2);
    if (r.npairs == 0) continue;
    r.pairs_off = off;
    off = align_up(off + pl.size() * sizeof(int32_t));
    in.rounds = static_cast<int>(p->fused_rounds.size());
    p->fused_rounds.push_back(std::move(r));
    round_pairs.push_back(std::move(pl));
    p->apply_fft_pairs += p->fused_rounds.back().npairs;
  }
  for (const Group& g : groups) {
    const Instance& in = p->inst[g.inst];
    const int nout = (g.k1 - g.k0) * in.nbands;
    const int npart = static_cast<int>(g.parts.size() / 2);
    if (npart == 0) continue;
    if (in.rounds >= 0) continue;  // served by its rounds
    if (in.fused) {
      FusedGroup fg;
      fg.inst = g.inst;
      fg.o0 = g.k0 * in.nbands;
      fg.nout = nout;
      fg.part_off = g.off;
      fg.npart = npart;
      // partner slices: fill the resident workgroup slots evenly (fewest slices wins ties)
      const size_t lds = fused_lds_bytes(prec, in.grid[0]);
      const int per_cu = std::max(1, std::min<int>(static_cast<int>(160 * 1024 / lds), 2048 / fused_threads(prec, in.grid[0])));
      const int slots = n_cus * per_cu;
      double best = -1.0;
      for (int sp = 1; sp <= 4 && sp <= npart; ++sp) {
        if (tn.fused_split > 0 && sp != std::min(tn.fused_split, npart)) continue;
        const long long items = static_cast<long long>(nout) * sp;
        const long long waves = (items + slots - 1) / slots;
        const double eff = static_cast<double>(items) / static_cast<double>(waves * slots);
        if (eff > best + 1e-9) {
          best = eff;
          fg.nsplit = sp;
        }
      }
      max_partial = std::max(max_partial, static_cast<size_t>(fg.nsplit - 1) * nout * in.npts * p->csize);
      p->fused_groups.push_back(fg);
      p->apply_fft_pairs += static_cast<int64_t>(nout) * npart;
      continue;
    }
    const size_t pair_bytes = static_cast<size_t>(in.npts) * p->csize;
    const int pmax = static_cast<int>(std::max<size_t>(1, std::min<size_t>(65535, tbuf_target / pair_bytes)));
    if (in.reg && !no_sym && g.k0 == 0 && g.k1 == in.nk && full_kset(in)) {
      // Pair symmetry: W_ba = conj(W_ab) (the Nyquist-averaged kernel is even
      // in c -> -c, q -> -q), so each unordered pair is transformed once.  The
      // orbitals (partner order = global order k' nbands + m) are cut into
      // blocks of bs; block pair (I, J), I < J, is one batch whose accumulate
      // pass serves I and whose mirror pass serves J; a block with itself is a
      // triangular batch of its unordered pairs.  Batches run in sequence on
      // one stream, so no output is written by two launches at once.
      int bs = std::max(1, std::min(nout, static_cast<int>(std::sqrt(static_cast<double>(pmax)))));
      const int nblk = (nout + bs - 1) / bs;
      bs = (nout + nblk - 1) / nblk;
      std::vector<char> touched(nblk, 0);
      for (int I = 0; I < nblk; ++I) {
        const int i0 = I * bs, ni = std::min(bs, nout - i0);
        for (int J = I; J < nblk; ++J) {
          const int j0 = J * bs, nj = std::min(bs, nout - j0);
          Batch b;
          b.inst = g.inst;
          b.o0 = i0;
          b.nO = ni;
          b.part_off = g.off + static_cast<size_t>(j0) * 2 * sizeof(int32_t);
          b.nP = nj;
          b.first = touched[I] ? 0 : 1;
          touched[I] = 1;
          if (J != I) {
            b.mirror = 1;
            b.first_mirror = touched[J] ? 0 : 1;
            touched[J] = 1;
            b.npairs = ni * nj;
          } else {
            b.tri = 1;  // the block with itself: its unordered pairs once
            b.npairs = ni * (ni + 1) / 2;
          }
          max_pairs_elems = std::max(max_pairs_elems, static_cast<size_t>(b.npairs) * in.npts);
          p->apply_batches.push_back(b);
          p->apply_fft_pairs += b.npairs;
        }
      }
      continue;
    }
    int nO = std::max(1, std::min(nout, (acc_wgs + in.grid[0] - 1) / in.grid[0]));
    nO = std::min(nO, pmax);
    const int nP = std::max(1, std::min(npart, pmax / nO));
    for (int ob = 0; ob < nout; ob += nO) {
      for (int pb = 0; pb < npart; pb += nP) {
        Batch b;
        b.inst = g.inst;
        b.o0 = g.k0 * in.nbands + ob;
        b.nO = std::min(nO, nout - ob);
        b.part_off = g.off + static_cast<size_t>(pb) * 2 * sizeof(int32_t);
        b.nP = std::min(nP, npart - pb);
        b.first = pb == 0 ? 1 : 0;
        b.npairs = b.nO * b.nP;
        max_pairs_elems = std::max(max_pairs_elems, static_cast<size_t>(b.npairs) * in.npts);
        p->apply_batches.push_back(b);
        p->apply_fft_pairs += b.npairs;
      }
    }
  }
  // outputs without partners (empty k-pair list for some k) are written as zero by
  // a dedicated apply batch with no partners: not needed, the wrapper zero-fills.
  // energy pair lists
  std::vector<std::vector<PairRef>> elists(n_inst);
  size_t max_epairs = 0, max_n2 = 0, max_fused_epairs = 0;
  int slot = 0;
  for (int i = 0; i < n_inst; ++i) {
    Instance& in = p->inst[i];
    std::vector<PairRef>& L = elists[i];
    for (int k = 0; k < in.nk; ++k)
      for (int n = 0; n < in.nbands; ++n)
        for (int kp : in.kpartners[k])
          for (int m = 0; m < in.nbands; ++m) {
            const int a = k * in.nbands + n, bidx = kp * in.nbands + m;
            int mult = 1;
            if (in.symmetric) {
              if (bidx < a) continue;
              mult = bidx > a ? 2 : 1;
            }
            L.push_back(PairRef{k, n, kp, m, in.qmap[static_cast<size_t>(k) * in.nk + kp], mult});
          }
    for (int k = 0; k < in.nk; ++k) p->ordered_pairs += static_cast<int64_t>(in.kpartners[k].size()) * in.nbands * in.nbands;
    const size_t pair_bytes = static_cast<size_t>(in.npts) * p->csize;
    size_t pmax = std::max<size_t>(1, std::min<size_t>(65535, tbuf_target / pair_bytes));
    if (in.fused) pmax = std::max<size_t>(1, L.size());  // one launch; no pair buffer
    in.first_ebatch = slot;
    in.n_ebatches = 0;
    const size_t base = off;
    off = align_up(off + L.size() * sizeof(PairRef));
    for (size_t s0 = 0; s0 < L.size(); s0 += pmax) {
      Batch b;
      b.inst = i;
      b.pair_off = base + s0 * sizeof(PairRef);
      b.npairs = static_cast<int32_t>(std::min(pmax, L.size() - s0));
      b.slot = slot++;
      in.n_ebatches++;
      if (in.fused) {
        b.per_wg = std::max(1, b.npairs / 1024);
        max_fused_epairs = std::max(max_fused_epairs, static_cast<size_t>(b.npairs));
      } else {
        max_epairs = std::max(max_epairs, static_cast<size_t>(b.npairs));
        max_pairs_elems = std::max(max_pairs_elems, static_cast<size_t>(b.npairs) * in.npts);
      }
      p->energy_batches.push_back(b);
      p->energy_fft_pairs += b.npairs;
    }
    max_n2 = std::max(max_n2, static_cast<size_t>(in.grid[1]));
  }
  // apply-with-energy sum slots: one per apply batch of a three-pass
  // instance, contiguous per instance
  size_t max_apply_epairs = 0;
  for (int i = 0; i < n_inst; ++i) {
    Instance& in = p->inst[i];
    in.first_aslot = slot;
    if (!in.fused) {
      for (Batch& b : p->apply_batches) {
        if (b.inst != i) continue;
        b.eslot = slot++;
        max_apply_epairs = std::max(max_apply_epairs, static_cast<size_t>(b.npairs));
      }
    }
    in.n_aslot = slot - in.first_aslot;
  }
  p->const_bytes = off;
  // ---- scratch ----
  p->tbuf_off = off;
  if (prec == FOCK_MIXED || prec == FOCK_MIXED_INV) {
    // FP32 pair buffer (plane pass out, pencil in), then the FP64 one
    p->tbuf64_off = align_up(off + max_pairs_elems * 8);
    p->tbuf_bytes = p->tbuf64_off - off + max_pairs_elems * 16;
  } else {
    p->tbuf_bytes = max_pairs_elems * p->csize;
  }
  off = align_up(off + p->tbuf_bytes);
  p->epart_off = off;
  // per (pair, line block) energy partials: energy batches and apply-with-energy batches
  p->epart_bytes = std::max(std::max(max_epairs, max_apply_epairs) * max_n2, max_fused_epairs) * sizeof(double);
  off = align_up(off + p->epart_bytes);
  p->partial_off = off;
  p->partial_bytes = max_partial;
  off = align_up(off + p->partial_bytes);
  p->ovl_off = off;
  for (const auto& in : p->inst) p->ovl_bytes = std::max(p->ovl_bytes, overlap_scratch_bytes(in));
  off = align_up(off + p->ovl_bytes);
  // energy partials of the whole-pair apply: one per block, contiguous per instance
  int neblk = 0;
  for (int i = 0; i < n_inst; ++i) {
    p->inst[i].first_eblk = neblk;
    for (FusedGroup& g : p->fused_groups) {
      if (g.inst != i) continue;
      g.eblk0 = neblk;
      neblk += g.nout * g.nsplit;
    }
    for (FusedRounds& r : p->fused_rounds) {
      if (r.inst != i) continue;
      r.eblk0 = neblk;
      neblk += r.npairs;
      r.eslot = slot++;
    }
    p->inst[i].n_eblk = neblk - p->inst[i].first_eblk;
  }
  p->eblk_off = off;
  p->eblk_bytes = static_cast<size_t>(std::max(neblk, 1)) * sizeof(double);
  off = align_up(off + p->eblk_bytes);
  p->ebsum_off = off;
  p->ebsum_bytes = static_cast<size_t>(std::max(slot, 1)) * sizeof(double);
  off = align_up(off + p->ebsum_bytes);
  p->total_bytes = off;
  for (const auto& in : p->inst) {
    const size_t plane = static_cast<size_t>(in.grid[1]) * in.grid[2], tile = static_cast<size_t>(in.grid[0]) * in.grid[2];
    const size_t need = in.fused ? fused_lds_bytes(prec, in.grid[0]) + 256
                        : in.reg ? reg_lds_bytes(prec, in.grid[1]) + 64
                                 : std::max(plane, tile) * p->csize + 64;
    p->lds_needed = std::max(p->lds_needed, need);
  }
  p->apply_launches = 0;
  for (const Batch& b : p->apply_batches) p->apply_launches += 3;
  for (const FusedGroup& g : p->fused_groups) p->apply_launches += g.nsplit > 1 ? 2 : 1;
  for (const FusedRounds& r : p->fused_rounds) p->apply_launches += static_cast<int64_t>(r.round_start.size());

  // ---- host image of the constant prefix ----
  p->host_image.assign(p->const_bytes, 0);
  unsigned char* img = p->host_image.data();
  for (int L = 2; L <= kNMax; ++L) {
    if (!smooth235(L)) continue;
    const int o = twiddle_offset(L);
    for (int t = 0; t < L; ++t) {
      // exp(-2 pi i t/L) in FP64, rounded once
      const double ang = -2.0 * M_PI * static_cast<double>(t) / static_cast<double>(L);
      const double c = std::cos(ang), s = std::sin(ang);
      if (prec != FOCK_C64) {
        double* w = reinterpret_cast<double*>(img + p->tw_off) + 2 * (o + t);
        w[0] = c;
        w[1] = s;
      } else {
        float* w = reinterpret_cast<float*>(img + p->tw_off) + 2 * (o + t);
        w[0] = static_cast<float>(c);
        w[1] = static_cast<float>(s);
      }
    }
  }
  for (int i = 0; i < n_inst; ++i) {
    Instance& in = p->inst[i];
    for (int q = 0; q < in.nq; ++q) {
      std::vector<double>& t = tables[i][q];
      if (in.fused) {
        // whole-pair path reads the table in C order: (c3*L + c2)*L + c1
        const int L = in.grid[0];
        std::vector<double> r(t.size());
        for (int c1 = 0; c1 < L; ++c1)
          for (int c2 = 0; c2 < L; ++c2)
            for (int c3 = 0; c3 < L; ++c3)
              r[(static_cast<size_t>(c3) * L + c2) * L + c1] = t[(static_cast<size_t>(c1) * L + c2) * L + c3];
        t.swap(r);
      } else if (in.reg && !in.slab) {
        // register-line three-pass path reads the table as [c1][c3][c2]
        // (grids N1 x L x L; the slab pencil reads it in grid order)
        const int n1 = in.grid[0], L = in.grid[1];
        std::vector<double> r(t.size());
        for (int c1 = 0; c1 < n1; ++c1)
          for (int c2 = 0; c2 < L; ++c2)
            for (int c3 = 0; c3 < L; ++c3)
              r[(static_cast<size_t>(c1) * L + c3) * L + c2] = t[(static_cast<size_t>(c1) * L + c2) * L + c3];
        t.swap(r);
      }
      if (prec != FOCK_C64) {
        std::memcpy(img + in.vtab_off + static_cast<size_t>(q) * in.npts * 8, t.data(), t.size() * 8);
      } else {
        float* dst = reinterpret_cast<float*>(img + in.vtab_off) + static_cast<size_t>(q) * in.npts;
        for (size_t e = 0; e < t.size(); ++e) dst[e] = static_cast<float>(t[e]);
      }
    }
    std::vector<int32_t> qm(in.qmap.begin(), in.qmap.end());
    std::memcpy(img + in.qmap_off, qm.data(), qm.size() * sizeof(int32_t));
    std::memcpy(img + in.kw_off, in.kweight.data(), in.kweight.size() * sizeof(double));
    tables[i].clear();
  }
  for (const Group& g : groups)
    if (!g.parts.empty()) std::memcpy(img + g.off, g.parts.data(), g.parts.size() * sizeof(int32_t));
  for (size_t i = 0; i < p->fused_rounds.size(); ++i)
    std::memcpy(img + p->fused_rounds[i].pairs_off, round_pairs[i].data(), round_pairs[i].size() * sizeof(int32_t));
  for (int i = 0; i < n_inst; ++i) {
    const Instance& in = p->inst[i];
    if (in.n_ebatches == 0) continue;
    const size_t base = p->energy_batches[in.first_ebatch].pair_off;
    std::memcpy(img + base, elists[i].data(), elists[i].size() * sizeof(PairRef));
  }
  *out = p.release();
  return FOCK_OK;
}

}  // namespace fock
