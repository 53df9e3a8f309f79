/*
 * fock.h - C ABI of the MI355X screened exact-exchange library (libfock.so).
 *
 * The library applies the exact-exchange (Fock) operator of plane-wave
 * hybrid-functional DFT and evaluates the exchange energy and its gradient:
 *
 *   (V_x u)_{k,n} = - sum_{k',m} w_{k'} f_{k',m} u_{k',m} * IDFT[ v_q * DFT( conj(u_{k',m}) u_{k,n} ) ]
 *   E_x           = -1/2 sum_{k,n,k',m} w_k f_{k,n} w_{k'} f_{k',m} (Omega/N^2) sum_c v_q(c) |DFT(conj(u_{k',m}) u_{k,n})(c)|^2
 *
 * which is the paper's Eq. (2) (section "Our Implementation": four nested
 * loops, k-points outer, band pairs inner) written on the FFT grid, with the
 * screened kernel of HSE06 (paper, Introduction):
 *
 *   v_q(c) = 4 pi/|K|^2 (1 - exp(-|K|^2/(4 mu^2))),  K = sum_i (g_i(c) + q_i) b_i,  v(K=0) = pi/mu^2,
 *   q = k - k' (fractional, never folded), g_i(c) the integer representative of
 *   class c_i in (-N_i/2, N_i/2); for even N_i the Nyquist class c_i = N_i/2 takes
 *   the mean of v over both representatives +-N_i/2 (and over all 2^d
 *   combinations when d axes sit at Nyquist).
 *
 * Conventions
 *   lattice   rows a1, a2, a3 in bohr (Cartesian); Omega = |det|; b_i = 2 pi (A^-T) rows.
 *   grid      N1, N2, N3; orbital element j = (j1*N2 + j2)*N3 + j3 is the value at
 *             r = sum_i (j_i/N_i) a_i of the PERIODIC PART u of the Bloch orbital.
 *   DFT       forward unnormalised with exp(-2 pi i c.j/N); inverse carries 1/N.
 *   psi       per instance, complex (interleaved re, im), [nk][nbands][band_stride];
 *             element (k, n, j) at psi[(k*nbands + n)*band_stride + j].
 *   occ       per instance, device FP64 [nk][nbands] (f_{k,n}; fractional allowed).
 *   weights   w_k from the descriptor (host), default 1/nk.
 *
 * Precision: FOCK_C128 computes in complex128 throughout.  FOCK_C64 takes
 * complex64 orbitals and runs co-densities, FFTs, the kernel multiply and the
 * accumulate in FP32; the kernel table and the twiddles are built in FP64 and
 * rounded once, and per-pair energies are accumulated in FP64.
 *
 * Errors: every function returns a fock_status and never aborts.  Argument
 * errors are detected before any device work and leave outputs untouched.
 * fock_last_error() returns a thread-local description of the last non-OK
 * status.  Asynchronous device faults surface at the caller's next
 * synchronisation.
 *
 * Concurrency: all device work is enqueued on the plan's stream with no host
 * synchronisation.  A plan is not thread-safe; distinct plans are independent.
 */
#ifndef FOCK_H
#define FOCK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fock_plan_s* fock_plan_t; /* opaque, owned by the library */

typedef enum {
  FOCK_OK = 0,
  FOCK_ERR_ARG = 1,         /* invalid argument (NULL, out of range, non-finite, singular cell) */
  FOCK_ERR_UNSUPPORTED = 2, /* valid but not supported (grid axis not {2,3,5}-smooth or > 72)     */
  FOCK_ERR_NOMEM = 3,       /* host allocation failed, or workspace smaller than required          */
  FOCK_ERR_DEVICE = 4,      /* no usable GPU, or a HIP call / kernel launch failed                */
  FOCK_ERR_STATE = 5,       /* call out of order (e.g. apply before fock_set_workspace)           */
  /* not statuses: they make the type span int32, so any int32 a caller passes
   * where an enum of this header is expected is a value the library may read
   * (and reject) */
  FOCK_STATUS_RANGE_MIN_ = -2147483647 - 1,
  FOCK_STATUS_RANGE_MAX_ = 2147483647
} fock_status;

/* FOCK_C128: complex128 throughout.  FOCK_C64: complex64 orbitals, FP32
 * arithmetic (FP64 tables, twiddles and energy sums).  The two mixed
 * policies (the paper's "some of the FFTs in single precision") take
 * complex128 orbitals and outputs:
 *   FOCK_MIXED      co-densities and forward transforms in FP32; kernel
 *                   multiply, inverse transforms and accumulate in FP64
 *   FOCK_MIXED_INV  co-densities, forward transforms, kernel multiply and
 *                   pair energies in FP64; inverse transforms and the
 *                   accumulate in FP32 (added into the FP64 outputs in FP64)
 * Both need grids N1 x L x L with N1 and L each 24, 32, 36, 40, 48, 50, 54,
 * 60, 64 or 72 (FOCK_ERR_UNSUPPORTED otherwise). */
typedef enum {
  FOCK_C128 = 0,
  FOCK_C64 = 1,
  FOCK_MIXED = 2,
  FOCK_MIXED_INV = 3,
  FOCK_PRECISION_RANGE_MIN_ = -2147483647 - 1, /* not precisions (see fock_status) */
  FOCK_PRECISION_RANGE_MAX_ = 2147483647
} fock_precision;

/* One exchange problem ("instance").  All pointers are HOST pointers and are
 * only read during fock_plan. */
typedef struct {
  double lattice[9];       /* rows a1, a2, a3, bohr                                          */
  int32_t grid[3];         /* N1, N2, N3: each in [2, 72] with prime factors in {2, 3, 5}    */
  int32_t nk;              /* k-points of the orbital set, >= 1                              */
  const double* kfrac;     /* [nk][3] fractional (reciprocal-basis) coordinates              */
  const double* kweight;   /* [nk] finite, >= 0; NULL means 1/nk                             */
  int32_t npairs;          /* 0: every k' for every k; else the number of (k, k') below      */
  const int32_t* kpairs;   /* [npairs][2] (ik, ik'): the k' summed for output k              */
  int32_t nbands;          /* bands per k, >= 1                                              */
  int64_t band_stride;     /* elements between consecutive bands, >= N1*N2*N3                */
  double mu;               /* screening parameter in bohr^-1, finite and > 0                 */
} fock_desc;

/* Build a plan for n_inst independent instances of one precision (paper,
 * "Our Implementation": the band loops of every k-point pair go to the GPU).
 * Host work only: validates the descriptors, builds the FP64 kernel tables
 * v_q for every distinct transfer q, the twiddle tables, and the batched
 * schedule of band pairs.  `hip_stream` is a hipStream_t (NULL: default
 * stream).  On success *out owns host memory only; release with fock_destroy. */
fock_status fock_plan(const fock_desc* descs, int32_t n_inst, fock_precision prec, void* hip_stream,
                      fock_plan_t* out);

/* Schedule knobs (0 = library default).  Chosen by measurement with the
 * autotuner (paper_1111_0716_amd/autotune.py) or left at the defaults.
 *   acc_workgroups  three-pass path: target workgroups of the accumulate pass,
 *                   which sets the output block |O| = ceil(target / N1)
 *   tbuf_mb         three-pass path: pair-buffer budget (MiB), which bounds
 *                   |O| x |P| pairs per batch
 *   fused_split     whole-pair path: partner slices per output (1..4)
 *   no_fused        1: use the three-pass path for every grid
 *   no_pair_symmetry 1: three-pass register-line path transforms every
 *                   ordered pair; 0: with the full k-pair set it transforms
 *                   each unordered pair once, W_nm(k,k') = conj W_mn(k',k)
 *                   serving both (blocks of outputs x partners of about
 *                   sqrt(tbuf_mb / pair size) orbitals each; acc_workgroups
 *                   is then unused)
 *   fused_rounds    1: whole-pair path on 32^3 FP32 grids by unordered pairs
 *                   (one workgroup per pair, rounds of pairwise disjoint
 *                   pairs, one launch per round; needs a k-pair list closed
 *                   under swapping); 0: one workgroup per output
 * Defaults: acc_workgroups 2048, tbuf_mb 4096, 8192 for FOCK_C128 (or
 * $FOCK_TBUF_MB), fused_split
 * chosen to fill the compute units evenly, pair symmetry on (off with
 * $FOCK_NO_PAIR_SYMMETRY=1), fused_rounds off (on with $FOCK_FUSED_ROUNDS=1). */
typedef struct {
  int32_t acc_workgroups;
  int32_t tbuf_mb;
  int32_t fused_split;
  int32_t no_fused;
  int32_t no_pair_symmetry;
  int32_t fused_rounds;
} fock_tuning;

/* fock_plan with explicit schedule knobs (tuning may be NULL = defaults). */
fock_status fock_plan_tuned(const fock_desc* descs, int32_t n_inst, fock_precision prec, void* hip_stream,
                            const fock_tuning* tuning, fock_plan_t* out);

/* Bytes of device workspace the plan needs (tables, schedule, scratch). */
fock_status fock_workspace_size(fock_plan_t plan, size_t* bytes);

/* Attach caller-owned device memory of at least fock_workspace_size bytes
 * (256-byte aligned) and upload the tables on the plan stream.  The memory
 * must stay valid until fock_destroy or the next fock_set_workspace, which
 * also drops every recorded graph (they address the old workspace).
 * Returns FOCK_ERR_DEVICE when no GPU is usable. */
fock_status fock_set_workspace(fock_plan_t plan, void* dev_ptr, size_t bytes);

/* Change the stream later calls enqueue on. */
fock_status fock_set_stream(fock_plan_t plan, void* hip_stream);

/* V_x u for every (k, n) of every instance (the paper's FOCK_ACC,
 * "CPU Performance Analysis").  psi[i], vx_psi[i]: device pointers in the psi
 * layout of instance i (vx_psi may not alias psi); occ[i]: device FP64
 * [nk][nbands].  vmat: NULL, or per instance a device pointer to the band
 * overlap M[k][i][j] = Omega/N sum_j conj(u_{k,i}) (V_x u)_{k,j} in the
 * instance's complex precision, layout [nk][nbands][nbands].  The pointer
 * arrays themselves are host arrays of length n_inst. */
fock_status fock_apply(fock_plan_t plan, const void* const* psi, const double* const* occ, void* const* vx_psi,
                       void* const* vmat);

/* E_x of every instance (paper Eq. (2), negative sign: exchange lowers the
 * energy) into device FP64 ex[n_inst].  Per-pair sums are FP64 and reduced in
 * a fixed order, so FP64 results are bitwise reproducible. */
fock_status fock_energy(fock_plan_t plan, const void* const* psi, const double* const* occ, double* ex);

/* fock_apply (V_x psi into vx_psi, the overlap into vmat if not NULL) and
 * fock_energy (E_x into device FP64 ex[n_inst]) in one call.  Both are sums
 * over the same band pairs of Eq. (2): the apply kernels (whole-pair kernel,
 * or the pencil pass of the three-pass paths) also form each pair's energy
 * from the spectrum they have already transformed (FP64 partials, summed in
 * a fixed order), so no transform runs twice.
 * vx_psi and vmat come out bitwise equal to fock_apply's.  E_x agrees with
 * fock_energy's to rounding (bitwise reproducible from call to call, but
 * summed over ordered pairs where fock_energy folds swapped ones).
 * Errors as fock_apply, and FOCK_ERR_ARG if ex is NULL. */
fock_status fock_apply_energy(fock_plan_t plan, const void* const* psi, const double* const* occ,
                              void* const* vx_psi, void* const* vmat, double* ex);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * fock_apply_energy with the plan's workspace taken from a library-owned
 * device array of FOCK_STATIC_WORKSPACE_BYTES bytes instead of one attached
 * with fock_set_workspace (which need not have been called).  The array is a
 * static __device__ object, one per device, held until the process ends; the
 * call runs on the current device and allocates nothing (no hipMalloc, no
 * events, no graphs: launches are always eager).  It uploads the plan's
 * tables into the array with hipMemcpyAsync on the plan stream unless the
 * previous call on this device was made with the same plan.
 * Outputs as fock_apply_energy (vx_psi, vmat and ex bitwise equal to its).
 * Errors: FOCK_ERR_NOMEM, before any other check, when fock_workspace_size
 * exceeds FOCK_STATIC_WORKSPACE_BYTES; otherwise as fock_apply_energy.
 * Every call on one device shares that device's array: calls that overlap in
 * time on one device (other threads or streams) race and give wrong results. */
#define FOCK_STATIC_WORKSPACE_BYTES (64u << 20)
fock_status fock_apply_energy_static(fock_plan_t plan, const void* const* psi, const double* const* occ,
                                     void* const* vx_psi, void* const* vmat, double* ex);

/* Gradient of E_x: grad_psi[i] (psi layout, device) receives
 *   grad_ex[i] * scale * w_k * f_{k,n} * (V_x u)_{k,n}
 * with grad_ex a device FP64 array [n_inst] and scale a host number; the
 * co-densities are recomputed, never stored.  dE_x/d conj(u_{k,n}) is
 * scale = Omega/N; torch's complex-gradient convention is scale = 2 Omega/N
 * (instances of different Omega/N: fold it into grad_ex[i], scale = 1).
 * The formula differentiates Eq. (2)'s double sum when every listed k-pair
 * (k, k') has its swap (k', k) listed (the full set always does); a plan
 * with another explicit list returns FOCK_ERR_UNSUPPORTED before any other
 * check. */
fock_status fock_energy_backward(fock_plan_t plan, const void* const* psi, const double* const* occ,
                                 const double* grad_ex, double scale, void* const* grad_psi);

/* ---- plane-wave boundary and batched 3-D DFT ------------------------------
 * A plane-wave code keeps each orbital as coefficients c(G) on the cutoff
 * sphere |k+G|^2/2 < E_cut and scatters them to the FFT grid around the
 * band-pair loop, gathering the results back (paper, "CPU Performance
 * Analysis": the scatter/gather of FOCK_ACC).  With
 *   psi(r) = Omega^-1/2 sum_G c(G) exp(i (k+G).r),  u = psi exp(-i k.r):
 *   to the grid    u[j] = Omega^-1/2 sum_G c(G) exp(+2 pi i sum_d c_d j_d / N_d)
 *   to the sphere  d(G) = (Omega^1/2 / N) sum_j f[j] exp(-2 pi i sum_d c_d j_d / N_d)
 * where c_d = g_d mod N_d is the grid class of G; d(G) is the exact
 * coefficient of f on the sphere, so sum_G conj(c_m(G)) d_n(G) equals the
 * grid overlap Omega/N sum_j conj(u_m[j]) f_n[j] for band-limited u_m.
 *
 * Sphere of instance i, all device memory owned by the caller:
 *   gidx[i]     int32 [nk][npw_max[i]]: flat grid class (c1 N2 + c2) N3 + c3
 *               of slot p of k; slots must be distinct within a k
 *   npw[i]      int32 [nk]: slots in use per k (values above npw_max[i] are
 *               read as npw_max[i])
 *   npw_max[i]  host int32 >= 1, slots per k
 *   coefficients: plan precision, [nk][nbands][npw_max[i]]
 * Slots whose class lies outside [0, N) are skipped by the scatter and read
 * as zero by the gather; nothing outside the arrays is touched.
 * All calls are asynchronous on the plan stream; argument errors are
 * reported before any launch. */

/* u (psi layout, written in full) from sphere coefficients coef. */
fock_status fock_pw_to_grid(fock_plan_t plan, const void* const* coef, const int32_t* const* gidx,
                            const int32_t* const* npw, const int32_t* npw_max, void* const* psi);

/* Sphere coefficients coef_out[i] ([nk][nbands][npw_max], slots past npw[k]
 * written as zero) of the grid functions f[i] (psi layout).  f is
 * overwritten: it is transformed in place. */
fock_status fock_grid_to_pw(fock_plan_t plan, void* const* f, const int32_t* const* gidx, const int32_t* const* npw,
                            const int32_t* npw_max, void* const* coef_out);

/* V_x psi on the sphere: fock_pw_to_grid(coef -> psi_work),
 * fock_apply(psi_work -> vx_work), fock_grid_to_pw(vx_work -> vx_coef).
 * psi_work and vx_work are caller buffers in the psi layout (distinct);
 * on return psi_work holds u and vx_work its transformed V_x u. */
fock_status fock_apply_pw(fock_plan_t plan, const void* const* coef, const int32_t* const* gidx,
                          const int32_t* const* npw, const int32_t* npw_max, const double* const* occ,
                          void* const* psi_work, void* const* vx_work, void* const* vx_coef);

/* In-place unnormalised 3-D DFT of `count` grids of instance `inst`'s shape
 * in the plan precision: grid b starts at data + b * stride elements
 * (stride >= N), element j = (j1 N2 + j2) N3 + j3.
 *   sign -1: F(c) = sum_j f(j) exp(-2 pi i sum_d c_d j_d / N_d)
 *   sign +1: the same with exp(+...), no 1/N. */
fock_status fock_dft3(fock_plan_t plan, int32_t inst, int32_t sign, int64_t count, void* data, int64_t stride);

/* Counters of the plan: ordered band pairs per apply (N_k^2 N_b^2 summed over
 * instances, or per the k-pair lists), band-pair FFT round trips per apply,
 * FFT pairs per energy evaluation, and kernel launches per apply. */
fock_status fock_plan_stats(fock_plan_t plan, int64_t* ordered_pairs, int64_t* apply_fft_pairs,
                            int64_t* energy_fft_pairs, int64_t* apply_launches);

/* Kernel kinds for per-kernel timing. */
typedef enum {
  FOCK_K_PLANE = 0,          /* apply: co-density + forward FFT of axes 3, 2       */
  FOCK_K_PENCIL = 1,         /* apply: FFT of axis 1, x v_q, inverse FFT of axis 1 */
  FOCK_K_ACCUMULATE = 2,     /* apply: inverse FFT of axes 2, 3 + accumulate       */
  FOCK_K_ENERGY_PLANE = 3,   /* energy: co-density + forward FFT of axes 3, 2      */
  FOCK_K_ENERGY_PENCIL = 4,  /* energy: FFT of axis 1 + FP64 sum of v_q |P|^2      */
  FOCK_K_ENERGY_REDUCE = 5,  /* energy: fixed-order reductions                     */
  FOCK_K_OVERLAP = 6,        /* band overlap M                                     */
  FOCK_K_OTHER = 7,          /* zero fills, sums of partner-slice partial outputs  */
  FOCK_K_FUSED = 8,          /* apply: whole pair per workgroup (cubic <= 32^3)    */
  FOCK_K_ENERGY_FUSED = 9,   /* energy: whole pair per workgroup (cubic <= 32^3)   */
  FOCK_K_DFT = 10,           /* batched 3-D DFT passes (fock_dft3, plane waves)    */
  FOCK_K_PW = 11,            /* scatter / gather between cutoff sphere and grid    */
  FOCK_K_COUNT = 12
} fock_kernel_kind;

/* Per-kernel timing: when enabled, every launch is bracketed by HIP events on
 * the plan stream.  fock_profile_read waits for the recorded events, returns
 * the summed elapsed time and launch count of one kind since the last read of
 * that kind, and resets them.  Off by default (no events are recorded). */
fock_status fock_profile_enable(fock_plan_t plan, int enable);
fock_status fock_profile_read(fock_plan_t plan, int kind, double* total_ms, int64_t* launches);

/* Graph replay: when enabled, each of fock_apply, fock_apply_energy,
 * fock_energy and fock_energy_backward records its whole launch sequence (every instance,
 * every batch) into one HIP graph on first use and replays it with a single
 * graph launch while the argument pointers stay the same (a new pointer set
 * records a new graph).  Needs a plan stream other than the legacy default
 * stream (FOCK_ERR_STATE otherwise).  Results are identical to eager launches. */
fock_status fock_set_graph(fock_plan_t plan, int enable);

/* Call records.  When the environment variable FOCK_LOG names a file (or is
 * "stderr") at fock_plan, the plan records every call of fock_apply,
 * fock_apply_energy, fock_energy, fock_energy_backward, fock_pw_to_grid,
 * fock_grid_to_pw, fock_apply_pw and fock_dft3 (not fock_apply_energy_static,
 * which creates nothing): one JSON line per call with the status, the host
 * enqueue time, the device time between events recorded on the plan stream
 * around the call (device_ms -1 where no workspace was attached), and the
 * plan's counters; at fock_destroy, one summary line per call name (calls,
 * device time, ordered pairs per second).  Lines are written at fock_destroy,
 * or when 1024 records are pending (the host then waits for their events).
 * Records add two events per call to the stream and nothing else. */

/* Release the plan (host memory; the caller frees the workspace). NULL is a no-op. */
fock_status fock_destroy(fock_plan_t plan);

const char* fock_status_string(fock_status s);
const char* fock_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FOCK_H */
