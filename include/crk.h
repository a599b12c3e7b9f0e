/*
 * crk.h -- C ABI of the chiral rank-k multigrid library for MI355X (gfx950).
 *
 * The library sets up and applies the multigrid hierarchy of
 *   T. Whyte, A. Stathopoulos, E. Romero, "Chiral rank-k truncations for the
 *   multigrid preconditioner of Wilson fermions in lattice QCD" (LATTICE2024),
 * for the Wilson-Dirac operator D on a periodic 4-D lattice:
 *   setup (Sec. 2, Eqs. (1), (2) and (4); Sec. 3, Eqs. (5) and (6)):
 *     MR smoother on D psi_i ~ 0 for m' random vectors -> chiral split per block
 *     -> per-(block, chirality) SVD truncated to k left singular vectors = P
 *     (R = P^dag, gamma5 P = P sigma3) -> Galerkin coarse stencil D_c = R D P;
 *   solve (Sec. 2, last paragraph): flexible GCR preconditioned by a K-cycle.
 *
 * Conventions shared by every entry point
 *   - Site index s = x0 + L0*(x1 + L1*(x2 + L2*x3)); direction mu = 0..3 = x,y,z,t.
 *   - Spinor component index 3*spin + colour (chiral gamma basis,
 *     gamma5 = diag(1,1,-1,-1)); "host layout" of a field set is
 *     complex128 interleaved (re, im) [nrhs][V][12].
 *   - Gauge field: complex128 [V][4][3][3], entry U_mu(x)[a][b].
 *   - D psi(x) = (m0 + sum_mu w_mu) psi(x)
 *       - 1/2 sum_mu w_mu [(1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu)],
 *     w = (1, 1, 1, 1/xi), periodic boundaries.
 *   - Coarse degrees of freedom: (coarse site j, chirality alpha, i), i < k.
 *   - Every call returns CRK_OK (0) or a negative crk_status; on error
 *     crk_last_error() returns a thread-local message.  No call aborts or
 *     exits; no exception crosses the ABI.
 *   - Host buffers are owned by the caller and copied before the call
 *     returns.  Device ("_dev") buffers are owned by the caller and used in
 *     order on the given HIP stream (NULL = the null stream); the caller keeps
 *     them alive until that stream has completed.
 *   - Handles are not thread-safe; use one handle per thread or serialise.
 *     Destroying a lattice while hierarchies built on it live is allowed
 *     (reference counted).
 *   - Same inputs on the same GPU and build give bitwise-identical results.
 */
#ifndef CRK_H
#define CRK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct crk_lattice_s* crk_lattice_t; /* opaque, library-owned */
typedef struct crk_mg_s* crk_mg_t;           /* opaque; holds a reference on its lattice */

enum crk_status {
  CRK_OK = 0,
  CRK_EINVAL = -1,    /* invalid argument (message says which) */
  CRK_ENOMEM = -2,    /* device or host allocation failed */
  CRK_EHIP = -3,      /* HIP runtime error */
  CRK_ENOCONV = -4,   /* solver hit max_iter or broke down; x and info hold the best iterate */
  CRK_ESTATE = -5,    /* call out of order (e.g. solve before gauge load) */
  CRK_EBUSY = -6,     /* would exceed the device memory budget */
  CRK_EINTERNAL = -7  /* internal inconsistency (a bug) */
};

/* Precision forms.  FP64: every kernel in double.  FP32: float storage and
 * arithmetic.  FP16S: IEEE binary16 storage of x/s with an fp32 scale s per
 * (site, rhs) for spinors and per (coarse site, link) for coarse links; fine
 * links stored unscaled in fp16; all arithmetic accumulates in fp32. */
enum crk_form { CRK_FORM_FP64 = 0, CRK_FORM_FP32 = 1, CRK_FORM_FP16S = 2 };

/* Library version (major*10000 + minor*100 + patch). */
int crk_version(void);

/* Thread-local text of the last error ("" if none). */
const char* crk_last_error(void);

/* Name of device 0 (NUL-terminated, truncated to n bytes), its HBM size in
 * bytes and compute-unit count.  Any pointer may be NULL. */
int crk_device_info(char* name, int32_t n, int64_t* hbm_bytes, int32_t* n_cu);

/* Device memory.  Buffers the library frees (a destroyed hierarchy or
 * lattice, a solve's work space) are kept per device and handed to later
 * requests of about the same size (at most 1/8, or 2 MiB, larger), so that
 * setups repeated on one lattice shape (one per gauge configuration) do not
 * give back and re-obtain their hundreds of GB each time.  A freed buffer is
 * cached only after its device has finished all queued work.  When a device
 * allocation does not fit, that device's cache is given back first.  Memory
 * the library reports as free (server budgets, batch sizes) includes the
 * cache. */

/* *bytes receives the bytes cached on the current device.  CRK_EINVAL if
 * bytes is NULL. */
int crk_cached_memory_bytes(int64_t* bytes);

/* Give every cached buffer back to the HIP runtime, on every device the
 * library has used (waits for those devices).  Call before large allocations
 * outside the library in the same process. */
int crk_release_cached_memory(void);

/* ------------------------------------------------------------------ lattice */

/* Create the lattice on which the Wilson-Dirac operator D of Sec. 2 (the
 * operator of D x = b in Sec. 1) acts: extent dims[4] (each >= 2), periodic,
 * Wilson mass m0 and temporal anisotropy xi > 0 (the temporal hop weighted by
 * 1/xi).  Allocates the device gauge storage (all forms) and the
 * lexicographic neighbour table.  *out receives a library-owned handle
 * (free with crk_lattice_destroy).  CRK_EINVAL for an extent < 2 or xi <= 0,
 * CRK_ENOMEM if the device storage does not fit. */
int crk_create_lattice(const int32_t dims[4], double m0, double xi, crk_lattice_t* out);

/* Turn the Wilson-clover operator on (c_sw != 0) or off (c_sw = 0).  The
 * paper's ensembles are clover actions (Sec. 4, both ensembles); its site term
 * becomes (m0 + sum_mu w_mu) 1 + C(x) with
 *   C(x) = -(c_sw/2) sum_{mu<nu} w_mu w_nu sigma_{mu nu} (x) F_{mu nu}(x),
 *   sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu],
 *   F_{mu nu}(x) = [(Q - Q^dag) - tr(Q - Q^dag)/3] / (8i),
 * Q_{mu nu}(x) the four plaquettes of the (mu, nu) plane at x.  C(x) is two
 * Hermitian 6 x 6 blocks per site (one per chirality of Eq. (2)), so
 * gamma5 D gamma5 = D^dag still holds.  May be called before or after
 * crk_load_gauge (the blocks are computed on the device from the FP64 links
 * when both are set).  A hierarchy keeps the clover blocks of its lattice at
 * the time of crk_mg_setup.  CRK_EINVAL for a NULL handle or a non-finite c_sw. */
int crk_lattice_set_clover(crk_lattice_t lat, double c_sw);

/* Upload the SU(3) gauge links U_mu(x) that define D (Sec. 2): host
 * complex128 [V][4][3][3] (entry [x][mu][a][b] = U_mu(x)[a][b]),
 * n_doubles = 2*V*36.  Copied before the call returns and converted on the
 * device to every precision form.  CRK_EINVAL if n_doubles does not match
 * the lattice or U is NULL. */
int crk_load_gauge(crk_lattice_t lat, const double* U, int64_t n_doubles);

/* Apply the Wilson-Dirac operator D of Sec. 2 (formula above) to nrhs
 * host-layout fields (complex128 [nrhs][V][12]) in the given form; in and
 * out are caller-owned host pointers and may not alias.  FP32/FP16S round
 * the input to the form, apply, and widen the result.  nrhs = 0 is a no-op.
 * CRK_ESTATE before crk_load_gauge, CRK_EINVAL for a bad form, nrhs < 0 or
 * NULL pointers. */
int crk_dirac_apply(crk_lattice_t lat, int32_t form, const double* in, double* out, int32_t nrhs);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation as crk_dirac_apply, staged through a fixed device array of
 * crk_dirac_apply_noalloc_max_bytes() bytes (64 MiB) that the library holds
 * on every GPU it runs on until the process ends, instead of three device
 * buffers allocated per call.  It calls no hipMalloc, hipFree or allocating
 * library routine.  The staging a call needs, 16*12*V*nrhs bytes plus twice
 * crk_field_bytes(lat, form, nrhs) (each rounded up to 256), must fit in the
 * array; larger calls return CRK_EINVAL and do nothing.  Results are bitwise
 * those of crk_dirac_apply.  All calls on one GPU share its array: calls that
 * overlap on one GPU (several host threads) race and must be serialised by
 * the caller.  Other errors as crk_dirac_apply. */
int crk_dirac_apply_noalloc(crk_lattice_t lat, int32_t form, const double* in, double* out, int32_t nrhs);
int64_t crk_dirac_apply_noalloc_max_bytes(void);

/* Device-resident variant on the lattice's native device layout of the form
 * (site-vectorised): with Vp = V rounded up to a multiple of 64, entry
 * (rhs r, component c, lexicographic site s) is complex element
 * (r*Vp + 64*floor(s/64))*12 + 64*c + s%64 of the buffer (FP64 double2,
 * FP32 float2, FP16S half2 of x/scale followed by the float scales [nrhs][Vp]
 * at byte offset nrhs*12*Vp*4).  in/out are device pointers; padding sites
 * are neither read nor written. */
int crk_dirac_apply_dev(crk_lattice_t lat, int32_t form, const void* in, void* out, int32_t nrhs,
                        void* hip_stream);

/* Bytes of one native device field set of nrhs right-hand sides in a form. */
int64_t crk_field_bytes(crk_lattice_t lat, int32_t form, int32_t nrhs);

/* Convert between host-layout complex128 device buffers ([nrhs][V][12]) and
 * the native device layout of a form (both device pointers). */
int crk_field_import_dev(crk_lattice_t lat, int32_t form, const void* host_layout_dev, void* native_dev,
                         int32_t nrhs, void* hip_stream);
int crk_field_export_dev(crk_lattice_t lat, int32_t form, const void* native_dev, void* host_layout_dev,
                         int32_t nrhs, void* hip_stream);

/* Site-indexed integer maps of the lattice (bit-exact with the definitions):
 * CRK_MAP_NEIGHBOR  int32 [V][8]  (column 2mu: x+mu, 2mu+1: x-mu)        */
enum crk_map { CRK_MAP_NEIGHBOR = 0 };
int crk_lattice_get_map(crk_lattice_t lat, int32_t what, void* out, int64_t n_bytes);

void crk_lattice_destroy(crk_lattice_t lat);

/* ------------------------------------------------------------------ setup */

#define CRK_MAX_LEVELS 3

typedef struct {
  int32_t n_levels;                    /* 2 or 3 (levels including the fine one) */
  int32_t m_prime[CRK_MAX_LEVELS];     /* test vectors per coarsening step (<= 128) */
  int32_t k[CRK_MAX_LEVELS];           /* kept per chirality; multiple of 8 in [8, 32], <= m', <= N_r */
  int32_t block[CRK_MAX_LEVELS][4];    /* block extent per coarsening step */
  int32_t n_smooth[CRK_MAX_LEVELS];    /* MR sweeps on D psi ~ 0 per step */
  int32_t setup_form;                  /* precision of the setup smoother (FP64 or FP32) */
  int32_t normalize;                   /* 1: psi_i <- psi_i/||psi_i|| before the SVD */
  uint64_t seed;                       /* device random vectors when init_vectors is NULL */
  const double* init_vectors[CRK_MAX_LEVELS]; /* optional host complex128 [m'][V_l][N_l] */
  int32_t smooth_chunk;                /* fine-level smoother: vectors per launch, 0 = all m' unless
                                          device memory is short (then halved until r, q fit) */
  int32_t svd_batch;                   /* blocks per SVD batch, 0 = all unless the work space would
                                          exceed a quarter of the free device memory */
  int32_t coarse_init;                 /* 1: a coarsening step l >= 1 without init_vectors[l] starts
                                          from the coarse test vectors of step l-1 instead of random
                                          vectors: per block and chirality Sigma_k V_k^dag of the
                                          truncated SVD (Sec. 3, after Eq. (5)), i.e. P^dag of the
                                          first m'_l (normalised) test vectors of step l-1, computed
                                          on the device by the restriction in the setup form.
                                          Requires m'_l <= m'_{l-1}.  0 (default): random vectors. */
  int32_t smooth_defer;                /* fine-level smoother: sweeps whose psi updates share one pass
                                          over psi (each sweep still forms its residual, into a ring
                                          of smooth_defer + 1 fields); 1 = every sweep updates psi,
                                          2..8 as given (at most n_smooth), 0 (default) = the
                                          largest of 8, 4, 2 (at most n_smooth) for
                                          which the ring and q take at most 30 % of the free device
                                          memory, else 1.  The hierarchy is bitwise the same for
                                          every value. */
} crk_mg_params;

/* Fill p with defaults (two levels, m'=48, k=24, 4^4 blocks, 20 sweeps, FP32 smoother). */
void crk_mg_params_default(crk_mg_params* p);

/* Build the hierarchy (Sec. 2-3).  Blocking must divide every level's extent.
 * Blocks until the setup is complete.  Per-stage device times are available
 * through crk_mg_get_timing. */
int crk_mg_setup(crk_lattice_t lat, const crk_mg_params* params, crk_mg_t* out);

/* ------------------------------------------------------------------ solve */

typedef struct {
  /* in */
  double tol;          /* relative TRUE residual ||b - D x|| / ||b|| (FP64) */
  int32_t max_iter;    /* outer iterations */
  int32_t form;        /* K-cycle precision (the outer GCR is always FP64) */
  int32_t restart;     /* outer GCR restart length (<= 32) */
  double tau;          /* inner relative tolerance of the coarse solves */
  int32_t inner_maxit; /* iterations of an intermediate-level coarse solve */
  int32_t coarsest_maxit; /* iterations of the coarsest solve */
  int32_t nu_post;     /* MR post-smoothing steps */
  int32_t post_defer;  /* fine-level post-smoothing steps whose e updates share one pass over e
                          (each step still forms its residual, into a ring of post_defer + 1
                          fields): 1 = every step updates e, 2..8 as given (at most nu_post),
                          0 (default) = min(nu_post, 4).  The solve is bitwise the same for
                          every value. */
  /* out (maxima over right-hand sides) */
  int32_t iters;                         /* outer iterations */
  int32_t level_iters[CRK_MAX_LEVELS];   /* total iterations per level */
  double true_rel_resid;                 /* max over RHS */
  double seconds;                        /* device wall time of the solve */
} crk_solve_info;

void crk_solve_info_default(crk_solve_info* info);

/* Solve D x = b (Sec. 1) for nrhs host-layout right-hand sides (complex128
 * [nrhs][V][12], caller-owned, copied in and out) with flexible GCR
 * preconditioned by the K-cycle of the hierarchy (Sec. 2, last paragraph),
 * to the relative TRUE residual info->tol in FP64.  Blocks until done.
 * CRK_ENOCONV when max_iter is reached (x and info hold the best iterate),
 * CRK_EINVAL for nrhs outside [1, 64], tol <= 0 or NULL pointers. */
int crk_mg_solve(crk_mg_t mg, const double* b, double* x, int32_t nrhs, crk_solve_info* info);

/* Same with device buffers in host layout (complex128 [nrhs][V][12]), stream ordered;
 * returns after the solve has completed on the stream (the outer loop reads
 * residual norms every iteration). */
int crk_mg_solve_dev(crk_mg_t mg, const void* b_dev, void* x_dev, int32_t nrhs, void* hip_stream,
                     crk_solve_info* info);

/* Per-RHS outer iteration counts and true residuals of the last solve. */
int crk_mg_last_solve_rhs(crk_mg_t mg, int32_t* iters, double* true_rel_resid, int32_t nrhs);

/* Per-RHS time to solution of the last solve (Sec. 2, last paragraph: the
 * outer flexible GCR): host wall seconds from the start of the solve to the
 * outer iteration at which that right-hand side's true residual was verified
 * (or it stopped).  nrhs must equal the last solve's; CRK_EINVAL otherwise. */
int crk_mg_last_solve_rhs_seconds(crk_mg_t mg, double* seconds, int32_t nrhs);

/* ------------------------------------------------------------------ inspection */

enum crk_mg_what {
  CRK_GET_P = 0,        /* complex128 [d][2][N_r][k]   prolongator blocks of level l (rows h*l+c') */
  CRK_GET_SIGMA = 1,    /* double     [d][2][min(m',N_r)] singular values, descending */
  CRK_GET_X = 2,        /* complex128 [Vc][2k][2k]     coarse site term of level l+1 */
  CRK_GET_YP = 3,       /* complex128 [4][Vc][2k][2k]  coarse hop Y_{+mu} */
  CRK_GET_YM = 4,       /* complex128 [4][Vc][2k][2k]  coarse hop Y_{-mu} */
  CRK_GET_VECTORS = 5,  /* complex128 [m'][V_l][N_l]   smoothed, normalised test vectors */
  CRK_GET_BLOCK_MAP = 6,/* int32 [V_l][2]  (block j, local index l) of every site */
  CRK_GET_DEVICE_ORDER = 7 /* int32 [V_l]  device position of every site */
};
/* Copy a hierarchy quantity of step l (0 = fine -> first coarse) to host memory
 * of exactly n_bytes (caller-owned): the prolongator blocks U_k of Sec. 3,
 * Eqs. (5)-(6), their singular values, the Galerkin links of D_{l+1} = R D_l P
 * (Sec. 2, Eq. (4)), the smoothed test vectors of Eq. (1), and the block maps
 * of the domains Lambda_j (Sec. 2).  CRK_EINVAL for an unknown quantity, a
 * level out of range or n_bytes != crk_mg_get_bytes. */
int crk_mg_get(crk_mg_t mg, int32_t level, int32_t what, void* out, int64_t n_bytes);

/* Bytes a quantity of crk_mg_get needs. */
int64_t crk_mg_get_bytes(crk_mg_t mg, int32_t level, int32_t what);

/* Device timing of the last setup, seconds:
 * 0 total, 1 smoother, 2 split+SVD+P, 3 Galerkin, 4 average dslash launch
 * inside the smoother, 5 number of those launches. */
int crk_mg_get_timing(crk_mg_t mg, int32_t level, double* out6);

/* Apply the operator of level l in a form to host complex128 vectors
 * [nrhs][V_l][N_l]: l = 1..n_levels-1 the Galerkin coarse operator (2k
 * components per coarse site), l = 0 the fine Wilson operator through the
 * hierarchy's own kernels and block-major site order, i.e. the operator the
 * smoother and the K-cycle apply (FP16S at level 0: FP16 spinors with one
 * scale per site and RHS and half links, as the FP16S form's post-smoother
 * uses them; the input is rounded to that storage). */
int crk_mg_coarse_apply(crk_mg_t mg, int32_t level, int32_t form, const double* in, double* out,
                        int32_t nrhs);

/* Device-resident variant of crk_mg_coarse_apply (paper, Sec. 2, Eq. (4) for
 * l >= 1; the Wilson operator for l = 0) on the hierarchy's own device layout
 * of level l, the one the smoother and the K-cycle use, for callers that keep
 * fields on the device and for timing the operator kernels:
 *   l = 0: the native layout of crk_dirac_apply_dev with every site at its
 *          CRK_GET_DEVICE_ORDER position (block-major) instead of its
 *          lexicographic index (FP16S: half2 spinors plus one float scale
 *          per site and RHS, after the data);
 *   l >= 1: entry (rhs r, component c, device site p) at complex element
 *          (p*N_l + c)*nrhs + r (FP64 double2; FP32 and FP16S float2, the
 *          FP16S form keeping FP16 links only).
 * in and out are device pointers of crk_mg_field_bytes(mg, l, form, nrhs)
 * bytes each and may not alias; the work is ordered on hip_stream (NULL: the
 * default stream) and the call returns without waiting.  nrhs = 0 is a no-op;
 * CRK_EINVAL for a bad level, form or pointer. */
int crk_mg_apply_dev(crk_mg_t mg, int32_t level, int32_t form, const void* in, void* out, int32_t nrhs,
                     void* hip_stream);

/* Bytes of nrhs fields of level l in a form for crk_mg_apply_dev; -1 on bad arguments. */
int64_t crk_mg_field_bytes(crk_mg_t mg, int32_t level, int32_t form, int32_t nrhs);

/* Restrict fine-level (level l) host vectors [nrhs][V_l][N_l] to level l+1, and prolong back. */
int crk_mg_restrict(crk_mg_t mg, int32_t level, int32_t form, const double* in, double* out, int32_t nrhs);
int crk_mg_prolong(crk_mg_t mg, int32_t level, int32_t form, const double* in, double* out, int32_t nrhs);

/* Device bytes held by the hierarchy plus the solver work space for nrhs
 * right-hand sides in the given form (used for admission). */
int64_t crk_mg_footprint_bytes(crk_mg_t mg, int32_t nrhs, int32_t form);

void crk_mg_destroy(crk_mg_t mg);

/* ------------------------------------------------------------------ serving
 * Continuously batched solve server (not in the paper: a serving loop around
 * the solve above).  Hierarchies stay resident; every registered lattice has a
 * FIFO of requests and up to max_lanes lanes.  A lane is one outer MG-GCR
 * solver with slots_per_lane RHS slots, its own buffers, HIP stream and host
 * thread.  Between two outer iterations a lane hands back finished RHS and
 * admits queued requests into its free slots while its other RHS keep
 * iterating.  A lane is opened when queued RHS exceed the free slots of the
 * lattice's lanes and the lane's buffers fit in the HBM budget; idle lanes
 * beyond a lattice's last close after idle_ms and return their memory.  Each
 * RHS follows exactly the iteration it would follow alone (every kernel treats
 * each RHS on its own), so results do not depend on the traffic mix.
 *
 * Threading: every call is thread-safe.  The caller keeps b and x of a request
 * alive and untouched until crk_server_wait has returned for it.  A hierarchy
 * registered with a server must not be solved through crk_mg_solve* at the
 * same time; the server holds a reference on it, so crk_mg_destroy may be
 * called at any time. */
typedef struct crk_server_s* crk_server_t;

typedef struct {
  int64_t hbm_budget_bytes; /* device memory the lanes may use; <= 0: 80% of the free memory at creation */
  int32_t slots_per_lane;   /* RHS slots per lane = the largest request size, 1..64 (default 12) */
  int32_t max_lanes;        /* lanes per lattice, 1..16 (default 4) */
  int32_t idle_ms;          /* an idle lane that is not its lattice's last closes after this long (default 200) */
  crk_solve_info solve;     /* tol, max_iter, form, restart, tau, inner_maxit, coarsest_maxit, nu_post, post_defer */
} crk_server_params;

typedef struct {
  int32_t status;           /* CRK_OK, CRK_ENOCONV or the error of the lane that ran it */
  int32_t lattice, nrhs;
  int32_t lane;             /* lane id within the lattice */
  int32_t joined;           /* 1 if admitted while other RHS were iterating in that lane */
  int32_t iters;            /* outer iterations (max over the request's RHS) */
  int32_t level_iters[CRK_MAX_LEVELS];
  double true_rel_resid;    /* max over the request's RHS, FP64 */
  double t_submit, t_admit, t_done; /* seconds since the server was created (steady clock) */
} crk_request_info;

typedef struct {
  int64_t submitted, completed, failed, joins;
  int64_t lanes_opened, lanes_closed, max_concurrent_lanes;
  int64_t bytes_in_use, peak_bytes, budget_bytes;
} crk_server_stats;

void crk_server_params_default(crk_server_params* p);
int crk_server_create(const crk_server_params* p, crk_server_t* out);
/* Register a hierarchy; *lattice_id receives its index.  CRK_ENOMEM if one lane does not fit the budget. */
int crk_server_add(crk_server_t srv, crk_mg_t mg, int32_t* lattice_id);
/* Queue nrhs right-hand sides b (complex128 host layout [nrhs][V][12]); x receives the solutions.
 * Returns at once; *request_id identifies the request. */
int crk_server_submit(crk_server_t srv, int32_t lattice_id, const double* b, double* x, int32_t nrhs,
                      uint64_t* request_id);
/* Wait for a request (timeout_s < 0: no limit).  CRK_EBUSY on timeout (the request stays queued),
 * otherwise the request's status; info is filled and the request id is released. */
int crk_server_wait(crk_server_t srv, uint64_t request_id, double timeout_s, crk_request_info* info);
int crk_server_get_stats(crk_server_t srv, crk_server_stats* out);
/* Device bytes one lane of a registered lattice takes from the budget (solver buffers + staging). */
int64_t crk_server_lane_bytes(crk_server_t srv, int32_t lattice_id);
/* Finish every queued request, stop the lanes and free the server. */
void crk_server_destroy(crk_server_t srv);

#ifdef __cplusplus
}
#endif

#endif /* CRK_H */
