// Internal declarations of the gfx950 ABD library (not part of the ABI).
#pragma once
#include <initializer_list>

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "../../include/abd.h"

// ------------------------------------------------------------ context ----

struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
};

// Per-kernel timing with HIP events (enabled by abd_profile): event pairs
// are recorded around instrumented launches and resolved at the next host
// synchronisation, so profiling adds no synchronisation of its own.
struct KStat {
  double ms = 0.0;
  int64_t launches = 0, units = 0;
};
// Host-side events of the same table (workspace growth, graph captures):
// wall time on the host, counted while profiling is on.
struct abd_ctx;
struct HostTimer {
  abd_ctx *ctx;
  const char *name;
  int64_t units;
  std::chrono::steady_clock::time_point t0;
  HostTimer(abd_ctx *c, const char *n, int64_t u) : ctx(c), name(n), units(u), t0(std::chrono::steady_clock::now()) {}
  ~HostTimer();
};
struct PendingEv {
  hipEvent_t a, b;
  std::string name;
  int64_t units;
};

// joint tables of a scene (abd_joint.hip), rebuilt when the key changes
struct JointTables {
  std::vector<uintptr_t> key;
  int32_t *joff = nullptr, *jent = nullptr, *run_off = nullptr, *run_joint = nullptr, *pairs = nullptr;
  int n_runs = 0;
  int64_t n_pairs = 0;  // joints between two free bodies (point-triangle-shaped pairs for the pattern)
};

struct abd_ctx {
  int device = 0;
  // launch shapes (abd_tune_set / abd_autotune); none changes a result
  abd_tune tune = {16, 1, 256, 1024, 256, 16, 64, 1};
  JointTables joints;
  std::string err;
  std::map<std::string, DevBuf> bufs;
  // buffers replaced by a larger one, freed after the next point where the
  // device is idle (ws_collect), so that growing never waits for the stream
  std::vector<void *> ws_old;
  size_t ws_old_bytes = 0;
  // counts of the last call per buffer family, used as capacities of the
  // next one (checked when the counts are read)
  std::map<std::string, int64_t> cap_hint;
  void *pinned = nullptr;  // small host staging area for scalar readbacks
  size_t pinned_bytes = 0;
  void *pinned_nt = nullptr;  // per-scene staging of the Newton driver
  void *pinned_nt_d = nullptr;  // (mapped: its device address)
  size_t pinned_nt_bytes = 0;
  // coherent mapped host memory that kernels write counts into directly
  // (read after the stream synchronises; allocated once, so its address
  // can be baked into captured graphs)
  int64_t *mirror_h = nullptr, *mirror_d = nullptr;
  // look-back status words and the tag of the last launch, one set per
  // stream that scans (the call's stream, the auxiliary stream): launches on
  // one stream run in order and each takes a new tag
  struct LbState {
    unsigned long long *status = nullptr;
    int64_t words = 0;
    unsigned int tag = 0;
  } lb[2];
  // auxiliary stream (default priority) for work that overlaps the call's
  // stream inside one call, and the events that order the two
  hipStream_t aux_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev[8] = {};
  bool profiling = false;
  bool count_box_tests = false;  // (abd_profile mode 2)
  std::map<std::string, KStat> kstats;
  // the device sums of box tests (workspace "prof_box_tests") restart at
  // the next profiled candidates call
  bool prof_box_tests_clear = true;
  bool prof_pcg_clear = true;  // (likewise the solver's algorithmic bytes)
  std::vector<PendingEv> pending;
  std::vector<hipEvent_t> ev_pool;
  // captured PCG iterations (short and long replays), re-captured when any
  // argument changes; pcg_hint: iterations of the last solve
  hipGraphExec_t pcg_exec[2] = {nullptr, nullptr};
  std::vector<uintptr_t> pcg_key[2];
  // one-kernel PCG replays of 2, 4, ..., 256 iterations (slot k: 2^(k+1)),
  // captured when first needed
  hipGraphExec_t cg_exec[8] = {};
  std::vector<uintptr_t> cg_key[8];
  int pcg_hint = 0;
  int ls_hint = 0;  // line-search halvings of the last Newton iteration
  hipStream_t capture_stream = nullptr;
  // friction lagged at the start of the current time step (set by
  // abd_friction_begin_step, used by the Newton iterations while set)
  bool fr_set = false;
  // adaptive barrier stiffness: per-scene kappa (device [S], workspace
  // "kappa_sc") while abd_time_step runs with kappa_adaptive; null otherwise,
  // and then every kernel takes the scalar kappa_b
  double *kappa_sc = nullptr;
  // dense off-diagonal pattern: the scene arrays its layout was read from,
  // and the total bytes of the per-scene pair matrices
  std::vector<uintptr_t> od_key;
  int64_t od_total = 0;
  // tables that depend only on a scene's body-to-scene map (per workspace
  // name: the scene key and the buffer they were written to)
  std::map<std::string, std::vector<uintptr_t>> scene_tables;
  int64_t fr_n_pt = 0, fr_n_ee = 0;
  // swept candidates of the last accepted Newton step (the segment holds the
  // new iterate, so its static candidates are a subset of these)
  bool sw_valid = false;
  const int32_t *sw_pt = nullptr, *sw_ee = nullptr;
  int64_t sw_n_pt = 0, sw_n_ee = 0;
};

// instrumentation: prof_begin returns an event recorded before the launch
// (or null when profiling is off); prof_end records the end event and
// queues the pair; prof_flush resolves queued pairs (call after a sync).
hipEvent_t prof_begin(abd_ctx *ctx, hipStream_t s);
void prof_end(abd_ctx *ctx, hipEvent_t a, const char *name, int64_t units, hipStream_t s);
void prof_flush(abd_ctx *ctx);
// the profile's device total of the solver's algorithmic bytes ("pcg_round"
// units), cleared on first use after a reset
int prof_pcg_bytes(abd_ctx *ctx, unsigned long long **acc, hipStream_t s);

#define ABD_TRY(expr)                 \
  do {                                \
    int _rc = (expr);                 \
    if (_rc != ABD_OK) return _rc;    \
  } while (0)

int abd_fail(abd_ctx *ctx, int code, const char *fmt, ...);
int abd_hip_check(abd_ctx *ctx, hipError_t e, const char *what);
#define HIP_TRY(ctx, expr) ABD_TRY(abd_hip_check((ctx), (expr), #expr))

// Growable named device workspace.  A grown buffer is new, zeroed memory
// (cleared on `stream`); the one it replaces stays allocated until
// ws_collect, so queued kernels may still read it.
int ws_get(abd_ctx *ctx, const char *name, size_t bytes, void **out, hipStream_t stream);
// frees the replaced buffers (synchronises the device when there are any)
int ws_collect(abd_ctx *ctx);
// true when workspace `buf` still holds the table `name` computed for the
// scene's body-to-scene map (same map, counts and buffer); otherwise
// records it as computed now (the caller then writes it)
bool scene_table_cached(abd_ctx *ctx, const abd_scene *sc, const char *name, const void *buf);
template <class T>
int ws(abd_ctx *ctx, const char *name, size_t count, T **out, hipStream_t stream) {
  return ws_get(ctx, name, count * sizeof(T) + 256, reinterpret_cast<void **>(out), stream);
}
int pinned_get(abd_ctx *ctx, size_t bytes, void **out);
// separate staging area of the Newton driver (never used by the operations
// it calls, so its contents survive them); coherent mapped host memory, so
// kernels may also write it through *dev (may be NULL)
int pinned_get_nt(abd_ctx *ctx, size_t bytes, void **out, void **dev = nullptr);
// MIRROR_SLOTS int64 of coherent mapped host memory: host and device
// addresses.  Fixed slots per use; a slot is read right after the
// synchronisation that follows its writer.
constexpr int MIRROR_SLOTS = 64;
constexpr int MIR_BROAD = 0;     // 8 slots: broad-phase totals
constexpr int MIR_OFFDIAG = 8;   // 1 slot: off-diagonal key count
constexpr int MIR_COMPACT = 12;  // 2 slots: compaction total and PT count
constexpr int MIR_PCG = 16;      // 2 slots (4 ints): PCG iteration state
int mirror_get(abd_ctx *ctx, int64_t **host, int64_t **dev);
// Counts that a scan wrote to mapped host memory are -1 when its look-back
// failed; a host that sizes buffers from them calls this first.
int mirror_counts_ok(abd_ctx *ctx, std::initializer_list<int64_t> counts, const char *where);
// at least `words` zero-or-stale look-back status words and a new tag for
// one launch (abd_lookback.h)
int lb_prepare(abd_ctx *ctx, int64_t words, unsigned long long **status, unsigned int *tag, hipStream_t s);

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// ---------------------------------------------------- device-wide scan ----
// Exclusive prefix sum of n int64 values (in != out allowed, or in-place);
// total (device, may be NULL) receives the sum.
// host (device address of mapped host memory, may be null) receives
// host[0] = total and, for 0 <= split <= n, host[1] = out[split] (the
// total when split == n); both written by the scan's own kernels.
int scan_exclusive_i64(abd_ctx *ctx, const int64_t *in, int64_t *out, int64_t n, int64_t *total, hipStream_t s,
                       int64_t *host = nullptr, int64_t split = -1);
// Stable sort of (key, value) pairs by key (keys in [0, 2^key_bits));
// *keys and *vals then point to the sorted arrays (context workspace, valid
// until the next sort).
int sort_pairs_u32(abd_ctx *ctx, uint32_t **keys, uint32_t **vals, int64_t n, int key_bits, hipStream_t s);

// ----------------------------------------------------- pair records ----
// Local record of a pair whose 12x12 Hessian and 12-gradient are assembled
// into body blocks (barrier and friction share the assembly).
struct alignas(16) PairInfo {
  int32_t vid[4];
  int32_t body[2];  // body of slot 0 and of slot 3
  int32_t is_ee;
  int32_t pad;
};

// Lagged friction pairs: PT pairs then EE pairs, per pair (in that combined
// order) lambda [n], tangent basis T [n][6] (columns t1, t2), closest-point
// weights w [n][4]; xt the vertex positions they were lagged at.
struct FrictionSet {
  const int32_t *pt = nullptr, *ee = nullptr;
  int64_t n_pt = 0, n_ee = 0;
  const double *lam = nullptr, *T = nullptr, *w = nullptr, *xt = nullptr;
  double mu = 0.0, eps = 0.0;
  int64_t n() const { return n_pt + n_ee; }
};

// ------------------------------------------------- internal operations ----
// (shared by the ABI wrappers and the Newton driver)
// (skip_scene, device, may be NULL: vertices of the scenes it marks keep x)
int op_vertex_map(abd_ctx *ctx, const abd_scene *sc, const double *q, double *x, hipStream_t s,
                  const uint8_t *skip_scene = nullptr);
// candidates; sub-scenes s with skip_scene[s] != 0 (device, may be NULL)
// contribute none
int op_candidates(abd_ctx *ctx, const abd_scene *sc, const double *x0, const double *x1, double inflate,
                  int32_t **pt, int64_t *n_pt, int32_t **ee, int64_t *n_ee, const char *tag, hipStream_t s,
                  const uint8_t *skip_scene = nullptr);
// candidates at x (static, inflate) taken from the swept candidates
// (spt, see) of a segment that contains x: equal to op_candidates at x
int op_candidates_within(abd_ctx *ctx, const abd_scene *sc, const double *x, double inflate, const int32_t *spt,
                         int64_t n_spt, const int32_t *see, int64_t n_see, int32_t **pt, int64_t *n_pt, int32_t **ee,
                         int64_t *n_ee, const char *tag, hipStream_t s);
// Row structure of a key list (keys sorted by (row, column), row < column)
// for the block solvers: lo_beg[b] (nb + 1) the first key with row b,
// hi_beg[b] (nb + 1) the first entry of body b in tperm, the key indices
// ordered by (column, row).
struct KeyPattern {
  const int64_t *lo_beg = nullptr, *hi_beg = nullptr;
  const uint32_t *tperm = nullptr;
  bool valid = false;
};
// pattern of the pairs (pt, ee) and, when given, the extra pairs (pt2, ee2)
// and point-triangle-shaped pairs pt3 (joints); pat (may be NULL) receives
// the keys' row structure when the dense path builds it (else pat->valid =
// false)
// (defer: only enqueue; *n_keys is then read by op_offdiag_count after the
// caller has synchronised s)
int op_offdiag(abd_ctx *ctx, const abd_scene *sc, const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee,
               int32_t **keys, int64_t *n_keys, const char *tag, hipStream_t s, const int32_t *pt2 = nullptr,
               int64_t n_pt2 = 0, const int32_t *ee2 = nullptr, int64_t n_ee2 = 0, KeyPattern *pat = nullptr,
               const int32_t *pt3 = nullptr, int64_t n_pt3 = 0, bool defer = false);
int op_offdiag_count(abd_ctx *ctx, int64_t *n_keys);
// the auxiliary stream and its events (created on first use)
int aux_stream_get(abd_ctx *ctx, hipStream_t *aux);
// joints: the scene's tables (NULL when it has none); per-body energy
// (added to e_items + t estride for trial t, q at q + t qstride), gradient
// and diagonal blocks, times c = kappa_j w; off-diagonal blocks into off
int joint_tables(abd_ctx *ctx, const abd_scene *sc, JointTables **out, hipStream_t s);
int op_joint_body(abd_ctx *ctx, const abd_scene *sc, double c, const double *q, int n_trials, int64_t qstride,
                  double *e_items, int64_t estride, double *grad, double *diag, hipStream_t s);
int op_joint_off(abd_ctx *ctx, const abd_scene *sc, double c, const int32_t *keys, int64_t n_keys, double *off,
                 hipStream_t s);
// barrier (and, when fr is given, the lagged friction of fr) energy,
// gradient and Hessian blocks, assembled in one pass.  Hooks (may be NULL):
// `active` runs once the active pairs are known (act [na]: indices into
// the list PT then EE, the na_pt PT pairs first; valid on s), before the
// pair kernels are enqueued; `join` supplies keys, their count and off
// (then not known at the call) after the pair kernels are enqueued and
// before the assembly.  Neither runs when there is nothing to assemble.
struct BarrierHooks {
  std::function<int(const int32_t *act, int64_t na, int64_t na_pt)> active;
  std::function<int(const int32_t **keys, int64_t *n_keys, double **off)> join;
};
int op_barrier(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x, const int32_t *pt,
               int64_t n_pt, const int32_t *ee, int64_t n_ee, const int32_t *keys, int64_t n_keys, double *energy,
               double *grad, double *diag, double *off, int project, int64_t *n_active_pt, int64_t *n_active_ee,
               hipStream_t s, const FrictionSet *fr = nullptr, const BarrierHooks *hooks = nullptr);
// the active pairs act [na] (as the hook above receives them) gathered into
// pair lists: PT [na_pt][2], then EE [na - na_pt][2] (context workspace)
int op_gather_active(abd_ctx *ctx, const int32_t *act, int64_t na, int64_t na_pt, int64_t n_pt, const int32_t *pt,
                     const int32_t *ee, int32_t **pt_out, int32_t **ee_out, hipStream_t s);
// fixed-order assembly of n local records (info, g_loc [n][12], H_loc
// [n][78] packed symmetric) into grad / diag / off (accumulated)
int op_assemble(abd_ctx *ctx, const abd_scene *sc, int64_t n, const PairInfo *info, const double *g_loc,
                const double *H_loc, const int32_t *keys, int64_t n_keys, double *grad, double *diag, double *off,
                hipStream_t s);
// friction: lagged quantities of candidate pairs at xt; local records of
// the pairs of fr at x (written at e/g/H/info); energy of fr at x
int op_friction_lag(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *xt, const int32_t *pt,
                    int64_t n_pt, const int32_t *ee, int64_t n_ee, double *lam, double *T, double *w, hipStream_t s);
int op_friction_local(abd_ctx *ctx, const abd_scene *sc, const FrictionSet *fr, const double *x, double *e_loc,
                      double *g_loc, double *H_loc, PairInfo *info, hipStream_t s);
int op_friction_energy(abd_ctx *ctx, const abd_scene *sc, const FrictionSet *fr, const double *x, double *energy,
                       hipStream_t s);
// friction Hessian of fr at x times the body vector v [nb][12], accumulated
// into out [nb][12]
int op_friction_hvp(abd_ctx *ctx, const abd_scene *sc, const FrictionSet *fr, const double *x, const double *v,
                    double *out, hipStream_t s);
// adjoint's lag term: J^T grad_{x^t} [(J l) . g(x; lambda, T, w)] through the
// lagged quantities of fr, accumulated into out [nb][12]
int op_friction_lag_vjp(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const FrictionSet *fr,
                        const double *x, const double *l, double *out, hipStream_t s);
// reads and clears the device error flags of the last operations (syncs)
int op_read_err(abd_ctx *ctx, hipStream_t s);
// the error flag copied to pinned host memory (enqueued only), and its
// translation into an error code (clears the flag)
int err_enqueue(abd_ctx *ctx, int *h_err, hipStream_t s);
int err_check(abd_ctx *ctx, int e, hipStream_t s);
// the friction state of the current time step (null when none is set)
int op_friction_state(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, FrictionSet *fr, bool *active,
                      hipStream_t s);
int op_barrier_energy(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x, const int32_t *pt,
                      int64_t n_pt, const int32_t *ee, int64_t n_ee, double *energy, hipStream_t s);
int op_ccd(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x0, const double *dx,
           const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee, double *t_pt, double *t_ee,
           double *alpha, hipStream_t s, const double *x1 = nullptr);
// adaptive barrier stiffness (abd_kappa.hip): per-scene kappa and the
// closest active distance at q (workspace "kappa_sc", "kappa_d2prev"), and
// the doubling rule before a Newton iteration at x over its candidates
int op_kappa_init(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q, const double *qt,
                  hipStream_t s);
int op_kappa_update(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *x, const int32_t *pt,
                    int64_t npt, const int32_t *ee, int64_t nee, hipStream_t s);
// (skip_scene, device, may be NULL: bodies of the scenes it marks add
// nothing and get energy 0)
int op_body_terms(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q, const double *qt,
                  double *energy, double *grad, double *diag, int project, hipStream_t s,
                  const uint8_t *skip_scene = nullptr);
int op_body_energy(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q, const double *qt,
                   double *energy, hipStream_t s);
// x0 (may be NULL = 0, may alias p): initial guess
// pre_diag: preconditioner blocks (NULL: diag); pat: the keys' row
// structure if already built (else built here)
// pre_sync (may be NULL) is enqueued after the iterations queued in a
// round, before the host synchronises to read the solver's state; it gets
// that state on the device (int[4]: iteration base, scenes stopped, largest
// final count, scenes stopped by the cap or a breakdown).  *pre_sync_final
// (may be NULL) tells whether its last enqueue followed the solve's final
// iterations with nothing changing p afterwards.  skip_scene (device, may be
// NULL) marks scenes whose right-hand side is zero and whose diagonal
// blocks need not be invertible: their preconditioner blocks are zero.
using PcgHook = std::function<int(const int *cg_state)>;
// relative tolerance at and above which a one-kernel solve whose scenes all
// stopped on the tolerance skips the residual check (nothing then changes
// its result after the last iterations)
constexpr double PCG_CHECK_RTOL = 1e-6;
int op_pcg(abd_ctx *ctx, const abd_scene *sc, const double *diag, const double *off, const int32_t *keys,
           int64_t n_keys, const double *rhs, double *p, double rtol, int max_iter, int *iters, hipStream_t s,
           const double *x0 = nullptr, const double *pre_diag = nullptr, const KeyPattern *pat = nullptr,
           const PcgHook *pre_sync = nullptr, bool *pre_sync_final = nullptr,
           const uint8_t *skip_scene = nullptr);
// preconditioned MINRES on the (possibly indefinite) symmetric block matrix,
// block-Jacobi preconditioner from the SPD diagonal blocks pre_diag; stops
// at |r|_{P} <= rtol |b|_{P} (syncs every iteration)
int op_minres(abd_ctx *ctx, const abd_scene *sc, const double *diag, const double *off, const int32_t *keys,
              int64_t n_keys, const double *pre_diag, const double *rhs, double *x_out, double rtol, int max_iter,
              int *iters, hipStream_t s);
// per-scene max_k |J_k p|_inf at (*out)[j * *stride] (device, context
// workspace; a NaN displacement gives NaN; scenes skip_scene marks, device,
// may be NULL, get 0)
int op_max_abs_disp_scenes(abd_ctx *ctx, const abd_scene *sc, const double *p, const double **out, int *stride,
                           hipStream_t s, const uint8_t *skip_scene = nullptr);
int op_orthogonality(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q, double weight,
                     double *energy, double *grad, double *diag, int project, hipStream_t s);
int op_inertia(abd_ctx *ctx, const abd_scene *sc, const double *q, const double *qt, double *energy, double *grad,
               double *diag, hipStream_t s);

// ------------------------------------------- exact (set-deciding) math ----
// Everything that decides a candidate or an active flag is evaluated with
// fused multiply-add disabled and in a fixed operation order, so the result
// is a pure function of the IEEE-754 inputs.
struct d3 {
  double x, y, z;
};

__host__ __device__ __forceinline__ d3 ld3(const double *p, int64_t i) { return {p[3 * i], p[3 * i + 1], p[3 * i + 2]}; }

// vertex v at the body state q (12 per body): p + A xbar_v, each component
// p_i + ((a_i0 xb0 + a_i1 xb1) + a_i2 xb2), the vertex map's arithmetic
__host__ __device__ __forceinline__ d3 map_vertex(const double *q, const int32_t *vert_body, const double *xbar,
                                                  int64_t v) {
#pragma clang fp contract(off)
  const double *qb = q + 12 * (int64_t)vert_body[v];
  const double xb0 = xbar[3 * v], xb1 = xbar[3 * v + 1], xb2 = xbar[3 * v + 2];
  return {qb[0] + ((qb[3] * xb0 + qb[4] * xb1) + qb[5] * xb2), qb[1] + ((qb[6] * xb0 + qb[7] * xb1) + qb[8] * xb2),
          qb[2] + ((qb[9] * xb0 + qb[10] * xb1) + qb[11] * xb2)};
}

__host__ __device__ __forceinline__ d3 xsub(d3 a, d3 b) {
#pragma clang fp contract(off)
  return {a.x - b.x, a.y - b.y, a.z - b.z};
}
__host__ __device__ __forceinline__ double xdot(d3 a, d3 b) {
#pragma clang fp contract(off)
  return (a.x * b.x + a.y * b.y) + a.z * b.z;
}
__host__ __device__ __forceinline__ d3 xcross(d3 a, d3 b) {
#pragma clang fp contract(off)
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

enum : int {
  PT_PP0 = 0, PT_PP1 = 1, PT_PP2 = 2, PT_PE01 = 3, PT_PE12 = 4, PT_PE02 = 5, PT_FACE = 6,
  EE_BASE = 16, EE_LL = 28
};

// Slots of each case. kind 0: point-point (i,j); 1: point-edge (i; j,k);
// 2: point-face (0; 1,2,3); 3: line-line (0,1; 2,3)
struct CaseSlots {
  int kind, i, j, k;
};
__host__ __device__ __forceinline__ CaseSlots case_slots(int type) {
  switch (type) {
    case PT_PP0: return {0, 0, 1, -1};
    case PT_PP1: return {0, 0, 2, -1};
    case PT_PP2: return {0, 0, 3, -1};
    case PT_PE01: return {1, 0, 1, 2};
    case PT_PE12: return {1, 0, 2, 3};
    case PT_PE02: return {1, 0, 1, 3};
    case PT_FACE: return {2, 0, 1, 2};
    case EE_LL: return {3, 0, 1, 2};
    default: break;
  }
  const int k = (type - EE_BASE) / 3, c = (type - EE_BASE) % 3;
  const int e0 = k < 2 ? 2 : 0, e1 = k < 2 ? 3 : 1;
  if (c == 0) return {0, k, e0, -1};
  if (c == 1) return {0, k, e1, -1};
  return {1, k, e0, e1};
}

// squared distance of a case as num/den.  Each case is instantiated with
// compile-time vertex slots (a switch over the case code), so no register
// array is indexed with a run-time value.
template <int I, int J>
__host__ __device__ __forceinline__ void nd_pp(const d3 X[4], double &num, double &den) {
#pragma clang fp contract(off)
  d3 d = xsub(X[I], X[J]);
  num = xdot(d, d);
  den = 1.0;
}
template <int I, int J, int K>
__host__ __device__ __forceinline__ void nd_pe(const d3 X[4], double &num, double &den) {
#pragma clang fp contract(off)
  d3 e = xsub(X[K], X[J]);
  d3 cr = xcross(xsub(X[I], X[J]), e);
  num = xdot(cr, cr);
  den = xdot(e, e);
}
__host__ __device__ __forceinline__ void nd_face(const d3 X[4], double &num, double &den) {
#pragma clang fp contract(off)
  d3 n = xcross(xsub(X[2], X[1]), xsub(X[3], X[1]));
  double h = xdot(xsub(X[0], X[1]), n);
  num = h * h;
  den = xdot(n, n);
}
__host__ __device__ __forceinline__ void nd_ll(const d3 X[4], double &num, double &den) {
#pragma clang fp contract(off)
  d3 n = xcross(xsub(X[1], X[0]), xsub(X[3], X[2]));
  double h = xdot(xsub(X[2], X[0]), n);
  num = h * h;
  den = xdot(n, n);
}

__host__ __device__ __forceinline__ void case_nd(int type, const d3 X[4], double &num, double &den) {
  switch (type) {
    case PT_PP0: nd_pp<0, 1>(X, num, den); break;
    case PT_PP1: nd_pp<0, 2>(X, num, den); break;
    case PT_PP2: nd_pp<0, 3>(X, num, den); break;
    case PT_PE01: nd_pe<0, 1, 2>(X, num, den); break;
    case PT_PE12: nd_pe<0, 2, 3>(X, num, den); break;
    case PT_PE02: nd_pe<0, 1, 3>(X, num, den); break;
    case PT_FACE: nd_face(X, num, den); break;
    case EE_BASE + 0: nd_pp<0, 2>(X, num, den); break;
    case EE_BASE + 1: nd_pp<0, 3>(X, num, den); break;
    case EE_BASE + 2: nd_pe<0, 2, 3>(X, num, den); break;
    case EE_BASE + 3: nd_pp<1, 2>(X, num, den); break;
    case EE_BASE + 4: nd_pp<1, 3>(X, num, den); break;
    case EE_BASE + 5: nd_pe<1, 2, 3>(X, num, den); break;
    case EE_BASE + 6: nd_pp<2, 0>(X, num, den); break;
    case EE_BASE + 7: nd_pp<2, 1>(X, num, den); break;
    case EE_BASE + 8: nd_pe<2, 0, 1>(X, num, den); break;
    case EE_BASE + 9: nd_pp<3, 0>(X, num, den); break;
    case EE_BASE + 10: nd_pp<3, 1>(X, num, den); break;
    case EE_BASE + 11: nd_pe<3, 0, 1>(X, num, den); break;
    default: nd_ll(X, num, den); break;
  }
}

// Point-triangle case from the Voronoi regions of the triangle (sign tests
// of dot products; vertices before edges before the face on ties).
__host__ __device__ __forceinline__ int classify_pt(d3 p, d3 t0, d3 t1, d3 t2) {
#pragma clang fp contract(off)
  d3 ab = xsub(t1, t0), ac = xsub(t2, t0), ap = xsub(p, t0);
  double d1 = xdot(ab, ap), d2 = xdot(ac, ap);
  if (d1 <= 0.0 && d2 <= 0.0) return PT_PP0;
  d3 bp = xsub(p, t1);
  double d3v = xdot(ab, bp), d4 = xdot(ac, bp);
  if (d3v >= 0.0 && d4 <= d3v) return PT_PP1;
  double vc = d1 * d4 - d3v * d2;
  if (vc <= 0.0 && d1 >= 0.0 && d3v <= 0.0) return PT_PE01;
  d3 cp = xsub(p, t2);
  double d5 = xdot(ab, cp), d6 = xdot(ac, cp);
  if (d6 >= 0.0 && d5 <= d6) return PT_PP2;
  double vb = d5 * d2 - d1 * d6;
  if (vb <= 0.0 && d2 >= 0.0 && d6 <= 0.0) return PT_PE02;
  double va = d3v * d6 - d5 * d4;
  if (va <= 0.0 && (d4 - d3v) >= 0.0 && (d5 - d6) >= 0.0) return PT_PE12;
  return PT_FACE;
}

// Edge-edge case: line-line when the lines' closest points are strictly
// inside both segments and the edges are not parallel; otherwise the
// smallest of the four endpoint-vs-segment distances (division-free
// comparison, first minimum wins).
__host__ __device__ __forceinline__ int classify_ee(const d3 X[4]) {
#pragma clang fp contract(off)
  d3 u = xsub(X[1], X[0]), v = xsub(X[3], X[2]), w = xsub(X[0], X[2]);
  double a = xdot(u, u), b = xdot(u, v), c = xdot(v, v), d = xdot(u, w), e = xdot(v, w);
  d3 n = xcross(u, v);
  double nn = xdot(n, n);
  double D = a * c - b * b;
  double sN = b * e - c * d, tN = a * e - b * d;
  if (nn > (1e-20 * a) * c && sN > 0.0 && sN < D && tN > 0.0 && tN < D) return EE_LL;
  int best = -1;
  double bn = 0.0, bd = 1.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const d3 P = X[k], E0 = X[k < 2 ? 2 : 0], E1 = X[k < 2 ? 3 : 1];
    d3 ev = xsub(E1, E0);
    double tn = xdot(xsub(P, E0), ev);
    int sub = tn <= 0.0 ? 0 : (tn >= xdot(ev, ev) ? 1 : 2);
    const int type = EE_BASE + 3 * k + sub;
    double num, den;
    case_nd(type, X, num, den);
    if (best < 0 || num * bd < bn * den) {
      best = type;
      bn = num;
      bd = den;
    }
  }
  return best;
}

__host__ __device__ __forceinline__ void pair_vids(int is_ee, const int32_t *pr, const int32_t *tris, const int32_t *edges,
                                          int vid[4]) {
  if (!is_ee) {
    const int t = pr[1];
    vid[0] = pr[0];
    vid[1] = tris[3 * t];
    vid[2] = tris[3 * t + 1];
    vid[3] = tris[3 * t + 2];
  } else {
    vid[0] = edges[2 * pr[0]];
    vid[1] = edges[2 * pr[0] + 1];
    vid[2] = edges[2 * pr[1]];
    vid[3] = edges[2 * pr[1] + 1];
  }
}

__host__ __device__ __forceinline__ int classify_pair(int is_ee, const d3 X[4]) {
  return is_ee ? classify_ee(X) : classify_pt(X[0], X[1], X[2], X[3]);
}

// ------------------------------------------------------ reductions ----
// Wave-level (64 lanes) sums via cross-lane moves; the lane order of the
// tree is fixed, so results are run-to-run reproducible.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Deterministic device-wide sums: per-block partials then one block folds them.
int reduce_sum_f64(abd_ctx *ctx, const double *in, int64_t n, double *out_accum, hipStream_t s);
// the same sum (same launches, same order) with the second pass's block
// partials in caller memory of REDUCE_MAX_PARTS doubles; allocates nothing
constexpr int REDUCE_MAX_PARTS = 1024;
void reduce_sum_f64_into(const double *in, int64_t n, double *part, double *out_accum, hipStream_t s);
// once per device, with the device current: the device address of the
// allocation-free entry point's scratch array (abd_narrow.hip)
int noalloc_scratch_init(int device);
int reduce_min_f64(abd_ctx *ctx, const double *in, int64_t n, double init, double *out, hipStream_t s);
// Per-scene reductions of items whose scene keys are non-decreasing (bodies,
// vertices and candidate pairs are all scene-contiguous): sums accumulate
// into out [n_scenes] (n_scenes <= 1: one device-wide sum, keys unused);
// maxima (of non-negative values) overwrite out.
// Sums of trial-major values (trial t's n items at vals + t * stride) per
// (trial, scene) into out_accum[t * n_scenes + scene] (accumulated); keys
// (non-decreasing item scenes) are needed when n_scenes > 1.
// Energies of n_trials configurations at once (trial t's q, x at
// q + 12 nb t, x + 3 nv t; the barrier maps its pairs' vertices from q
// itself): each op accumulates into energy[t S + scene]; with items
// non-NULL it instead writes the per-item energies (trial t's at
// items + t estride) and sums nothing.
// With defer non-NULL (several scenes) an op writes its per-item energies
// and their scenes and appends the segments to *defer instead of summing;
// seg_sum_trials_multi then sums every segment in one launch.
struct TrialSeg {
  const double *vals;  // trial t's items at vals + t stride
  int64_t stride, n;
  const int32_t *keys;  // non-decreasing item scenes
};
struct TrialSums {
  TrialSeg seg[5];
  int k = 0;
  const uint8_t *skip = nullptr;  // (device, may be NULL) scenes whose sums are 0
};
// (with defer, bodies of the scenes defer->skip marks get energy 0)
int op_body_energy_trials(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q,
                          const double *qt, int n_trials, double *energy, hipStream_t s, double *items = nullptr,
                          int64_t estride = 0, TrialSums *defer = nullptr);
int op_barrier_energy_trials(abd_ctx *ctx, const abd_scene *sc, const abd_params *prm, const double *q,
                             int n_trials, const int32_t *pt, int64_t n_pt, const int32_t *ee, int64_t n_ee,
                             double *energy, hipStream_t s, double *items = nullptr, int64_t estride = 0,
                             TrialSums *defer = nullptr);
int op_friction_energy_trials(abd_ctx *ctx, const abd_scene *sc, const FrictionSet *fr, const double *x,
                              int n_trials, double *energy, hipStream_t s, double *items = nullptr,
                              int64_t estride = 0, TrialSums *defer = nullptr);
// out[t S + scene] = the sum, segment after segment in order, of each
// segment's sum over the scene's items (each in the fixed order of
// seg_sum_trials, so the result equals accumulating the segments one by
// one into zeros); n_scenes > 1
int seg_sum_trials_multi(abd_ctx *ctx, const TrialSums &ts, int n_trials, int n_scenes, double *out,
                         hipStream_t s);
int seg_sum_trials(abd_ctx *ctx, const double *vals, int64_t stride, int64_t n, const int32_t *keys, int n_trials,
                   int n_scenes, double *out_accum, hipStream_t s,
                   bool assign = false);
// first body of every scene, [n_scenes + 1] (device, context workspace)
int op_scene_offsets(abd_ctx *ctx, const abd_scene *sc, const int32_t **off, hipStream_t s);
