/*
 * opf.h -- C ABI of libopf: per-iteration model evaluation of a multi-period
 * AC optimal power flow on one AMD MI355X (gfx950), FP64.
 *
 * The model is the multi-period AC OPF of Shin et al., "Scalable Multi-Period
 * AC Optimal Power Flow Utilizing GPUs with High Memory Capacities"
 * (arXiv 2405.14032), Sec. II, eq. (1a)-(1k), evaluated the way an
 * interior-point iteration needs it (Sec. III): objective, gradient,
 * constraints, sparse Jacobian and Lagrangian Hessian in COO form with
 * sparsity fixed per repeated pattern (Sec. III-A), and the condensed KKT
 * matrix W + delta_w I + Sigma_x + A^T D A of the lifted-KKT method
 * (Sec. III-B).
 *
 * Conventions
 *  - Indices are 0-based.  Value arrays are double.  Index arrays are int32,
 *    CSR row pointers int64.  Creation fails with OPF_ERANGE if any global
 *    row or column index would not fit int32, or if one period's block of
 *    x, c, J, H or K (or of the line scratch, 22 doubles per line) would
 *    exceed 4 GiB (the kernels address inside a block by 32-bit byte
 *    offsets; at most 2^29 - 1 doubles per block).
 *  - Status: every function returns OPF_OK (0) or a negative code; the
 *    thread-local message of the last failure is opf_last_error().  No C++
 *    exception crosses this boundary.
 *  - Unless stated otherwise, array arguments of the evaluation calls are
 *    DEVICE pointers (hipMalloc'd or torch CUDA tensors on the model's
 *    device), owned by the caller, and the work is enqueued asynchronously on
 *    the model's stream (opf_set_stream); the caller synchronises.
 *  - A model is not re-entrant: calls on one model must not overlap (they
 *    share the model's scratch).  Distinct models are independent.
 *  - A model may hold several instances (ninst > 1, the batched form): it is
 *    block-diagonal; x, c, the J/H COO arrays and the K CSR are the
 *    instance-major concatenation of the per-instance arrays, with row and
 *    column indices offset by the instance's x / c offsets
 *    (opf_instance_offsets).  Every call evaluates all instances.
 *
 * Canonical per-instance layouts (N buses, B lines, G generators, T periods):
 *  x, per period t:  [vm N | va N | pg G | qg G | pf B | qf B | pt B | qt B]
 *                    (pf, qf: complex power entering line l = (i -> j) at
 *                    its from end i; pt, qt: entering at its to end j)
 *  c, per period t:  [balP N | balQ N | ref 1 | cpf B | cqf B | cpt B |
 *                     cqt B | thf B | tht B | ang B]
 *                    then ramp rows (t-1)*G + g for t = 1..T-1.
 *  J COO, per period t (offset t*(2G+30B+1)); index = base + local*cnt + e:
 *     gen-balance   2 x G : (balP[bus_g], pg_g), (balQ[bus_g], qg_g)
 *     line-balance  4 x B : (balP[i],pf) (balQ[i],qf) (balP[j],pt) (balQ[j],qt)
 *     ref           1     : (ref, va[ref_bus])
 *     flows        20 x B : local = kind*5 + {own, vm_i, vm_j, va_i, va_j},
 *                           kind in {pf, qf, pt, qt}
 *     thermal       4 x B : (thf,pf) (thf,qf) (tht,pt) (tht,qt)
 *     angle         2 x B : (ang, va_i) (ang, va_j)
 *   then the ramp block at T*(2G+30B+1): (t-1)*2G + local*G + g with
 *   local 0 = (ramp, pg_t), 1 = (ramp, pg_{t-1}).
 *  H COO (lower, row >= col, duplicates kept), per period t (offset
 *   t*(G+40B)): objective G x (pg,pg); flows 36 x B with local = kind*9 + p
 *   over the row-major lower triangle of (vm_i, vm_j, va_i, va_j) without
 *   its structural zero ((vm_j,vm_j) for pf/qf, (vm_i,vm_i) for pt/qt);
 *   thermal 4 x B: (pf,pf) (qf,qf) (pt,pt) (qt,qt).
 *  K CSR: rows in x order, lower triangle, strictly ascending columns,
 *   duplicates merged, diagonal always present.
 */
#ifndef OPF_H
#define OPF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  OPF_OK = 0,
  OPF_EINVAL = -1, /* bad descriptor, NULL required pointer, misuse          */
  OPF_ERANGE = -2, /* a count or index does not fit the index types         */
  OPF_ENOMEM = -3, /* device or host allocation failed                      */
  OPF_EHIP = -4,   /* HIP runtime error (message holds hipGetErrorString)   */
  OPF_ENODEV = -5  /* the call needs a device but the model is host-only    */
};

typedef struct opf_model opf_model;

/* One instance, as HOST arrays (copied at creation; the caller keeps
 * ownership).  Sec. II, eq. (1): buses N, lines B with pi-model data,
 * generators G with quadratic cost c2 p^2 + c1 p + c0 (eq. (1a)) and bounds
 * (eq. (1g)-(1h), (1k)), voltage bounds (eq. (1i)), line rating (eq. (1f)),
 * angle-difference limits (eq. (1j)) and the per-period bus load profile
 * (eq. (1b)-(1c)).  Multiple lines between one bus pair and several
 * generators per bus are allowed. */
typedef struct {
  int32_t nbus, nbranch, ngen, nperiod, ref_bus; /* N>=1, B>=0, G>=1, T>=1    */
  const double *vmin, *vmax;                     /* [N]                       */
  const int32_t *f_bus, *t_bus;                  /* [B], in [0,N), f != t     */
  const double *r, *x, *b_charge;                /* [B] series r + jx, charging */
  const double *rate, *angmin, *angmax;          /* [B]                       */
  const double *tap, *shift;                     /* [B] or NULL => 1, 0 (rad) */
  const int32_t *gen_bus;                        /* [G], in [0,N)             */
  const double *c2, *c1, *c0;                    /* [G]; c0 may be NULL => 0  */
  const double *pmin, *pmax, *qmin, *qmax, *ramp;/* [G]                       */
  const double *pd, *qd;                         /* [T*N], pd[t*N + n]        */
} opf_instance_desc;

typedef struct {
  int64_t n, m, nnz_jac, nnz_hess, nnz_kkt; /* totals over all instances      */
  int32_t ninst;
} opf_dims;

/* Arguments of one whole evaluation sweep.  Device pointers; an output left
 * NULL is not computed (its inputs may then be NULL too).  kvals needs
 * jvals and hvals (the sweep computes them first). */
typedef struct {
  const double *x;      /* [n]                                             */
  const double *lambda; /* [m] multipliers of the Hessian                  */
  double sigma;         /* objective weight of the Hessian                 */
  const double *v;      /* [m] vector of the J^T v product                  */
  const double *diag_x; /* [n] or NULL: diagonal added to K                */
  const double *dcon;   /* [m] row weights D of K                          */
  double *f;            /* [ninst] objective per instance                  */
  double *grad;         /* [n]                                             */
  double *c;            /* [m]                                             */
  double *jvals;        /* [nnz_jac]                                       */
  double *hvals;        /* [nnz_hess]                                      */
  double *jtv;          /* [n]                                             */
  double *kvals;        /* [nnz_kkt]                                       */
} opf_sweep_args;

/* Checks a descriptor array on the host (no device needed): sizes, index
 * ranges, f != t, NULL pointers, finite admittances, int32 index limits,
 * per-period blocks within 4 GiB (the K block is checked at creation, once
 * its pattern is known).  Returns OPF_OK, OPF_EINVAL or OPF_ERANGE. */
int opf_validate(const opf_instance_desc *desc, int32_t ninst);

/* Builds a model of ninst instances.  device >= 0: element tables, the
 * per-period symbolic plans (Sec. III-A: sparsity analysed once per pattern
 * and expanded over the data) and scratch are uploaded to that HIP device.
 * device < 0: host-only model, only dims / offsets / opf_kkt_structure
 * (into HOST arrays) are available; evaluation calls return OPF_ENODEV.
 * *out receives the model (NULL on failure).  Errors: those of
 * opf_validate; OPF_ENOMEM / OPF_EHIP on device allocation or upload
 * failure; OPF_EINVAL if the condensed matrix's rows for one tile of lines
 * or buses cannot be staged in on-chip memory at any launch shape (a bus
 * joined to thousands of lines), or a bus's K rows would exceed 65534
 * partner slots (OPF_ERANGE). */
int opf_model_create(const opf_instance_desc *desc, int32_t ninst, int device,
                     opf_model **out);
void opf_model_destroy(opf_model *model); /* NULL is a no-op */

int opf_model_dims(const opf_model *model, opf_dims *dims); /* host out */

/* Host arrays of ninst+1 entries each (any may be NULL): starting offsets of
 * each instance in x, c, J, H and K (the last entry is the total). */
int opf_instance_offsets(const opf_model *model, int64_t *x_off, int64_t *c_off,
                         int64_t *j_off, int64_t *h_off, int64_t *k_off);

/* Stream for all later calls on this model (a hipStream_t; NULL = the null
 * stream). */
int opf_set_stream(opf_model *model, void *hip_stream);

/* Variable and row bounds (eq. (1f)-(1k); flows, angles unbounded = +-inf,
 * equality rows [0,0], ref row [0,0]).  Device [n], [n], [m], [m]. */
int opf_bounds(const opf_model *model, double *lvar, double *uvar, double *lcon,
               double *ucon);

/* COO index arrays of J ([nnz_jac] each) and of the lower Hessian
 * ([nnz_hess] each, row >= col), canonical order (Sec. III-A). Device. */
int opf_jac_structure(const opf_model *model, int32_t *rows, int32_t *cols);
int opf_hess_structure(const opf_model *model, int32_t *rows, int32_t *cols);

/* CSR pattern of the lower triangle of K (Sec. III-B, M_cond; the optional
 * compressed form of Sec. III-A): rowptr [n+1], colind [nnz_kkt].  Device
 * arrays for a device model, HOST arrays for a host-only model. */
int opf_kkt_structure(const opf_model *model, int64_t *rowptr, int32_t *colind);

/* f = sum_t sum_g c2 pg^2 + c1 pg + c0 (eq. (1a)); f: device [ninst].
 * Deterministic two-pass reduction. */
int opf_eval_obj(opf_model *model, const double *x, double *f);
/* grad f (eq. (1a)): [n], zero outside the pg entries. */
int opf_eval_grad(opf_model *model, const double *x, double *g);
/* All rows c(x) in canonical order (eq. (1b)-(1f), (1j), (1k), ref). [m] */
int opf_eval_cons(opf_model *model, const double *x, double *c);
/* Jacobian values of the rows of eq. (1b)-(1f), (1j), (1k) and the ref row,
 * in the canonical COO order (Sec. III-A: each pattern's sparsity analysed
 * once and expanded over the data; the order is that of
 * opf_jac_structure).  x: device [n]; jvals: device [nnz_jac], overwritten.
 * Errors: OPF_EINVAL (NULL), OPF_ENODEV (host-only model), OPF_EHIP. */
int opf_eval_jac(opf_model *model, const double *x, double *jvals);
/* Lower COO values of sigma Hess f + sum_i lambda_i Hess c_i (Sec. III-B:
 * W, the Hessian of the Lagrangian; an IPM written with p_x = grad f -
 * A^T y passes lambda = -y). [nnz_hess] */
int opf_eval_hess(opf_model *model, const double *x, const double *lambda,
                  double sigma, double *hvals);
/* Matrix-free J(x)^T v (the A^T y term of p_x, Sec. III-B). [n] */
int opf_jtprod(opf_model *model, const double *x, const double *v, double *jtv);
/* Replace the load profile by device arrays pd, qd (concatenation over
 * instances of [T*N] each). */
int opf_set_load(opf_model *model, const double *pd, const double *qd);
/* d(lambda^T c)/d(pd, qd) = (-lambda_balP, -lambda_balQ) (the load enters
 * eq. (1b)-(1c) with coefficient -1), each the concatenation of [T*N]. */
int opf_load_adjoint(opf_model *model, const double *lambda, double *gpd,
                     double *gqd);
/* K = lower(H + diag(diag_x) + J^T diag(dcon) J) into the fixed CSR of
 * opf_kkt_structure (Sec. III-B: M_cond with diag_x = delta_w + Sigma_x and
 * dcon = D supplied by the caller).  hvals / jvals as produced by
 * opf_eval_hess / opf_eval_jac; diag_x may be NULL (= 0).  Every slot is
 * written by exactly one thread: no atomics, bitwise reproducible. */
int opf_assemble_condensed(opf_model *model, const double *hvals,
                           const double *jvals, const double *diag_x,
                           const double *dcon, double *kvals);

/* ---- lifted-KKT condensation around the condensed matrix (Sec. III-B) ----
 *
 * One iterate of the lifted interior-point method: the rows are relaxed to
 * c(x) - s = 0 with sl <= s <= su (equality rows get a small band chosen by
 * the solver), and the variables keep xl <= x <= xu.  All arrays are device
 * pointers over the concatenated instances; a bound of +-inf is absent (its
 * multiplier entry is ignored and every term of that bound vanishes).  The
 * caller owns every array; none is retained. */
typedef struct {
  const double *x;         /* [n] primal point (strictly inside finite bounds) */
  const double *s;         /* [m] slacks (strictly inside finite bounds) */
  const double *y;         /* [m] multipliers of c(x) - s = 0 (the paper's y) */
  const double *zl, *zu;   /* [n] multipliers of x >= xl and x <= xu (>= 0) */
  const double *vl, *vu;   /* [m] multipliers of s >= sl and s <= su (>= 0) */
  const double *xl, *xu;   /* [n] variable bounds */
  const double *sl, *su;   /* [m] slack bounds */
  double mu;               /* barrier parameter (>= 0) */
  double delta_w, delta_c; /* primal and dual regularisation (>= 0) */
} opf_ipm_state;

/* Forward product J(x) v: the A dx term of the step recovery.  [m] */
int opf_jprod(opf_model *model, const double *x, const double *v, double *jv);

/* The condensed system's weights and right-hand side (Sec. III-B):
 *   diag_x = delta_w + Sigma_x,  Sigma_x = Zl (X - Xl)^-1 + Zu (Xu - X)^-1,
 *   dcon   = D = (Sigma_s + delta_w) C,
 *            C = (delta_c Sigma_s + (1 + delta_c delta_w))^-1,
 *   rhs    = q_x + J^T (C q_s + D q_y),
 * with p_x = grad - J^T y - zl + zu, p_s = -vl + vu + y, q_y = c - s,
 * q_x = p_x + (X - Xl)^-1 p_zl - (Xu - X)^-1 p_zu and the same for q_s, and
 * the complementarity residuals p_zl = zl (x - xl) - mu,
 * p_zu = zu (xu - x) - mu (likewise for s).  grad = grad f(x) [n] and
 * c = c(x) [m] as produced by opf_eval_grad / opf_eval_cons at st->x.
 * Outputs: diag_x [n], dcon [m], rhs [n]; they feed opf_assemble_condensed
 * and the solve of K dx = rhs.  Outputs must not alias inputs.  Uses the
 * model's work vector: calls on one model must not overlap. */
int opf_condensed_rhs(opf_model *model, const opf_ipm_state *st,
                      const double *grad, const double *c, double *diag_x,
                      double *dcon, double *rhs);

/* Recovery of the other step components from the condensed solution dx
 * (Sec. III-B):
 *   ds  = C (J dx + delta_c q_s - q_y),  dy = (Sigma_s + delta_w) ds - q_s,
 *   dzl = (X - Xl)^-1 (-zl dx + p_zl),   dzu = (Xu - X)^-1 (zu dx + p_zu),
 *   dvl = (S - Sl)^-1 (-vl ds + p_vl),   dvu = (Su - S)^-1 (vu ds + p_vu),
 * (the slack step takes +J dx: eliminating the relaxed rows of the full
 * system gives that sign; the paper's printed formula has the other one);
 * entries of absent bounds are 0.  c = c(x) [m]; outputs ds, dy, dvl, dvu
 * [m] and dzl, dzu [n], none aliasing an input.  Uses the model's work
 * vector. */
int opf_recover_step(opf_model *model, const opf_ipm_state *st,
                     const double *c, const double *dx, double *ds, double *dy,
                     double *dzl, double *dzu, double *dvl, double *dvu);

/* Jacobian, Hessian and condensed matrix in one pass over x: the values of
 * opf_eval_jac, opf_eval_hess and opf_assemble_condensed (bitwise identical
 * to those three calls), with K built from the J / H values while they are
 * in registers instead of reading them back (the per-pattern evaluation of
 * Sec. III-A feeding the condensation of Sec. III-B directly).  diag_x may
 * be NULL. */
int opf_eval_jhk(opf_model *model, const double *x, const double *lambda,
                 double sigma, const double *diag_x, const double *dcon,
                 double *jvals, double *hvals, double *kvals);

/* Every requested output of one iteration's evaluation, enqueued as
 * persistent tile-list kernels covering all instances; when jvals, hvals and
 * kvals are all requested the fused pass of opf_eval_jhk is used.  With
 * every output requested, the objective is summed inside the two sweep
 * passes in their own tile order: equal to opf_eval_obj up to the rounding
 * of a reordered sum, and bitwise equal from call to call. */
int opf_sweep(opf_model *model, const opf_sweep_args *args);
/* The same sweep recorded once into a HIP graph (re-recorded when the
 * argument set changes) and replayed with a single graph launch. */
int opf_sweep_graph(opf_model *model, const opf_sweep_args *args);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sweep as opf_sweep, with the same kernels and bitwise identical results,
 * but its scratch (the line -> bus hand-off records and the objective's
 * partial sums) lives in a static device array of the library, 32 MiB per
 * device, instead of the model's buffers.  The call itself allocates nothing
 * (no hipMalloc, no event creation) and only enqueues kernels on the model's
 * stream; the model is still created beforehand with opf_model_create.
 * Returns OPF_ERANGE when the model needs more scratch than the static array
 * holds (22 doubles per line-period, one per 64 generators and period, and
 * one per tile of the separate objective pass: e.g. 2000
 * buses / 3200 lines over 24 periods fit, the 13000-line grid over 168
 * periods does not).  Every call on one device shares that array and it
 * keeps the last call's contents: calls that overlap on one device (two
 * streams, two models, two threads) race and must be serialised by the
 * caller.  Per-kernel timing (opf_set_timing) does not cover this call. */
int opf_sweep_noalloc(opf_model *model, const opf_sweep_args *args);
/* Status of the one-launch sweep (opf_sweep, opf_sweep_graph and
 * opf_sweep_noalloc with every per-element output requested run the line,
 * generator and bus passes of Sec. III-A / III-B as one persistent launch in
 * which bus tiles wait, with a bounded spin, for the line tiles of their
 * periods).  Waits for the model's stream, then returns in *status (host
 * int32) the bits raised by the launches since the last call and clears
 * them: bit 0 = a bus tile's wait ran out (its outputs are not valid),
 * bit 1 = a work queue was left unfinished.  0 means every sweep since the
 * last call completed as designed. */
int opf_sweep_check(opf_model *model, int32_t *status);

/* Per-kernel timing.  opf_set_timing(model, 1) clears the statistics and
 * brackets every later kernel launch of the model with HIP events on the
 * model's stream (launches recorded into a graph are not timed);
 * opf_set_timing(model, 0) stops.  opf_kernel_stats returns, for kernel
 * family index (0 .. until OPF_ERANGE), its name, the number of timed
 * launches and their summed duration in milliseconds (it waits for the
 * pending events).  For profiling the evaluation path; the events cost a
 * few microseconds of host time per launch. */
int opf_set_timing(opf_model *model, int enable);
int opf_kernel_stats(opf_model *model, int32_t index, const char **name,
                     int64_t *launches, double *total_ms);

/* Chooses tile shapes (lines / buses / generators per tile, periods per
 * tile, persistent grid size) per kernel by timing candidates on the device.
 * cache_path (host string or NULL): JSON file read for a previous result
 * for this model shape and written after tuning. */
int opf_autotune(opf_model *model, const char *cache_path);

/* ---- static-pivot sparse Cholesky of the condensed matrix (Sec. III-B) ----
 *
 * After inertia correction the condensed matrix K is positive definite, so
 * it is factored as K = L L^T without numerical pivoting; a pivot that is not
 * above the caller's threshold is replaced (static pivoting) and counted, so
 * the caller can tell that K was not positive definite and correct the
 * inertia.  Structure used (Sec. II, eq. (1k)): periods couple only through
 * the ramp rows, i.e. through the pg variables, and every period block has
 * the same pattern.  One ordering of a period's variables serves all
 * periods: the other variables first (approximate minimum degree), the pg
 * variables last; the interior fronts of all periods are factored together,
 * then the pg fronts form a chain over the periods (block elimination in
 * time), eliminated from both ends of the horizon towards its middle period.
 * Instances of a batched model are factored one after another. */
typedef struct opf_chol opf_chol;

typedef struct {
  int64_t factor_entries; /* stored factor doubles, all instances and periods */
  int64_t arena_entries;  /* update-matrix workspace doubles                  */
  double flops;           /* factorization flops (multiply-add = 2)           */
  double flops_interior;  /* of which in the per-period interior fronts       */
  int32_t nodes;          /* interior fronts per period, summed over instances */
  int32_t levels;         /* largest interior tree height                      */
  int32_t chunk;          /* periods whose interior fronts are factored together
                             (smallest over instances)                         */
  int32_t large_nodes;    /* fronts factored by the blocked kernels            */
} opf_chol_info;

/* Symbolic analysis of the model's K pattern (opf_kkt_structure): ordering,
 * assembly tree, front sizes, assembly maps; on a device model it also
 * allocates the factor and its workspace on the model's device.  Works on a
 * host-only model (analysis only).  *out receives the factor object (NULL on
 * failure); it refers to the model, which must outlive it.  Errors:
 * OPF_EINVAL (NULL arguments, a front too large for the kernels),
 * OPF_ENOMEM (host or device allocation), OPF_EHIP.  The update-matrix
 * workspace holds the fronts of as many periods as fit in 16 GiB (the
 * environment variable OPF_CHOL_ARENA_BYTES, read here, overrides the
 * budget); those periods are factored together.  The large trailing
 * updates of the pg chain's fronts (one from each end per step) run as rocBLAS
 * strided-batched DGEMMs (atomics off: reproducible); OPF_CHOL_BLAS=0, read
 * here, keeps them on the library's own kernel. */
int opf_chol_analyze(opf_model *model, opf_chol **out);
void opf_chol_destroy(opf_chol *chol); /* NULL is a no-op */
int opf_chol_get_info(const opf_chol *chol, opf_chol_info *info);

/* The analysis of instance inst, into HOST arrays (for checking it):
 * opf_chol_tree_size gives the number of interior fronts per period and the
 * total count of their update rows; opf_chol_tree fills perm [n_p] (position
 * in the elimination order -> position in the period block of x), first,
 * npiv, parent [nodes] (front s eliminates positions first[s] ..
 * first[s] + npiv[s] - 1; parent -1 = the period's pg front), rowptr
 * [nodes + 1] and rows [rows] (update rows of each front, in elimination
 * positions, ascending).  Positions n_p - G .. n_p - 1 are the pg
 * variables in their natural order. */
int opf_chol_tree_size(const opf_chol *chol, int32_t inst, int32_t *nodes,
                       int64_t *rows);
int opf_chol_tree(const opf_chol *chol, int32_t inst, int32_t *perm,
                  int32_t *first, int32_t *npiv, int32_t *parent,
                  int64_t *rowptr, int32_t *rows);

/* Numeric factorization of K from its values kvals [nnz_kkt] (device, the
 * order of opf_kkt_structure).  A pivot d (the diagonal entry after the
 * updates of the columns before it) with !(d > pivot_tol) is replaced by
 * pivot_repl (> 0) and counted into *npert (device int32, overwritten).
 * Enqueued on the model's stream: the work of the call starts after what
 * is already queued there and later work queued there sees the finished
 * factor (internally the pg chain, and every other large front of a level,
 * run on two streams of the object's own, ordered by events and joined back
 * into the model's stream).  The factor
 * stays in the opf_chol object.  Errors: OPF_EINVAL (NULL, pivot_repl not
 * > 0), OPF_ENODEV (host-only model), OPF_EHIP. */
int opf_chol_factor(opf_chol *chol, const double *kvals, double pivot_tol,
                    double pivot_repl, int32_t *npert);

/* Solves L L^T x = b with the last factorization: b, x device [n] (may be
 * the same array).  Enqueued on the model's stream; uses the factor
 * object's work vectors, so solves on one object must not overlap. */
int opf_chol_solve(opf_chol *chol, const double *b, double *x);
/* By default a solve is recorded once into a HIP graph per (b, x) pointer
 * pair and replayed (the launch sequence is fixed for the object; the
 * graph reads the factor's current values).  enable = 0 launches the
 * kernels one by one instead. */
int opf_chol_set_graph(opf_chol *chol, int enable);
/* enable != 0: opf_chol_factor stops at its first static pivot -- every
 * later kernel of that factorization returns at once, *npert is then >= 1
 * (not the full count) and the factor is not usable.  For callers that
 * discard a factorization with static pivots, as the inertia correction of
 * Sec. III-B does (opf_ipm_solve turns it on for its own factorizations and
 * restores the setting afterwards).  A factorization without static pivots
 * is unchanged, bitwise.  Default 0. */
int opf_chol_set_stop_on_pivot(opf_chol *chol, int enable);
/* The current setting (0 or 1; 0 for NULL). */
int opf_chol_stop_on_pivot(const opf_chol *chol);

/* ---- the lifted-KKT interior-point loop (Sec. III-B) ----
 *
 * Solves the multi-period AC OPF of the model (all instances jointly) to
 * tolerance by a primal-dual interior-point method on the lifted
 * formulation: rows relaxed to sl <= s <= su with c(x) - s = 0 (equality
 * rows widened by +-relax), each iteration condensing (opf_condensed_rhs),
 * building K at lambda = -y (opf_eval_jhk), factoring with the static-pivot
 * Cholesky and correcting the inertia (delta_w = 0, then dw_first, times
 * dw_grow, while the factorization reports static pivots), solving and
 * recovering the step (opf_recover_step; with line_search the correction
 * starts from the last delta_w used, see dw_shrink).  Sec. III-B takes the inertia
 * correction from the filter interior-point method of Waechter and Biegler
 * (2006) and says a line search chooses the step length; with line_search
 * (the default) this loop takes that method's filter line search: a
 * monotone barrier parameter (mu_init; while the barrier problem's error is
 * at most kappa_eps mu, mu = max(tol / 10, min(kappa_mu mu, mu^theta_mu))
 * and the filter is emptied), fraction to the boundary
 * tau_k = max(tau_min, 1 - mu), then backtracking (halving) on the barrier
 * function phi = f - mu sum ln(distance to each finite bound) and the
 * violation theta = |c(x) - s|_1 with the filter, switching (delta,
 * s_theta, s_phi), Armijo (eta_phi) and sufficient-decrease (gamma_theta,
 * gamma_phi) tests of that method; y moves with the accepted primal length
 * and each bound multiplier is kept within [mu / (kappa_sigma gap),
 * kappa_sigma mu / gap].  When no length above alpha_min (gamma_alpha times
 * the smallest length at which a decrease can still be required) is
 * accepted, or theta has not fallen below 0.9 of its best value for
 * stall_iter iterations while max |c - s| > tol (steps accepted, no progress
 * towards feasibility), the loop stops with status OPF_IPM_STALLED (the
 * method's restoration phase is not implemented: a stall reports the
 * instance as not solved, e.g. infeasible).  With or without the line
 * search, an iteration whose inertia correction would need delta_w >
 * dw_max (no positive definite condensed matrix found) also ends the loop
 * with OPF_IPM_STALLED and the last iterate.  Without line_search: mu = sigma * (mean
 * complementarity product) and the fraction-to-the-boundary lengths (tau,
 * one primal, one dual; y moves with the dual length) are taken as they
 * are.  Both stop when max(|p_x| / sd, |p_s| / sd, |c - s|,
 * complementarity) <= tol with sd = max(1, mean |multiplier| / 100).
 * Start: flat voltages, generation at the middle of its box, consistent
 * flows, every bounded entry pushed 1e-2 max(1, |bound|) inside; y = 0,
 * bound multipliers 1. */
typedef struct {
  double tol;      /* stopping tolerance (1e-4)                          */
  int32_t max_iter; /* iteration limit (100)                             */
  double relax;    /* half-width of the relaxed equality rows (1e-4)     */
  double sigma;    /* centring factor of mu without line search (0.1)    */
  double tau;      /* fraction to the boundary without line search (0.99995) */
  double delta_c;  /* dual regularisation (1e-8)                         */
  double dw_first, dw_grow, dw_max; /* inertia correction (1e-4, 8, 1e10) */
  double pivot_tol; /* static pivot threshold of the factorization (0)   */
  int32_t verbose;  /* 1: progress lines per iteration on stderr, 2: also
                       each factorization's delta_w and static pivots (0) */
  int32_t line_search; /* 1: filter line search, monotone mu (1)         */
  double mu_init, kappa_eps, kappa_mu, theta_mu, tau_min; /* (0.1, 10, 0.2, 1.5, 0.99) */
  double gamma_theta, gamma_phi, eta_phi, s_theta, s_phi, delta; /* (1e-5, 1e-8, 1e-8, 1.1, 2.3, 1) */
  double gamma_alpha, kappa_sigma; /* (0.05, 1e10)                       */
  int32_t stall_iter; /* line search: stop as stalled when theta has not
                         fallen below 0.9 of its best for this many
                         iterations while max |c - s| > tol; 0: never (25) */
  double dw_grow_first, dw_shrink, dw_min; /* inertia correction with the
                         line search: first nonzero delta_w = dw_first if no
                         earlier iteration needed one, else
                         max(dw_min, dw_shrink * last); growth dw_grow_first
                         while none was needed before, else dw_grow
                         (100, 1/3, 1e-20) */
} opf_ipm_options;

enum { OPF_IPM_CONVERGED = 0, OPF_IPM_MAX_ITER = 1, OPF_IPM_STALLED = 2 };

typedef struct {
  int32_t converged;      /* 1 if the tolerance was met                  */
  int32_t iterations;     /* Newton steps taken                           */
  int32_t factorizations; /* including inertia-correction refactorizations */
  double objective;       /* sum over instances                           */
  double err;             /* final value of the stopping measure          */
  double seconds;         /* wall time of the call                        */
  double t_eval, t_factor, t_solve; /* evaluation + condensation, factorization, solve + recovery + step */
  int32_t status;         /* OPF_IPM_CONVERGED / _MAX_ITER / _STALLED      */
  int32_t trials;         /* line-search trial points evaluated           */
  double theta;           /* final |c(x) - s|_1                           */
} opf_ipm_result;

void opf_ipm_default_options(opf_ipm_options *opt);
/* chol: opf_chol_analyze of the same model.  x_out: device [n], receives
 * the final primal point; y_out: device [m] or NULL, the final multipliers
 * of c(x) - s = 0.  opt NULL = defaults.  Allocates its work vectors on the
 * model's device for the duration of the call and synchronises the model's
 * stream once per iteration (and once per line-search trial).  Returns
 * OPF_OK also when the iteration limit or a stall stops it
 * (res->converged = 0, res->status says which); OPF_EINVAL on bad options, a non-finite
 * iterate (any non-finite residual) or a failed inertia correction;
 * OPF_ENODEV on a host-only model. */
int opf_ipm_solve(opf_model *model, opf_chol *chol, const opf_ipm_options *opt,
                  double *x_out, double *y_out, opf_ipm_result *res);

/* Last error message of the calling thread ("" if none). */
const char *opf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* OPF_H */
