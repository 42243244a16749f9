/*
 * hps.h -- C ABI of the MI355X Hierarchical Poincare-Steklov (HPS) direct
 * solver: build (factor) and solve stages for
 *
 *     A u = g in Omega,  u = f on Gamma = boundary of Omega,
 *     A u = -c11 u_xx - 2 c12 u_xy - c22 u_yy + c1 u_x + c2 u_y + c u,
 *
 * on a rectangle Omega split into a binary tree of boxes whose leaves carry
 * a p x p Chebyshev grid and q Gauss nodes per side (Babb, Gillman, Hao,
 * Martinsson, arXiv:1612.02736: problem statement eqs. basic/defA, leaf
 * discretisation Sec. 3, merge Sec. 4, Algorithms 1 and 2, local refinement
 * Sec. 6).
 *
 * Conventions shared by every entry point
 *  - Return value: HPS_OK (0) or a negative HPS_E* code; a thread-local text
 *    explaining the last failure is available from hps_last_error().  No C++
 *    exception crosses this interface.
 *  - Floating point arrays are IEEE binary64 unless stated.  "host" arrays
 *    live in ordinary CPU memory; "device" arrays are HIP device pointers on
 *    the current device (for example torch CUDA tensors).  The caller owns
 *    every array it passes; the library never frees or keeps them.
 *  - Leaf order ("canonical"): leaves sorted by (problem, y0, x0).
 *  - Chebyshev grid of a leaf: node (ix, iy), 0 <= ix, iy < p, has index
 *    iy*p + ix; coordinates ascend.  Interior nodes 1 <= ix, iy <= p-2 are
 *    numbered (iy-1)*(p-2) + (ix-1).
 *  - Domain boundary Gauss nodes of a problem ("canonical"): sides S, E, N, W
 *    in that order, each in increasing coordinate; problems one after
 *    another.
 *  - Boundary flux convention of the paper (Sec. 3.1): +d/dx on vertical
 *    sides and +d/dy on horizontal sides.
 *  - Multiple right-hand sides are stored one after another ("RHS-major").
 *  - Work is enqueued on the HIP stream given in the options (0 = the null
 *    stream) and the calls return after the stream has drained, unless
 *    stated otherwise.
 */
#ifndef HPS_H
#define HPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HPS_OK = 0,
  HPS_EINVAL = -1,      /* bad argument (size, pointer, q >= p, nrhs <= 0) */
  HPS_ETREE = -2,       /* malformed tree (non-dyadic split, bad problem) */
  HPS_ESINGULAR = -3,   /* zero pivot in a leaf or interface block */
  HPS_ENONFINITE = -4,  /* NaN/Inf met in a pivot */
  HPS_ENOCONV = -5,     /* iterative refinement missed its tolerance */
  HPS_EHIP = -6,        /* a HIP runtime call failed */
  HPS_ENOMEM = -7       /* device or host allocation failed */
};

typedef struct hps_tree hps_tree;
typedef struct hps_handle hps_handle;

typedef struct {
  int n_problems;
  int n_leaves;          /* all problems together */
  int n_boxes;           /* leaves + merges, all problems */
  int n_levels;          /* distinct merge heights */
  int max_depth;         /* deepest refinement level below the base grid */
} hps_tree_info_t;

/* Options of hps_build; pass NULL for the defaults. */
typedef struct {
  int q;                 /* Gauss nodes per leaf side; 0 -> p - 1 */
  void *stream;          /* hipStream_t; 0 -> null stream */
  int keep_fp32;         /* 1: also keep FP32 copies of the solve operators
                            (needed for HPS_PREC_MIXED solves) */
  int economic;          /* 1: storage-economic version (the remark on a
                            storage efficient version, Sec. 5.4): the leaf
                            solution operators F are not kept, and every
                            solve redoes the leaf Gauss-Jordan eliminations
                            in chunks of 1024 leaves to apply F g.  Removes
                            the N q^2 storage term; FP64 forward solves only
                            (no keep_fp32, no adjoint). */
  int translation_invariant; /* 1: the coefficients are the same on every
                            leaf (a constant-coefficient operator on a tree
                            without refined interfaces; the remark after the
                            timings of Sec. 7.1): leaves, and merges within a
                            level, that have the same shape and position in
                            their parent get one shared copy of their
                            operators, built once.  hps_build and
                            hps_refactor compare the coefficients of every
                            leaf with the first leaf's on the device and
                            return HPS_EINVAL if any differ (bitwise); not
                            combined with economic. */
  void *workspace;       /* optional caller-owned device memory for the FP64
                            operators (for example a torch tensor), at least
                            hps_build_workspace_size() bytes, 256-byte
                            aligned; it also holds the reference matrices the
                            build uploads once, so the caller leaves it
                            untouched while the handle lives, and it must
                            outlive the handle, which never frees it.  NULL:
                            the library allocates the operator memory itself.
                            Build scratch, solve work vectors and FP32 copies
                            stay library-owned. */
  size_t workspace_bytes; /* size of workspace (ignored when it is NULL) */
} hps_build_opts;

enum { HPS_PREC_FP64 = 0, HPS_PREC_MIXED = 1, HPS_PREC_FP32 = 2 };

/* Options of hps_solve / hps_solve_adjoint; pass NULL for the defaults. */
typedef struct {
  int precision;         /* HPS_PREC_*; MIXED = FP32 sweeps + FP64 residual
                            iterative refinement */
  double ir_tol;         /* MIXED: relative error target (0 -> 1e-10).  Each
                            FP32 sweep solves the correction equation to a
                            relative accuracy rho (~1e-6), so after a
                            correction du the remaining error is about
                            rho max|du|; rho is estimated as the ratio of
                            successive corrections (the first sweep's u
                            counting as the first).  The refinement stops
                            when max|du| <= ir_tol max|u|, or when
                            rho <= 1e-3 and 100 rho max|du| <= ir_tol max|u|;
                            a solve that ends above it returns HPS_ENOCONV,
                            one that meets a NaN or Inf HPS_ENONFINITE */
  int max_iter;          /* MIXED: refinement steps (0 -> 6) */
  void *stream;          /* hipStream_t; 0 -> null stream */
  double *u_gauss;       /* optional device out [nrhs][n_gauss] */
  int *iters_out;        /* optional host out: refinement steps taken */
  double *resid_out;     /* optional host out: the estimated relative error
                            at exit (the smaller of max|du|/max|u| and rho
                            times it) */
} hps_solve_opts;

/* -- trees (host objects) ------------------------------------------------- */

/* A forest of n_problems copies of [x0,x1] x [y0,y1], each split into a
 * uniform nx x ny grid of leaf boxes (Sec. 2, Fig. 1).  A box covering
 * several leaves is cut across the direction with more leaves (x on ties);
 * the west/south part is child alpha.  Returns HPS_EINVAL for non-positive
 * sizes or an empty rectangle. */
int hps_tree_uniform(double x0, double x1, double y0, double y1, int nx,
                     int ny, int n_problems, hps_tree **out);

/* Side conditions (Sec. 7.6 solves a problem with zero Neumann data on two
 * sides and periodicity on the other two).  bc[4] gives sides S, E, N, W of
 * problem `problem` (-1: every problem):
 *  - HPS_BC_DIRICHLET: u is given (the default);
 *  - HPS_BC_NEUMANN: the flux is given, in the convention above (+d/dx on
 *    vertical sides, +d/dy on horizontal sides; the outward normal derivative
 *    is minus the data on the S and W sides);
 *  - HPS_BC_PERIODIC: opposite sides are identified (both of a pair).
 * A periodic pair shares one set of Gauss nodes, and the merge whose two
 * children meet across the seam eliminates it.  Neumann nodes stay exterior
 * up to the root, and one more elimination above the root solves the root's
 * relation flux = T u + h on them (the merge of Sec. 4 with a sibling whose
 * T is zero and whose flux is the data).  Build-time rules: a periodic
 * direction needs at least 4 leaves and no refined leaf on its sides; a
 * problem with a Neumann side needs at least 2 leaves; a problem without a
 * Dirichlet side needs q <= p - 2 (with q = p - 1 its discrete system is
 * singular).  The tree rules fail with HPS_ETREE in the node queries and
 * hps_build, the q rule with HPS_EINVAL in hps_build.  HPS_PREC_MIXED refines against the residual's flux rows at
 * the periodic seams and the Neumann nodes too, and hps_solve_adjoint
 * returns fbar = d/dpsi at Neumann entries and 0 at periodic entries.  A
 * translation_invariant build keys a seam-closing merge by its two shared
 * blocks and a closure by its root, so both get their own operators.
 * Errors: HPS_EINVAL (unknown code, unpaired periodic side, bad problem). */
enum { HPS_BC_DIRICHLET = 0, HPS_BC_NEUMANN = 1, HPS_BC_PERIODIC = 2 };
int hps_tree_set_bc(hps_tree *tree, int problem, const int *bc);

/* Sec. 6.1: n_ref rounds of splitting into 2 x 2 every leaf of problem
 * `problem` whose distance to (px, py) is <= t * (half its side); t = sqrt(2)
 * in the paper.  Must be called before hps_build; invalidates earlier
 * node queries. */
int hps_tree_refine_point(hps_tree *tree, int problem, double px, double py,
                          int n_ref, double t);

/* Sizes of the tree of boxes (Sec. 2: the domain is split into a binary
 * tree whose leaves carry the discretisation; Sec. 6.1 for refined trees):
 * problems, leaves, boxes, merge levels and refinement depth. */
int hps_tree_info(const hps_tree *tree, hps_tree_info_t *info);

/* Number of Gauss nodes for a given q (Sec. 2 and 3.1: q Gauss-Legendre
 * nodes on each leaf side, shared by the two leaves of an interior side):
 * all nodes, and those on the domain boundary (the length of f per
 * right-hand side). */
int hps_tree_counts(const hps_tree *tree, int q, int64_t *n_gauss,
                    int64_t *n_bdry);

/* host out [n_leaves][p*p][2]: (x, y) of every leaf Chebyshev node (the
 * p x p tensor grid of Sec. 3.1 on each leaf, where the coefficients and g
 * are sampled and u is returned). */
int hps_leaf_cheb_nodes(const hps_tree *tree, int p, double *xy);

/* host out [n_leaves][4]: x0, x1, y0, y1 of every leaf (Sec. 2). */
int hps_leaf_boxes(const hps_tree *tree, double *boxes);

/* host out [n_bdry][2]: canonical boundary Gauss nodes, where f is given
 * (Sec. 3.1 places q Gauss nodes on every leaf side; on a periodic side these
 * are the seam nodes it shares with its partner, at the partner's
 * coordinates). */
int hps_bdry_gauss_nodes(const hps_tree *tree, int q, double *xy);

/* host out [n_gauss][2]: every Gauss node in the order of u_gauss (the
 * vector u of Gauss-node values of Sec. 3.1 and Algorithm 2). */
int hps_gauss_nodes(const hps_tree *tree, int q, double *xy);

void hps_tree_free(hps_tree *tree);

/* -- build stage (Algorithm 1) -------------------------------------------- */

/* coeffs: device [n_leaves][6][p*p], nodal c11, c12, c22, c1, c2, c.
 * Builds F, S, H, T on every leaf (Sec. 3) and X, S, T on every merge
 * (Sec. 4), with P_up/P_down on refined interfaces (Sec. 6.3).  The
 * operators live in opts->workspace when one is given (caller-owned) and in
 * device memory of the handle otherwise; the handle keeps a copy of the
 * tree.  A workspace smaller than hps_build_workspace_size() or not 256-byte
 * aligned fails with HPS_EINVAL.
 * Errors: HPS_EINVAL (p < 4, q < 2, q >= p, NULL), HPS_ESINGULAR (message
 * names the first failing box), HPS_ENONFINITE, HPS_EHIP, HPS_ENOMEM.  On
 * failure *out is NULL. */
int hps_build(const hps_tree *tree, const double *coeffs, int p,
              const hps_build_opts *opts, hps_handle **out);

/* Algorithm 1 again on an existing handle for new coefficients (same tree,
 * p, q and layouts as hps_build): no device memory is allocated, the stored
 * operators are overwritten.  stream: hipStream_t (0 = null stream).
 * Errors as hps_build; on failure the handle's operators are undefined until
 * a successful refactor. */
int hps_refactor(hps_handle *h, const double *coeffs, void *stream);

/* Device bytes of the FP64 operators a build with these options stores
 * (opts may be NULL; its q, economic and translation_invariant fields
 * count): the size hps_build_opts.workspace must have.  Stored per leaf:
 * [S_ci | F], H and T (Sec. 3, eqs. alpine3-alpine4; without F for an
 * economic build, the storage-efficient version of Sec. 5.4), per merge X,
 * S and T (Sec. 4), and the refinement tables P (Sec. 6.3).  0 for bad
 * arguments. */
size_t hps_build_workspace_size(const hps_tree *tree, int p, const hps_build_opts *opts);

/* -- solve stage (Algorithm 2) -------------------------------------------- */

/* f: device [nrhs][n_bdry] (canonical boundary order): u on Dirichlet
 *    sides, the flux on Neumann sides, ignored on periodic sides;
 * g: device [nrhs][n_leaves][(p-2)^2] (interior Chebyshev nodes);
 * u: device out [nrhs][n_leaves][p*p].
 * Upward pass h = H g, w = X(h3b - h3a), h = [h1a; h2b] + [T13a; T23b] w;
 * downward pass u_gi = S u_ge + w, u_c = S u_ge + F g (Algorithm 2); on an
 * economic build F g is recomputed through the leaf Gauss-Jordan
 * eliminations, one chunk of leaves at a time (FP64 only). */
int hps_solve(hps_handle *h, const double *f, const double *g, int nrhs,
              double *u, const hps_solve_opts *opts);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): hps_solve
 * with the same arguments and results, whose work vectors and split-K
 * partials live in one fixed device array of the library
 * (HPS_SOLVE_NOALLOC_MAX_BYTES per device, held by every device that loads
 * the library until the process ends) instead of buffers the handle grows
 * on demand.  No hipMalloc, hipFree or allocating library routine runs.
 * The array's device address is looked up once per device, on the first
 * call with that device current.
 *  - precision: HPS_PREC_FP64 or HPS_PREC_FP32 only (HPS_EINVAL for MIXED);
 *    stored builds only (HPS_EINVAL for an economic handle); iters_out and
 *    resid_out, when given, receive 0.
 *  - HPS_EINVAL, with the bytes needed in the message, when nrhs right-hand
 *    sides need more work memory than the array holds (64 x 64 leaves,
 *    p = 16: 34.5 MB per right-hand side, so up to 7 fit; 32 x 32 leaves:
 *    7.6 MB, up to 35).
 *  - Every call on one device shares that device's array: calls that
 *    overlap on one device (other host threads, or other streams before
 *    this call's stream has drained) race and give undefined results.  The
 *    array keeps the last call's contents; every entry a solve reads it has
 *    written first, so nothing needs clearing between calls. */
#define HPS_SOLVE_NOALLOC_MAX_BYTES ((size_t)256 << 20)
int hps_solve_noalloc(hps_handle *h, const double *f, const double *g, int nrhs,
                      double *u, const hps_solve_opts *opts);

/* Transpose of the linear map (f, g) -> u_c of hps_solve (not in the
 * paper): given ubar [nrhs][n_leaves][p*p] (device) returns
 * fbar [nrhs][n_bdry] and gbar [nrhs][n_leaves][(p-2)^2] (device) by the
 * transposed sweeps, reusing the stored operators (HPS_EINVAL on an economic
 * build, which keeps no F).  Entries of fbar on periodic sides are 0 (their
 * data is not used). */
int hps_solve_adjoint(hps_handle *h, const double *ubar, int nrhs,
                      double *fbar, double *gbar, const hps_solve_opts *opts);

/* dL/dc for the zeroth-order coefficient c from the adjoint load gbar and the
 * forward solution u (both device, layouts as above):
 * cbar [nrhs][n_leaves][p*p] = -gbar * u on interior nodes, 0 on exterior
 * nodes (only the collocated PDE rows depend on c). */
int hps_coeff_grad_c(hps_handle *h, const double *u, const double *gbar,
                     int nrhs, double *cbar, void *stream);

/* sigma u - A u at the interior Chebyshev nodes of every leaf, with A the
 * handle's collocated operator (Sec. 3.2, the coefficients of the last build
 * or refactor).  u: device [nrhs][n_leaves][p*p]; out: device
 * [nrhs][n_leaves][(p-2)^2].  An implicit step u_t = A' u with the handle
 * built for L = I/k - A'/2 (Crank-Nicolson, Sec. 7.6) takes the right side
 * (I/k + A'/2) u = (2/k) u - L u, i.e. sigma = 2/k. */
int hps_apply_operator(hps_handle *h, const double *u, int nrhs, double sigma, double *out,
                       void *stream);

void hps_handle_free(hps_handle *h);

/* Thread-local description of the last failure on this thread. */
const char *hps_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HPS_H */
