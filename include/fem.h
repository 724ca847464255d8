/*
 * fem.h -- C ABI of the MI355X cell-loop finite element assembler.
 *
 * The library implements, on one AMD Instinct MI355X (gfx950), the parallel
 * loop of PyOP2 (Rathgeber et al., "Firedrake: automating the finite element
 * method by composing abstractions", section "PyOP2"): a local kernel is
 * executed for every cell of the mesh, reading coordinates and coefficients
 * gathered through Maps (access descriptor READ) and adding its element
 * tensor into a global sparse matrix (Mat) or vector (Dat) (access
 * descriptor INC).  The vocabulary follows the paper's data model:
 *
 *   Set       -- a number of entities (cells, vertices, nodes)      (Sets)
 *   Map       -- constant-arity table from one Set to another        (Maps)
 *   Dat       -- values attached to the members of a Set             (Data)
 *   Mat       -- sparse bilinear operator over a row and a column Set,
 *                assembled through two Maps; only WRITE and INC      (Matrix arguments)
 *   par_loop  -- for all e in E: kernel(f_0(m_0(e)), ..., f_n(m_n(e)))
 *                                                          (Parloops and kernels)
 *
 * Argument roles follow the Firedrake layer ("Assembling forms"): the output
 * tensor first, then the coordinate field, then the coefficients.
 *
 * Forms (integrand on each cell K, P_k Lagrange test v / trial u, P1
 * coefficient fields):
 *   FEM_HELMHOLTZ  kappa grad(u).grad(v) + u v
 *   FEM_LAPLACE    kappa grad(u).grad(v)
 *   FEM_MASS       u v
 *   FEM_SOURCE     f v              (linear form)
 *   FEM_NL_RESIDUAL  kappa grad(u).grad(v) + u^3 v - f v   (nonlinear residual,
 *                  P1 only; u, kappa, f are P1 fields on the nodes; its
 *                  vector-Jacobian products come from
 *                  fem_par_loop_assemble_adjoint)
 *   FEM_ELASTICITY 2 mu eps(u):eps(v) + lam div(u) div(v)   (linear
 *                  elasticity, eps the symmetric gradient; vector P2 on
 *                  tetrahedra, form dim 3; mu, lam P1 fields; the element
 *                  contraction may run in FP32, BF16 or FP16 on the matrix
 *                  cores, geometry and the global sums stay FP64)
 *
 * Memory, ownership, ordering
 *   - Every pointer inside fem_map, fem_dat, fem_sparsity and fem_mat is a
 *     DEVICE pointer owned by the caller; it must stay valid until the work
 *     queued on the context stream has completed.
 *   - fem_ctx and fem_plan are library-owned (create/destroy pairs).
 *   - All work is queued on the context's HIP stream.  Calls that must
 *     return a host-visible result synchronise that stream and say so:
 *     fem_build_sparsity (counting pass returns nnz), fem_plan_create,
 *     fem_renumber, fem_sync.  The assembly calls and the action never
 *     synchronise and never allocate.
 *
 * Errors
 *   - Every call returns fem_status; no exception crosses the ABI and the
 *     library never aborts.  Argument errors are detected on the host before
 *     anything is queued.  Out-of-range Map entries are detected on the device
 *     by fem_build_sparsity and fem_plan_create (which read every entry) and
 *     reported as FEM_E_RANGE.  Device faults surface as FEM_E_DEVICE at the
 *     next synchronising call.  fem_last_error() describes the last failure.
 *
 * Local (per-cell) node order, shared by every Map of a P_k space:
 *   vertices 0..d in the cell-to-vertex Map's order; then edges in
 *   lexicographic order of local vertex pairs ((0,1),(0,2),(0,3),(1,2),(1,3),
 *   (2,3) on a tetrahedron; (0,1),(0,2),(1,2) on a triangle), the two P3
 *   nodes of an edge ordered from its lower local vertex; then P3
 *   tetrahedron faces (0,1,2),(0,1,3),(0,2,3),(1,2,3) or the P3 triangle's
 *   interior node.  Vector-valued spaces number DOF = node*dim + component
 *   (Firedrake layer, "Function spaces and functions").
 *
 * Determinism: results are bitwise reproducible run to run on the same
 * inputs and plan (the paper's colouring is deterministic, "Parloops and
 * kernels"); every sum is taken in an order fixed by the plan.
 */
#ifndef FEM_H
#define FEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fem_status {
    FEM_OK = 0,
    FEM_E_ARG = 1,          /* bad argument: null pointer, size/arity mismatch */
    FEM_E_RANGE = 2,        /* a Map entry outside its target Set               */
    FEM_E_OVERFLOW = 3,     /* a count exceeds an index type of the library     */
    FEM_E_UNSUPPORTED = 4,  /* (cell, degree, form, precision) not provided     */
    FEM_E_NOMEM = 5,        /* device or host allocation failed                 */
    FEM_E_DEVICE = 6        /* HIP runtime or kernel error                      */
} fem_status;

/* Access descriptors ("Access descriptors"; SUM, MIN and MAX are the
 * reductions of a Global, "Global arguments").  READ for inputs; a Mat or an
 * output Dat accepts WRITE (overwrite with the assembled sum) or INC (add the
 * assembled sum to the existing values). */
typedef enum fem_access { FEM_READ = 0, FEM_WRITE = 1, FEM_INC = 2, FEM_SUM = 3, FEM_MIN = 4, FEM_MAX = 5 } fem_access;

typedef enum fem_cell { FEM_TRIANGLE = 2, FEM_TETRAHEDRON = 3 } fem_cell;

/* Arithmetic of the local kernel.  FEM_FP64 everywhere.  FEM_FP32 for
 * FEM_NL_RESIDUAL (its residual and adjoint: element values and the per-row
 * sums in binary32 after FP64 edge vectors, results stored as float64).
 * FEM_FP32, FEM_BF16, FEM_FP16 for FEM_ELASTICITY: the operands of the
 * element contraction (the reference tensor and the per-cell geometry
 * factor, scaled per cell by a power of two) are rounded to that type and
 * multiplied on the matrix cores with FP32 accumulation; the element blocks
 * are kept in FP32 (FEM_FP32), bfloat16 (FEM_BF16) or binary16 with a
 * power-of-two scale per cell (FEM_FP16) until they are summed; the
 * Jacobian, its determinant and inverse are FP64 for every cell, and the
 * global sums are FP64.  Other combinations return
 * FEM_E_UNSUPPORTED. */
typedef enum fem_prec { FEM_FP64 = 0, FEM_FP32 = 1, FEM_BF16 = 2, FEM_FP16 = 3 } fem_prec;

typedef enum fem_kind {
    FEM_MASS = 0, FEM_LAPLACE = 1, FEM_HELMHOLTZ = 2, FEM_SOURCE = 3, FEM_NL_RESIDUAL = 4,
    FEM_ELASTICITY = 5
} fem_kind;

/* A Set: only a size ("Sets"). */
typedef struct fem_set { int64_t size; } fem_set;

/* A Map from->to of constant arity: values[e*arity + l] in [0, to->size),
 * int32, row-major [from->size][arity], device memory ("Maps").  version:
 * the caller's count of changes to the contents of values.  A plan records
 * the array and the version of every Map it was built from; a call with the
 * same array at another version (contents rewritten in place) is refused
 * with FEM_E_ARG, so that a stale plan is never applied. */
typedef struct fem_map {
    const fem_set *from;
    const fem_set *to;
    int32_t arity;
    const int32_t *values;
    uint64_t version;
} fem_map;

/* A Dat: set->size * dim float64 values, node-major [size][dim], device
 * memory ("Data").  Coordinates are a Dat of dim = geometric dimension on the
 * vertex Set. */
typedef struct fem_dat {
    const fem_set *set;
    int32_t dim;
    double *data;
} fem_dat;

/* CSR sparsity of a Mat: row_ptr int64 [nrows+1], col_idx int32 [nnz], columns
 * of each row ascending and unique; structural zeros kept; device memory. */
typedef struct fem_sparsity {
    int64_t nrows, ncols, nnz;
    int64_t *row_ptr;
    int32_t *col_idx;
} fem_sparsity;

/* A Mat: float64 values[nnz] in the CSR order of sp, device memory. */
typedef struct fem_mat {
    const fem_sparsity *sp;
    double *values;
} fem_mat;

/* A Global: one float64 value in device memory, visible from every cell
 * ("Global arguments"). */
typedef struct fem_global {
    double *data;
} fem_global;

/* The local kernel: form kind, cell shape, Lagrange degree of the test and
 * trial space (1..3), value dimension of that space (1; 3 for
 * FEM_ELASTICITY), contraction precision, quadrature degree.
 * qdegree: 0 (or any degree at least the integrand's) selects exact
 * integration, which is what every kernel does: each integrand is a
 * polynomial (degree 2k of P_k test and trial functions with a P1
 * coefficient, k+1 for the source, 4 for the P1 residual, 3 for elasticity)
 * integrated by exact reference tensors rounded once, so any exact rule gives
 * the same values up to rounding.  A positive qdegree below the integrand's
 * degree (an under-integrated form) is FEM_E_UNSUPPORTED. */
typedef struct fem_form {
    fem_kind kind;
    fem_cell cell;
    int32_t degree;
    int32_t dim;
    fem_prec prec;
    int32_t qdegree;
} fem_form;

/* par_loop data arguments other than the output: the iteration Set (cells),
 * the coordinate field (a P1 vector Dat read through cell_vertex), the
 * cell-to-node Map of the P_k space, and coefficient Dats.  For the linear
 * and bilinear forms they are P1 fields read through cell_vertex: coeff[0]
 * is kappa for the bilinear forms and f for FEM_SOURCE.  For
 * FEM_NL_RESIDUAL they are fields of the P1 space itself, on the node Set,
 * read through cell_node: coeff[0] = u, coeff[1] = kappa, coeff[2] = f (f is
 * not read by the adjoint).  For FEM_ELASTICITY coeff[0] = mu and coeff[1] =
 * lam (P1, through cell_vertex), and the coordinates are read through
 * cell_coord.  cell_coord: optional Map from the cells to the Set that
 * coords lives on (arity d+1); NULL means coords is a vertex Dat read
 * through cell_vertex.  FEM_ELASTICITY requires it, so that the coordinate
 * field may be discontinuous (per cell) and single cells may be reshaped
 * without moving their neighbours (coordinates are an ordinary field, "The
 * mesh abstraction"). */
typedef struct fem_args {
    const fem_set *cells;
    const fem_map *cell_vertex;
    const fem_dat *coords;
    const fem_map *cell_node;
    const fem_dat *coeff[4];
    int32_t ncoeff;
    const fem_map *cell_coord;
} fem_args;

typedef struct fem_ctx fem_ctx;
typedef struct fem_plan fem_plan;

/* Create a context on HIP device `device` queuing on `hip_stream` (a
 * hipStream_t; NULL = the null stream). */
fem_status fem_ctx_create(int device, void *hip_stream, fem_ctx **ctx);
void fem_ctx_destroy(fem_ctx *ctx);
fem_status fem_ctx_set_stream(fem_ctx *ctx, void *hip_stream);
/* Device memory of the context from the caller's allocator (for instance
 * torch's caching allocator): alloc(bytes, user) returns device memory on the
 * context's device, usable on the context's stream, or NULL (the call then
 * fails with FEM_E_NOMEM); release(ptr, user) gives it back.  Plans created
 * afterwards take their arrays from it and release them in fem_plan_destroy
 * (the allocator must outlive them); temporaries of the setup calls
 * (fem_build_sparsity without a work buffer, fem_plan_create,
 * fem_renumber, fem_facet_plan_create) are allocated and released inside
 * the call: a release may come before work queued on the context stream has
 * run, so the allocator must order reuse on that stream (torch's caching
 * allocator does, for memory allocated on it).  alloc == NULL and
 * release == NULL restore the HIP runtime (hipMalloc for plans, stream-
 * ordered hipMallocAsync for temporaries).  FEM_E_ARG if exactly one of the
 * two is NULL. */
fem_status fem_ctx_set_allocator(fem_ctx *ctx, void *(*alloc)(size_t bytes, void *user),
                                 void (*release)(void *ptr, void *user), void *user);
/* Text of the last failure on this context ("" if none); owned by ctx. */
const char *fem_last_error(const fem_ctx *ctx);
/* Synchronise the context stream; FEM_E_DEVICE on a pending device error. */
fem_status fem_sync(fem_ctx *ctx);

/*
 * Sparsity of the Mat assembled through row Map rmap and column Map cmap
 * (same source Set): row i holds every column that any cell incident to i
 * reaches through cmap (paper: PyOP2 builds the sparsity OP2 lacks, from a
 * pair of Maps; "Matrix arguments").  Two calls:
 *   1. sp->col_idx == NULL: writes sp->row_ptr (caller-allocated, nrows+1)
 *      and sets sp->nnz, sp->nrows = rmap->to->size, sp->ncols =
 *      cmap->to->size.  Synchronises (nnz is returned to the host).
 *   2. sp->col_idx != NULL (nnz entries, caller-allocated), row_ptr from the
 *      first call: fills the columns.  Does not synchronise.
 * FEM_E_RANGE if a Map entry is out of range, FEM_E_OVERFLOW if nnz or the
 * incidence count does not fit the library's int32 column/entry indices,
 * FEM_E_UNSUPPORTED if one row has more than 8192 distinct columns (rows
 * whose cells reach up to 2048 candidate columns, counted with repetition,
 * are formed in LDS; longer rows go through an LDS hash set of 8192
 * columns).
 * Scratch device memory: work_bytes == NULL: the call takes it from the
 * context's allocator and gives it back before returning.  work_bytes !=
 * NULL and work == NULL: a query; *work_bytes receives the bytes the call
 * needs for these Maps (the same for both passes) and nothing else is done.
 * work != NULL: the caller's buffer of *work_bytes bytes (at least the
 * queried size, else FEM_E_ARG, 256-byte aligned), used as scratch; the call
 * then allocates nothing.  The buffer is in use until the queued work has
 * run.
 */
fem_status fem_build_sparsity(fem_ctx *ctx, const fem_map *rmap, const fem_map *cmap,
                              fem_sparsity *sp, void *work, size_t *work_bytes);

/*
 * fem_build_sparsity for callers that cannot allocate device memory at all
 * (code under stream capture, serving loops, harnesses that forbid
 * allocation) and have no buffer to lend: the same two passes and results,
 * with the scratch taken from a fixed 32 MiB array in the device's global
 * memory that the library holds for the life of the process (one per GPU).
 * The call allocates nothing, neither on the device nor through the
 * context's allocator.  Maps whose scratch (the size the work_bytes query of
 * fem_build_sparsity reports) exceeds 32 MiB are refused with FEM_E_ARG
 * before anything is queued; FEM_E_DEVICE if the array's address could not
 * be looked up at fem_ctx_create.  Every call on one GPU uses the same
 * array: calls that overlap in time on one GPU (other streams, other
 * contexts of the process) race and must be serialised by the caller.
 */
fem_status fem_build_sparsity_noalloc(fem_ctx *ctx, const fem_map *rmap, const fem_map *cmap,
                                      fem_sparsity *sp);

/*
 * Sparsity of a vector-valued space from the node sparsity: every node entry
 * (n, m) becomes the bs x bs block of rows bs*n + a, columns bs*m + b
 * (node-major DOFs, "Function spaces and functions": the vector CSR is the
 * node CSR with each entry replaced by a dense block).  Row bs*n + a holds
 * bs * len(n) columns in ascending order.  Two calls, like
 * fem_build_sparsity:
 *   1. out->col_idx == NULL: writes out->row_ptr (caller-allocated,
 *      bs*node->nrows + 1) and sets out->nrows, ncols, nnz (= bs^2 node->nnz).
 *   2. out->col_idx != NULL (out->nnz entries): fills the columns.
 * node is a CSR built by fem_build_sparsity.  bs in 1..8.  FEM_E_OVERFLOW if
 * bs * ncols exceeds int32.  Neither call synchronises or allocates.
 */
fem_status fem_expand_sparsity(fem_ctx *ctx, const fem_sparsity *node, int32_t bs, fem_sparsity *out);

/*
 * Execution plan of the deterministic INC for one (form, args) pair.
 * With sp != NULL the plan serves fem_par_loop_assemble_mat on that
 * sparsity; with sp == NULL it serves fem_par_loop_assemble_vec and
 * fem_apply_action.  The plan partitions the rows of the output into
 * contiguous blocks, each owned by one workgroup that gathers every
 * contribution to its rows in an order fixed by the plan (conflict-free INC without
 * atomics; "Access descriptors": only INC needs a schedule).  It references
 * the Maps' device arrays: rebuild it if their contents change.  Synchronises;
 * allocates device memory owned by the plan.  A Mat row with more values than
 * one block holds in LDS is split into blocks of consecutive value slices;
 * FEM_E_UNSUPPORTED if the cells of one row of a Dat plan do not fit one
 * block.  FEM_E_ARG if the sparsity lacks an entry the Maps reach;
 * FEM_E_NOMEM if a device or host allocation fails.
 *
 * FEM_ELASTICITY plans (sp = the vector CSR, the 3x3-block expansion of the
 * node sparsity, e.g. from fem_expand_sparsity) hold, per node pair, the
 * list of its (cell, local pair) contributions in ascending cell id, and a
 * workspace for the element blocks of every cell ([cells][55][9] values of
 * float64 for FEM_FP64, float32 for FEM_FP32; [cells][55][10] 16-bit values
 * for FEM_BF16, bfloat16 with the tenth unused, and FEM_FP16, binary16 with
 * the tenth holding the cell's scale exponent).  Assembly calls on one plan
 * share that workspace: they must not overlap in time (queue them on one
 * stream).  FEM_E_OVERFLOW for 2^24 cells or more.
 */
fem_status fem_plan_create(fem_ctx *ctx, const fem_form *form, const fem_args *args,
                           const fem_sparsity *sp, fem_plan **plan);
void fem_plan_destroy(fem_plan *plan);
/* Plan statistics: number of row blocks, total (block, cell) pairs, bytes of
 * device memory held.  Any output pointer may be NULL. */
fem_status fem_plan_info(const fem_plan *plan, int64_t *nblocks, int64_t *cell_visits,
                         int64_t *device_bytes);

/*
 * A[rmap(c,i), cmap(c,j)] (+)= integral over cell c of the bilinear form, for
 * every cell c (par_loop with the Mat argument INC'd through two Maps).
 * acc = FEM_WRITE overwrites A->values with the sum, FEM_INC adds to them.
 * Asynchronous on the context stream; allocates nothing.  FEM_ELASTICITY
 * runs two kernels: the element blocks into the plan's workspace (matrix
 * cores, the form's precision), then the FP64 sums into A in ascending cell
 * order per value.
 */
fem_status fem_par_loop_assemble_mat(fem_ctx *ctx, const fem_plan *plan, const fem_form *form,
                                     const fem_args *args, fem_mat *A, fem_access acc);

/* b[cell_node(c,i)] (+)= integral over cell c of the linear form: f v_i
 * (FEM_SOURCE) or the residual kappa grad(u).grad(v_i) + u^3 v_i - f v_i
 * (FEM_NL_RESIDUAL). */
fem_status fem_par_loop_assemble_vec(fem_ctx *ctx, const fem_plan *plan, const fem_form *form,
                                     const fem_args *args, fem_dat *b, fem_access acc);

/*
 * Adjoint (vector-Jacobian product) assembly of the FEM_NL_RESIDUAL residual
 * F(u, kappa): for a P1 field lambda on the nodes,
 *   g_u[j]     (+)= sum_i lambda_i dF_i/du_j
 *               = sum over cells of integral of kappa grad(v_j).grad(lambda)
 *                                             + 3 u^2 v_j lambda,
 *   g_kappa[k] (+)= sum_i lambda_i dF_i/dkappa_k
 *               = sum over cells of integral of v_k grad(u).grad(lambda),
 * assembled like a Dat (the reverse mode of the residual; the paper's closing
 * discussion of adjoints through the same abstractions).  args as for the
 * residual (coeff[0] = u, coeff[1] = kappa); lambda, g_u, g_kappa are Dats on
 * the node Set; either output may be NULL.  Plan: a Dat plan (sp == NULL).
 * Asynchronous; allocates nothing.
 */
fem_status fem_par_loop_assemble_adjoint(fem_ctx *ctx, const fem_plan *plan, const fem_form *form,
                                         const fem_args *args, const fem_dat *lambda, fem_dat *g_u,
                                         fem_dat *g_kappa, fem_access acc);

/*
 * Global reduction over the cells ("Global arguments": globally integrated
 * quantities such as energy).  Each cell contributes q_K:
 *   bilinear forms (FEM_MASS, FEM_LAPLACE, FEM_HELMHOLTZ): the cell energy
 *     x_K^T A_K x_K of the field x (a Dat on the nodes), so that the SUM is
 *     the energy x^T A x without forming A;
 *   FEM_SOURCE: the integral of the P1 field f = coeff[0] over K (x unused,
 *     may be NULL), so that the SUM is the integral of f.
 * acc = FEM_SUM adds the sum of the q_K to g, FEM_MIN / FEM_MAX replace g by
 * the minimum / maximum of g and the q_K (initialise g to 0 or +/-inf as
 * wanted).  Plan: a Dat plan (sp == NULL), whose partial buffer the call uses,
 * so calls on one plan must not overlap.  The combination order is fixed by
 * cell index, so the value is bitwise reproducible.  Asynchronous; allocates
 * nothing.
 */
fem_status fem_par_loop_reduce(fem_ctx *ctx, const fem_plan *plan, const fem_form *form, const fem_args *args,
                               const fem_dat *x, fem_global *g, fem_access acc);

/*
 * Mixed function spaces by blocks ("Factorisation of mixed function spaces"):
 * a bilinear form on W = V^nfields (nfields copies of the scalar space of
 * `form` -- cell, degree; its kind is ignored) is split into its (test field
 * a, trial field b) parts, each of which is assembled by the scalar kernel
 * into its own Mat, mats[a*nfields + b] (a nested matrix; a block whose
 * values are NULL is zero and skipped).  Block (a, b) is
 *   blocks[a*nfields + b].scale * (the form of blocks[..].kind),
 * kind FEM_MASS, FEM_LAPLACE or FEM_HELMHOLTZ, with its own P1 coefficient
 * Dat (kappa of the stiffness term; NULL only for FEM_MASS).  Every block
 * shares the scalar sparsity and the Mat plan of (form, args, sp).  The
 * monolithic matrix over DOF f*nnodes + node is the block matrix of these.
 * Asynchronous; allocates nothing.
 */
typedef struct fem_block {
    fem_kind kind;
    double scale;
    const fem_dat *coeff;
} fem_block;
fem_status fem_par_loop_assemble_mixed(fem_ctx *ctx, const fem_plan *plan, const fem_form *form, const fem_args *args,
                                       int32_t nfields, const fem_block *blocks, fem_mat *mats, fem_access acc);

/*
 * Exterior facet integrals ("The mesh abstraction": the mesh's exterior
 * facets are an iteration Set of the parallel loop, the source of their own
 * Maps).  For a triangle mesh the facets are segments, for a tetrahedral mesh
 * triangles.  facet_vertex: the facet's d vertices (arity d); facet_node: the
 * nodes of the degree-k Lagrange element of the facet, in the facet's own
 * local order (its vertices in facet_vertex order, then its edges in
 * lexicographic order with the two P3 nodes from the lower vertex, then a P3
 * triangle's face node); coords: the vertex Dat (dim d); g: a P1 vertex Dat.
 * form: FEM_SOURCE with the mesh's cell and degree.
 *   b[i] (+)= sum over facets F of the integral over F of g v_i ds.
 * fem_facet_plan_create builds the node-to-facet incidence and a facet
 * workspace (synchronises, allocates); fem_par_loop_assemble_facets runs one
 * kernel over the facets and one over the node rows, summing each row in
 * ascending facet id (deterministic, no atomics; asynchronous, allocates
 * nothing; calls on one plan must not overlap).  b covers all nodes: WRITE
 * zeroes the rows no facet touches.
 */
typedef struct fem_facets {
    const fem_set *facets;
    const fem_map *facet_vertex;
    const fem_map *facet_node;
    const fem_dat *coords;
    const fem_dat *g;
} fem_facets;
fem_status fem_facet_plan_create(fem_ctx *ctx, const fem_form *form, const fem_facets *facets, fem_plan **plan);
fem_status fem_par_loop_assemble_facets(fem_ctx *ctx, const fem_plan *plan, const fem_form *form,
                                        const fem_facets *facets, fem_dat *b, fem_access acc);

/*
 * Dirichlet boundary conditions on an assembled system, in place (the paper's
 * Firedrake example assembles A with a DirichletBC and applies it to b).  For
 * every row r with mask[r] != 0: row r and column r of A become zero except
 * A[r][r] = diag, and b[r] = diag g[r].  Every other row i first lifts the
 * boundary values, b[i] -= sum of A[i][r] g[r] over its boundary columns r
 * (summed in a fixed order: bitwise reproducible), so that the modified
 * system keeps the solution and stays symmetric.  mask: uint8 [nrows] device; values: the Mat's values in sp's
 * order; b and g: float64 [nrows] device, g NULL for homogeneous conditions,
 * b NULL to modify A only (then g must be NULL).  Square Mats only.
 * Asynchronous; allocates nothing.
 */
fem_status fem_apply_dirichlet(fem_ctx *ctx, const fem_sparsity *sp, double *values, const uint8_t *mask,
                               double diag, double *b, const double *g);

/* Matrix-free action y (+)= A x with A the assembled bilinear form, computed
 * cell by cell without forming the CSR matrix (the paper's wave benchmark
 * assembles exactly such an action, grad(v).grad(phi), every time step). */
fem_status fem_apply_action(fem_ctx *ctx, const fem_plan *plan, const fem_form *form,
                            const fem_args *args, const fem_dat *x, fem_dat *y, fem_access acc);

/*
 * Locality renumbering (setup; the paper renumbers the mesh with RCM for
 * cache locality, experiments section "Problem setup"): host int32 outputs
 *   cell_perm[new]   = old cell    (size cells->size)
 *   vertex_perm[new] = old vertex  (size cell_vertex->to->size)
 *   node_perm[new]   = old node    (size cell_node->to->size)
 * ordering cells by the Hilbert index of their centroid and vertices and
 * nodes by the Hilbert index of their position, so that contiguous rows and
 * cells are compact in space.  Any output may be NULL.  The caller applies
 * the permutations to its inputs (outputs are then numbered in the new
 * order); nothing is hidden inside the library.  Synchronises.
 */
fem_status fem_renumber(fem_ctx *ctx, const fem_form *form, const fem_args *args,
                        int32_t *cell_perm, int32_t *vertex_perm, int32_t *node_perm);

/*
 * Request server: continuous batching of assemblies and actions on resident
 * models (the paper keeps data on the device across parallel loops; its fixed
 * per-call overheads are what batching amortises, "Experiments").
 *
 * A model is a mesh with the FP64 Helmholtz form of some degree: args as for
 * fem_plan_create with coeff[0] = kappa and coeff[1] = f (P1 vertex Dats).
 * fem_server_add_model builds its sparsity and Mat and Dat plans once and
 * keeps them resident (synchronises).  The caller's device arrays (Maps,
 * coordinates, fields, action inputs) must outlive the server; the Set/Map/
 * Dat descriptors are copied.
 *
 * A request is FEM_REQ_ASSEMBLE (the CSR matrix and the right-hand side
 * integral of f v, WRITE) or FEM_REQ_ACTION (y = A x for the caller's x on the
 * model's nodes).  Submitted requests queue in arrival order.
 * fem_server_poll, which never blocks, retires batches whose work has
 * finished and, while one of the `slots` is free, admits a batch: queued
 * requests taken in admission order (the queue head first, or by
 * fem_server_set_order the smallest) up to fem_server_set_batch's limits (64
 * requests and a bound on their estimated work by default) and as long as
 * each request's outputs fit the HBM budget
 * (hbm_budget bytes for resident models plus outputs in flight).  A batch's
 * work is queued on its slot's stream as one persistent launch per kernel
 * (Mat, source vector, action) and (dimension, degree) present, whose
 * workgroups take (request, row blocks) work items from a device counter:
 * requests of different meshes and degrees share launches, and batches
 * admitted while others run overlap with them on the device.  A request
 * completes with its batch.  Outputs come from an arena of the budget left
 * after the resident models, allocated at the first admission (so models
 * must be added before the first poll that admits a request) and carved on
 * the host without driver calls.  Its outputs
 * (device pointers from fem_server_result: CSR values in the model's
 * sparsity order and the vector, or y) stay valid until fem_server_release
 * returns their memory to the budget.  Results do not depend on the mix:
 * every row block is computed by the same code and in the same order as by
 * the single-request kernels and reads only its own request's inputs, so a
 * result is bitwise the same alone, batched with any other requests, and as
 * fem_par_loop_assemble_mat / _vec and fem_apply_action compute it.
 * `now` and `arrival_time` are the caller's clock (seconds); the server
 * stamps admission and completion with the `now` of the poll that saw them.
 * The server owns its slot streams (default priority); it restores the
 * context's stream before returning.  One host thread drives a server.
 */
typedef struct fem_server fem_server;
typedef enum fem_req_op { FEM_REQ_ASSEMBLE = 0, FEM_REQ_ACTION = 1 } fem_req_op;

fem_status fem_server_create(fem_ctx *ctx, int32_t slots, int64_t hbm_budget, fem_server **server);
void fem_server_destroy(fem_server *server);
fem_status fem_server_add_model(fem_server *server, const fem_form *form, const fem_args *args,
                                int32_t *model_id, int64_t *resident_bytes);
fem_status fem_server_submit(fem_server *server, int32_t model, int32_t op, const double *x,
                             double arrival_time, int64_t *request_id);
fem_status fem_server_poll(fem_server *server, double now, int32_t *completed, int32_t *running,
                           int32_t *queued);
fem_status fem_server_result(fem_server *server, int64_t request_id, const double **values,
                             const double **vec, double *t_admit, double *t_done);
fem_status fem_server_release(fem_server *server, int64_t request_id);
/* Hand out up to cap ids of requests completed (by earlier polls) and not yet
 * handed out, in completion order; *n receives the count. */
fem_status fem_server_take_completed(fem_server *server, int64_t *ids, int32_t cap, int32_t *n);
/* Admission policy: use only the first `slots` slots (1..the number created;
 * batches already running elsewhere finish normally); with share_cus != 0
 * (the default) a batch admitted while other batches run or requests wait
 * launches its persistent Mat kernels on half the compute units, so that it
 * does not shut the others out for its whole duration. */
fem_status fem_server_configure(fem_server *server, int32_t slots, int32_t share_cus);
/* Batch limits: at most max_requests requests (1..64; 1: every request runs
 * in launches of its own) and at most max_work of estimated work (the unit
 * of fem_server_set_order: cell visits times the local tensor size, plus the
 * Mat values of an assembly; 1e8 by default, about 0.1 ms of an MI355X).  A
 * request above max_work runs in a batch of its own, so that small requests
 * batched together do not wait for a large one (a request completes with its
 * batch).  FEM_E_ARG outside those ranges. */
fem_status fem_server_set_batch(fem_server *server, int32_t max_requests, double max_work);
/* Which queued request admission takes next.  FEM_SERVE_FIFO (the default):
 * the queue head.  FEM_SERVE_SHORTEST: the queued request of least estimated
 * work (cell visits of its plan times the local tensor size, plus the Mat
 * values of an assembly; ties go to the earlier), except that a head which
 * has waited max_wait seconds or more (by the poll's `now`) is taken first,
 * which bounds how long large requests can be passed over.  Results do not
 * depend on the order.  FEM_E_ARG for an unknown order or max_wait < 0. */
typedef enum fem_serve_order { FEM_SERVE_FIFO = 0, FEM_SERVE_SHORTEST = 1 } fem_serve_order;
fem_status fem_server_set_order(fem_server *server, int32_t order, double max_wait);
/* A resident model's sizes and its sparsity (device pointers owned by the server). */
fem_status fem_server_model_info(const fem_server *server, int32_t model, int64_t *cells, int64_t *nrows,
                                 int64_t *nnz, const int64_t **row_ptr, const int32_t **col_idx);

#ifdef __cplusplus
}
#endif

#endif /* FEM_H */
