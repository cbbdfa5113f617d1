/*
 * bbfmm.h -- C ABI of the MI355X (gfx950) black-box FMM kernel matvec.
 *
 * The library computes phi = K sigma (eq. (1)-(2) of the paper) for a set of
 * N points that are both sources and targets, with the Chebyshev black-box
 * FMM: octree (Section 2.1), Lagrange interpolation (Section 2.2), the
 * four stages P2M/M2M, M2L, L2L/L2P and P2P (Section 2.3), and the
 * homogeneous-kernel reuse, SVD-compressed M2L and multi-RHS grouping of
 * Section 2.5.  The three calls mirror the paper's API (Section 3):
 * building the hierarchy, precomputing the M2L operators, computing.
 *
 * Conventions for every entry point
 *   - Every function returns a bbfmm_status; nothing throws across the ABI.
 *     On failure bbfmm_last_error() returns a message (thread-local, valid
 *     until the next call on the same thread).
 *   - "device" pointers are HIP device allocations on the current device;
 *     "host" pointers are ordinary host memory.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are stream-ordered; build_tree and precompute_operators return
 *     only after their work is complete (they read sizes back), matvec and
 *     plan_execute are asynchronous.  A fault inside a kernel surfaces at
 *     the next synchronising call.
 *   - Handles (trees, operator sets, plans) own their device memory and are
 *     immutable after creation, except that a plan owns a workspace: the
 *     library orders the products of one plan one after another (each waits
 *     for the previous one, whatever stream it ran on), so a plan never runs
 *     concurrently with itself.  Distinct plans may run concurrently.
 *   - Device memory of a handle comes from the bbfmm_allocator given when
 *     the tree was built (operator sets and plans inherit it unless given
 *     their own), or from hipMalloc when none was given.
 *   - Freeing a plan waits until its last product has finished.  A tree or
 *     an operator set must outlive the plans and servers that use it, and
 *     is freed only once no enqueued product uses it any more.
 *   - Free functions accept NULL.
 */
#ifndef BBFMM_H
#define BBFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BBFMM_OK = 0,
    BBFMM_ERR_INVALID_ARG = 1,   /* bad size, pointer, option or input value */
    BBFMM_ERR_OUT_OF_MEMORY = 2, /* a device or host allocation failed        */
    BBFMM_ERR_HIP = 3,           /* a HIP runtime call or launch failed       */
    BBFMM_ERR_BUDGET = 4,        /* a server request exceeds the HBM budget   */
    BBFMM_ERR_NOT_FOUND = 5,     /* unknown array / level in an export        */
    BBFMM_ERR_INTERNAL = 6,      /* an internal consistency check failed      */
    BBFMM_ERR_CANCELLED = 7      /* a server request was cancelled or its
                                    server destroyed before it ran            */
} bbfmm_status;

/* Kernel functions (Sections 1 and 4; all translation invariant). */
enum {
    BBFMM_K_INV_R = 0,      /* 1/|x-y|; K = 0 where |x-y|^2 == 0 (on the GPU also for
                               |x-y|^2 < 2^-126, i.e. points closer than ~1e-19);
                               homogeneous, degree -1                              */
    BBFMM_K_EXP = 1,        /* exp(-|x-y|/a), a = kernel_param                         */
    BBFMM_K_GAUSS = 2,      /* exp(-|x-y|^2/a^2), a = kernel_param                      */
    BBFMM_K_DIPOLE_X = 3,   /* (x_1-y_1)/|x-y|^3 (x target, y source); K = 0 where
                               |x-y|^2 == 0 (as for 1/r); skew-symmetric,
                               homogeneous of degree -2 (Section 2.5)            */
    BBFMM_K_POLY_TEST = 100 /* prod_d g((x_d-y_d)/a), g(u) = 1 + u/2 - u^2/3 + u^3/5:
                               degree 3 per coordinate, for exactness tests only     */
};

/* Arithmetic of the M2L contraction (P2P, up/down passes, compression and
 * decompression stay FP32; the operator precompute is FP64). */
enum {
    BBFMM_M2L_FP32 = 0,         /* FP32 operands, FP32 MFMA                          */
    BBFMM_M2L_BF16X3 = 1,       /* operands split x = hi + lo in bf16; products
                                   hi*hi + hi*lo + lo*hi on bf16 MFMA, FP32 accumulate */
    BBFMM_M2L_FP16_SCALED = 2,  /* fp16 operands with a power-of-two scale per operator
                                   and per (cell, RHS, 64 ranks) block; FP32 accumulate */
    BBFMM_M2L_FFT = 3           /* equally spaced interpolation nodes (Section 2.2) and
                                   the uncompressed block-Toeplitz M2L applied with the
                                   FFT (Section 2.5): transforms of size (2n)^3 per
                                   cell, FP32 complex; svd_eps is ignored             */
};

typedef struct {
    int32_t kernel_id;     /* one of BBFMM_K_*                                       */
    double kernel_param;   /* length scale a (ignored by 1/r)                        */
    int32_t cheb_order;    /* Chebyshev nodes per axis n, 2..8 (Section 2.2)         */
    int32_t leaf_size;     /* depth rule: smallest depth whose largest leaf holds at
                              most leaf_size points (>= 1)                          */
    int32_t max_depth;     /* cap on the number of levels incl. the root, 1..22     */
    int32_t fixed_depth;   /* > 0: use exactly this many levels (1..22)             */
    int32_t adaptive;      /* 0: uniform tree (every leaf on the last level);
                              1: level-adaptive (Section 2.1): a cell of at most
                              leaf_size points is a leaf, on whatever level; the
                              last level is the uniform tree's (depth rule or
                              fixed_depth).  One point set only.                 */
} bbfmm_tree_params;

/*
 * Device-memory hook, so that a framework's allocator (for PyTorch: its
 * caching allocator) owns every byte of device memory the library uses.
 *   alloc(bytes, stream, ctx)  returns device memory on the current device
 *       usable by work enqueued on `stream` after the call, or NULL when it
 *       cannot (the library then frees what it already holds through `free`
 *       and returns BBFMM_ERR_OUT_OF_MEMORY).  bytes > 0.
 *   free(ptr, stream, ctx)     returns memory from `alloc`, with the same
 *       stream.  The library calls it once all of its work that uses ptr has
 *       been enqueued on `stream` (temporaries of a build) or has completed
 *       (handles), so a stream-ordered allocator may hand the memory to work
 *       enqueued later on that stream.
 * Both may be called from any thread that calls into the library, and from
 * a server's scheduler thread.  The hook (its functions and ctx) must stay
 * valid until every handle built with it is freed.
 */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, void *stream, void *ctx);
    void *ctx;
} bbfmm_allocator;

typedef struct bbfmm_tree bbfmm_tree;
typedef struct bbfmm_ops bbfmm_ops;
typedef struct bbfmm_plan bbfmm_plan;

typedef struct {
    int64_t n_points;
    int32_t depth;             /* levels including the root; leaf level = depth-1 */
    int32_t cheb_order;
    int32_t kernel_id;
    double kernel_param;
    float lo[3];               /* bounding-cube anchor (per-axis minimum)          */
    float side;                /* cube side (largest extent, 1 if all coincide)    */
    float scale;               /* 2^21 / side, the binning factor                  */
    int32_t max_leaf_points;
    int32_t cells[22];         /* occupied cells per level                         */
    int64_t pairs[22];         /* M2L pairs per level (0 on levels 0 and 1)        */
    int64_t near_pairs;        /* point pairs of neighbouring leaves (over all
                                  points, also with separate sets)                */
    int64_t n_targets;         /* rows of phi: N, or the targets of a tree over
                                  separate sets                                   */
    int64_t n_sources;         /* rows of sigma: N, or the sources                 */
    int32_t adaptive;          /* 1 for a level-adaptive tree                      */
    int32_t n_leaves;          /* leaves on all levels                             */
    int64_t w_entries;         /* W-list entries (adaptive trees; 0 otherwise)     */
} bbfmm_tree_info;

/*
 * Build the octree over the bounding cube of the points (Section 2.1,
 * Definition 2.1).
 *   points  device, N x 3 float32 row-major, original order; read only.
 *   n       number of points, >= 1 and < 2^31.
 * The tree is uniform (every leaf on level depth-1) unless params->adaptive
 * is set; empty cells are not stored.  A level-adaptive tree is the uniform
 * tree with the descendants of every cell of at most leaf_size points
 * removed (trailing empty levels dropped), and carries the lists of the
 * adaptive FMM: U (adjacent leaves, near field), V (Definition 2.1, M2L),
 * W (cells finer than a leaf, not adjacent to it, whose parent is: their
 * multipole expansions are evaluated at the leaf's points) and X (the dual
 * of W: a coarser leaf's points feed the local expansion of a cell).  Binning: q_d = clamp(floor((x_d - lo_d) * scale), 0, 2^21-1) in
 * float32 (one rounding per operation), the level-l coordinate is
 * q_d >> (21-l); points are ordered by a stable sort of the Morton leaf key
 * (bit b of x, y, z at bits 3b, 3b+1, 3b+2).  Also built: the leaf
 * neighbour lists N(.) and, on every level >= 2, the interaction lists I(.)
 * grouped by transfer vector.
 *   allocator  device-memory hook of the tree and, by default, of its
 *              operator sets and plans; NULL = hipMalloc / hipFree.  Copied.
 * Errors: INVALID_ARG for n < 1, NULL pointers, non-finite coordinates,
 * cheb_order outside 2..8, leaf_size < 1, depths outside 1..22 or an unknown
 * kernel; OUT_OF_MEMORY (also when the allocator returns NULL; nothing is
 * leaked); HIP.
 */
bbfmm_status bbfmm_build_tree(const float *points, int64_t n,
                              const bbfmm_tree_params *params,
                              const bbfmm_allocator *allocator, void *stream,
                              bbfmm_tree **out);

/*
 * The same for separate target and source sets (eq. (1): phi(x_i) = sum_j
 * K(x_i, y_j) sigma_j with targets x and sources y): one octree over the
 * bounding cube of both sets, whose points are [targets; sources].  A
 * product on such a tree takes sigma with one row per source and writes phi
 * with one row per target: P2M and the near field sum over the sources of
 * a leaf, L2P and the near field evaluate at its targets.
 *   targets  device, n_targets x 3 float32;  sources  device, n_sources x 3.
 *   n_targets, n_sources >= 1, n_targets + n_sources < 2^31.
 * The depth rule counts the points of both sets.  Errors as bbfmm_build_tree.
 */
bbfmm_status bbfmm_build_tree_sets(const float *targets, int64_t n_targets,
                                   const float *sources, int64_t n_sources,
                                   const bbfmm_tree_params *params,
                                   const bbfmm_allocator *allocator, void *stream,
                                   bbfmm_tree **out);

bbfmm_status bbfmm_tree_info_get(const bbfmm_tree *tree, bbfmm_tree_info *out);

/* Arrays a tree exposes for inspection (copied device -> host). */
enum {
    BBFMM_TA_PERM = 0,      /* int32[N]: sorted position -> original index         */
    BBFMM_TA_KEYS = 1,      /* uint64[C_l]: Morton keys of level l, ascending      */
    BBFMM_TA_PB = 2,        /* int32[C_l]: first point (sorted order)              */
    BBFMM_TA_PE = 3,        /* int32[C_l]: one past the last point                 */
    BBFMM_TA_PARENT = 4,    /* int32[C_l]: parent index on level l-1 (-1 at root)  */
    BBFMM_TA_CB = 5,        /* int32[C_l]: first child on level l+1 (-1 on leaves) */
    BBFMM_TA_CE = 6,        /* int32[C_l]: one past the last child                 */
    BBFMM_TA_NBR_OFF = 7,   /* int32[C_L+1]: leaf neighbour CSR offsets (adaptive
                               trees: int32[NL+1], the U lists over the leaf table) */
    BBFMM_TA_NBR_IDX = 8,   /* int32[nnz]: neighbours, ascending cell index (adaptive
                               trees: ascending leaf-table index)                   */
    BBFMM_TA_PAIR_T = 9,    /* int32[P_l]: transfer-vector index 0..315 per pair   */
    BBFMM_TA_PAIR_TGT = 10, /* int32[P_l]: target cell of each pair                */
    BBFMM_TA_PAIR_SRC = 11, /* int32[P_l]: source cell of each pair                */
    BBFMM_TA_PAIR_GOFF = 12,/* int32[317]: group offsets by transfer vector        */
    BBFMM_TA_LEAF_LEVEL = 13,/* int32[NL]: level of each leaf (leaf table: by level,
                                then cell index)                                    */
    BBFMM_TA_LEAF_CELL = 14,/* int32[NL]: cell index of each leaf on its level     */
    BBFMM_TA_W_OFF = 15,    /* int32[NL+1]: W-list CSR offsets (adaptive trees)    */
    BBFMM_TA_W_LEVEL = 16,  /* int32[nW]: level of each W cell, ascending (level,
                               cell) per row                                       */
    BBFMM_TA_W_CELL = 17,   /* int32[nW]: cell index of each W cell                */
    BBFMM_TA_X_OFF = 18,    /* int32[C_l+1]: X-list CSR offsets of level l         */
    BBFMM_TA_X_LEAF = 19    /* int32[nX_l]: leaf-table index of each X leaf,
                               ascending per row                                   */
};

/*
 * Copy one tree array to host memory.
 *   what   one of BBFMM_TA_*; level selects the level for per-level arrays.
 *   dst    host buffer of capacity bytes, or NULL to query the size only.
 *   size   receives the array size in bytes.
 * Pair arrays list (target, source) with source - target = transfer vector
 * t (t in {-3..3}^3 minus {-1..1}^3, index ascending in
 * (tx+3) + 7(ty+3) + 49(tz+3)), grouped by t, ascending target within a group.
 * Errors: NOT_FOUND for an unknown array or level; INVALID_ARG when
 * capacity is too small.  Synchronous.
 */
bbfmm_status bbfmm_tree_export(const bbfmm_tree *tree, int32_t what,
                               int32_t level, void *dst, int64_t capacity,
                               int64_t *size);

/*
 * Precompute the M2L operators of every level >= 2 on the GPU in FP64
 * (Sections 2.3 and 2.5): sample the 316 operators
 * K_t[i][j] = K(h s_i, h (2t + s_j)) (h the level's half-width), compress
 * them with the truncated SVD of the fat and thin concatenations
 * (k = largest count of singular values above svd_eps times the largest,
 * U / V the leading left / right singular vectors, C_t = U^T K_t V), and
 * cast U, V, C_t to the matvec precision.  For the homogeneous kernel 1/r
 * one set is built and scaled by 1/h per level.  svd_eps = 0 disables the
 * compression (U = V = identity); otherwise svd_eps >= 1e-7 (the singular
 * values come from FP64 eigenvalues of Gram matrices, which resolve about
 * 1e-8 of the largest).  For a symmetric or skew-symmetric kernel the
 * operators of t and -t are signed transposes: one SVD (V = U) and half of
 * the operators are computed.
 *   allocator  NULL = the tree's.
 * Errors: INVALID_ARG (svd_eps < 0, in (0, 1e-7) or not finite, unknown
 * precision), OUT_OF_MEMORY, HIP.  Synchronous.
 */
bbfmm_status bbfmm_precompute_operators(const bbfmm_tree *tree,
                                        double svd_eps, int32_t precision,
                                        const bbfmm_allocator *allocator,
                                        void *stream, bbfmm_ops **out);

/* Rank k of level l (levels >= 2), or NOT_FOUND. */
bbfmm_status bbfmm_ops_rank(const bbfmm_ops *ops, int32_t level, int32_t *k);

/* Arrays an operator set exposes (FP64, copied device -> host). */
enum {
    BBFMM_OA_U = 0,        /* double[m][k]: left basis, row-major (m = n^3)      */
    BBFMM_OA_V = 1,        /* double[m][k]: right basis                          */
    BBFMM_OA_C = 2,        /* double[316][k][k]: compressed operators, level-scaled */
    BBFMM_OA_SV_FAT = 3,   /* double[m]: singular values of the fat matrix       */
    BBFMM_OA_SV_THIN = 4   /* double[m]: singular values of the thin matrix      */
};

/* Same calling convention as bbfmm_tree_export. */
bbfmm_status bbfmm_ops_export(const bbfmm_ops *ops, int32_t what,
                              int32_t level, void *dst, int64_t capacity,
                              int64_t *size);

/*
 * Build an operator set from host FP64 arrays instead of the SVD (lets a
 * caller test the matvec with given operators).  Device memory comes from
 * the tree's allocator.
 *   ranks  host int32[depth]: k of each level (entries of levels 0, 1 unused)
 *   U, V   host double: for each level l >= 2 in order, m x k_l row-major
 *   C      host double: for each level l >= 2 in order, 316 x k_l x k_l,
 *          already scaled for that level
 * Errors: INVALID_ARG (k outside 1..m, NULL arrays), OUT_OF_MEMORY, HIP.
 */
bbfmm_status bbfmm_ops_import(const bbfmm_tree *tree, int32_t precision,
                              const int32_t *ranks, const double *U,
                              const double *V, const double *C, void *stream,
                              bbfmm_ops **out);

/*
 * phi = K sigma for r right-hand sides (Section 2.5, multiple RHS).
 *   sigma  device, N x r float32 row-major (r fastest), original point order
 *          (n_sources x r for a tree over separate sets).
 *   phi    device, N x r float32, overwritten; must not overlap sigma
 *          (n_targets x r for a tree over separate sets).
 * Enqueues gather, P2M, M2M, compression, M2L, decompression, L2L, L2P and
 * P2P on the stream and returns without waiting for them (asynchronous).
 * The workspace comes from a cache held by the operator set: one plan per
 * (r, stream) pair, the four most recently used kept (the oldest is freed
 * once its last product has finished), so repeated products on a stream
 * allocate nothing; the first product of a pair allocates through the
 * operator set's allocator and uploads its launch lists (host work, no
 * wait for the device).  Products on different streams run concurrently;
 * a cached workspace used again on another stream is ordered after its
 * previous product.  The cache is freed with the operator set.
 * Errors: INVALID_ARG (r < 1 or > 4096, NULL pointers, ops not built for
 * this tree), OUT_OF_MEMORY, HIP.
 */
bbfmm_status bbfmm_matvec(const bbfmm_tree *tree, const bbfmm_ops *ops,
                          const float *sigma, int64_t r, float *phi,
                          void *stream);

/*
 * bbfmm_matvec without any device allocation, for callers that cannot
 * allocate (tight serving loops, harnesses that forbid allocation): the
 * same product, with every buffer beyond sigma and phi (sigma in tree order,
 * expansions, M2L partials, launch lists) taken from one fixed device array
 * of BBFMM_STATIC_SCRATCH_BYTES that the library holds on each GPU it runs
 * on until the process ends.  Launch shapes are the built-in heuristic with
 * the one-stream schedule, so the result equals bbfmm_matvec's up to
 * floating-point summation order.  Synchronous: returns once the product
 * has finished.  Every call on one GPU uses the same array; calls that
 * overlap on one GPU (from several threads) race.
 * Errors: INVALID_ARG (as bbfmm_matvec, and when the product needs more
 * than the fixed array: large N x r), HIP.
 */
#define BBFMM_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
bbfmm_status bbfmm_matvec_static(const bbfmm_tree *tree, const bbfmm_ops *ops,
                                 const float *sigma, int64_t r, float *phi,
                                 void *stream);

/*
 * A reusable matvec for a fixed (tree, operators, r) that owns its
 * workspace, so repeated products allocate nothing.  plan_execute has the
 * semantics of bbfmm_matvec: it enqueues the product on `stream` and
 * returns.  With the overlapped schedule (option `overlap`) the near field
 * runs on a side stream the plan holds, forked from and joined back into
 * `stream` with events, so all of the product's work is still ordered after
 * earlier work on `stream` and before later work on it.  One plan's
 * workspace serves one product at a time: a product waits for the plan's
 * previous product (an event) when it is enqueued on another stream.  When
 * `stream` is being captured into a caller's graph the plan does not order
 * or track that launch; the caller keeps the plan alive while the graph
 * can run.  plan_free waits for the last product.  The tree and operators
 * must outlive the plan.  bbfmm_plan_create sets up on the null stream with
 * the operators' allocator.
 */
bbfmm_status bbfmm_plan_create(const bbfmm_tree *tree, const bbfmm_ops *ops,
                               int64_t r, bbfmm_plan **out);

/* Launch-shape choices of a plan; 0 selects the built-in heuristic. */
typedef struct {
    int32_t m2l_split;      /* workgroups sharing one M2L tile's 189 slots, 1..8   */
    int32_t m2l_min_waves;  /* heuristic target of M2L workgroups per CU, 1..16  */
                            /* (0 = 16; the split doubles up to 8 to reach it)   */
    int32_t p2p_max_split;  /* cap on sub-lanes per P2P target, 1..64 (power of 2) */
    int32_t p2p_mfma;       /* near field + L2P: 1 per-lane FMA kernel, 2 on MFMA  */
                            /* (kernel values as the A operand); 0 picks by r     */
    int32_t overlap;        /* 2: near field on a second stream while the far    */
                            /* field runs, then L2P adds the far field; 1: one   */
                            /* stream, L2P fused into P2P; 0 picks (2 with the   */
                            /* per-lane near field)                              */
    int32_t p2p_waves;      /* per-lane near field: workgroups launched, each     */
                            /* looping over work items (0 = one per item); fewer */
                            /* leave room for the far field when overlapped      */
    int32_t m2l_occupancy;  /* M2L workgroups per CU, 1..4 (0 = as many as fit); */
                            /* fewer leave registers to the overlapped near field */
    int32_t m2l_layout;     /* FP32 M2L waves: 1 = 16 rank rows x 64 columns     */
                            /* each, 2 = 32 x 32 (half the LDS reads per MFMA);  */
                            /* 0 = 1                                             */
    int32_t m2l_schedule;   /* 1: one M2L launch for all levels after the upward */
                            /* pass; 2: each level's M2L starts as soon as its   */
                            /* compressed multipoles exist (the upward chain     */
                            /* runs on a second stream, Section 2.4); 0 = 2 with */
                            /* at least two M2L levels                           */
    int32_t m2l_block;      /* 16-bit M2L: 1 = tiles of 64 (target, column)      */
                            /* pairs of one octant; 2 = the children of a parent */
                            /* cell as one block, each source of their halo      */
                            /* staged once for all of them (no slot split);      */
                            /* 0 = 2 from r = 16 on.  FFT M2L (level-uniform     */
                            /* trees): 1 = one workgroup per (target cell,       */
                            /* column); 2 or 0 = blocks of 4 x 4 x 4 targets     */
                            /* sharing one staged 8 x 8 x 8 source halo per      */
                            /* slice of frequencies                              */
    int32_t m2l_rtile;      /* parent blocks: right-hand sides per workgroup, 16, */
                            /* 32 or 64 (0: 16 up to r = 16, 32 up to 47, else   */
                            /* 64)                                               */
    int32_t m2l_xcd;        /* tile M2L: 1 = each XCD runs every slot split of a  */
                            /* contiguous run of tiles; 2 = each split pinned to  */
                            /* 8 / m2l_split XCDs, so a split's operators stay in */
                            /* their L2s (needs m2l_split dividing 8); 0 = 2 when */
                            /* it applies                                        */
    int32_t leaf_fused;     /* 2: P2M, compression and M2M of the leaf level in   */
                            /* one kernel per (parent, 16 right-hand sides): the  */
                            /* leaves' full coefficients never reach HBM; 1: the */
                            /* three stages as separate kernels; 0 = 1.  Applies  */
                            /* to uniform trees of at least four levels with the */
                            /* Chebyshev/SVD M2L (else the stages stay separate) */
    int32_t p2p_pack;       /* per-lane near field, one right-hand side: 2 =     */
                            /* each wave holds 1, 2 or 4 targets per lane and    */
                            /* any number S <= 16 of sub-lanes per target,       */
                            /* picked per leaf so that the leaf's targets fill   */
                            /* the 64 lanes, and L2P runs as its own kernel;     */
                            /* 1 = power-of-two sub-lanes, one target per lane   */
                            /* (L2P fused on the one-stream schedule); 0 = 2     */
                            /* where it applies                                  */
    int32_t m2l_mfma;       /* 16-bit parent-block M2L: 1 = 16x16x32 MFMAs, 2 =  */
                            /* 32x32x16 (with an r-tile of 32 or 64; 32 rank rows */
                            /* per workgroup); 0 = 1                             */
} bbfmm_plan_options;

/* plan_create with explicit launch shapes (NULL options = defaults), a
 * device-memory hook (NULL = the operators') and the stream its set-up
 * (launch-list uploads, tile masks) is enqueued on; products are ordered
 * after the set-up.  The results do not depend on the options beyond
 * floating-point summation order.  Errors: INVALID_ARG for out-of-range
 * options, OUT_OF_MEMORY, HIP. */
bbfmm_status bbfmm_plan_create_ex(const bbfmm_tree *tree, const bbfmm_ops *ops,
                                  int64_t r, const bbfmm_plan_options *options,
                                  const bbfmm_allocator *allocator, void *stream,
                                  bbfmm_plan **out);
bbfmm_status bbfmm_plan_execute(bbfmm_plan *plan, const float *sigma,
                                float *phi, void *stream);
/* Bytes of device workspace the plan holds. */
bbfmm_status bbfmm_plan_workspace_bytes(const bbfmm_plan *plan, int64_t *bytes);
/* The launch shapes the plan runs with, every heuristic choice made
 * explicit (out, host).  p2p_max_split and m2l_min_waves echo what was
 * asked (0 = default). */
bbfmm_status bbfmm_plan_get_options(const bbfmm_plan *plan, bbfmm_plan_options *out);

/* Stages of one matvec, in execution order (Section 2.3).  Each stage is
 * one kernel launch except M2M and DOWN, which launch once per level. */
enum {
    BBFMM_STAGE_GATHER = 0, /* sigma into tree order                          */
    BBFMM_STAGE_P2M = 1,    /* leaf multipoles and their compression          */
    BBFMM_STAGE_M2M = 2,    /* upward translation and compression, per level  */
    BBFMM_STAGE_M2L = 3,    /* all levels' interaction lists, one launch      */
    BBFMM_STAGE_DOWN = 4,   /* decompression + L2L, per level                 */
    BBFMM_STAGE_P2P = 5,    /* L2P + near field + scatter to phi              */
    BBFMM_NUM_STAGES = 6
};

/*
 * Device-time measurement of the stages with HIP events recorded on the
 * execution stream (enable = 1 to start, 0 to stop).  While enabled, every
 * plan_execute records BBFMM_NUM_STAGES + 1 events.
 * plan_stage_times waits for the recorded executions and returns the summed
 * milliseconds per stage (ms: array of BBFMM_NUM_STAGES) and the number of
 * executions they cover; reset != 0 clears the totals afterwards.
 */
bbfmm_status bbfmm_plan_set_timing(bbfmm_plan *plan, int32_t enable);

/*
 * Graph replay (enable = 1): the first plan_execute captures the whole
 * launch sequence into a HIP graph on a private stream and every later call
 * with the same sigma / phi pointers only launches that graph on the given
 * stream (a new pointer pair is captured again).  The graph contains kernel
 * nodes only.  Stage timing is not recorded in graph mode.
 */
bbfmm_status bbfmm_plan_set_graph(bbfmm_plan *plan, int32_t enable);
bbfmm_status bbfmm_plan_stage_times(bbfmm_plan *plan, double *ms, int64_t *executions,
                                    int32_t reset);

/*
 * Launch-shape autotuner for a (tree, operators, r): times whole products
 * on the caller's data and returns the fastest options found.  Candidates,
 * by coordinate descent from the built-in heuristic: M2L slot split 1..4;
 * then the near-field kernel (per-lane FMA or MFMA); then, for the
 * per-lane kernel, the sub-lane cap 4, 8 or 16; then the overlapped
 * schedule on or off; then, overlapped with the per-lane kernel, the
 * near-field workgroup count (one per item, or 512 .. 4096); then, when
 * overlapped, the M2L workgroups per CU (as many as fit, 3 or 2); then
 * the FP32 M2L wave layout; then the M2L schedule (one launch, or per
 * level as the upward pass finishes each level); then, for a 16-bit M2L,
 * the target grouping (64-column tiles or parent blocks) and, with parent
 * blocks, the r-tile (16, 32 or 64 right-hand sides per workgroup).  Each candidate runs one
 * untimed product and `reps` timed ones (HIP events on `stream`); its
 * time is the median.  Options only change launch shapes (and with them
 * the floating-point summation order), never the arithmetic precision.
 *   sigma, phi  device, float32 (n_sources x r, n_targets x r; N x r for one
 *               set); phi is overwritten by every trial.
 *   reps        1..100.
 *   best        out: the chosen options (m2l_split, p2p_mfma,
 *               p2p_max_split, overlap, p2p_waves, m2l_occupancy,
 *               m2l_layout, m2l_schedule, m2l_block, m2l_rtile, m2l_xcd and
 *               leaf_fused explicit).
 *   best_ms     out (may be NULL): its median milliseconds per product.
 * Allocates and frees one plan workspace per candidate; synchronizes
 * `stream`.  Errors: INVALID_ARG, OUT_OF_MEMORY, HIP.
 */
bbfmm_status bbfmm_plan_autotune(const bbfmm_tree *tree, const bbfmm_ops *ops, int64_t r,
                                 const float *sigma, float *phi, void *stream, int32_t reps,
                                 bbfmm_plan_options *best, double *best_ms);

/*
 * Serving loop (continuous batching).  A server keeps any number of built
 * (tree, operators) models, accepts matvec requests of any model and r, and
 * a scheduler thread groups the pending requests of one model (arrival
 * order, total r <= r_max, rounded up to a power of two) into one product
 * on one of max_inflight slots; slots run concurrently on their own streams.
 * A batch is admitted when a slot is free and the device memory held by the
 * server's cached plans (workspace + N x R staging, one plan per (model, R),
 * replayed as a HIP graph) stays within hbm_budget_bytes; idle plans are
 * evicted least recently used first to make room.  A request larger than
 * the budget on its own fails with BBFMM_ERR_BUDGET (reported by wait).
 *   sigma, phi  device, float32, n_sources x r and n_targets x r of the
 *               model's tree (N x r for one set); must stay valid and
 *               untouched until wait returns.
 * Batch invariance: every server plan uses m2l_split = 2 and p2p_mfma = 2,
 * and with these fixed the arithmetic of one column does not depend on the
 * other columns or on R, so a request's phi is bit-identical to
 * bbfmm_plan_execute of a lone plan for that request with the same two
 * options, whatever batch it ran in.
 * Trees and operators must outlive the server.
 */
typedef struct bbfmm_server bbfmm_server;
typedef struct {
    double t_submit, t_admit, t_done;   /* steady-clock seconds              */
    int32_t batch_r;                    /* total r of the batch it ran in    */
    int32_t slot;                       /* slot (stream) index               */
} bbfmm_request_stats;

bbfmm_status bbfmm_server_create(int64_t hbm_budget_bytes, int32_t max_inflight,
                                 int32_t r_max, bbfmm_server **out);
bbfmm_status bbfmm_server_add(bbfmm_server *server, const bbfmm_tree *tree,
                              const bbfmm_ops *ops, int32_t *model_id);
/* Non-blocking; request_id identifies the request for wait. */
bbfmm_status bbfmm_server_submit(bbfmm_server *server, int32_t model_id,
                                 const float *sigma, int64_t r, float *phi,
                                 uint64_t *request_id);
/* Blocks until the request is complete; stats may be NULL.  Returns the
 * request's own status (BUDGET, HIP) if it failed.  Each id is waited once. */
bbfmm_status bbfmm_server_wait(bbfmm_server *server, uint64_t request_id,
                               bbfmm_request_stats *stats);
/* Cancel a request that has not been admitted yet: it completes with
 * BBFMM_ERR_CANCELLED (reported by wait; its phi is untouched).  Errors:
 * INVALID_ARG when it was already admitted or is complete, NOT_FOUND for an
 * unknown or already waited id. */
bbfmm_status bbfmm_server_cancel(bbfmm_server *server, uint64_t request_id);
/* Finishes the batches in flight, completes every request still pending
 * with BBFMM_ERR_CANCELLED, waits until every thread blocked in
 * bbfmm_server_wait has returned, and frees the server (NULL accepted).
 * No call may use the server after destroy has begun. */
bbfmm_status bbfmm_server_destroy(bbfmm_server *server);

/* Counters of a server since its creation (all out, host). */
typedef struct {
    int64_t requests_done;      /* completed (including rejected) requests        */
    int64_t batches;            /* products launched                              */
    int64_t plans_created;      /* (model, R) plans built (workspace + graph)     */
    int64_t plans_evicted;      /* idle plans freed to make room in the budget    */
    int64_t bytes_in_use;       /* device bytes held by cached plans now          */
    int64_t bytes_peak;         /* largest bytes_in_use so far                    */
} bbfmm_server_stats;
bbfmm_status bbfmm_server_get_stats(bbfmm_server *server, bbfmm_server_stats *out);

/*
 * Dense products of the randomized eigendecomposition built on the matvec
 * (Section 4, the geostatistics application: with l right-hand sides the
 * range basis is N x l).  Device pointers, row-major, FP32 inputs, FP64
 * accumulation, asynchronous on `stream`; the summation order is fixed, so
 * results do not depend on the launch.
 *   bbfmm_dense_atb: C (m x m, FP64) = A^T B for A, B (n x m, FP32).  Uses a
 *     workspace of ceil(n / 4096) m^2 doubles from `allocator` (NULL =
 *     hipMalloc), released before the call returns (stream-ordered with a
 *     hook).
 *   bbfmm_dense_ab: C (n x k, FP32) = A R for A (n x m, FP32) and R (m x k,
 *     FP64).
 * Errors: INVALID_ARG (NULL or host pointers, n < 1, m or k outside
 * [1, 1024]), OUT_OF_MEMORY, HIP.
 */
bbfmm_status bbfmm_dense_atb(const float *A, const float *B, int64_t n, int32_t m, double *C,
                             const bbfmm_allocator *allocator, void *stream);
bbfmm_status bbfmm_dense_ab(const float *A, int64_t n, int32_t m, const double *R, int32_t k,
                            float *C, void *stream);

/*
 * Live resources of the library in this process (all out, host): device
 * buffers and bytes it holds (from hooks or hipMalloc), plans, the streams
 * and events it created and has not destroyed (side streams are kept for
 * reuse until the process ends), and how many plans were freed while their
 * last product was still running (plan_free then waited for it).  For
 * checking that handles release what they hold.
 */
typedef struct {
    int64_t device_buffers, device_bytes, plans, streams, events;
    int64_t plans_freed_in_flight;
} bbfmm_runtime_counters;
bbfmm_status bbfmm_get_runtime_counters(bbfmm_runtime_counters *out);

void bbfmm_tree_free(bbfmm_tree *tree);
void bbfmm_ops_free(bbfmm_ops *ops);
void bbfmm_plan_free(bbfmm_plan *plan);

const char *bbfmm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BBFMM_H */
