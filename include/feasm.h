/*
 * feasm: finite-element sparse-matrix assembly on MI355X (gfx950).
 *
 * C ABI of libfeasm.so.  The library turns per-element dense FP64 stiffness
 * matrices into a global sparse matrix, following Sky, Polindara, Muench,
 * Birk, "A flexible sparse matrix data format and parallel algorithms for
 * the assembly of sparse matrices in general finite element applications
 * using atomic synchronisation primitives" (arXiv 2012.00585):
 *
 *   symbolic phase  pattern_build   -> CSR and CRAC sparsity structure
 *   numeric phase   assemble_csr / assemble_crac / reassemble_values
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - An element is a dense n x n matrix K plus its DOF index array D
 *    (Section 2.1).  With k nodes per element and d DOFs per node,
 *    n = k*d; DOFs are node-major: local row a*d + c of K maps to global
 *    DOF d*conn[e][a] + c (the contiguous per-node numbering of Section 2.1).
 *  - Global matrix G has n_rows = n_cols = d*n_nodes.  Its pattern is the
 *    union over elements of {(D_e[r], D_e[s])}; columns of a row are sorted
 *    ascending; no entry is dropped, whatever its value (Section 3 intro).
 *  - All indices are 0-based.  Pattern arrays are int32; building a pattern
 *    whose nnz, number of CRAC integers or number of rows reaches 2^31
 *    fails with FEASM_EOVERFLOW.
 *  - "dev" pointers are HIP device memory on the current device; "host"
 *    pointers are ordinary host memory.  Streams are hipStream_t (NULL is
 *    the legacy default stream).
 *  - Every call returns a feasm_status.  No C++ exception crosses the ABI:
 *    the host running out of memory inside a call gives FEASM_ENOMEM.
 *    last_error() returns a thread-local message for the latest failure.
 *  - Threads: calls on different handles (and batches) are independent.
 *    Several threads may make numeric calls (assemble_*, reassemble_values,
 *    spmv_*, assemble_hex8, hex8_element_matrices) on one handle at once;
 *    the state those calls create on first use is created once, under a
 *    lock of the handle.  pattern_tune, spin_aborts and pattern_free must
 *    not overlap any other call on the same handle, and calls writing the
 *    same values buffer race as usual.
 *  - Numeric calls are asynchronous on the given stream; pattern_build
 *    synchronises with its stream before returning.
 */
#ifndef FEASM_H
#define FEASM_H

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct feasm_pattern feasm_pattern; /* opaque handle */

enum feasm_status {
    FEASM_OK = 0,
    FEASM_EINVAL = -1,    /* bad argument (null pointer, non-positive size, unknown flag) */
    FEASM_ERANGE = -2,    /* a node id outside [0, n_nodes) */
    FEASM_ENOMEM = -3,    /* device or host memory allocation failed */
    FEASM_EHIP = -4,      /* a HIP runtime call failed */
    FEASM_EOVERFLOW = -5, /* nnz, CRAC length, rows or element entries reach 2^31 */
    FEASM_ELIMIT = -6,    /* a documented implementation limit is exceeded */
    FEASM_EINCOMPLETE = -7 /* spin_aborts: row-lock lanes gave up, so the results
                              of those launches miss their rows' contributions */
};

/* pattern_build flags (bitwise or) */
enum {
    FEASM_BUILD_CSR = 1,    /* row_ptr[n_rows+1], col_idx[nnz] */
    FEASM_BUILD_CRAC = 2,   /* crac_row_ptr[n_rows+1], col_align[n_ca] */
    FEASM_BUILD_COLOUR = 4, /* element colouring for the atomic-free scatter */
    FEASM_BUILD_TILES = 8,  /* element tiles for the atomic scatter (see FEASM_SCATTER_ATOMIC) */
    FEASM_BUILD_OWNER_MAP = 16 /* the row-owned lookup record, built with the pattern */
};

/* format selector for reassemble_values */
enum { FEASM_FMT_CSR = 0, FEASM_FMT_CRAC = 1 };

/* scatter strategy of the numeric calls */
enum {
    FEASM_SCATTER_AUTO = 0,     /* the library's choice for this handle (row-owned) */
    FEASM_SCATTER_ATOMIC = 1,   /* hardware FP64 atomic adds.  Without tiles: one atomic
                                   per contribution.  With tiles (FEASM_BUILD_TILES): a
                                   workgroup sums the contributions of a tile of nearby
                                   elements per distinct (row, column) in LDS, then writes
                                   each sum once -- a plain store where the tile holds
                                   every element coupling the two nodes, one atomic add
                                   otherwise */
    FEASM_SCATTER_COLOURED = 2, /* one launch per colour, plain read-modify-write
                                   (per colour and element-id block, blocks one
                                   after another: FEASM_TUNE_COLOUR_BLOCKS) */
    FEASM_SCATTER_OWNER = 3,    /* row-owned: each node row is summed by one wavefront
                                   from the incident elements, in element order, and
                                   written once (no atomics, no reset pass) */
    FEASM_SCATTER_SPIN = 4,     /* row locks (the spin-lock methods of Section 3.3): one
                                   lane per element row locks its global row, adds the
                                   row slice with device-coherent reads and writes, and
                                   unlocks; element rows of at most 32 entries (ELIMIT
                                   otherwise).  Each acquire loop is bounded by the spin
                                   limit (FEASM_TUNE_SPIN_LIMIT, default 2^20 attempts);
                                   a lane that reaches it leaves its row out and is
                                   counted by spin_aborts.  Sums in lock order (values
                                   within rounding of the sequential assembly) */
    FEASM_ACCUMULATE = 0x100    /* or-ed into `scatter`: add into `values` without
                                   resetting it first (values += sum_e scatter(K_e)) */
};

/*
 * pattern_build -- symbolic phase (Section 3 intro: the pattern is set up
 * once, before any assembly; Section 2.2 and Fig. 1 for CSR and CRAC).
 *
 *   conn            dev  int32 [n_elem][nodes_per_elem], row-major; read only,
 *                        copied into the handle, may be freed afterwards.
 *   n_elem          > 0
 *   nodes_per_elem  k > 0
 *   dofs_per_node   d > 0
 *   n_nodes         > 0; every conn entry must lie in [0, n_nodes)
 *   build_flags     FEASM_BUILD_* bits, at least one of CSR and CRAC
 *   out             host; receives the new handle (NULL on failure)
 *
 * CSR (Section 2.2, Fig. 1c): row_ptr[i] = entries in rows < i, col_idx
 * sorted within each row.  CRAC (Section 2.2, Fig. 1d): for each maximal
 * run of consecutive columns of a row, the pair (first column, position of
 * its first value in the CSR values array), row by row; crac_row_ptr counts
 * integers of col_align (two per run); a final pair (n_cols, nnz) closes
 * col_align, so n_ca = 2*runs + 2.  CRAC shares the CSR values layout.
 *
 * Colouring (Section 3.3): elements sharing a node get different colours;
 * the element list is grouped by colour, increasing element id within a
 * colour.  The colouring is the greedy one in element order: each element
 * takes the smallest colour unused by the smaller elements it shares a node
 * with.
 *
 * Tiles (FEASM_BUILD_TILES): elements grouped into small sets of
 * neighbouring elements (aggregates around a distance-2 independent set of
 * the element graph, cut into tiles of a few dozen elements) with each
 * tile's distinct node pairs, for the atomic scatter.  Any element order
 * and mesh is accepted; elements whose tile has more distinct node pairs
 * than the accumulator holds fall back to one atomic per contribution.
 *
 * Lookup record (FEASM_BUILD_OWNER_MAP): for every node, incident element
 * and element node, the offset of that node's first column inside the
 * owned row (int32, n_elem * k^2 entries, the same for both formats).  The
 * row-owned strategy then reads it instead of the element's connectivity
 * row and the search in the owned row, from the first assembly on (without
 * the flag it is built by the first row-owned reassemble_values).  Pays on
 * meshes whose node numbering is scattered (the permuted tet10 mesh) and on
 * elements with many nodes (tet10; high-order quads, where it makes the
 * row-owned strategy faster than atomics); on 8-node hexahedra numbered
 * along a grid the connectivity rows are cache hits and the record only
 * adds reads.
 *
 * Errors: EINVAL for bad arguments; ERANGE if a node id is out of range
 * (checked on the device, reported before returning); EOVERFLOW for int32
 * overflow of the pattern; ELIMIT if a node is shared by so many elements
 * that its candidate column list exceeds 8192 entries, or (with
 * FEASM_BUILD_OWNER_MAP) its row index words exceed 64 KiB of LDS; ENOMEM;
 * EHIP.
 * Synchronises `stream` before returning, so no asynchronous error is lost.
 */
int pattern_build(const int32_t* conn, int64_t n_elem, int32_t nodes_per_elem,
                  int32_t dofs_per_node, int64_t n_nodes, uint32_t build_flags,
                  hipStream_t stream, feasm_pattern** out);

/*
 * assemble_csr / assemble_crac -- numeric phase (Section 3: values are reset
 * to zero, then every element matrix is added, G(D(r),D(s)) += K(r,s), as in
 * the sequential, atomic and colouring listings).
 *
 *   p        handle from pattern_build (built with CSR, resp. CRAC; the
 *            coloured strategy also needs FEASM_BUILD_COLOUR)
 *   ke       dev  double [n_elem][n][n], row-major, element order of conn
 *   values   dev  double [nnz]; overwritten with sum_e scatter(K_e)
 *   scatter  FEASM_SCATTER_*, optionally | FEASM_ACCUMULATE (no reset: the
 *            sums are added to what `values` holds, e.g. to assemble several
 *            element blocks into one matrix)
 *
 * assemble_csr finds positions by binary search of col_idx in each row;
 * assemble_crac by linear block search over the row's CRAC pairs (Section
 * 2.2 listing) followed by contiguous slice adds over the element's DOF runs
 * (Section 3.3).  Both produce the same values array.
 *
 * Asynchronous on `stream`; nothing is checked on the device.  The caller
 * guarantees buffer sizes and that `values` does not alias `ke`; concurrent
 * calls on one values buffer race.  Returns EINVAL for a null handle or
 * buffer, a format the handle lacks, or an unknown strategy.
 */
int assemble_csr(const feasm_pattern* p, const double* ke, double* values, int scatter,
                 hipStream_t stream);
int assemble_crac(const feasm_pattern* p, const double* ke, double* values, int scatter,
                  hipStream_t stream);

/*
 * reassemble_values -- value-only re-assembly on an existing pattern
 * (Section 3 intro: between assemblies the values are reset to zero and the
 * pattern is kept).  `fmt` is FEASM_FMT_CSR or FEASM_FMT_CRAC.  Returns the
 * same values as assemble_<fmt> with the same arguments (bitwise for the
 * row-owned and coloured strategies; within FP64 reordering for the atomic
 * one).  The first call on a handle records the lookup results on the
 * device and synchronises `stream` (hence the non-const handle): for the
 * atomic and coloured strategies each element's (row node, run) offsets,
 * for the row-owned strategy the column offset of every element node in
 * every owned row (int32 [n_elem*k][k]); each record is made once, by the
 * first call of its strategy family.  Later calls, on any stream and
 * concurrently, read the record instead of searching.  A recording call
 * must not race another call on the same handle.  Otherwise asynchronous.
 */
int reassemble_values(feasm_pattern* p, int fmt, const double* ke, double* values, int scatter,
                      hipStream_t stream);

/* Sizes of the pattern.  Any output pointer may be NULL. */
int pattern_info(const feasm_pattern* p, int64_t* n_rows, int64_t* nnz, int64_t* n_ca,
                 int32_t* n_colours);

/*
 * Borrowed device pointers to the pattern arrays (valid until pattern_free;
 * NULL for a format that was not built): row_ptr[n_rows+1], col_idx[nnz],
 * crac_row_ptr[n_rows+1], col_align[n_ca].  Any output may be NULL.
 */
int pattern_arrays(const feasm_pattern* p, const int32_t** row_ptr, const int32_t** col_idx,
                   const int32_t** crac_row_ptr, const int32_t** col_align);

/*
 * Colouring of a handle built with FEASM_BUILD_COLOUR.  colour_ptr is a
 * borrowed HOST array [n_colours+1] of offsets into colour_elems, a borrowed
 * DEVICE array [n_elem] of element ids grouped by colour; element_colour is
 * a borrowed DEVICE array [n_elem].  Any output may be NULL.
 */
int pattern_colouring(const feasm_pattern* p, const int64_t** colour_ptr,
                      const int32_t** colour_elems, const int32_t** element_colour);

/*
 * Launch-shape tuning of one handle (used by the autotuner; 0 restores the
 * library default).  Results do not depend on these settings.
 *   FEASM_TUNE_OWNER_BLOCKS_PER_CU  row-owned strategy: 0 = one 64-lane block
 *                                   per node-row tile; n > 0 = a persistent
 *                                   grid of n blocks per compute unit
 *   FEASM_TUNE_THREADS_PER_ELEM     atomic/coloured strategies: lanes per
 *                                   element, one of 16, 32, 64, 128, 256
 *   FEASM_TUNE_OWNER_ROWS           row-owned strategy with elements of more
 *                                   than 64 entries per node row: node rows per
 *                                   wavefront, 1, 2 or 4
 *   FEASM_TUNE_OWNER_BATCH          row-owned strategy: element rows loaded per
 *                                   batch, 8 or 16
 *   FEASM_TUNE_STRATEGY             the strategy FEASM_SCATTER_AUTO resolves to
 *                                   for this handle (and in batches)
 *   FEASM_TUNE_OWNER_FLAT           row-owned strategy: one node row per
 *                                   wavefront, the element rows of a batch of 4,
 *                                   8 or 16 entries read as one flat array; 0 =
 *                                   auto (4 for d*n > 192, else 8 if no node has
 *                                   more than 8 incident entries, else 16), -1 =
 *                                   off.  Compiled for 8-node hexes and 10-node
 *                                   tets with 3 DOFs per node, and, for rows of
 *                                   at most 4 or 8 entries, for Q3/Q4 quads with
 *                                   4 DOFs and Q1 quads with 4 to 8; other
 *                                   shapes keep the launch the settings above
 *                                   choose
 *   FEASM_TUNE_OWNER_PREFETCH       flat batches, rows longer than one batch:
 *                                   1 = issue the next batch's loads before the
 *                                   current batch is added (more registers)
 *   FEASM_TUNE_SPMV_CHUNK           spmv_csr / spmv_crac: values a wavefront
 *                                   stages in LDS at a time, 256, 512, 1024 or
 *                                   2048 (0: 1024, or 512 for CRAC with at most
 *                                   96 values per row on average); rows per
 *                                   wavefront follow
 *   FEASM_TUNE_HEX8_PIPE            assemble_hex8: 0 = nodes with at most 8
 *                                   incident entries by the pipelined kernel
 *                                   (a grid the compute units hold at once,
 *                                   each wavefront a contiguous range of
 *                                   nodes), the rest one node per wavefront;
 *                                   n in [1, 16] = the pipelined grid with n
 *                                   blocks per compute unit; -1 = every node
 *                                   one per wavefront
 *   FEASM_TUNE_TILE_CAP             handles with tiles: elements per tile at
 *                                   most, 1 to 64 (0: chosen from the element
 *                                   size); rebuilds the tiles (synchronises
 *                                   the device)
 *   FEASM_TUNE_SPIN_LIMIT           FEASM_SCATTER_SPIN: lock acquire attempts
 *                                   per lane before it gives up (0: 2^20;
 *                                   -1: none, every lane gives up at once,
 *                                   which exercises the give-up path)
 *   FEASM_TUNE_COLOUR_BLOCKS        handles with colouring: element-id blocks
 *                                   the coloured scatter runs one after
 *                                   another, every colour within each block,
 *                                   1 to 256 (0: the values array's size over
 *                                   the 256 MiB memory-side cache, rounded);
 *                                   reads the colour lists back to the host
 *                                   (a synchronous copy)
 * Returns EINVAL for an unknown key or value.
 */
enum {
    FEASM_TUNE_OWNER_BLOCKS_PER_CU = 1,
    FEASM_TUNE_THREADS_PER_ELEM = 2,
    FEASM_TUNE_OWNER_ROWS = 3,
    FEASM_TUNE_OWNER_BATCH = 4,
    FEASM_TUNE_STRATEGY = 5,
    FEASM_TUNE_OWNER_FLAT = 6,
    FEASM_TUNE_OWNER_PREFETCH = 7,
    FEASM_TUNE_SPMV_CHUNK = 8,
    FEASM_TUNE_HEX8_PIPE = 9,
    FEASM_TUNE_SPIN_LIMIT = 10,
    FEASM_TUNE_TILE_CAP = 11,
    FEASM_TUNE_COLOUR_BLOCKS = 12
};
int pattern_tune(feasm_pattern* p, int key, int64_t value);

/*
 * spmv_csr / spmv_crac -- sparse matrix-vector product y = G x with an
 * assembled matrix (the conclusions and outlook name the product as the use
 * of the CRAC runs; the definition is the usual one, n_cols = n_rows).
 *   values  dev double [nnz]: the assembled values (the same array for both
 *           formats)
 *   x       dev double [n_rows]
 *   y       dev double [n_rows], overwritten; must not overlap x
 * spmv_csr reads row_ptr and col_idx; spmv_crac reads crac_row_ptr and the
 * CRAC pairs, each run covering consecutive columns from its first column.
 * Each y[i] sums its row's products values[p] * x[col] in increasing column
 * order with every product and sum rounded separately, so both give the
 * same bits as a sequential loop over the row.  Asynchronous on `stream`.
 * Returns EINVAL for a null handle or buffer, a format the handle lacks, or
 * overlapping x and y.
 */
int spmv_csr(const feasm_pattern* p, const double* values, const double* x, double* y,
             hipStream_t stream);
int spmv_crac(const feasm_pattern* p, const double* values, const double* x, double* y,
              hipStream_t stream);

/*
 * Element stiffness of 8-node trilinear hexahedra (the computation the paper
 * replaces by a dummy matrix, Remark 1; textbook isoparametric element).
 * The handle's elements must have k = 8 nodes, in the order: bottom face
 * (zeta = -1) counter-clockwise from (-1,-1), then the top face in the same
 * order; d = 1 gives the scalar Laplace matrix K_ab = sum_q kappa (g_a . g_b)
 * det J, d = 3 isotropic linear elasticity K_(a,i)(b,j) = sum_q [lambda
 * g_a,i g_b,j + mu (g_a,j g_b,i + delta_ij g_a . g_b)] det J (local DOF
 * 3a + i), with the 2x2x2 Gauss rule (points +-1/sqrt(3), xi fastest), J_ij
 * = dx_i/dxi_j and g_a,i = sum_j C_ij / det J * dN_a/dxi_j (C: cofactors of
 * J).  The device evaluates each entry as one fixed sequence of correctly
 * rounded operations and fused multiply-adds (fma(a,b,c) = a*b + c rounded
 * once), so its results are reproducible bit for bit and differ from any
 * other evaluation of the same formulas by rounding only:
 *   J_ij  = fma over a = 0..7 of (x_a,i, dN_a,j), from 0
 *   C_ij  = fma(J_i1j1, J_i2j2, -(J_i1j2 * J_i2j1)), i1 = i+1, i2 = i+2 mod 3
 *   det   = fma(J_00, C_00, fma(J_01, C_01, J_02 * C_02))
 *   g_a,i = fma over j = 0..2 of (C_ij / det, dN_a,j), from 0
 *   dot   = fma(g_a,2, g_b,2, fma(g_a,1, g_b,1, g_a,0 * g_b,0))
 *   d = 1: K_ab += (kappa * det) * dot
 *   d = 3: l = lambda * det, m = mu * det; s = (i == j ? m * dot : 0);
 *          s = fma(m * g_a,j, g_b,i, s); s = fma(l * g_a,i, g_b,j, s);
 *          K_(a,i)(b,j) += s
 * with the quadrature points summed in order.
 *   coords    dev double [n_nodes][3]
 *   material  dev double [n_elem] (kappa) for d = 1, [n_elem][2] (lambda,
 *             mu) for d = 3
 * hex8_element_matrices writes ke (dev double [n_elem][8d][8d]), for the
 * two-pass path (then assemble_csr / assemble_crac).
 * assemble_hex8 fuses the two: values (dev double [nnz]) := G, or += G with
 * flags = FEASM_ACCUMULATE, computing each node's row block of every
 * incident element inside the row-owned assembly (no element matrices in
 * memory); fmt is FEASM_FMT_CSR or FEASM_FMT_CRAC.  Values are summed in
 * element order, as the sequential listing, so they equal a sequential
 * (or row-owned) assembly of hex8_element_matrices' output bit for bit.
 * Asynchronous on `stream`; elements must not be inverted (det J > 0; not
 * checked).  Returns EINVAL for a null handle or buffer, k != 8, d not 1 or
 * 3, a format the handle lacks or an unknown flag; ELIMIT (assemble_hex8)
 * if a node row does not fit the LDS accumulator.
 */
int hex8_element_matrices(const feasm_pattern* p, const double* coords, const double* material,
                          double* ke, hipStream_t stream);
int assemble_hex8(const feasm_pattern* p, int fmt, const double* coords, const double* material,
                  double* values, int flags, hipStream_t stream);

/*
 * Lanes of FEASM_SCATTER_SPIN launches on this handle that reached the spin
 * limit since the last call (their rows' contributions are missing from
 * those results); synchronises the device and clears the count.  0 when
 * the handle never ran that strategy.  Returns FEASM_OK when the count is
 * 0 and FEASM_EINCOMPLETE (with *count set) when it is not, so a caller of
 * the asynchronous row-lock scatter learns here whether its results are
 * complete.  EINVAL for a null argument.
 */
int spin_aborts(feasm_pattern* p, int64_t* count);

/*
 * assemble_spin_noalloc -- FEASM_SCATTER_SPIN (assemble_csr / assemble_crac
 * with row locks) for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It allocates nothing: the lock words sit in a static device
 * array of the library (2^21 int32, 8 MiB, held by each GPU the library
 * runs on until the process ends), and the give-up count goes to the
 * caller's `aborts`.
 *   p        handle from pattern_build with the format `fmt`, built on the
 *            current device; at most 2^21 rows (n_rows), element rows of
 *            at most 32 entries
 *   fmt      FEASM_FMT_CSR or FEASM_FMT_CRAC (position lookup as in
 *            assemble_csr / assemble_crac)
 *   ke       dev double [n_elem][n][n], as for assemble_csr
 *   values   dev double [nnz]; overwritten with sum_e scatter(K_e), or added
 *            to with flags = FEASM_ACCUMULATE
 *   aborts   dev int32 [1], caller-owned: the kernel adds the number of
 *            lanes that reached the spin limit (their rows are missing);
 *            the caller zeroes it and reads it after the stream completes
 *   flags    0 or FEASM_ACCUMULATE
 * Same values as assemble_<fmt>(p, ke, values, FEASM_SCATTER_SPIN [|
 * FEASM_ACCUMULATE], stream) up to summation order.  Each call first
 * clears the lock words of the handle's rows and (flags = 0) the values,
 * with kernels (no memset nodes), then launches the row-lock scatter;
 * asynchronous.  Every call on one GPU shares the one lock array, so calls
 * that overlap on a GPU (other streams, other threads) race and must be
 * serialised by the caller.  Errors: EINVAL (null argument, unknown fmt or
 * flag, a format the handle lacks, the handle's device not current);
 * ELIMIT (more than 2^21 rows, element rows longer than 32); EHIP.
 */
int assemble_spin_noalloc(const feasm_pattern* p, int fmt, const double* ke, double* values,
                          int32_t* aborts, int flags, hipStream_t stream);

/* Releases the handle and its device arrays (synchronises the device). NULL is ignored. */
void pattern_free(feasm_pattern* p);

/*
 * Batched assembly: many independent meshes in one graph launch.
 *
 * batch_create prepares the batch for `count` handles (host array; the
 * handles must outlive the batch and all share `fmt`, FEASM_FMT_CSR or
 * FEASM_FMT_CRAC).  Each mesh runs the strategy its handle's
 * FEASM_TUNE_STRATEGY selects (AUTO = row-owned; row-owned meshes whose rows
 * do not fit the LDS accumulator fall back to atomics) with its launch-shape
 * knobs, except that element lanes are capped at 64.  The meshes' work is
 * cut into tiles (node rows of row-owned meshes, element blocks otherwise)
 * grouped by kernel path.  The whole sequence -- zero fill of the atomic and
 * coloured meshes, then for each path of the row-owned and atomic meshes
 * one launch over all of its tiles, and beside them, on a second graph
 * branch, one launch per colour for coloured meshes in colour order -- is
 * captured into one hipGraph.  `flags` may hold
 * FEASM_ACCUMULATE (no reset) and one mode:
 *   (none)                      a workgroup per tile, scheduled by the
 *                               hardware dispatcher (fastest measured);
 *   FEASM_BATCH_PERSISTENT      persistent launches: as many workgroups as
 *                               are resident, popping tiles from device
 *                               counters (one per XCD and path);
 *   FEASM_BATCH_PER_MESH_GRAPH  every mesh's own single-mesh kernels
 *                               (largest first, on 4 parallel branches); the
 *                               graph is recaptured whenever the pointer
 *                               tables change.
 * Synchronises the device.  EINVAL for an unknown flag or both modes.
 *
 * assemble_batch replays it on `stream`: ke[i] (dev double [n_elem_i][n][n])
 * and values[i] (dev double [nnz_i]) are host arrays of device pointers; the
 * values of every mesh are overwritten (or accumulated) exactly as
 * assemble_<fmt> would.  When the pointer tables differ from the previous
 * call they are uploaded first (and the host waits for that upload).  Calls
 * on one batch must not overlap.
 *
 * batch_info reports the number of phases, work tiles, the largest launch's
 * grid and each mesh's kernel path (host array of `count` ints, may be NULL;
 * zeros in per-mesh-graph mode).
 */
enum { FEASM_BATCH_PER_MESH_GRAPH = 0x200, FEASM_BATCH_PERSISTENT = 0x400 };
/*
 * Workload generator (benchmarks and serving; not part of the assembly
 * method): fills ke (dev double [n_elem][n][n]) with reproducible element
 * matrices from counter-based Philox4x32-10 draws.  recipe 0: symmetric
 * zero-row-sum ("laplacian", off-diagonals uniform in [-1, 1)); recipe 1:
 * symmetric positive definite B B^T / n + I with unit-variance B.  Element
 * e uses counter ((entry), e + elem_offset, recipe) under key `seed`, with
 * exact or correctly rounded operations only, so any implementation of the
 * same definition reproduces the bits.  Asynchronous; n*(n+1)*8 <= 64 KiB.
 */
int generate_ke(int recipe, int64_t n_elem, int32_t n, uint64_t seed, int64_t elem_offset,
                double* ke, hipStream_t stream);

typedef struct feasm_batch feasm_batch;
int batch_create(const feasm_pattern* const* patterns, int64_t count, int fmt, uint32_t flags,
                 feasm_batch** out);
int assemble_batch(feasm_batch* b, const double* const* ke, double* const* values,
                   hipStream_t stream);
int batch_info(const feasm_batch* b, int32_t* n_phases, int64_t* n_tiles, int64_t* grid,
               int32_t* paths);
void batch_free(feasm_batch* b);

/* Thread-local message describing the latest failed call on this thread. */
const char* last_error(void);

/*
 * Device allocator of the library (for the caller's memory pool, e.g. a
 * framework's caching allocator).  Every device array the library creates
 * from then on -- pattern arrays, the re-assembly lookup record and cache,
 * batch tables, serving buffers and the temporaries of pattern_build --
 * comes from alloc(bytes, stream, ctx), which returns device memory of the
 * current device, aligned to at least 256 bytes and usable in stream order
 * on `stream`, or NULL when it cannot (the library call then fails with
 * FEASM_ENOMEM).  The library gives each array back with
 * release(ptr, stream, ctx) once no work of its own uses it any longer
 * (stream may be NULL when the release happens outside a stream, as in
 * pattern_free).  An object remembers the allocator that created it and
 * releases its arrays through that one, whatever is set later.  Both NULL
 * restores the default, hipMalloc / hipFree; exactly one NULL is EINVAL.
 * Process-wide; the callbacks may be called from any thread that calls the
 * library.  Unlike every other entry point it is not tied to a pattern or
 * to the paper: it is the library's memory-ownership hook.
 */
typedef void* (*feasm_alloc_fn)(size_t bytes, hipStream_t stream, void* ctx);
typedef void (*feasm_release_fn)(void* ptr, hipStream_t stream, void* ctx);
int set_allocator(feasm_alloc_fn alloc, feasm_release_fn release, void* ctx);

/*
 * Serving engine: requests for one assembly followed by n_reassembly
 * value-only re-assemblies of a mesh, continuously batched.
 *
 * Meshes (host array [n_meshes] of feasm_serve_mesh): the connectivity and
 * sizes as for pattern_build (conn: dev int32 [n_elem][nodes_per_elem],
 * kept alive by the caller for the call), and either
 *   - pattern: a resident handle of the caller (never freed by the engine;
 *     its re-assembly state is built before the clock starts), or
 *   - pattern = NULL: the engine builds the pattern with pattern_build on the
 *     first request that needs it (a miss; the loop stalls for the build and
 *     the first re-assembly's record) and keeps it in a cache of at most
 *     config->pattern_cache_bytes bytes of pattern arrays (<= 0: unbounded),
 *     evicting the least recently used patterns no admitted request uses; it
 *     frees them at the end.
 * Element matrices of iteration i of a request with key s: with ke_pool ==
 * NULL, fresh ones from generate_ke(recipe, ..., key s*1000003 + i*7919 + 1
 * mod 2^64) on a side stream into the slot's ping-pong buffers; otherwise
 * block (s + i) mod pool_size of ke_pool (dev double [pool_size][n_elem][n][n],
 * pre-generated by the caller), read in place.
 *
 * Continuous batching: arriving requests are admitted FIFO into free slots
 * (each with its own streams) whenever the sum of admitted footprints (the
 * two generator buffers unless the mesh has a pool, plus the values; for a
 * pattern not yet built the values are bounded by n_elem*n*n) stays within
 * config->hbm_budget (<= 0: no limit; a request is always admitted when
 * nothing else runs); every slot issues its next iteration as soon as the
 * previous completes, so admitted requests overlap on the device.  The
 * strategy is each handle's AUTO choice.  Synchronous; runs until every
 * request is done.
 *
 * Times (seconds since the start of the run): admitted_s is host time;
 * assembled_s and done_s are the device completion times of the assembly
 * and of the request (timing events, relative to an event recorded at the
 * start); reassembly_latency (optional host array [sum of n_reassembly],
 * request order) holds each re-assembly's device time from its issue on the
 * slot's stream to its completion.  stats (optional) receives pattern cache
 * counts, the host time spent building patterns on misses, and the summed
 * device times of the generator kernels and of the assemblies.
 */
typedef struct {
    const int32_t* conn;  /* dev [n_elem][nodes_per_elem] (may be NULL when pattern is given) */
    int64_t n_elem;
    int32_t nodes_per_elem;
    int32_t dofs_per_node;
    int64_t n_nodes;
    int32_t recipe;                 /* generate_ke recipe (0 or 1) when ke_pool is NULL */
    int32_t pool_size;              /* blocks in ke_pool */
    const double* ke_pool;          /* optional dev [pool_size][n_elem][n][n] */
    const feasm_pattern* pattern;   /* optional resident handle of the caller */
} feasm_serve_mesh;

typedef struct {
    double arrival_s;     /* seconds after the start of the run */
    int32_t mesh;         /* index into the mesh table */
    int32_t n_reassembly; /* value-only re-assemblies after the assembly */
    uint64_t seed;        /* element-matrix key of the request */
    double* keep_values;  /* optional dev double [nnz]: receives the final values */
} feasm_request;

typedef struct {
    double admitted_s, assembled_s, done_s;
} feasm_request_result;

typedef struct {
    int32_t fmt;                  /* FEASM_FMT_CSR or FEASM_FMT_CRAC */
    int32_t slots;                /* 1 .. 256; 1 = one request at a time (FIFO) */
    int64_t hbm_budget;           /* admission budget in bytes (<= 0: none) */
    int64_t pattern_cache_bytes;  /* engine-built patterns kept (<= 0: no limit) */
} feasm_serve_config;

typedef struct {
    int64_t pattern_hits, pattern_misses, pattern_evictions;
    int64_t pattern_cache_peak_bytes, patterns_resident_at_end;
    double pattern_build_s;   /* host seconds in pattern_build + first record on misses */
    double generate_ms;       /* device time of the generator kernels */
    double assemble_ms;       /* device time of the assemblies and re-assemblies */
    int64_t generated_bytes;  /* element-matrix bytes generated */
} feasm_serve_stats;

int serve_run(const feasm_serve_mesh* meshes, int64_t n_meshes, const feasm_request* requests,
              int64_t n_requests, const feasm_serve_config* config, feasm_request_result* results,
              double* reassembly_latency, feasm_serve_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* FEASM_H */
