/*
 * Serial CPU oracle for finite-element sparse-matrix assembly.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the device library and must never be used as a
 * fallback for it.
 *
 * Everything here is the plain definition, written for a reader to check by
 * eye against the paper (Sky, Polindara, Muench, Birk, arXiv 2012.00585):
 *
 *   - element DOF map and its run-length form ............. Section 2.1
 *   - CSR pattern = union of element cliques, sorted ...... Section 2.2, Fig. 1(b,c), Section 3 intro
 *   - CRAC column-alignment pairs + final pair ............ Section 2.2, Fig. 1(d)
 *   - CRAC linear block search ............................ Section 2.2, "Linear block search" listing
 *   - sequential assembly G(D(r),D(c)) += K(r,c) .......... Section 3.1, "Sequential assembly" listing
 *   - greedy first-fit element colouring .................. Section 3.3 (colouring listing and text)
 *   - matrix-vector product y = G x, CSR and over CRAC runs  Conclusions and outlook
 *   - 8-node hexahedron stiffness (Laplace, elasticity) .... Remark 1 (the element
 *     matrix the paper replaces by a dummy); textbook trilinear element
 *
 * Indices are 0-based and 64-bit.  Floating point is plain FP64 with
 * round-to-nearest adds in the stated order; build with -O2
 * -ffp-contract=off and no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ERANGE (-2)
#define ORC_ENOMEM (-3)
#define ORC_ENOTFOUND (-4)
#define ORC_ECAP (-5)

void orc_free(void* p) { free(p); }

/* ------------------------------------------------------------------ */
/* Section 2.1: the element DOF map.  DOFs of one node are contiguous and
 * numbered node-major: global DOF of (node, component c) is d*node + c,
 * and the local row of (local node a, component c) is a*d + c.          */
void orc_dof_map(const int32_t* conn_e, int32_t k, int32_t d, int64_t* D)
{
    for (int32_t a = 0; a < k; ++a)
        for (int32_t c = 0; c < d; ++c)
            D[(int64_t)a * d + c] = (int64_t)d * conn_e[a] + c;
}

/* Section 2.1: run-length form of an element DOF array.  Runs follow the
 * local order (they are not sorted): pairs[2j] = first DOF of run j,
 * pairs[2j+1] = its length.  Returns the number of runs.               */
int32_t orc_dof_runs(const int64_t* D, int32_t n, int64_t* pairs)
{
    int32_t nr = 0;
    int32_t s = 0;
    while (s < n) {
        int32_t len = 1;
        while (s + len < n && D[s + len] == D[s + len - 1] + 1)
            ++len;
        pairs[2 * nr] = D[s];
        pairs[2 * nr + 1] = len;
        ++nr;
        s += len;
    }
    return nr;
}

/* ------------------------------------------------------------------ */
/* CSR pattern: every row's column bucket is sorted and duplicates are
 * removed; row_ptr[i] counts the entries of rows < i.                   */
static int cmp_i64(const void* a, const void* b)
{
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

/* buf holds, for row i, the candidate columns buf[start[i] .. start[i+1]).
 * Sorts and compacts in place.  Returns nnz.                            */
static int64_t compact_rows(int64_t n_rows, const int64_t* start, int64_t* buf, int64_t* row_ptr)
{
    int64_t w = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n_rows; ++i) {
        int64_t b = start[i], e = start[i + 1];
        qsort(buf + b, (size_t)(e - b), sizeof(int64_t), cmp_i64);
        for (int64_t j = b; j < e; ++j)
            if (j == b || buf[j] != buf[j - 1])
                buf[w++] = buf[j];
        row_ptr[i + 1] = w;
    }
    return w;
}

/* Sparsity pattern of an arbitrary list of coordinates (rows[q], cols[q]).
 * Fills row_ptr[n_rows+1]; *col_idx_out is malloc'd (free with orc_free).
 * Returns nnz or a negative error.                                      */
int64_t orc_pattern_pairs(int64_t m, const int64_t* rows, const int64_t* cols, int64_t n_rows,
                          int64_t n_cols, int64_t* row_ptr, int64_t** col_idx_out)
{
    for (int64_t q = 0; q < m; ++q)
        if (rows[q] < 0 || rows[q] >= n_rows || cols[q] < 0 || cols[q] >= n_cols)
            return ORC_ERANGE;
    int64_t* start = calloc((size_t)n_rows + 1, sizeof(int64_t));
    int64_t* buf = malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    if (!start || !buf) {
        free(start);
        free(buf);
        return ORC_ENOMEM;
    }
    for (int64_t q = 0; q < m; ++q)
        start[rows[q] + 1] += 1;
    for (int64_t i = 0; i < n_rows; ++i)
        start[i + 1] += start[i];
    int64_t* fill = malloc(sizeof(int64_t) * (size_t)(n_rows + 1));
    if (!fill) {
        free(start);
        free(buf);
        return ORC_ENOMEM;
    }
    memcpy(fill, start, sizeof(int64_t) * (size_t)(n_rows + 1));
    for (int64_t q = 0; q < m; ++q)
        buf[fill[rows[q]]++] = cols[q];
    free(fill);
    int64_t nnz = compact_rows(n_rows, start, buf, row_ptr);
    free(start);
    *col_idx_out = buf;
    return nnz;
}

/* Sparsity pattern of an element mesh: the union over elements e of the
 * cliques {(D_e[r], D_e[s]) : 0 <= r, s < n}, with n = k*d and
 * n_rows = n_cols = d*n_nodes.  No entry is ever dropped.               */
int64_t orc_pattern(const int32_t* conn, int64_t E, int32_t k, int32_t d, int64_t n_nodes,
                    int64_t* row_ptr, int64_t** col_idx_out)
{
    if (E < 0 || k <= 0 || d <= 0 || n_nodes < 0)
        return ORC_EINVAL;
    for (int64_t q = 0; q < E * k; ++q)
        if (conn[q] < 0 || conn[q] >= n_nodes)
            return ORC_ERANGE;
    const int32_t n = k * d;
    const int64_t n_rows = (int64_t)d * n_nodes;
    int64_t* D = malloc(sizeof(int64_t) * (size_t)n);
    int64_t* start = calloc((size_t)n_rows + 1, sizeof(int64_t));
    if (!D || !start) {
        free(D);
        free(start);
        return ORC_ENOMEM;
    }
    for (int64_t e = 0; e < E; ++e) {
        orc_dof_map(conn + e * k, k, d, D);
        for (int32_t r = 0; r < n; ++r)
            start[D[r] + 1] += n;
    }
    for (int64_t i = 0; i < n_rows; ++i)
        start[i + 1] += start[i];
    int64_t total = start[n_rows];
    int64_t* buf = malloc(sizeof(int64_t) * (size_t)(total > 0 ? total : 1));
    int64_t* fill = malloc(sizeof(int64_t) * (size_t)(n_rows + 1));
    if (!buf || !fill) {
        free(D);
        free(start);
        free(buf);
        free(fill);
        return ORC_ENOMEM;
    }
    memcpy(fill, start, sizeof(int64_t) * (size_t)(n_rows + 1));
    for (int64_t e = 0; e < E; ++e) {
        orc_dof_map(conn + e * k, k, d, D);
        for (int32_t r = 0; r < n; ++r)
            for (int32_t s = 0; s < n; ++s)
                buf[fill[D[r]]++] = D[s];
    }
    free(fill);
    int64_t nnz = compact_rows(n_rows, start, buf, row_ptr);
    free(start);
    free(D);
    *col_idx_out = buf;
    return nnz;
}

/* ------------------------------------------------------------------ */
/* Coefficient lookup in CSR: binary search of column j in row i
 * (Section 2.2).  Returns the 0-based value position or -1 if absent. */
int64_t orc_csr_find(const int64_t* row_ptr, const int64_t* col_idx, int64_t i, int64_t j)
{
    int64_t lo = row_ptr[i], hi = row_ptr[i + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col_idx[mid] < j)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < row_ptr[i + 1] && col_idx[lo] == j) ? lo : -1;
}

/* Section 2.2, Fig. 1(d): a CRAC run is a maximal sequence of consecutive
 * column indices within a row.  Returns the number of runs B.           */
int64_t orc_crac_count(const int64_t* row_ptr, const int64_t* col_idx, int64_t n_rows)
{
    int64_t B = 0;
    for (int64_t i = 0; i < n_rows; ++i)
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
            if (p == row_ptr[i] || col_idx[p] != col_idx[p - 1] + 1)
                ++B;
    return B;
}

/* Builds the CRAC arrays from CSR.  For each run, in row order, the pair
 * (first column, position of its first value) is appended to ca; the
 * CRAC row pointer counts integers of ca (two per run), as in Fig. 1(d).
 * A final pair (n_cols, nnz) closes ca, so n_ca = 2B + 2.  The values
 * array is the CSR one.                                                 */
void orc_crac_fill(const int64_t* row_ptr, const int64_t* col_idx, int64_t n_rows, int64_t n_cols,
                   int64_t* crac_row_ptr, int64_t* ca)
{
    int64_t w = 0;
    for (int64_t i = 0; i < n_rows; ++i) {
        crac_row_ptr[i] = w;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
            if (p == row_ptr[i] || col_idx[p] != col_idx[p - 1] + 1) {
                ca[w] = col_idx[p];
                ca[w + 1] = p;
                w += 2;
            }
    }
    crac_row_ptr[n_rows] = w;
    ca[w] = n_cols;
    ca[w + 1] = row_ptr[n_rows];
}

/* Linear block search in CRAC (Section 2.2 listing).  Steps over the pairs
 * of row i while the next run's first column is <= j; the last run of the
 * row is the default (the listing's loop bound would otherwise read the
 * next row's pair).  Returns the value position or -1 if (i,j) is not
 * stored.                                                               */
int64_t orc_crac_find(const int64_t* crac_row_ptr, const int64_t* ca, int64_t i, int64_t j)
{
    int64_t b = crac_row_ptr[i], e = crac_row_ptr[i + 1];
    if (b == e)
        return -1;
    int64_t q = b;
    while (q + 2 < e && ca[q + 2] <= j)
        q += 2;
    int64_t first_col = ca[q];
    int64_t vpos = ca[q + 1];
    int64_t vend = ca[q + 3]; /* value position of the following pair */
    if (j >= first_col && j < first_col + (vend - vpos))
        return vpos + (j - first_col);
    return -1;
}

/* ------------------------------------------------------------------ */
/* Section 3.1, "Sequential assembly": values are reset to zero, then for
 * every element e, row r and column s (in this order)
 *     values[pos(D_e[r], D_e[s])] += Ke[e][r][s].
 * abssum (optional) accumulates |Ke[e][r][s]| at the same positions; it
 * bounds the rounding error of any other summation order.               */
int orc_assemble(const int32_t* conn, int64_t E, int32_t k, int32_t d, const double* Ke,
                 const int64_t* row_ptr, const int64_t* col_idx, int64_t n_rows, double* values,
                 double* abssum)
{
    const int32_t n = k * d;
    const int64_t nnz = row_ptr[n_rows];
    for (int64_t p = 0; p < nnz; ++p)
        values[p] = 0.0;
    if (abssum)
        for (int64_t p = 0; p < nnz; ++p)
            abssum[p] = 0.0;
    int64_t* D = malloc(sizeof(int64_t) * (size_t)n);
    if (!D)
        return ORC_ENOMEM;
    for (int64_t e = 0; e < E; ++e) {
        orc_dof_map(conn + e * k, k, d, D);
        const double* K = Ke + e * (int64_t)n * n;
        for (int32_t r = 0; r < n; ++r) {
            if (D[r] < 0 || D[r] >= n_rows) {
                free(D);
                return ORC_ERANGE;
            }
            for (int32_t s = 0; s < n; ++s) {
                int64_t p = orc_csr_find(row_ptr, col_idx, D[r], D[s]);
                if (p < 0) {
                    free(D);
                    return ORC_ENOTFOUND;
                }
                values[p] = values[p] + K[(int64_t)r * n + s];
                if (abssum)
                    abssum[p] = abssum[p] + fabs(K[(int64_t)r * n + s]);
            }
        }
    }
    free(D);
    return ORC_OK;
}

/* Assembly of explicit coordinate contributions (rows[q], cols[q], vals[q])
 * in q order into an existing CSR pattern.                              */
int orc_assemble_pairs(int64_t m, const int64_t* rows, const int64_t* cols, const double* vals,
                       const int64_t* row_ptr, const int64_t* col_idx, int64_t n_rows,
                       double* values)
{
    for (int64_t p = 0; p < row_ptr[n_rows]; ++p)
        values[p] = 0.0;
    for (int64_t q = 0; q < m; ++q) {
        int64_t p = orc_csr_find(row_ptr, col_idx, rows[q], cols[q]);
        if (p < 0)
            return ORC_ENOTFOUND;
        values[p] = values[p] + vals[q];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Node -> incident elements, each list in increasing element order.
 * An element that lists a node twice appears twice.                     */
static int incidence(const int32_t* conn, int64_t E, int32_t k, int64_t n_nodes, int64_t** ptr_out,
                     int64_t** elem_out)
{
    int64_t* ptr = calloc((size_t)n_nodes + 1, sizeof(int64_t));
    int64_t* el = malloc(sizeof(int64_t) * (size_t)(E * k > 0 ? E * k : 1));
    int64_t* fill = malloc(sizeof(int64_t) * (size_t)(n_nodes + 1));
    if (!ptr || !el || !fill) {
        free(ptr);
        free(el);
        free(fill);
        return ORC_ENOMEM;
    }
    for (int64_t q = 0; q < E * k; ++q)
        ptr[conn[q] + 1] += 1;
    for (int64_t v = 0; v < n_nodes; ++v)
        ptr[v + 1] += ptr[v];
    memcpy(fill, ptr, sizeof(int64_t) * (size_t)(n_nodes + 1));
    for (int64_t e = 0; e < E; ++e)
        for (int32_t a = 0; a < k; ++a)
            el[fill[conn[e * k + a]]++] = e;
    free(fill);
    *ptr_out = ptr;
    *elem_out = el;
    return ORC_OK;
}

/* Greedy first-fit colouring in natural element order (the greedy
 * algorithm the paper uses for its colouring method, Section 3.3): two
 * elements conflict when they share a node; each element takes the
 * smallest colour not used by an already-coloured conflicting element.
 * Returns the number of colours or a negative error.                    */
int32_t orc_greedy_colour(const int32_t* conn, int64_t E, int32_t k, int64_t n_nodes,
                          int32_t* colour)
{
    int64_t *ptr, *el;
    if (incidence(conn, E, k, n_nodes, &ptr, &el) != ORC_OK)
        return ORC_ENOMEM;
    int64_t* seen = malloc(sizeof(int64_t) * (size_t)(E + 1)); /* seen[c] == e: c is taken */
    if (!seen) {
        free(ptr);
        free(el);
        return ORC_ENOMEM;
    }
    for (int64_t c = 0; c <= E; ++c)
        seen[c] = -1;
    int32_t n_colours = 0;
    for (int64_t e = 0; e < E; ++e) {
        for (int32_t a = 0; a < k; ++a) {
            int64_t v = conn[e * k + a];
            for (int64_t q = ptr[v]; q < ptr[v + 1]; ++q)
                if (el[q] < e)
                    seen[colour[el[q]]] = e;
        }
        int32_t c = 0;
        while (seen[c] == e)
            ++c;
        colour[e] = c;
        if (c + 1 > n_colours)
            n_colours = c + 1;
    }
    free(seen);
    free(ptr);
    free(el);
    return n_colours;
}

/* A colouring is valid when no two distinct elements sharing a node have
 * the same colour (Section 3.3).  Returns 1 if valid, 0 if not.         */
int orc_colouring_valid(const int32_t* conn, int64_t E, int32_t k, int64_t n_nodes,
                        const int32_t* colour, int32_t n_colours)
{
    for (int64_t e = 0; e < E; ++e)
        if (colour[e] < 0 || colour[e] >= n_colours)
            return 0;
    int64_t *ptr, *el;
    if (incidence(conn, E, k, n_nodes, &ptr, &el) != ORC_OK)
        return ORC_ENOMEM;
    int64_t* owner = malloc(sizeof(int64_t) * (size_t)(n_colours > 0 ? n_colours : 1));
    int64_t* stamp = malloc(sizeof(int64_t) * (size_t)(n_colours > 0 ? n_colours : 1));
    int ok = 1;
    for (int32_t c = 0; c < n_colours; ++c)
        stamp[c] = -1;
    for (int64_t v = 0; v < n_nodes && ok; ++v)
        for (int64_t q = ptr[v]; q < ptr[v + 1]; ++q) {
            int32_t c = colour[el[q]];
            if (stamp[c] == v && owner[c] != el[q]) {
                ok = 0;
                break;
            }
            stamp[c] = v;
            owner[c] = el[q];
        }
    free(owner);
    free(stamp);
    free(ptr);
    free(el);
    return ok;
}

/* ------------------------------------------------------------------ */
/* Selected rows of the assembled matrix, one by one, for checks on meshes
 * too large to assemble whole.  For DOF row i, cols receives its sorted
 * columns and vals/abssum the sums, accumulated in the same (element, r, s)
 * order as orc_assemble, so the results are bit-identical to it.
 * Row q of the output occupies [q*cap, q*cap + len[q]).                 */
int orc_rows(const int32_t* conn, int64_t E, int32_t k, int32_t d, int64_t n_nodes,
             const double* Ke, int64_t n_req, const int64_t* req_rows, int64_t cap, int64_t* len,
             int64_t* cols, double* vals, double* abssum)
{
    const int32_t n = k * d;
    int64_t *ptr, *el;
    if (incidence(conn, E, k, n_nodes, &ptr, &el) != ORC_OK)
        return ORC_ENOMEM;
    int64_t* D = malloc(sizeof(int64_t) * (size_t)n);
    int64_t* pc = malloc(sizeof(int64_t) * (size_t)cap);
    double* pv = malloc(sizeof(double) * (size_t)cap);
    double* pa = malloc(sizeof(double) * (size_t)cap);
    int64_t* ord = malloc(sizeof(int64_t) * (size_t)cap);
    int rc = ORC_OK;
    for (int64_t q = 0; q < n_req && rc == ORC_OK; ++q) {
        int64_t i = req_rows[q];
        int64_t v = i / d;
        int64_t m = 0;
        for (int64_t t = ptr[v]; t < ptr[v + 1] && rc == ORC_OK; ++t) {
            if (t > ptr[v] && el[t] == el[t - 1])
                continue; /* element lists node v twice: visit it once */
            int64_t e = el[t];
            orc_dof_map(conn + e * k, k, d, D);
            const double* K = Ke + e * (int64_t)n * n;
            for (int32_t r = 0; r < n && rc == ORC_OK; ++r) {
                if (D[r] != i)
                    continue;
                for (int32_t s = 0; s < n; ++s) {
                    int64_t w = 0;
                    while (w < m && pc[w] != D[s])
                        ++w;
                    if (w == m) {
                        if (m == cap) {
                            rc = ORC_ECAP;
                            break;
                        }
                        pc[m] = D[s];
                        pv[m] = 0.0;
                        pa[m] = 0.0;
                        ++m;
                    }
                    pv[w] = pv[w] + K[(int64_t)r * n + s];
                    pa[w] = pa[w] + fabs(K[(int64_t)r * n + s]);
                }
            }
        }
        /* selection sort of the (few) columns, carrying the sums along */
        for (int64_t a = 0; a < m; ++a)
            ord[a] = a;
        for (int64_t a = 0; a < m; ++a) {
            int64_t best = a;
            for (int64_t b = a + 1; b < m; ++b)
                if (pc[ord[b]] < pc[ord[best]])
                    best = b;
            int64_t tmp = ord[a];
            ord[a] = ord[best];
            ord[best] = tmp;
        }
        len[q] = m;
        for (int64_t a = 0; a < m; ++a) {
            cols[q * cap + a] = pc[ord[a]];
            vals[q * cap + a] = pv[ord[a]];
            abssum[q * cap + a] = pa[ord[a]];
        }
    }
    free(D);
    free(pc);
    free(pv);
    free(pa);
    free(ord);
    free(ptr);
    free(el);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Matrix-vector product y = G x, the use of the CRAC runs the paper names
 * in its conclusions and outlook.  Definition: y[i] = sum over the stored
 * entries (i, j) of row i of values * x[j], summed in increasing column
 * order, each product and each sum rounded (no fused multiply-add).
 * yabs (optional) receives sum |values * x[j]|, which bounds the rounding
 * error of any other order.                                             */
void orc_spmv_csr(const int64_t* row_ptr, const int64_t* col_idx, int64_t n_rows,
                  const double* values, const double* x, double* y, double* yabs)
{
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0, a = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            const double t = values[p] * x[col_idx[p]];
            s = s + t;
            a = a + fabs(t);
        }
        y[i] = s;
        if (yabs)
            yabs[i] = a;
    }
}

/* The same product read through the CRAC arrays: row i holds the pairs
 * ca[crac_row_ptr[i] .. crac_row_ptr[i+1]) (two integers per run: first
 * column, position of its first value).  A run's values are consecutive
 * and end where the next pair's values begin (the next run of the row, the
 * next row's first run, or the final pair (n_cols, nnz)); value t of the
 * run multiplies x[first column + t].                                   */
void orc_spmv_crac(const int64_t* crac_row_ptr, const int64_t* ca, int64_t n_rows,
                   const double* values, const double* x, double* y)
{
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t q = crac_row_ptr[i]; q < crac_row_ptr[i + 1]; q += 2) {
            const int64_t col = ca[q], pos = ca[q + 1], end = ca[q + 3];
            for (int64_t t = 0; t < end - pos; ++t)
                s = s + values[pos + t] * x[col + t];
        }
        y[i] = s;
    }
}

/* ------------------------------------------------------------------ */
/* Element stiffness of the 8-node trilinear hexahedron -- the computation
 * the paper replaces by a dummy matrix (Remark 1); textbook isoparametric
 * element.  Local nodes: the bottom face (zeta = -1) counter-clockwise from
 * (-1,-1), then the top face (zeta = +1) in the same order.  Shape function
 * N_a = (1 + xi_a xi)(1 + eta_a eta)(1 + zeta_a zeta) / 8.  Quadrature: the
 * 2x2x2 Gauss rule, points +-1/sqrt(3), weights 1, in the order xi fastest,
 * then eta, then zeta.  With J_ij = dx_i/dxi_j and g_a = J^-T grad_xi N_a:
 *   d = 1 (Laplace, mat[0] = kappa):
 *       K_ab = sum_q kappa (g_a . g_b) det J
 *   d = 3 (isotropic elasticity, mat[0] = lambda, mat[1] = mu), local DOF
 *       3a + i:
 *       K_(a,i)(b,j) = sum_q [lambda g_a,i g_b,j + mu (g_a,j g_b,i +
 *                       delta_ij g_a . g_b)] det J
 * Each formula is evaluated as written, left to right, with a separately
 * rounded multiply or add per operation (build without contraction); any
 * other evaluation order, fused multiply-adds included, differs from it by
 * rounding only.  x holds the 8 nodes' coordinates (x[3a + i]); K is n x n
 * row-major with n = 8 d; kabs (optional) receives sum_q |each term| per
 * entry, the scale of the rounding error of any other evaluation order.
 * Returns ORC_OK, or ORC_ERANGE if det J <= 0 at a quadrature point.     */
static const int HEX8_REF[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                                   {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

int orc_hex8_stiffness(const double* x, int32_t d, const double* mat, double* K, double* kabs)
{
    const int32_t n = 8 * d;
    for (int32_t i = 0; i < n * n; ++i) {
        K[i] = 0.0;
        if (kabs)
            kabs[i] = 0.0;
    }
    const double gp = 1.0 / sqrt(3.0);
    for (int q = 0; q < 8; ++q) {
        const double xi[3] = {(q & 1) ? gp : -gp, (q & 2) ? gp : -gp, (q & 4) ? gp : -gp};
        double dN[8][3]; /* d N_a / d xi_j */
        for (int a = 0; a < 8; ++a) {
            double f[3];
            for (int j = 0; j < 3; ++j)
                f[j] = 1.0 + HEX8_REF[a][j] * xi[j];
            dN[a][0] = HEX8_REF[a][0] * f[1] * f[2] / 8.0;
            dN[a][1] = f[0] * HEX8_REF[a][1] * f[2] / 8.0;
            dN[a][2] = f[0] * f[1] * HEX8_REF[a][2] / 8.0;
        }
        double J[3][3] = {{0}};
        for (int a = 0; a < 8; ++a)
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j)
                    J[i][j] += x[3 * a + i] * dN[a][j];
        /* inverse by cofactors: Jinv = adj(J) / det J */
        double C[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
                C[i][j] = J[i1][j1] * J[i2][j2] - J[i1][j2] * J[i2][j1]; /* cofactor of J_ij */
            }
        const double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
        if (!(det > 0.0))
            return ORC_ERANGE;
        /* g_a,i = sum_j (J^-1)_ji dN_a,j and (J^-1)_ji = C_ij / det */
        double g[8][3];
        for (int a = 0; a < 8; ++a)
            for (int i = 0; i < 3; ++i) {
                double s = 0.0;
                for (int j = 0; j < 3; ++j)
                    s += C[i][j] / det * dN[a][j];
                g[a][i] = s;
            }
        for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b) {
                const double dot = g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2];
                if (d == 1) {
                    const double t = mat[0] * dot * det;
                    K[a * n + b] += t;
                    if (kabs)
                        kabs[a * n + b] += fabs(t);
                    continue;
                }
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        const double t1 = mat[0] * g[a][i] * g[b][j] * det;
                        const double t2 = mat[1] * g[a][j] * g[b][i] * det;
                        const double t3 = i == j ? mat[1] * dot * det : 0.0;
                        const int64_t p = (int64_t)(3 * a + i) * n + 3 * b + j;
                        K[p] += t1 + t2 + t3;
                        if (kabs)
                            kabs[p] += fabs(t1) + fabs(t2) + fabs(t3);
                    }
            }
    }
    return ORC_OK;
}

/* Element matrices of a whole hexahedral mesh: K[e] from the coordinates of
 * conn[e] and mat[e * (d == 1 ? 1 : 2)].                                 */
int orc_hex8_matrices(const int32_t* conn, int64_t E, const double* coords, int32_t d,
                      const double* mat, double* K, double* kabs)
{
    const int32_t n = 8 * d, m = d == 1 ? 1 : 2;
    for (int64_t e = 0; e < E; ++e) {
        double x[24];
        for (int a = 0; a < 8; ++a)
            for (int i = 0; i < 3; ++i)
                x[3 * a + i] = coords[3 * (int64_t)conn[8 * e + a] + i];
        const int rc = orc_hex8_stiffness(x, d, mat + m * e, K + e * (int64_t)n * n,
                                          kabs ? kabs + e * (int64_t)n * n : NULL);
        if (rc != ORC_OK)
            return rc;
    }
    return ORC_OK;
}
