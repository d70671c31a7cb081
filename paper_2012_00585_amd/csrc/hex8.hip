// Element stiffness of 8-node trilinear hexahedra computed on the device --
// the computation the paper replaces by a dummy matrix (Remark 1) -- either
// written out as element matrices (hex8_element_matrices) or fused into the
// row-owned assembly (assemble_hex8), which then reads node coordinates and
// material parameters instead of an n x n matrix per element.
//
// Element: local nodes are the bottom face (zeta = -1) counter-clockwise
// from (-1,-1), then the top face in the same order; N_a = (1 + xi_a xi)
// (1 + eta_a eta)(1 + zeta_a zeta) / 8; 2x2x2 Gauss rule (points
// +-1/sqrt(3), weights 1, xi fastest).  With J_ij = dx_i/dxi_j, C the
// cofactor matrix of J and g_a,i = sum_j C_ij / det J * dN_a/dxi_j:
//   d = 1 (Laplace, kappa):   K_ab = sum_q kappa (g_a . g_b) det J
//   d = 3 (elasticity, lambda, mu), local DOF 3a + i:
//     K_(a,i)(b,j) = sum_q [lambda g_a,i g_b,j + mu (g_a,j g_b,i + delta_ij g_a . g_b)] det J
// Every quantity is evaluated as one fixed sequence of correctly rounded
// operations and fused multiply-adds (stated at each step below and in the
// header), so the matrices are the same bits as any evaluation that keeps
// the sequence.
//
// Fused kernel: one 64-lane wavefront owns one node row, as the flat
// row-owned kernel, and walks its incident elements in batches of 8.  Lane
// (t, q) computes the geometry of entry t at quadrature point q into LDS,
// lane (t, b) the d x d block of the owner's rows against element node b,
// and the batch's row blocks are then added into the LDS accumulator entry
// by entry, so every value receives its contributions in element order.
#include <algorithm>

#include "scatter_device.h"

namespace feasm {
namespace {

using scatter::kCRAC;
using scatter::kCSR;
using scatter::row_lookup;

constexpr double kGauss = 0.5773502691896258;  // the double nearest 1/sqrt(3), as 1.0/sqrt(3.0)

struct Hex8Args {
    const int32_t* conn;
    const int64_t* inc_ptr;
    const int32_t* inc_q;
    const int32_t* row_ptr;
    const int32_t* col_idx;
    const int32_t* crac_row_ptr;
    const int32_t* ca;
    const double* coords;  // [n_nodes][3]
    const double* mat;     // [n_elem][d == 1 ? 1 : 2]
    const int32_t* node_list;  // one-node kernel: node of block b (null: node b)
    double* values;
    double* ke;  // element matrices (hex8_element_matrices)
    int64_t n_nodes, n_elem;
    int64_t n_light;  // pipelined kernel: positions [0, n_light) of node_list
    int32_t acc_doubles, idx_ints;
    int32_t accumulate;
};

// Reference corner a: (xi_a, eta_a, zeta_a) in {-1, 1}^3.
__device__ inline double ref_coord(int a, int j) {
    const int f = a & 3;
    const bool plus = j == 0 ? (f == 1 || f == 2) : j == 1 ? (f >= 2) : (a >= 4);
    return plus ? 1.0 : -1.0;
}

// Reference gradients dN[a][j] = dN_a/dxi_j at quadrature point q.
__device__ inline void hex8_ref_gradients(int q, double (&dN)[8][3]) {
    const double xi[3] = {(q & 1) ? kGauss : -kGauss, (q & 2) ? kGauss : -kGauss,
                          (q & 4) ? kGauss : -kGauss};
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        double f[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) f[j] = 1.0 + ref_coord(a, j) * xi[j];
        dN[a][0] = ref_coord(a, 0) * f[1] * f[2] / 8.0;
        dN[a][1] = f[0] * ref_coord(a, 1) * f[2] / 8.0;
        dN[a][2] = f[0] * f[1] * ref_coord(a, 2) / 8.0;
    }
}

// Gradients g[a][i] and det J at a quadrature point with reference
// gradients dN, for the element whose node coordinates are x[3a + i].
__device__ inline void hex8_geometry(const double* x, const double (&dN)[8][3], double (&g)[8][3],
                                     double& det) {
    // J_ij: fused multiply-adds over a, from 0
    double J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < 8; ++a) s = fma(x[3 * a + i], dN[a][j], s);
            J[i][j] = s;
        }
    double C[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            C[i][j] = fma(J[i1][j1], J[i2][j2], -(J[i1][j2] * J[i2][j1]));
        }
    det = fma(J[0][0], C[0][0], fma(J[0][1], C[0][1], J[0][2] * C[0][2]));
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) s = fma(C[i][j] / det, dN[a][j], s);
            g[a][i] = s;
        }
}

// Gradients g[a][i] and det J at quadrature point q of the element whose
// node coordinates are x[3a + i].
__device__ inline void hex8_point(const double* x, int q, double (&g)[8][3], double& det) {
    double dN[8][3];
    hex8_ref_gradients(q, dN);
    hex8_geometry(x, dN, g, det);
}

// The point data of hex8_geometry with its operands in LDS (x: 24
// coordinates, dn: [8][3] reference gradients of the point): cd[3i + j] =
// C_ij / det J and cd[9] = det J, from which the gradients follow as
// g_a,i = sum_j fma(cd[3i + j], dn[a][j]) (hex8_gradient).  One node at a
// time is read, so that few values are live; every value is the same
// sequence of operations as in hex8_geometry.
constexpr int kCd = 10;
// LDS strides of the pipelined kernel, padded so that the eight lane groups
// (t, *) and the eight points fall on different banks: point data per entry
// (8 points), coordinates per entry (8 nodes), reference gradients per point.
constexpr int kCdEntry = 8 * kCd + 2, kXsEntry = 25, kDnPoint = 25;
constexpr int kPointRegion = 8 * kCdEntry;

__device__ inline void hex8_point_lds(const double* x, const double* dn, double* cd) {
    double J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) J[i][j] = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        double xa[3], da[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            xa[k] = x[3 * a + k];
            da[k] = dn[3 * a + k];
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) J[i][j] = fma(xa[i], da[j], J[i][j]);
    }
    double C[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            C[i][j] = fma(J[i1][j1], J[i2][j2], -(J[i1][j2] * J[i2][j1]));
        }
    const double det = fma(J[0][0], C[0][0], fma(J[0][1], C[0][1], J[0][2] * C[0][2]));
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) cd[3 * i + j] = C[i][j] / det;
    cd[9] = det;
}

__device__ inline void hex8_gradient(const double* cd, const double* da, double (&g)[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) t = fma(cd[3 * i + j], da[j], t);
        g[i] = t;
    }
}

// One quadrature term of the (a, b) block, added to blk (d*d values).
template <int D>
__device__ inline void hex8_block_term(const double* ga, const double* gb, double det,
                                       const double* mat, double* blk) {
    const double dot = fma(ga[2], gb[2], fma(ga[1], gb[1], ga[0] * gb[0]));
    if (D == 1) {
        blk[0] = blk[0] + (mat[0] * det) * dot;
    } else {
        const double l = mat[0] * det, m = mat[1] * det;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double s = i == j ? m * dot : 0.0;
                s = fma(m * ga[j], gb[i], s);
                s = fma(l * ga[i], gb[j], s);
                blk[3 * i + j] = blk[3 * i + j] + s;
            }
    }
}

// LDS geometry of a batch of 8 (element, point) x 8 points: gradients and
// det J per (t, q), [t][q][25].
constexpr int kGeo = 25;

// Lane (t = l / 8, q = l % 8): geometry of element e (if valid) at point q.
__device__ inline void geometry_lane(const Hex8Args& A, int64_t e, int q, double* geo) {
    double x[24];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        const int64_t v = A.conn[8 * e + a];
#pragma unroll
        for (int i = 0; i < 3; ++i) x[3 * a + i] = A.coords[3 * v + i];
    }
    double g[8][3], det;
    hex8_point(x, q, g, det);
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) geo[3 * a + i] = g[a][i];
    geo[24] = det;
}

// The (a, b) block of element e summed over the 8 points, from the batch
// geometry of its entry (geo_t: [8 points][kGeo]).
template <int D>
__device__ inline void block_from_geometry(const double* geo_t, int a, int b, const double* mat,
                                           double (&blk)[D * D]) {
#pragma unroll
    for (int r = 0; r < D * D; ++r) blk[r] = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const double* gq = geo_t + q * kGeo;
        hex8_block_term<D>(gq + 3 * a, gq + 3 * b, gq[24], mat, blk);
    }
}

// block_from_geometry from the point data of hex8_point_lds (cd_t: [8
// points][kCd]) and the reference gradients (dnt: [8 points, stride
// kDnPoint][8 nodes][3]).
template <int D>
__device__ inline void block_from_point_data(const double* cd_t, const double* dnt, int a, int b,
                                             const double* mat, double (&blk)[D * D]) {
#pragma unroll
    for (int r = 0; r < D * D; ++r) blk[r] = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const double* cq = cd_t + q * kCd;
        double ga[3], gb[3];
        hex8_gradient(cq, dnt + kDnPoint * q + 3 * a, ga);
        hex8_gradient(cq, dnt + kDnPoint * q + 3 * b, gb);
        hex8_block_term<D>(ga, gb, cq[9], mat, blk);
    }
}

// Element matrices: 8 elements per 64-lane block.
template <int D>
__global__ void __launch_bounds__(64) k_hex8_ke(Hex8Args A) {
    constexpr int N = 8 * D, M = D == 1 ? 1 : 2;
    __shared__ double geo[64 * kGeo];
    // one element matrix, written out by consecutive lanes so that every
    // store instruction covers whole cache lines (non-temporal stores are
    // not merged across instructions)
    __shared__ double slab[N * N];
    const int l = threadIdx.x, t = l >> 3, s = l & 7;
    const int64_t e0 = xcd_block(blockIdx.x, gridDim.x) * 8;
    const int64_t e = e0 + t;
    if (e < A.n_elem) geometry_lane(A, e, s, geo + l * kGeo);
    __syncthreads();
    // lane (a = t, b = s) of every element of the block
    for (int te = 0; te < 8 && e0 + te < A.n_elem; ++te) {
        const int64_t ee = e0 + te;
        double mat[M];
#pragma unroll
        for (int m = 0; m < M; ++m) mat[m] = A.mat[M * ee + m];
        double blk[D * D];
        block_from_geometry<D>(geo + te * 8 * kGeo, t, s, mat, blk);
#pragma unroll
        for (int i = 0; i < D; ++i)
#pragma unroll
            for (int j = 0; j < D; ++j) slab[(D * t + i) * N + D * s + j] = blk[D * i + j];
        __syncthreads();
        double* K = A.ke + ee * (int64_t)N * N;
#pragma unroll
        for (int u = 0; u < N * N / 64; ++u) __builtin_nontemporal_store(slab[64 * u + l], K + 64 * u + l);
        __syncthreads();
    }
}

// Fused: one node row per wavefront.
template <int FMT, int D>
__global__ void __launch_bounds__(64) k_hex8_fused(Hex8Args A) {
    constexpr int N = 8 * D, DN = D * N, M = D == 1 ? 1 : 2;
    extern __shared__ double lds[];
    double* geo = lds;                      // [64][kGeo]
    double* slab = geo + 64 * kGeo;         // [8 entries][D rows][N]
    double* acc = slab + 8 * DN;            // [D rows][ncols]
    int32_t* sidx = reinterpret_cast<int32_t*>(acc + A.acc_doubles);
    int32_t* scol = sidx + A.idx_ints;      // [8 entries][8 nodes]
    const int l = threadIdx.x, t = l >> 3, s = l & 7;
    const int64_t b = xcd_block(blockIdx.x, gridDim.x);
    const int64_t v = A.node_list ? A.node_list[b] : b;
    const int64_t tbeg = A.inc_ptr[v], T = A.inc_ptr[v + 1] - tbeg;
    const int32_t Rw = D * (int32_t)v;
    int32_t rs, ncols, npairs = 0;
    if (FMT == kCSR) {
        rs = A.row_ptr[Rw];
        ncols = A.row_ptr[Rw + 1] - rs;
        for (int x = l; x < ncols; x += 64) sidx[x] = A.col_idx[rs + x];
    } else {
        const int32_t pb = A.crac_row_ptr[Rw], pe = A.crac_row_ptr[Rw + 1];
        npairs = (pe - pb) >> 1;
        rs = npairs > 0 ? A.ca[pb + 1] : 0;
        ncols = npairs > 0 ? A.ca[pe + 1] - rs : 0;
        if (npairs > 0)
            for (int x = l; x < 2 * npairs + 2; x += 64) sidx[x] = A.ca[pb + x];
    }
    for (int x = l; x < D * ncols; x += 64) acc[x] = 0.0;
    __syncthreads();
    for (int64_t t0 = 0; t0 < T; t0 += 8) {
        // lane (t, s): geometry of entry t at point s, and the column offset
        // of element node s in the owned row
        const bool valid = t0 + t < T;
        int32_t q = 0;
        if (valid) {
            q = A.inc_q[tbeg + t0 + t];
            const int64_t e = q >> 3;
            geometry_lane(A, e, s, geo + l * kGeo);
            scol[l] = row_lookup<FMT>(sidx, ncols, npairs, rs, D * A.conn[8 * e + s]);
        }
        __syncthreads();
        // lane (t, s): the (a, s) block of entry t into the slab
        if (valid) {
            const int64_t e = q >> 3;
            const int a = q & 7;
            double mat[M];
#pragma unroll
            for (int m = 0; m < M; ++m) mat[m] = A.mat[M * e + m];
            double blk[D * D];
            block_from_geometry<D>(geo + t * 8 * kGeo, a, s, mat, blk);
#pragma unroll
            for (int i = 0; i < D; ++i)
#pragma unroll
                for (int j = 0; j < D; ++j) slab[t * DN + i * N + D * s + j] = blk[D * i + j];
        }
        __syncthreads();
        // entry by entry, in element order
        const int nt = (int)std::min<int64_t>(8, T - t0);
        for (int te = 0; te < nt; ++te) {
            for (int x = l; x < DN; x += 64) {
                const int c1 = x / N, col = x - c1 * N, b = col / D, c = col - b * D;
                const int32_t off = scol[te * 8 + b];
                if (off >= 0) atomicAdd(acc + c1 * ncols + off + c, slab[te * DN + x]);
            }
        }
        __syncthreads();
    }
    double* out = A.values + rs;
    if (A.accumulate)
        for (int x = l; x < D * ncols; x += 64) out[x] += acc[x];
    else
        for (int x = l; x < D * ncols; x += 64) __builtin_nontemporal_store(acc[x], out + x);
}

// Pipelined fused kernel over the light nodes (at most 8 incident entries,
// one batch per node).  A wavefront walks a contiguous range of positions
// of the node order.  A node's loads form a dependent chain of five steps:
//   A  node number (node order)
//   B  incidence range and the first row's pointer pair
//   C  entry q of lane (t, s) and the row's index words
//   D  element node c of the entry, and the element's materials
//   E  coordinates of c
// While node i is computed, E of node i + 1, D of i + 2, C of i + 3, B of
// i + 4 and A of i + 5 are in flight, so a node waits for memory once, not
// five times.  Each lane loads one element node's coordinates (not all
// eight), which lanes (t, *) exchange through LDS.  The geometry, blocks
// and adds are those of k_hex8_fused, in the same order.
struct PipeB {
    int64_t tbeg;
    int32_t T, pb, pe;
};
struct PipeC {
    int32_t q;
    int32_t w[3];  // index words l, l + 64, l + 128 of the first row
};
struct PipeD {
    int32_t c;
    double mat[2];
};

// A zero the optimiser cannot see through: added to a uniform index, it
// turns the load into a vector load, whose completion is counted in order
// with the other vector loads instead of with the LDS operations.
__device__ inline int32_t vector_zero() {
    int32_t z = 0;
    asm volatile("" : "+v"(z));
    return z;
}

__device__ inline int32_t uniform32(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline PipeB uniform_b(const PipeB& b) {
    PipeB r;
    r.tbeg = (int64_t)(((uint64_t)(uint32_t)uniform32((int32_t)(b.tbeg >> 32)) << 32) |
                       (uint32_t)uniform32((int32_t)b.tbeg));
    r.T = uniform32(b.T);
    r.pb = uniform32(b.pb);
    r.pe = uniform32(b.pe);
    return r;
}

template <int FMT, int D>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) k_hex8_pipe(Hex8Args A) {
    constexpr int N = 8 * D, DN = D * N, M = D == 1 ? 1 : 2;
    extern __shared__ double lds[];
    // kPointRegion values: coordinates [8 entries, stride kXsEntry][8
    // nodes][3], then the point data of lane (t, q) at t kCdEntry + q kCd,
    // then the slab [8 entries, stride SL][D rows][N]
    constexpr int SL = D == 1 ? DN : DN + 1;
    static_assert(8 * SL <= kPointRegion && 8 * kXsEntry <= kPointRegion, "LDS layout");
    double* geo = lds;
    double* dnt = geo + kPointRegion;  // [8 points, stride kDnPoint][8 nodes][3]
    double* acc = dnt + 8 * kDnPoint;  // [D rows][ncols]
    int32_t* sidx = reinterpret_cast<int32_t*>(acc + A.acc_doubles);
    int32_t* scol = sidx + A.idx_ints;  // [8 entries][8 nodes]
    const int l = threadIdx.x, t = l >> 3, s = l & 7;
    const int64_t wv = xcd_block(blockIdx.x, gridDim.x);
    const int64_t per = ceil_div(A.n_light, (int64_t)gridDim.x);
    const int64_t i0 = wv * per, i1 = std::min<int64_t>(i0 + per, A.n_light);
    if (i0 >= i1) return;
    const int32_t* rp = FMT == kCSR ? A.row_ptr : A.crac_row_ptr;
    const int32_t* idx = FMT == kCSR ? A.col_idx : A.ca;
    const int32_t z = vector_zero();
    {
        double dN[8][3];
        hex8_ref_gradients(l >> 3, dN);
        // lane (q, a) keeps row a of point q: the same values as evaluated above
#pragma unroll
        for (int a = 0; a < 8; ++a)
            if (a == (l & 7))
#pragma unroll
                for (int j = 0; j < 3; ++j) dnt[kDnPoint * (l >> 3) + 3 * a + j] = dN[a][j];
    }

    auto load_a = [&](int64_t i) -> int32_t { return A.node_list[(i < i1 ? i : i1 - 1) + z]; };
    auto load_b = [&](int32_t v) -> PipeB {
        PipeB r;
        r.tbeg = A.inc_ptr[(int64_t)v + z];
        r.T = (int32_t)(A.inc_ptr[(int64_t)v + 1 + z] - r.tbeg);
        r.pb = rp[(int64_t)D * v + z];
        r.pe = rp[(int64_t)D * v + 1 + z];
        return r;
    };
    auto load_c = [&](const PipeB& b) -> PipeC {
        PipeC r;
        // the incidence array is padded, so entries past the node's own are
        // readable (and belong to valid elements)
        r.q = A.inc_q[b.tbeg + t];
        const int32_t nidx = FMT == kCSR ? b.pe - b.pb : (b.pe > b.pb ? b.pe - b.pb + 2 : 0);
#pragma unroll
        for (int k = 0; k < 3; ++k) r.w[k] = l + 64 * k < nidx ? idx[b.pb + l + 64 * k] : 0;
        return r;
    };
    auto load_d = [&](const PipeC& c) -> PipeD {
        PipeD r;
        const int64_t e = c.q >> 3;
        r.c = A.conn[8 * e + s];
#pragma unroll
        for (int m = 0; m < M; ++m) r.mat[m] = A.mat[M * e + m];
        return r;
    };

    // fill the pipeline: after it, stage X holds the data of the node that
    // is (X's distance) ahead of node i0
    int32_t a4 = uniform32(load_a(i0 + 4));
    PipeB b3 = uniform_b(load_b(uniform32(load_a(i0 + 3)))),
          b2 = uniform_b(load_b(uniform32(load_a(i0 + 2)))),
          b1 = uniform_b(load_b(uniform32(load_a(i0 + 1)))),
          b0 = uniform_b(load_b(uniform32(load_a(i0))));
    PipeC c2 = load_c(b2), c1 = load_c(b1), c0 = load_c(b0);
    PipeD d1 = load_d(c1), d0 = load_d(c0);
    double x0[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) x0[k] = A.coords[3 * (int64_t)d0.c + k];

    for (int64_t i = i0; i < i1; ++i) {
        // issue the next nodes' steps
        double x1[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) x1[k] = A.coords[3 * (int64_t)d1.c + k];
        const PipeD d2 = load_d(c2);
        const PipeC c3 = load_c(b3);
        const PipeB b4 = load_b(a4);
        const int32_t a5 = load_a(i + 5);

        // node i
        const int32_t T = b0.T, pb = b0.pb, pe = b0.pe;
        int32_t rs, ncols, npairs = 0, nidx;
        if (FMT == kCSR) {
            rs = pb;
            ncols = pe - pb;
            nidx = ncols;
        } else {
            npairs = (pe - pb) >> 1;
            nidx = npairs > 0 ? 2 * npairs + 2 : 0;
            rs = npairs > 0 ? __builtin_amdgcn_readlane(c0.w[0], 1) : 0;
            const int32_t last = nidx - 1;
            const int32_t wl = last < 64 ? c0.w[0] : last < 128 ? c0.w[1] : c0.w[2];
            ncols = npairs > 0 ? __builtin_amdgcn_readlane(wl, last & 63) - rs : 0;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (l + 64 * k < nidx) sidx[l + 64 * k] = c0.w[k];
        for (int x = l + 192; x < nidx; x += 64) sidx[x] = idx[pb + x];
        for (int x = l; x < D * ncols; x += 64) acc[x] = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) geo[kXsEntry * t + 3 * s + k] = x0[k];
        __syncthreads();
        const bool valid = t < T;
        scol[l] = valid ? row_lookup<FMT>(sidx, ncols, npairs, rs, D * d0.c) : -1;
        // the coordinates are read (into J) before any lane's geometry
        // overwrites them: lanes of one wavefront issue LDS operations in
        // program order
        if (valid) hex8_point_lds(geo + kXsEntry * t, dnt + kDnPoint * s, geo + kCdEntry * t + kCd * s);
        __syncthreads();
        double blk[D * D];
        if (valid) block_from_point_data<D>(geo + kCdEntry * t, dnt, c0.q & 7, s, d0.mat, blk);
        __syncthreads();
        if (valid) {
#pragma unroll
            for (int r = 0; r < D; ++r)
#pragma unroll
                for (int j = 0; j < D; ++j) geo[t * SL + r * N + D * s + j] = blk[D * r + j];
        }
        __syncthreads();
        // entry by entry, in element order
        for (int te = 0; te < T; ++te) {
            for (int x = l; x < DN; x += 64) {
                const int c1r = x / N, col = x - c1r * N, bn = col / D, cc = col - bn * D;
                const int32_t off = scol[te * 8 + bn];
                if (off >= 0) atomicAdd(acc + c1r * ncols + off + cc, geo[te * SL + x]);
            }
        }
        __syncthreads();
        double* out = A.values + rs;
        if (A.accumulate)
            for (int x = l; x < D * ncols; x += 64) out[x] += acc[x];
        else
            for (int x = l; x < D * ncols; x += 64) __builtin_nontemporal_store(acc[x], out + x);
        __syncthreads();

        // advance the stages
#pragma unroll
        for (int k = 0; k < 3; ++k) x0[k] = x1[k];
        d0 = d1;
        d1 = d2;
        c0 = c1;
        c1 = c2;
        c2 = c3;
        b0 = b1;
        b1 = b2;
        b2 = b3;
        b3 = uniform_b(b4);
        a4 = uniform32(a5);
    }
}

int check_hex8(const feasm_pattern* p, const double* coords, const double* material,
               const std::string& who) {
    if (!p) FEASM_FAIL(FEASM_EINVAL, who + ": null handle");
    if (p->k != 8) FEASM_FAIL(FEASM_EINVAL, who + ": elements must have 8 nodes");
    if (p->d != 1 && p->d != 3) FEASM_FAIL(FEASM_EINVAL, who + ": d must be 1 or 3");
    if (!coords || !material) FEASM_FAIL(FEASM_EINVAL, who + ": null coords or material");
    return FEASM_OK;
}

Hex8Args hex8_args(const feasm_pattern* p, const double* coords, const double* material) {
    Hex8Args A{};
    A.conn = p->conn;
    A.inc_ptr = p->inc_ptr;
    A.inc_q = p->inc_q;
    A.row_ptr = p->row_ptr;
    A.col_idx = p->col_idx;
    A.crac_row_ptr = p->crac_row_ptr;
    A.ca = p->ca;
    A.coords = coords;
    A.mat = material;
    A.n_nodes = p->n_nodes;
    A.n_elem = p->n_elem;
    return A;
}

// Light nodes by the pipelined kernel over the node order, heavy nodes one
// per wavefront; or every node one per wavefront (tune value -1, or a handle
// without a node order).
template <int FMT, int D>
int launch_hex8(const feasm_pattern* p, Hex8Args A, size_t lds, hipStream_t s) {
    const int64_t nl = p->node_order ? p->n_light : 0, nn = p->n_nodes;
    if (p->tune_hex8_pipe < 0 || nl == 0) {
        k_hex8_fused<FMT, D><<<(unsigned)nn, 64, lds, s>>>(A);
        FEASM_HIP(hipGetLastError());
        return FEASM_OK;
    }
    const size_t lds_pipe = sizeof(double) * (kPointRegion + 8 * kDnPoint + (size_t)A.acc_doubles) +
                            sizeof(int32_t) * ((size_t)A.idx_ints + 64);
    int dev = 0, cus = 0, lds_cu = 0;
    FEASM_HIP(hipGetDevice(&dev));
    FEASM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int per_cu = p->tune_hex8_pipe;
    if (per_cu == 0) {
        // every block of the grid must be resident at once (a block that
        // starts late adds a whole range to the run time), so the count is
        // also capped by LDS in 512-byte allocation units
        FEASM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(&k_hex8_pipe<FMT, D>), 64, lds_pipe));
        FEASM_HIP(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev));
        if (lds_cu > 0)
            per_cu = std::min<int>(per_cu, lds_cu / (int)(ceil_div((int64_t)lds_pipe, 512) * 512));
        if (per_cu < 1) per_cu = 1;
    }
    const int64_t grid = std::min<int64_t>(nl, (int64_t)(cus > 0 ? cus : 256) * per_cu);
    Hex8Args L = A;
    L.node_list = p->node_order;
    L.n_light = nl;
    k_hex8_pipe<FMT, D><<<(unsigned)grid, 64, lds_pipe, s>>>(L);
    FEASM_HIP(hipGetLastError());
    if (nn > nl) {
        Hex8Args H = A;
        H.node_list = p->node_order + nl;
        k_hex8_fused<FMT, D><<<(unsigned)(nn - nl), 64, lds, s>>>(H);
        FEASM_HIP(hipGetLastError());
    }
    return FEASM_OK;
}

}  // namespace
}  // namespace feasm

extern "C" int hex8_element_matrices(const feasm_pattern* p, const double* coords,
                                     const double* material, double* ke, hipStream_t stream) {
    return feasm::guarded("hex8_element_matrices", [&]() -> int {
        using namespace feasm;
        int rc = check_hex8(p, coords, material, "hex8_element_matrices");
        if (rc != FEASM_OK) return rc;
        if (!ke) FEASM_FAIL(FEASM_EINVAL, "hex8_element_matrices: null ke");
        if (p->n_elem == 0) return FEASM_OK;
        Hex8Args A = hex8_args(p, coords, material);
        A.ke = ke;
        const unsigned blocks = (unsigned)ceil_div(p->n_elem, 8);
        if (p->d == 1)
            k_hex8_ke<1><<<blocks, 64, 0, stream>>>(A);
        else
            k_hex8_ke<3><<<blocks, 64, 0, stream>>>(A);
        FEASM_HIP(hipGetLastError());
        return FEASM_OK;
    });
}

extern "C" int assemble_hex8(const feasm_pattern* p, int fmt, const double* coords,
                             const double* material, double* values, int flags,
                             hipStream_t stream) {
    return feasm::guarded("assemble_hex8", [&]() -> int {
        using namespace feasm;
        int rc = check_hex8(p, coords, material, "assemble_hex8");
        if (rc != FEASM_OK) return rc;
        if (!values) FEASM_FAIL(FEASM_EINVAL, "assemble_hex8: null values");
        if (fmt != FEASM_FMT_CSR && fmt != FEASM_FMT_CRAC)
            FEASM_FAIL(FEASM_EINVAL, "assemble_hex8: fmt must be FEASM_FMT_CSR or FEASM_FMT_CRAC");
        if (fmt == FEASM_FMT_CSR && !(p->flags & FEASM_BUILD_CSR))
            FEASM_FAIL(FEASM_EINVAL, "assemble_hex8: handle was built without CSR");
        if (fmt == FEASM_FMT_CRAC && !(p->flags & FEASM_BUILD_CRAC))
            FEASM_FAIL(FEASM_EINVAL, "assemble_hex8: handle was built without CRAC");
        if ((flags & ~FEASM_ACCUMULATE) != 0) FEASM_FAIL(FEASM_EINVAL, "assemble_hex8: unknown flag");
        if (p->n_nodes == 0) return FEASM_OK;
        Hex8Args A = hex8_args(p, coords, material);
        A.values = values;
        A.accumulate = (flags & FEASM_ACCUMULATE) ? 1 : 0;
        const int d = p->d;
        A.acc_doubles = d * d * p->max_deg;
        A.idx_ints = fmt == FEASM_FMT_CSR ? d * p->max_deg : 2 * p->max_deg + 2;
        const size_t lds = sizeof(double) * (64 * kGeo + 8 * d * 8 * d + (size_t)A.acc_doubles) +
                           sizeof(int32_t) * ((size_t)A.idx_ints + 64);
        if (lds > 64 * 1024)
            FEASM_FAIL(FEASM_ELIMIT, "assemble_hex8: node rows too long for the LDS accumulator");
        if (fmt == FEASM_FMT_CSR)
            return d == 1 ? launch_hex8<kCSR, 1>(p, A, lds, stream) : launch_hex8<kCSR, 3>(p, A, lds, stream);
        return d == 1 ? launch_hex8<kCRAC, 1>(p, A, lds, stream) : launch_hex8<kCRAC, 3>(p, A, lds, stream);
    });
}

