// Membrane and immersed-boundary kernels (gfx950).
//
// Node positions are an integer anchor per capsule plus an FP32 offset
// (off_hi), with an FP32 compensation term (off_lo) carried by the forward
// Euler update (Sec. II.B) so that many small displacements accumulate
// without FP32 rounding loss.  All geometry uses anchor + off_hi.
//
// Per step:
//   k_clear_tiles   zero the immersed-boundary fields of last step's tiles
//   k_cap_volume    FP64 enclosed volume per capsule (Sec. II.B, eq.
//                   method:volume), one thread per triangle
//   k_faces         Skalak (Sec. II.B, eq. method:strain) and volume
//                   forces per triangle and corner, F = -dE/dX
//   k_node_gather   sixteen lanes per node: gather its triangles' corner
//                   forces, count the node into its home bin
//   k_bin_alloc     disjoint slot runs for the occupied bins (wavefront scan
//                   plus one global atomic per wavefront)
//   k_bin_scatter   counting-sort scatter of node ids into the bins; flag
//                   the 8^3 tiles the bins' stencils can reach
//   k_bend_geo, k_bend_force  (when enabled) Helfrich bending: discrete
//                   curvatures per node, then the cot Laplacian and the force
//   k_repulse       (when enabled) particle-particle repulsion between nodes
//                   of different capsules, searched through the bins
//   k_spread        one workgroup per occupied bin: add the wettability
//                   reaction of its nodes (psi staged on a 9^3 LDS cube,
//                   sixteen lanes per node), accumulate F_b delta and
//                   the virtual density in 7^3 LDS boxes (one per wavefront,
//                   one lane per stencil point, no LDS atomics), then flush
//                   the non-zero cells to HBM with global atomics
//   k_interp_advect sixteen lanes per node: U_b = sum u delta, X += U_b
// Only k_spread reads the densities of the step: the kernels before it
// (after the previous step's advection) can overlap the density pass.
#include "lbm_internal.h"

namespace lbmx {

namespace {

constexpr int CNT_TOUCHED = 0;   // counters[0..1]
constexpr int CNT_HOME = 2;      // counters[2..3]
constexpr int CNT_ALLOC = 4;     // counters[4..5]
#ifndef LBM_CLEAR_GRID
#define LBM_CLEAR_GRID 2048
#endif
constexpr int CLEAR_GRID = LBM_CLEAR_GRID;   // blocks of the tile clearing (a grid-stride loop over the tiles)

__device__ __forceinline__ int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Periodic wrap without a division, for v in [-n, 3n) (stencil and box
// offsets from an already wrapped base; every lattice edge is >= 4).
__device__ __forceinline__ int wrap3(int v, int n) {
    v += v < 0 ? n : 0;
    v -= v >= n ? n : 0;
    v -= v >= n ? n : 0;
    return v;
}

// The index of this lane's wavefront within the block, as a wave-uniform
// (scalar) value: everything derived from it (node ids, positions) then
// lives in scalar registers and is read with scalar loads.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Peskin 4-point kernel
__device__ __forceinline__ float peskin(float r) {
    const float a = fabsf(r);
    if (a <= 1.0f) return (3.0f - 2.0f * a + sqrtf(1.0f + 4.0f * a - 4.0f * a * a)) * 0.125f;
    if (a <= 2.0f) return (5.0f - 2.0f * a - sqrtf(-7.0f + 12.0f * a - 4.0f * a * a)) * 0.125f;
    return 0.0f;
}

// its derivative
__device__ __forceinline__ float peskin_d(float r) {
    const float a = fabsf(r), sg = r < 0.0f ? -1.0f : 1.0f;
    if (a <= 1.0f) return sg * (-2.0f + (4.0f - 8.0f * a) / (2.0f * sqrtf(1.0f + 4.0f * a - 4.0f * a * a))) * 0.125f;
    if (a <= 2.0f) return sg * (-2.0f - (12.0f - 8.0f * a) / (2.0f * sqrtf(-7.0f + 12.0f * a - 4.0f * a * a))) * 0.125f;
    return 0.0f;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct NodePos {
    int fl[3];      // floor(X), absolute (unwrapped)
    float r[3];     // X - floor(X)
};

__device__ __forceinline__ NodePos node_pos(const Dev& d, int b) {
    const int4 an = d.node_anc[b];
    const int A[3] = {an.x, an.y, an.z};
    NodePos p;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float o = d.off_hi[3 * b + k];
        const float fo = floorf(o);
        p.fl[k] = A[k] + (int)fo;
        p.r[k] = o - fo;
    }
    return p;
}

// floor(X) wrapped into the lattice
__device__ __forceinline__ void wrapped_floor(const Lattice& L, const NodePos& p, int w[3]) {
    w[0] = wrapi(p.fl[0], L.nx);
    w[1] = wrapi(p.fl[1], L.ny);
    w[2] = wrapi(p.fl[2], L.nz);
}

__device__ __forceinline__ int tile_of(const Lattice& L, int x, int y, int z) {
    return ((z >> 3) * L.nty + (y >> 3)) * L.ntx + (x >> 3);
}

__device__ __forceinline__ int bin_of(const Lattice& L, int x, int y, int z) {
    return ((z / BIN) * L.nby + (y / BIN)) * L.nbx + (x / BIN);
}

// One workgroup per touched tile of the previous step (tile coordinates are
// wave-uniform): zero its immersed-boundary fields and flag; then the
// previous step's bin counts, this step's counters and capsule volumes.
// (blk of nblk blocks: the kernel also runs as a part of k_advect_clear)
__device__ __forceinline__ void clear_tiles(const Lattice& L, const Dev& d, int pp, int pc, int n_caps, int blk,
                                            int nblk) {
    const int nt = d.counters[CNT_TOUCHED + pp];
    const int nh = d.counters[CNT_HOME + pp];
    const int64_t N = L.n;
    for (int e = blk; e < nt; e += nblk) {
        const int t = d.touched[pp][e];
        const int tx = t % L.ntx, ty = (t / L.ntx) % L.nty, tz = t / (L.ntx * L.nty);
        for (int c = threadIdx.x; c < TILE * TILE * TILE; c += blockDim.x) {
            const int x = tx * TILE + (c & 7), y = ty * TILE + ((c >> 3) & 7), z = tz * TILE + (c >> 6);
            if (x < L.nx && y < L.ny && z < L.nz) {
                const uint32_t node = (uint32_t)((z * L.ny + y) * L.nx + x);
#pragma unroll
                for (int f = 0; f < 5; ++f) d.fib[f * N + node] = 0.0f;
                if (d.lam_u)   // the adjoint velocity field lives in the same tiles
                    for (int f = 0; f < 3; ++f) d.lam_u[f * N + node] = 0.0f;
            }
        }
        if (threadIdx.x == 0) d.tile_flag[t] = 0;
    }
    for (int64_t k = blk * (int64_t)blockDim.x + threadIdx.x; k < nh; k += (int64_t)nblk * blockDim.x)
        d.tile_count[d.home[pp][k]] = 0;
    if (blk == 0) {
        if (threadIdx.x == 0) {
            d.counters[CNT_TOUCHED + pc] = 0;
            d.counters[CNT_HOME + pc] = 0;
            d.counters[CNT_ALLOC + pc] = 0;
        }
        for (int k = threadIdx.x; k < n_caps; k += blockDim.x) {
            d.capV[k] = 0.0;
            if (d.capdV) d.capdV[k] = 0.0;
        }
    }
}

__global__ __launch_bounds__(256) void k_clear_tiles(Lattice L, Dev d, int pp, int pc, int n_caps) {
    clear_tiles(L, d, pp, pc, n_caps, blockIdx.x, gridDim.x);
}

// Triangle f's part of its capsule's volume, X1 . (X2 x X3) / 6 over
// anchor-relative offsets, in FP64.
__device__ __forceinline__ double face_volume(const Dev& d, int f) {
    double X[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int b = d.tri[3 * f + k];
#pragma unroll
        for (int j = 0; j < 3; ++j) X[k][j] = (double)d.off_hi[3 * b + j];
    }
    return (X[0][0] * (X[1][1] * X[2][2] - X[1][2] * X[2][1])
          + X[0][1] * (X[1][2] * X[2][0] - X[1][0] * X[2][2])
          + X[0][2] * (X[1][0] * X[2][1] - X[1][1] * X[2][0])) / 6.0;
}

// FP64 enclosed volume per capsule, V = sum_T face_volume: one thread per
// triangle, a block reduction when the block's triangles belong to one
// capsule, FP64 atomics otherwise.
__global__ __launch_bounds__(256) void k_cap_volume(Dev d, int n_faces) {
    __shared__ double sh[256];
    __shared__ int cap_first, cap_last;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    const int f_last = min((int)(blockIdx.x * blockDim.x + blockDim.x), n_faces) - 1;
    double v = 0.0;
    int cap = -1;
    if (f < n_faces) {
        cap = d.face_cap[f];
        v = face_volume(d, f);
    }
    if (threadIdx.x == 0) {
        cap_first = d.face_cap[blockIdx.x * blockDim.x];
        cap_last = d.face_cap[f_last];
    }
    __syncthreads();
    if (cap_first != cap_last) {
        if (f < n_faces) unsafeAtomicAdd(&d.capV[cap], v);
        return;
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) unsafeAtomicAdd(&d.capV[cap_first], sh[0]);
}

// Deterministic mode.  Three sums of the default step take their order
// from atomics, which differs from run to run: the capsule volumes above,
// the node ranks within a bin (the order in which the spreading and the
// repulsion visit a bin's nodes) and the flush of the bins' boxes into the
// lattice fields.  With deterministic sums each capsule's volume is one
// block's fixed-order reduction, each bin's nodes are ranked by id, and the
// force and virtual-density fields are gathered per lattice cell over the
// nodes in (bin, id) order, so that a step is the same bit for bit from run
// to run (the default step differs from it by rounding order only).

// one block per capsule: its triangles strided over the threads, then a
// fixed tree
__global__ __launch_bounds__(256) void k_cap_volume_det(Dev d) {
    __shared__ double sh[256];
    const CapDev& C = d.caps[blockIdx.x];
    double v = 0.0;
    for (int f = C.face_start + (int)threadIdx.x; f < C.face_start + C.face_count; f += 256) v += face_volume(d, f);
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) d.capV[blockIdx.x] = sh[0];
}

// Scalars that carry a tangent: v + e * epsilon.  The face forces below are
// written once, as a template; with Dual they give the directional
// derivative of the forces, which for forces derived from an energy is the
// Hessian-vector product the adjoint needs.
struct Dual {
    float v, e;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.e + b.e}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.e - b.e}; }
__device__ __forceinline__ Dual operator-(Dual a) { return {-a.v, -a.e}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.v * b.e + a.e * b.v}; }
__device__ __forceinline__ Dual operator*(float a, Dual b) { return {a * b.v, a * b.e}; }
__device__ __forceinline__ Dual operator*(Dual a, float b) { return {a.v * b, a.e * b}; }
__device__ __forceinline__ Dual operator+(Dual a, float b) { return {a.v + b, a.e}; }
__device__ __forceinline__ Dual operator-(Dual a, float b) { return {a.v - b, a.e}; }

template <typename T>
__device__ __forceinline__ void cross3(const T* a, const T* b, T* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// Skalak energy per triangle, E_T = A0 (kS/4)(I1^2 + 2 I1 - 2 I2 + C I2^2),
// I1 = tr(M0^-1 M) - 2, I2 = det M / det M0 - 1, with its analytic gradient
// (Fsk = -dE_T/dX per corner); plus the volume-penalty corner forces
// vfac * dV_T/dX with vfac = -kV (V - V0) / (6 V0).
template <typename T>
__device__ __forceinline__ void face_forces(const T X[3][3], const FaceRef& R, float kS, float C, T vfac,
                                            T Fsk[3][3], T F[3][3]) {
    T e1[3], e2[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        e1[j] = X[1][j] - X[0][j];
        e2[j] = X[2][j] - X[0][j];
    }
    const T m11 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
    const T m12 = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
    const T m22 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
    const T I1 = R.q11 * m11 + (2.0f * R.q12) * m12 + R.q22 * m22 - 2.0f;
    const T I2 = (m11 * m22 - m12 * m12) * R.inv_det0 - 1.0f;
    const T W1 = (0.25f * kS) * (2.0f * I1 + 2.0f);
    const T W2 = ((0.25f * kS) * (2.0f * C * I2 - 2.0f)) * R.inv_det0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        // d tr/d e1 = 2 (q11 e1 + q12 e2), d det/d e1 = 2 (m22 e1 - m12 e2)
        const T g1 = R.A0 * (W1 * (2.0f * (R.q11 * e1[j] + R.q12 * e2[j])) + W2 * (2.0f * (m22 * e1[j] - m12 * e2[j])));
        const T g2 = R.A0 * (W1 * (2.0f * (R.q12 * e1[j] + R.q22 * e2[j])) + W2 * (2.0f * (m11 * e2[j] - m12 * e1[j])));
        Fsk[0][j] = g1 + g2;
        Fsk[1][j] = -g1;
        Fsk[2][j] = -g2;
    }
    T c0[3], c1[3], c2[3];
    cross3(X[1], X[2], c0);
    cross3(X[2], X[0], c1);
    cross3(X[0], X[1], c2);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        F[0][j] = Fsk[0][j] + vfac * c0[j];
        F[1][j] = Fsk[1][j] + vfac * c1[j];
        F[2][j] = Fsk[2][j] + vfac * c2[j];
    }
}

__global__ __launch_bounds__(256) void k_faces(Dev d, int n_faces) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n_faces) return;
    const int cap = d.face_cap[f];
    const CapDev& C = d.caps[cap];
    float X[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int b = d.tri[3 * f + k];
#pragma unroll
        for (int j = 0; j < 3; ++j) X[k][j] = d.off_hi[3 * b + j];
    }
    const float vfac = C.kV != 0.0f ? -(float)((double)C.kV * (d.capV[cap] - C.V0) / C.V0) * (1.0f / 6.0f) : 0.0f;
    float Fsk[3][3], F[3][3];
    face_forces<float>(X, d.fref[f], C.kS, C.C, vfac, Fsk, F);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float* o = d.face_F + 3 * (int64_t)d.corner_slot[3 * f + k];
#pragma unroll
        for (int j = 0; j < 3; ++j) o[j] = F[k][j];
    }
}

// Node forces: the sum of the corner forces of the incident triangles, and
// the node's count into its home bin (4^3).  It reads no density, so it can
// run beside the density pass; the wettability reaction, which needs this
// step's densities, is added in k_spread.  Four nodes per wavefront, sixteen
// lanes per node, sixteen nodes per block.
__global__ __launch_bounds__(256) void k_node_gather(Lattice L, Dev d, int n_nodes, int par) {
    const int lane = threadIdx.x & 63, l16 = lane & 15;
    const int b = blockIdx.x * 16 + wave_id() * 4 + (lane >> 4);
    const bool valid = b < n_nodes;
    float gx = 0.f, gy = 0.f, gz = 0.f;
    int t = 0, rank = 0;
    if (valid) {
        const int beg = d.csr_ptr[b], end = d.csr_ptr[b + 1];
        for (int k = beg + l16; k < end; k += 16) {
            gx += d.face_F[3 * (int64_t)k + 0];
            gy += d.face_F[3 * (int64_t)k + 1];
            gz += d.face_F[3 * (int64_t)k + 2];
        }
        if (l16 == 1) {
            const NodePos p = node_pos(d, b);
            int pw[3];
            wrapped_floor(L, p, pw);
            t = bin_of(L, pw[0], pw[1], pw[2]);
            rank = atomicAdd(&d.tile_count[t], 1);
        }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
        gx += __shfl_xor(gx, o, 16);
        gy += __shfl_xor(gy, o, 16);
        gz += __shfl_xor(gz, o, 16);
    }
    if (valid && l16 == 0) {
        d.node_F[3 * b + 0] = gx;
        d.node_F[3 * b + 1] = gy;
        d.node_F[3 * b + 2] = gz;
    } else if (valid && l16 == 1) {
        d.node_tile[b] = t;
        d.node_rank[b] = rank;
        if (rank == 0) d.home[par][atomicAdd(&d.counters[CNT_HOME + par], 1)] = t;
    }
}

// Segments of the counting sort: each occupied bin gets a disjoint run of
// slots.  A wavefront scans its 64 bins' counts and takes one run for all
// of them from a global counter (segment order is immaterial to the sort).
__global__ __launch_bounds__(256) void k_bin_alloc(Dev d, int par) {
    const int nh = d.counters[CNT_HOME + par];
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int h = 0, cnt = 0;
    if (e < nh) {
        h = d.home[par][e];
        cnt = d.tile_count[h];
    }
    int v = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    const int total = __shfl(v, 63, 64);
    int base = 0;
    if (lane == 63 && total > 0) base = atomicAdd(&d.counters[CNT_ALLOC + par], total);
    base = __shfl(base, 63, 64);
    if (e < nh) {
        const int start = base + v - cnt;
        d.home_start[e] = start;
        d.tile_offset[h] = start;
    }
}

// Counting-sort scatter of the node ids, and the lattice tiles that the
// delta stencils can reach: a node of home bin c (floor(X) in [4c, 4c+3] per
// axis) has its stencil in [4c-1, 4c+5], so each occupied bin flags every
// tile that range meets on each axis (at most three when an edge is not a
// multiple of the tile).  A small superset of the exact set, from one
// thread per (bin, tile combination) instead of per node.
__global__ __launch_bounds__(256) void k_bin_scatter(Lattice L, Dev d, int n_nodes, int par) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n_nodes) d.sorted[d.tile_offset[d.node_tile[b]] + d.node_rank[b]] = b;
    const int nh = d.counters[CNT_HOME + par];
    const int nn[3] = {L.nx, L.ny, L.nz};
    for (int it = b; it < nh * 27; it += gridDim.x * blockDim.x) {
        const int e = it / 27, cmb = it - 27 * e;
        const int sel[3] = {cmb % 3, (cmb / 3) % 3, cmb / 9};
        const int h = d.home[par][e];
        const int bc[3] = {h % L.nbx, (h / L.nbx) % L.nby, h / (L.nbx * L.nby)};
        int tsel[3];
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // the sel[a]-th distinct tile met by cells 4c-1 .. 4c+5 of axis a
            int tt[3], nt = 0;
#pragma unroll
            for (int k = 0; k < BIN + 3; ++k) {
                const int tk = wrap3(BIN * bc[a] - 1 + k, nn[a]) >> 3;
                bool seen = false;
                for (int q = 0; q < nt; ++q) seen = seen || tt[q] == tk;
                if (!seen && nt < 3) tt[nt++] = tk;
            }
            ok = ok && sel[a] < nt;
            tsel[a] = tt[sel[a] < nt ? sel[a] : 0];
        }
        if (ok) {
            const int t = (tsel[2] * L.nty + tsel[1]) * L.ntx + tsel[0];
            if (atomicExch(&d.tile_flag[t], 1) == 0)
                d.touched[par][atomicAdd(&d.counters[CNT_TOUCHED + par], 1)] = t;
        }
    }
}

// Deterministic mode: each node's rank in its home bin becomes the number
// of the bin's nodes with a lower id (read from the order the scatter left,
// which any rank order gives), then the nodes are placed again by it.
__global__ __launch_bounds__(256) void k_bin_rank_det(Dev d, int n_nodes) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_nodes) return;
    const int t = d.node_tile[b], start = d.tile_offset[t], cnt = d.tile_count[t];
    int r = 0;
    for (int k = 0; k < cnt; ++k) r += d.sorted[start + k] < b;
    d.node_rank[b] = r;
}

__global__ __launch_bounds__(256) void k_bin_place_det(Dev d, int n_nodes) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < n_nodes) d.sorted[d.tile_offset[d.node_tile[b]] + d.node_rank[b]] = b;
}

// Particle-particle repulsion (Sec. III.E): a node pair of different
// capsules at separation d < d0 repels along the separation with
// eps (d0 - d)^{3/2}.
//
// for_each_contact calls fn(e, v, r2) for every node e of another capsule
// with |v|^2 = r2 < d0^2, v = X_b - X_e on the nearest periodic image:
// node b searches this step's 4^3 bins that its d0-ball meets.  Positions
// are anchor + (hi + lo) offsets; both nodes of a pair compute the same
// separation from negated differences.  The search range is widened by
// 1e-3 so that the bins (taken from the hi offsets alone) cover every pair.
// A capsule's nodes have consecutive ids, so same-capsule candidates are
// skipped by a range test without loading anything of theirs.  The caller
// takes the candidates sub, sub + nsub, ... of each bin (several lanes
// sharing one node's search).
template <typename Fn>
__device__ __forceinline__ void for_each_contact(const Lattice& L, const Dev& d, int b, float d0, int sub, int nsub,
                                                 Fn&& fn) {
    const NodePos p = node_pos(d, b);
    int pw[3];
    wrapped_floor(L, p, pw);
    const int4 an = d.node_anc[b];
    const CapDev& C = d.caps[d.node_cap[b]];
    const unsigned own0 = (unsigned)C.node_start, own_n = (unsigned)C.node_count;
    const int A[3] = {an.x, an.y, an.z};
    float oh[3], ol[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        oh[k] = d.off_hi[3 * b + k];
        ol[k] = d.off_lo[3 * b + k];
    }
    const int nn[3] = {L.nx, L.ny, L.nz};
    const float reach = d0 + 1e-3f;
    // distinct bins met by the cells floor(X - reach) .. floor(X + reach) per axis
    int bins[3][4], nb[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        nb[a] = 0;
        const int c0 = pw[a] + (int)floorf(p.r[a] - reach), c1 = pw[a] + (int)floorf(p.r[a] + reach);
        for (int c = c0; c <= c1; ++c) {
            int cw = c;
            if (a == 1 && (L.walls || L.onsite)) {
                if (c < 0 || c >= nn[a]) continue;
            } else {
                cw = wrap3(c, nn[a]);
            }
            const int bb = cw / BIN;
            bool seen = false;
            for (int q = 0; q < nb[a]; ++q) seen = seen || bins[a][q] == bb;
            if (!seen && nb[a] < 4) bins[a][nb[a]++] = bb;
        }
    }
    const float d02 = d0 * d0;
    for (int iz = 0; iz < nb[2]; ++iz)
        for (int iy = 0; iy < nb[1]; ++iy)
            for (int ix = 0; ix < nb[0]; ++ix) {
                const int t = (bins[2][iz] * L.nby + bins[1][iy]) * L.nbx + bins[0][ix];
                const int cnt = d.tile_count[t];
                const int start = cnt > 0 ? d.tile_offset[t] : 0;
                for (int k = sub; k < cnt; k += nsub) {
                    const int e = d.sorted[start + k];
                    if ((unsigned)e - own0 < own_n) continue;
                    const int4 ae = d.node_anc[e];
                    const int Ae[3] = {ae.x, ae.y, ae.z};
                    float v[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        float x = (float)(A[a] - Ae[a]) + ((oh[a] - d.off_hi[3 * e + a]) + (ol[a] - d.off_lo[3 * e + a]));
                        if (!(a == 1 && (L.walls || L.onsite))) {
                            const float nf = (float)nn[a];
                            x -= nf * rintf(x / nf);
                        }
                        v[a] = x;
                    }
                    const float r2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
                    if (r2 < d02 && r2 > 0.0f) fn(e, v, r2);
                }
            }
}

// Forward: node b's repulsion, f_b = sum_e m(d) (X_b - X_e) with
// m(d) = eps (d0 - d)^{3/2} / d, added to its force at X^n.
// REP_LANES lanes per node, each taking every REP_LANES-th candidate of a
// bin: crowded contacts (pressed capsules) split over the lanes, while a
// sparse suspension does not pay the bin search many times over.
constexpr int REP_LANES = 4;
__global__ __launch_bounds__(256) void k_repulse(Lattice L, Dev d, int n_nodes, float eps, float d0) {
    const int sl = threadIdx.x & (REP_LANES - 1);
    const int b = blockIdx.x * (256 / REP_LANES) + (int)(threadIdx.x / REP_LANES);
    float F[3] = {0.f, 0.f, 0.f};
    if (b < n_nodes)
        for_each_contact(L, d, b, d0, sl, REP_LANES, [&](int, const float* v, float r2) {
            const float r = sqrtf(r2), g = d0 - r;
            const float m = eps * g * sqrtf(g) / r;
            F[0] += m * v[0];
            F[1] += m * v[1];
            F[2] += m * v[2];
        });
#pragma unroll
    for (int o = REP_LANES / 2; o > 0; o >>= 1) {
        F[0] += __shfl_xor(F[0], o, REP_LANES);
        F[1] += __shfl_xor(F[1], o, REP_LANES);
        F[2] += __shfl_xor(F[2], o, REP_LANES);
    }
    if (b < n_nodes && sl == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a) d.node_F[3 * b + a] += F[a];
    }
}

// Adjoint: with J = dF_b/dX_b = m I + (m'(d) / d) v v^T (symmetric) and
// dF_e/dX_b = -J for the partner, lambda_X_b += sum_e J (lambda_F_b -
// lambda_F_e), where m'(d) = -eps (1.5 (d0 - d)^{1/2} / d + (d0 - d)^{3/2} / d^2).
__global__ __launch_bounds__(256) void k_adj_repulse(Lattice L, Dev d, int n_nodes, float eps, float d0) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_nodes) return;
    const float lb[3] = {d.lam_Fb[3 * b], d.lam_Fb[3 * b + 1], d.lam_Fb[3 * b + 2]};
    float acc[3] = {0.f, 0.f, 0.f};
    for_each_contact(L, d, b, d0, 0, 1, [&](int e, const float* v, float r2) {
        const float r = sqrtf(r2), g = d0 - r, sg = sqrtf(g);
        const float m = eps * g * sg / r;
        const float mp = -eps * (1.5f * sg / r + g * sg / r2);
        const float w[3] = {lb[0] - d.lam_Fb[3 * e], lb[1] - d.lam_Fb[3 * e + 1], lb[2] - d.lam_Fb[3 * e + 2]};
        const float vw = (v[0] * w[0] + v[1] * w[1] + v[2] * w[2]) * (mp / r);
        acc[0] += m * w[0] + vw * v[0];
        acc[1] += m * w[1] + vw * v[1];
        acc[2] += m * w[2] + vw * v[2];
    });
#pragma unroll
    for (int a = 0; a < 3; ++a) d.lam_X[3 * b + a] += acc[a];
}

// Helfrich bending (Sec. II.B, eq. surf_dens with zero spontaneous
// curvature): F_i = 2 kB [2 H (H^2 - K) + Lap_s H] n A at each node of a
// capsule with kB > 0, from the discrete operators of Meyer et al. (2003)
// on the current mesh.  Per triangle (i, j, k) seen from node i: the cot of
// the angle at a corner is (dot of its two edges) / |cross|; the mixed area
// is the Voronoi part (|x_ij|^2 cot_k + |x_ik|^2 cot_j) / 8 for a triangle
// without an obtuse angle, else area / 2 (obtuse at i) or area / 4; the
// mean curvature normal sums cot_k (x_i - x_j) + cot_j (x_i - x_k) over
// 2 A; the Gaussian curvature is the angle deficit over A; n is the
// normalised sum of the triangles' area normals, H = (K_vec . n) / 2.
// Two passes, one thread per node walking its corners: the geometry, then
// the cot Laplacian of H (which needs the neighbours' H) and the force.
// Positions are the capsule-relative hi + lo offsets (one anchor per capsule).
__device__ __forceinline__ void bend_pos(const Dev& d, int b, float x[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = d.off_hi[3 * b + a] + d.off_lo[3 * b + a];
}

struct BendCorner {
    int j, k;                 // the other two nodes, in the triangle's cyclic order after i
    float eij[3], eik[3];     // x_j - x_i, x_k - x_i
    float cn;                 // |e_ij x e_ik| (twice the area)
    float cr[3];              // e_ij x e_ik (outward area normal, doubled)
    float di, cot_j, cot_k;   // dot at i, cots at j and k
};

__device__ __forceinline__ BendCorner bend_corner(const Dev& d, int sc, const float xi[3]) {
    BendCorner q;
    const int f = sc / 3, c = sc - 3 * f;
    q.j = d.tri[3 * f + (c + 1) % 3];
    q.k = d.tri[3 * f + (c + 2) % 3];
    float xj[3], xk[3];
    bend_pos(d, q.j, xj);
    bend_pos(d, q.k, xk);
    float ejk[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        q.eij[a] = xj[a] - xi[a];
        q.eik[a] = xk[a] - xi[a];
        ejk[a] = xk[a] - xj[a];
    }
    q.cr[0] = q.eij[1] * q.eik[2] - q.eij[2] * q.eik[1];
    q.cr[1] = q.eij[2] * q.eik[0] - q.eij[0] * q.eik[2];
    q.cr[2] = q.eij[0] * q.eik[1] - q.eij[1] * q.eik[0];
    q.cn = sqrtf(q.cr[0] * q.cr[0] + q.cr[1] * q.cr[1] + q.cr[2] * q.cr[2]);
    q.di = q.eij[0] * q.eik[0] + q.eij[1] * q.eik[1] + q.eij[2] * q.eik[2];
    const float dj = -(q.eij[0] * ejk[0] + q.eij[1] * ejk[1] + q.eij[2] * ejk[2]);
    const float dk = q.eik[0] * ejk[0] + q.eik[1] * ejk[1] + q.eik[2] * ejk[2];
    q.cot_j = dj / q.cn;
    q.cot_k = dk / q.cn;
    return q;
}

__global__ __launch_bounds__(256) void k_bend_geo(Dev d, int n_nodes) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_nodes || d.caps[d.node_cap[b]].kB == 0.0f) return;
    float xi[3];
    bend_pos(d, b, xi);
    float A = 0.f, th = 0.f, Kv[3] = {0.f, 0.f, 0.f}, nr[3] = {0.f, 0.f, 0.f};
    for (int s = d.csr_ptr[b]; s < d.csr_ptr[b + 1]; ++s) {
        const BendCorner q = bend_corner(d, d.slot_corner[s], xi);
        const float area = 0.5f * q.cn;
        const float lij = q.eij[0] * q.eij[0] + q.eij[1] * q.eij[1] + q.eij[2] * q.eij[2];
        const float lik = q.eik[0] * q.eik[0] + q.eik[1] * q.eik[1] + q.eik[2] * q.eik[2];
        const bool obt_other = q.cot_j < 0.0f || q.cot_k < 0.0f;
        A += q.di < 0.0f ? 0.5f * area : (obt_other ? 0.25f * area : 0.125f * (lij * q.cot_k + lik * q.cot_j));
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Kv[a] -= q.cot_k * q.eij[a] + q.cot_j * q.eik[a];
            nr[a] += q.cr[a];
        }
        th += atan2f(q.cn, q.di);
    }
    const float inr = 1.0f / sqrtf(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
    const float n[3] = {nr[0] * inr, nr[1] * inr, nr[2] * inr};
    float* o = d.node_bend + 6 * (int64_t)b;
    o[0] = 0.5f * (Kv[0] * n[0] + Kv[1] * n[1] + Kv[2] * n[2]) / (2.0f * A);
    o[1] = (6.28318530717958648f - th) / A;
    o[2] = A;
    o[3] = n[0];
    o[4] = n[1];
    o[5] = n[2];
}

__global__ __launch_bounds__(256) void k_bend_force(Dev d, int n_nodes) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_nodes) return;
    const float kB = d.caps[d.node_cap[b]].kB;
    if (kB == 0.0f) return;
    float xi[3];
    bend_pos(d, b, xi);
    const float* g = d.node_bend + 6 * (int64_t)b;
    const float H = g[0], K = g[1], A = g[2];
    float lap = 0.f;
    for (int s = d.csr_ptr[b]; s < d.csr_ptr[b + 1]; ++s) {
        const BendCorner q = bend_corner(d, d.slot_corner[s], xi);
        lap += q.cot_k * (d.node_bend[6 * (int64_t)q.j] - H) + q.cot_j * (d.node_bend[6 * (int64_t)q.k] - H);
    }
    lap /= 2.0f * A;
    const float sF = 2.0f * kB * (2.0f * H * (H * H - K) + lap) * A;
#pragma unroll
    for (int a = 0; a < 3; ++a) d.node_F[3 * b + a] += sF * g[3 + a];
}

// ---- LBM-free reference model (Sec. III.B, eq. emulatetension) ----------
// Membrane-only relaxation: the elastic and bending forces plus the
// emulated tension gamma A / w on the part A of each element's area inside
// the slab |z - z_interface| <= w / 2, horizontal and radially away from the
// vertical axis through the capsule's centre of mass at the start of the
// relaxation (cap_mom[2..3] / node count, capsule-relative), shared evenly by
// the element's three nodes; then X += mu F.  The slab area uses the closed
// form of the area fraction below a plane (quadratic on each side of the
// middle vertex height).

__global__ void k_ref_zero_volume(Dev d, int n_caps) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n_caps) d.capV[k] = 0.0;
}

__device__ __forceinline__ float frac_below(float z0, float z1, float z2, float h) {
    // sort the three heights
    float a = fminf(z0, fminf(z1, z2)), c = fmaxf(z0, fmaxf(z1, z2));
    float b = z0 + z1 + z2 - a - c;
    if (h <= a) return 0.0f;
    if (h >= c) return 1.0f;
    if (h <= b) return (h - a) * (h - a) / ((b - a) * (c - a));
    return 1.0f - (c - h) * (c - h) / ((c - b) * (c - a));
}

__global__ __launch_bounds__(256) void k_ref_tension(Dev d, int n_faces, float gamma, float w, double z_interface) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n_faces) return;
    const int cap = d.face_cap[f];
    const CapDev& C = d.caps[cap];
    float x[3][3];
    for (int k = 0; k < 3; ++k) {
        const int b = d.tri[3 * f + k];
        for (int a = 0; a < 3; ++a) x[k][a] = d.off_hi[3 * b + a] + d.off_lo[3 * b + a];
    }
    // the slab in capsule-relative heights
    const float zi = (float)(z_interface - (double)C.anchor[2]);
    const float lo = zi - 0.5f * w, hi = zi + 0.5f * w;
    const float fb = frac_below(x[0][2], x[1][2], x[2][2], hi) - frac_below(x[0][2], x[1][2], x[2][2], lo);
    if (fb == 0.0f) return;
    float e1[3], e2[3];
    for (int a = 0; a < 3; ++a) {
        e1[a] = x[1][a] - x[0][a];
        e2[a] = x[2][a] - x[0][a];
    }
    const float cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2], cz = e1[0] * e2[1] - e1[1] * e2[0];
    const float area = 0.5f * sqrtf(cx * cx + cy * cy + cz * cz);
    const double inv_n = 1.0 / (double)C.node_count;
    const float ax = (float)(d.cap_mom[cap * MOM_STRIDE + 2] * inv_n), ay = (float)(d.cap_mom[cap * MOM_STRIDE + 3] * inv_n);
    const float dx = (x[0][0] + x[1][0] + x[2][0]) * (1.0f / 3.0f) - ax;
    const float dy = (x[0][1] + x[1][1] + x[2][1]) * (1.0f / 3.0f) - ay;
    const float dn = sqrtf(dx * dx + dy * dy);
    if (dn == 0.0f) return;
    const float m = gamma * area * fb / w * (1.0f / 3.0f) / dn;
    for (int k = 0; k < 3; ++k) {
        const int sl = d.corner_slot[3 * f + k];
        d.face_F[3 * (int64_t)sl + 0] += m * dx;
        d.face_F[3 * (int64_t)sl + 1] += m * dy;
    }
}

__global__ __launch_bounds__(256) void k_ref_gather(Dev d, int n_nodes) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_nodes) return;
    float g[3] = {0.f, 0.f, 0.f};
    for (int k = d.csr_ptr[b]; k < d.csr_ptr[b + 1]; ++k)
        for (int a = 0; a < 3; ++a) g[a] += d.face_F[3 * (int64_t)k + a];
    for (int a = 0; a < 3; ++a) d.node_F[3 * b + a] = g[a];
}

__global__ __launch_bounds__(256) void k_ref_advance(Dev d, int n_nodes, float mu) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_nodes) return;
    for (int k = 0; k < 3; ++k) {
        // compensated (hi, lo) += mu F, as in the coupled advection
        const float a = d.off_hi[3 * b + k];
        const float bb = d.off_lo[3 * b + k] + mu * d.node_F[3 * b + k];
        const float s = a + bb;
        const float bv = s - a;
        const float err = (a - (s - bv)) + (bb - bv);
        d.off_hi[3 * b + k] = s;
        d.off_lo[3 * b + k] = err;
    }
}

constexpr int SPREAD_GRID = 2048;

// Spreading, with the wettability reaction of the wetting nodes added first
// (it needs this step's densities; the rest of the node force does not).
// Per occupied bin: stage the bin's nodes; stage the pseudo-potential of the
// components its wetting nodes read (usually one: most bins meet one
// capsule) on the 9^3 cube that the stencils of the bin's nodes and their
// lattice neighbours reach; add each wetting node's reaction
// -G |rho_v| A_b sum_y delta(y - X_b) sum_i w_i psi^np(y + c_i) c_i, sixteen
// nodes at a time with sixteen lanes each (lane (kx, ky) takes the stencil
// column kz = 0..3), storing the node's total force back; then accumulate
// F_b delta and the virtual density in the boxes and flush them.
template <bool PSI>     // the exponential pseudo-potential (a compile-time choice, as in the collide)
__global__ __launch_bounds__(256) void k_spread(Lattice L, Dev d, int par, const float* __restrict__ rho_n,
                                                const float* __restrict__ cs) {
    constexpr int B3 = BOX * BOX * BOX;
    constexpr int WC = BIN + 5;                 // psi cube edge: bin cells -2 .. +6
    constexpr int W3 = WC * WC * WC;
    constexpr int CH = 128;                     // nodes staged per round
    // one box per wavefront: a wavefront adds its nodes one after another
    // with plain LDS read-modify-writes (the 64 lanes of one node hit
    // distinct cells), which is far cheaper than LDS float atomics; the
    // flush sums the four boxes
    __shared__ float box[4][5][B3];
    __shared__ float psi[2][W3];
    // the bin's nodes, staged by one thread each: per-axis delta weights,
    // force, virtual-density weight, the box and cube cells of the stencil
    // origin, the field the virtual density goes to and the node id
    __shared__ float sw[12][CH];
    __shared__ float sf[4][CH];
    __shared__ int scell[CH], swc[CH], sfield[CH], sid[CH];
    const int nh = d.counters[CNT_HOME + par];
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int kx = lane & 3, ky = (lane >> 2) & 3, kz = lane >> 4;
    const int l16 = lane & 15, q16 = threadIdx.x >> 4;       // wettability: node slot and lane
    const int64_t N = L.n;
    float* mybox = &box[wave][0][0];
    const float sc[2] = {cs ? cs[0] : 1.0f, cs ? cs[1] : 1.0f};   // FP16 form: this step's mass compensation
    // deterministic mode: the wettability reactions only (k_spread_gather_det fills the fields)
    const bool flush = d.det == 0;
    for (int e = blockIdx.x; e < nh; e += gridDim.x) {
        const int t = d.home[par][e];
        const int start = d.home_start[e], cnt = d.tile_count[t];
        if (cnt == 0) continue;                 // (a home bin holds a node; block-uniform)
        const int ox = (t % L.nbx) * BIN, oy = ((t / L.nbx) % L.nby) * BIN, oz = (t / (L.nbx * L.nby)) * BIN;
        if (flush)
            for (int k = threadIdx.x; k < 4 * 5 * B3; k += 256) (&box[0][0][0])[k] = 0.0f;
        // (the barrier after staging also orders the zeroing above)
        for (int c0 = 0; c0 < cnt; c0 += CH) {
            const int m = min(cnt - c0, CH);
            int need0 = 0, need1 = 0;           // components whose psi a wetting node reads
            if ((int)threadIdx.x < m) {
                const int b = d.sorted[start + c0 + threadIdx.x];
                const NodePos p = node_pos(d, b);
                int pw[3];
                wrapped_floor(L, p, pw);
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int k = 0; k < 4; ++k) sw[4 * a + k][threadIdx.x] = peskin(p.r[a] + 1.0f - k);
                sf[0][threadIdx.x] = d.node_F[3 * b + 0];
                sf[1][threadIdx.x] = d.node_F[3 * b + 1];
                sf[2][threadIdx.x] = d.node_F[3 * b + 2];
                const float wet = d.node_wet[b];
                const int pref = d.node_anc[b].w;
                need0 = wet != 0.0f && pref == 1;   // it reads the component it does not prefer
                need1 = wet != 0.0f && pref == 0;
                sf[3][threadIdx.x] = wet;
                sfield[threadIdx.x] = wet != 0.0f ? 3 + pref : -1;
                scell[threadIdx.x] = ((pw[2] - oz) * BOX + (pw[1] - oy)) * BOX + (pw[0] - ox);
                swc[threadIdx.x] = ((pw[2] - oz + 1) * WC + (pw[1] - oy + 1)) * WC + (pw[0] - ox + 1);
                sid[threadIdx.x] = b;
            }
            const int n0 = __syncthreads_or(need0) != 0, n1 = __syncthreads_or(need1) != 0;
            if (n0 || n1) {
                // (most bins meet one capsule, so one component)
                for (int k = threadIdx.x; k < (n0 + n1) * W3; k += 256) {
                    const int c = (k >= W3 || !n0) ? 1 : 0, cell = k >= W3 ? k - W3 : k;
                    const int iz = cell / (WC * WC), iy = (cell / WC) % WC, ix = cell % WC;
                    int gy = wrap3(oy - 2 + iy, L.ny);
                    if (L.walls) gy = gy == 0 ? 1 : (gy == L.ny - 1 ? L.ny - 2 : gy);
                    if (L.onsite) gy = min(max(oy - 2 + iy, 0), L.ny - 1);
                    const int gx = wrap3(ox - 2 + ix, L.nx), gz = wrap3(oz - 2 + iz, L.nz);
                    const float r = sc[c] * rho_n[c * N + (uint32_t)((gz * L.ny + gy) * L.nx + gx)];
                    psi[c][cell] = PSI ? psi_exp(r) : r;
                }
                __syncthreads();
                for (int j0 = 0; j0 < m; j0 += 16) {
                    const int j = j0 + q16;
                    const bool on = j < m && sfield[min(j, m - 1)] >= 0;      // (uniform per sixteen lanes)
                    const int jj = on ? j : 0;
                    // an idle group reads from the origin of a node at bin cell
                    // (1, 1, 1), inside the cube, with zero weight
                    const int base = on ? swc[jj] : ((2 * WC) + 2) * WC + 2;
                    const float* qp = psi[on ? 4 - sfield[jj] : 0];        // component np = 1 - (field - 3)
                    const int qx = l16 & 3, qy = l16 >> 2;
                    const float wxy = on ? sw[qx][jj] * sw[4 + qy][jj] : 0.0f;
                    float S[3] = {0.f, 0.f, 0.f};
#pragma unroll
                    for (int qz = 0; qz < 4; ++qz) {
                        const float w = wxy * sw[8 + qz][jj];
                        const int y0 = base + (qz * WC + qy) * WC + qx;
                        float T[3] = {0.f, 0.f, 0.f};
#pragma unroll
                        for (int k = 1; k < Q; k += 2) {
                            const int o = (cz(k) * WC + cy(k)) * WC + cx(k);
                            const float dd = wgt(k) * (qp[y0 + o] - qp[y0 - o]);
                            if (cx(k)) T[0] += cx(k) * dd;
                            if (cy(k)) T[1] += cy(k) * dd;
                            if (cz(k)) T[2] += cz(k) * dd;
                        }
                        S[0] += w * T[0];
                        S[1] += w * T[1];
                        S[2] += w * T[2];
                    }
#pragma unroll
                    for (int o = 8; o > 0; o >>= 1) {
                        S[0] += __shfl_xor(S[0], o, 16);
                        S[1] += __shfl_xor(S[1], o, 16);
                        S[2] += __shfl_xor(S[2], o, 16);
                    }
                    if (on && l16 < 3) {
                        const float s0 = -L.G * sf[3][jj];
                        const float F = sf[l16][jj] + s0 * (l16 == 0 ? S[0] : (l16 == 1 ? S[1] : S[2]));
                        sf[l16][jj] = F;
                        d.node_F[3 * sid[jj] + l16] = F;
                    }
                }
                __syncthreads();
            }
            for (int j = wave; flush && j < m; j += 4) {
                const float w = sw[kx][j] * sw[4 + ky][j] * sw[8 + kz][j];
                const int cell = scell[j] + (kz * BOX + ky) * BOX + kx;
                mybox[0 * B3 + cell] += w * sf[0][j];
                mybox[1 * B3 + cell] += w * sf[1][j];
                mybox[2 * B3 + cell] += w * sf[2][j];
                const int fld = sfield[j];
                if (fld >= 0) mybox[fld * B3 + cell] += w * sf[3][j];
            }
            __syncthreads();
        }
        for (int k = threadIdx.x; flush && k < 5 * B3; k += 256) {
            const float* bx = &box[0][0][0];
            const float v = (bx[k] + bx[5 * B3 + k]) + (bx[10 * B3 + k] + bx[15 * B3 + k]);
            if (v != 0.0f) {
                const int f = k / B3, cell = k - f * B3;
                const int iz = cell / (BOX * BOX), iy = (cell / BOX) % BOX, ix = cell % BOX;
                const int gx = wrap3(ox - 1 + ix, L.nx), gy = wrap3(oy - 1 + iy, L.ny), gz = wrap3(oz - 1 + iz, L.nz);
                unsafeAtomicAdd(&d.fib[f * N + (uint32_t)((gz * L.ny + gy) * L.nx + gx)], v);
            }
        }
        __syncthreads();
    }
}

// Deterministic mode: one block per touched tile writes the five fields of
// each of its cells, F_b delta and the virtual densities summed over the
// nodes of the bins whose stencils can reach the tile, bins in (z, y, x)
// order and each bin's nodes in id order (after k_spread has added the
// wettability reactions to node_F).  A node of wrapped floor cell p reaches
// the cells p - 1 .. p + 2 of each axis, so the tile's cells t0 .. t1 are
// reached from the floor cells t0 - 2 .. t1 + 1; their distinct bins, in
// the order met, are the candidates (at most 11 per axis).
__global__ __launch_bounds__(256) void k_spread_gather_det(Lattice L, Dev d, int par) {
    constexpr int CH = 128;
    __shared__ float sw[12][CH];
    __shared__ float sf[4][CH];
    __shared__ int sp[3][CH], sfield[CH];
    __shared__ int sb[3][11], snb[3];
    const int nt = d.counters[CNT_TOUCHED + par];
    const int64_t N = L.n;
    const int nn[3] = {L.nx, L.ny, L.nz};
    for (int e = blockIdx.x; e < nt; e += gridDim.x) {
        const int t = d.touched[par][e];
        const int T[3] = {t % L.ntx, (t / L.ntx) % L.nty, t / (L.ntx * L.nty)};
        if (threadIdx.x < 3) {
            const int a = threadIdx.x, t0 = TILE * T[a], t1 = min(t0 + TILE - 1, nn[a] - 1);
            int nb = 0;
            for (int c = t0 - 2; c <= t1 + 1; ++c) {
                const int bb = wrap3(c, nn[a]) / BIN;
                bool seen = false;
                for (int q = 0; q < nb; ++q) seen = seen || sb[a][q] == bb;
                if (!seen) sb[a][nb++] = bb;
            }
            snb[a] = nb;
        }
        // this thread's cells: c and c + 256 of the tile's 512
        int cell[2][3];
        bool in[2];
        float acc[2][5];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = (int)threadIdx.x + 256 * h;
            cell[h][0] = T[0] * TILE + (c & 7);
            cell[h][1] = T[1] * TILE + ((c >> 3) & 7);
            cell[h][2] = T[2] * TILE + (c >> 6);
            in[h] = cell[h][0] < L.nx && cell[h][1] < L.ny && cell[h][2] < L.nz;
#pragma unroll
            for (int f = 0; f < 5; ++f) acc[h][f] = 0.0f;
        }
        __syncthreads();
        for (int iz = 0; iz < snb[2]; ++iz)
            for (int iy = 0; iy < snb[1]; ++iy)
                for (int ix = 0; ix < snb[0]; ++ix) {
                    const int bin = (sb[2][iz] * L.nby + sb[1][iy]) * L.nbx + sb[0][ix];
                    const int cnt = d.tile_count[bin];
                    const int start = cnt > 0 ? d.tile_offset[bin] : 0;
                    for (int c0 = 0; c0 < cnt; c0 += CH) {
                        const int m = min(cnt - c0, CH);
                        if ((int)threadIdx.x < m) {
                            const int b = d.sorted[start + c0 + threadIdx.x];
                            const NodePos p = node_pos(d, b);
                            int pw[3];
                            wrapped_floor(L, p, pw);
#pragma unroll
                            for (int a = 0; a < 3; ++a) {
                                sp[a][threadIdx.x] = pw[a];
#pragma unroll
                                for (int k = 0; k < 4; ++k) sw[4 * a + k][threadIdx.x] = peskin(p.r[a] + 1.0f - k);
                            }
                            sf[0][threadIdx.x] = d.node_F[3 * b + 0];
                            sf[1][threadIdx.x] = d.node_F[3 * b + 1];
                            sf[2][threadIdx.x] = d.node_F[3 * b + 2];
                            const float wet = d.node_wet[b];
                            sf[3][threadIdx.x] = wet;
                            sfield[threadIdx.x] = wet != 0.0f ? 3 + d.node_anc[b].w : -1;
                        }
                        __syncthreads();
                        for (int j = 0; j < m; ++j) {
#pragma unroll
                            for (int h = 0; h < 2; ++h) {
                                // stencil index of the cell on each axis (n >= 4: at most one)
                                float w = 1.0f;
                                bool hit = in[h];
#pragma unroll
                                for (int a = 0; a < 3; ++a) {
                                    int k = cell[h][a] - sp[a][j] + 1;
                                    if (k < 0) k += nn[a];
                                    if (k >= nn[a]) k -= nn[a];
                                    hit = hit && k < 4;
                                    w *= sw[4 * a + min(k, 3)][j];
                                }
                                if (hit) {
                                    acc[h][0] += w * sf[0][j];
                                    acc[h][1] += w * sf[1][j];
                                    acc[h][2] += w * sf[2][j];
                                    const int fld = sfield[j];
                                    if (fld == 3) acc[h][3] += w * sf[3][j];
                                    if (fld == 4) acc[h][4] += w * sf[3][j];
                                }
                            }
                        }
                        __syncthreads();
                    }
                }
#pragma unroll
        for (int h = 0; h < 2; ++h)
            if (in[h]) {
                const uint32_t node = (uint32_t)((cell[h][2] * L.ny + cell[h][1]) * L.nx + cell[h][0]);
#pragma unroll
                for (int f = 0; f < 5; ++f) d.fib[f * N + node] = acc[h][f];
            }
        __syncthreads();      // (sb, snb are rewritten for the next tile)
    }
}

// Four nodes per wavefront, sixteen lanes per node: lane (kx, ky) of a
// node sums its stencil column kz = 0..3, then the sixteen lanes reduce.
__device__ __forceinline__ void interp_advect(const Lattice& L, const Dev& d, int n_nodes, int blk) {
    const int lane = threadIdx.x & 63;
    const int q = lane >> 4, kx = lane & 3, ky = (lane >> 2) & 3;
    const int b = (blk * 4 + wave_id()) * 4 + q;
    float ux = 0.f, uy = 0.f, uz = 0.f;
    NodePos p;
    if (b < n_nodes) {
        p = node_pos(d, b);
        int pw[3];
        wrapped_floor(L, p, pw);
        const float wxy = peskin(p.r[0] + 1.0f - kx) * peskin(p.r[1] + 1.0f - ky);
        const uint32_t rxy = (uint32_t)(wrap3(pw[1] - 1 + ky, L.ny) * L.nx + wrap3(pw[0] - 1 + kx, L.nx));
#pragma unroll
        for (int kz = 0; kz < 4; ++kz) {
            const float w = wxy * peskin(p.r[2] + 1.0f - kz);
            const uint32_t node = (uint32_t)(wrap3(pw[2] - 1 + kz, L.nz) * L.ny * L.nx) + rxy;
            ux += w * d.u[node];
            uy += w * d.u[L.n + node];
            uz += w * d.u[2 * L.n + node];
        }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
        ux += __shfl_xor(ux, o, 16);
        uy += __shfl_xor(uy, o, 16);
        uz += __shfl_xor(uz, o, 16);
    }
    if (b < n_nodes && (lane & 15) == 0) {
        const float U[3] = {ux, uy, uz};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            // compensated forward Euler: (hi, lo) += U exactly up to the lo rounding
            const float a = d.off_hi[3 * b + k];
            const float bb = d.off_lo[3 * b + k] + U[k];
            const float s = a + bb;
            const float bv = s - a;
            const float err = (a - (s - bv)) + (bb - bv);
            d.off_hi[3 * b + k] = s;
            d.off_lo[3 * b + k] = err;
        }
    }
}

__global__ __launch_bounds__(256) void k_interp_advect(Lattice L, Dev d, int n_nodes) {
    interp_advect(L, d, n_nodes, blockIdx.x);
}

// The previous step's advection and this step's tile clearing in one launch
// (they touch disjoint data): the first n_ib blocks advect, the rest clear.
__global__ __launch_bounds__(256) void k_advect_clear(Lattice L, Dev d, int n_nodes, int n_ib, int pp, int pc,
                                                      int n_caps) {
    if ((int)blockIdx.x < n_ib)
        interp_advect(L, d, n_nodes, blockIdx.x);
    else
        clear_tiles(L, d, pp, pc, n_caps, blockIdx.x - n_ib, gridDim.x - n_ib);
}

// FP64 shape moments per capsule, origin at the anchor:
// [0] V, [1] A, [2..4] sum of node offsets, [5..7] int x dV,
// [8..13] int x x^T dV (xx, yy, zz, xy, xz, yz).
__global__ __launch_bounds__(256) void k_cap_moments(Dev d) {
    __shared__ double sh[14][256];
    const CapDev C = d.caps[blockIdx.x];
    double acc[14];
    for (int j = 0; j < 14; ++j) acc[j] = 0.0;
    for (int f = C.face_start + threadIdx.x; f < C.face_start + C.face_count; f += blockDim.x) {
        double X[3][3];
        for (int k = 0; k < 3; ++k) {
            const int b = d.tri[3 * f + k];
            for (int j = 0; j < 3; ++j) X[k][j] = (double)d.off_hi[3 * b + j] + (double)d.off_lo[3 * b + j];
        }
        const double* a = X[0];
        const double* bq = X[1];
        const double* c = X[2];
        const double v = (a[0] * (bq[1] * c[2] - bq[2] * c[1]) + a[1] * (bq[2] * c[0] - bq[0] * c[2])
                          + a[2] * (bq[0] * c[1] - bq[1] * c[0])) / 6.0;
        double e1[3], e2[3];
        for (int j = 0; j < 3; ++j) { e1[j] = bq[j] - a[j]; e2[j] = c[j] - a[j]; }
        const double n0 = e1[1] * e2[2] - e1[2] * e2[1], n1 = e1[2] * e2[0] - e1[0] * e2[2],
                     n2 = e1[0] * e2[1] - e1[1] * e2[0];
        acc[0] += v;
        acc[1] += 0.5 * sqrt(n0 * n0 + n1 * n1 + n2 * n2);
        double s[3];
        for (int j = 0; j < 3; ++j) { s[j] = a[j] + bq[j] + c[j]; acc[5 + j] += v * s[j] * 0.25; }
        const int pi[6] = {0, 1, 2, 0, 0, 1}, pj[6] = {0, 1, 2, 1, 2, 2};
        for (int q = 0; q < 6; ++q) {
            const int i = pi[q], j = pj[q];
            acc[8 + q] += v / 20.0 * (a[i] * a[j] + bq[i] * bq[j] + c[i] * c[j] + s[i] * s[j]);
        }
    }
    for (int b = C.node_start + threadIdx.x; b < C.node_start + C.node_count; b += blockDim.x)
        for (int j = 0; j < 3; ++j) acc[2 + j] += (double)d.off_hi[3 * b + j] + (double)d.off_lo[3 * b + j];
    for (int j = 0; j < 14; ++j) sh[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int j = 0; j < 14; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 14) d.cap_mom[blockIdx.x * MOM_STRIDE + threadIdx.x] = sh[threadIdx.x][0];
}

// ---- adjoint -----------------------------------------------------------

// Spread a 3-vector per node with the same bins and LDS boxes as k_spread.
// mode 0: into target[axis][N]; mode 1: into the non-preferred component's
// block of a [2][3][N] target.
__global__ __launch_bounds__(256) void k_spread_vec(Lattice L, Dev d, int par, const float* __restrict__ val,
                                                    float* __restrict__ target, int mode) {
    constexpr int B3 = BOX * BOX * BOX;
    // one box per wavefront, plain LDS adds (as in k_spread)
    __shared__ float box[4][6][B3];
    const int nh = d.counters[CNT_HOME + par];
    const int lane = threadIdx.x & 63, wave = wave_id();
    const int kx = lane & 3, ky = (lane >> 2) & 3, kz = lane >> 4;
    const int64_t N = L.n;
    const int nf = mode == 0 ? 3 : 6;
    float* mybox = &box[wave][0][0];
    for (int e = blockIdx.x; e < nh; e += gridDim.x) {
        const int t = d.home[par][e];
        const int start = d.home_start[e], cnt = d.tile_count[t];
        const int ox = (t % L.nbx) * BIN, oy = ((t / L.nbx) % L.nby) * BIN, oz = (t / (L.nbx * L.nby)) * BIN;
        for (int k = threadIdx.x; k < 4 * 6 * B3; k += 256) (&box[0][0][0])[k] = 0.0f;
        __syncthreads();
        for (int j = wave; j < cnt; j += 4) {
            const int b = d.sorted[start + j];
            const NodePos p = node_pos(d, b);
            int pw[3];
            wrapped_floor(L, p, pw);
            const float w = peskin(p.r[0] + 1.0f - kx) * peskin(p.r[1] + 1.0f - ky) * peskin(p.r[2] + 1.0f - kz);
            const int cell = ((pw[2] - oz + kz) * BOX + (pw[1] - oy + ky)) * BOX + (pw[0] - ox + kx);
            const int base = mode == 0 ? 0 : 3 * (1 - d.node_anc[b].w);
            for (int a = 0; a < 3; ++a) mybox[(base + a) * B3 + cell] += w * val[3 * b + a];
        }
        __syncthreads();
        for (int k = threadIdx.x; k < nf * B3; k += 256) {
            const float* bx = &box[0][0][0];
            const float v = (bx[k] + bx[6 * B3 + k]) + (bx[12 * B3 + k] + bx[18 * B3 + k]);
            if (v != 0.0f) {
                const int f = k / B3, cell = k - f * B3;
                const int iz = cell / (BOX * BOX), iy = (cell / BOX) % BOX, ix = cell % BOX;
                const int gx = wrap3(ox - 1 + ix, L.nx), gy = wrap3(oy - 1 + iy, L.ny), gz = wrap3(oz - 1 + iz, L.nz);
                unsafeAtomicAdd(&target[f * N + (uint32_t)((gz * L.ny + gy) * L.nx + gx)], v);
            }
        }
        __syncthreads();
    }
}

// Adjoint of the node-side coupling, one wavefront per node (64 lanes =
// the delta stencil).  With lambda_U = lambda_X of the step's output:
//   lambda_Fb = sum_y delta lambda_Fib(y)          (spreading of F_b)
//   lambda_a  = sum_y delta lambda_phi(y) - G lambda_Fb . I_b
//               (phi and the wettability reaction R_b = -G a_b I_b,
//                I_b = sum_y delta S^np(y))
//   lambda_X += sum_y grad_X delta(y - X) [lambda_U . u + lambda_Fib . F_b
//               + a_b lambda_phi - G a_b lambda_Fb . S^np]
//   dJ/dG += -a_b lambda_Fb . I_b,  dJ/dtheta += lambda_a da_b/dtheta,
// and lambda_q = -G a_b lambda_Fb, to be spread into lambda_S^np.
// lambda_phi^pref(y) = sum_i w_i c_i . lambda_S^pref(y - c_i) comes from a
// 6^3 LDS cube of lambda_S, S^np from a 6^3 cube of rho^np.  Stencils must
// stay two nodes away from solid rows.
__global__ __launch_bounds__(256) void k_adj_nodes(Lattice L, Dev d, const float* __restrict__ rho_n, int n_nodes) {
    constexpr int CB = 6, C3 = CB * CB * CB;
    __shared__ float cube_r[4][C3];
    __shared__ float cube_s[4][3][C3];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int b = blockIdx.x * 4 + wv;
    if (b >= n_nodes) return;                   // whole wavefront; no block barrier below
    const int64_t N = L.n;
    const NodePos p = node_pos(d, b);
    const CapDev& C = d.caps[d.node_cap[b]];
    const float a_b = d.node_wet[b];
    const int pref = C.pref, np = 1 - pref;
    for (int j = lane; j < C3; j += 64) {
        const int qz = j / (CB * CB), qy = (j / CB) % CB, qx = j % CB;
        int gy = wrapi(p.fl[1] - 2 + qy, L.ny);
        const int64_t idx = ((int64_t)wrapi(p.fl[2] - 2 + qz, L.nz) * L.ny + gy) * L.nx + wrapi(p.fl[0] - 2 + qx, L.nx);
        for (int a = 0; a < 3; ++a) cube_s[wv][a][j] = d.lam_S[(3 * pref + a) * N + idx];
        if (L.walls) gy = gy == 0 ? 1 : (gy == L.ny - 1 ? L.ny - 2 : gy);
        const float r = rho_n[np * N + ((int64_t)wrapi(p.fl[2] - 2 + qz, L.nz) * L.ny + gy) * L.nx +
                              wrapi(p.fl[0] - 2 + qx, L.nx)];
        cube_r[wv][j] = L.psi_exp ? psi_exp(r) : r;     // the pseudo-potential, as in the forward
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int kx = lane & 3, ky = (lane >> 2) & 3, kz = lane >> 4;
    const float px = peskin(p.r[0] + 1.0f - kx), py = peskin(p.r[1] + 1.0f - ky), pz = peskin(p.r[2] + 1.0f - kz);
    const float w = px * py * pz;
    const float gw[3] = {peskin_d(p.r[0] + 1.0f - kx) * py * pz, px * peskin_d(p.r[1] + 1.0f - ky) * pz,
                         px * py * peskin_d(p.r[2] + 1.0f - kz)};
    const int64_t node = ((int64_t)wrapi(p.fl[2] - 1 + kz, L.nz) * L.ny + wrapi(p.fl[1] - 1 + ky, L.ny)) * L.nx
                       + wrapi(p.fl[0] - 1 + kx, L.nx);
    float lfib[3], uu[3];
    for (int a = 0; a < 3; ++a) {
        lfib[a] = d.lam_Fib[a * N + node];
        uu[a] = d.u[a * N + node];
    }
    const int c0 = ((kz + 1) * CB + (ky + 1)) * CB + (kx + 1);
    float lphi = 0.f, S[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 1; k < Q; k += 2) {
        const int o = (cz(k) * CB + cy(k)) * CB + cx(k);
        // lambda_phi: sum_i w_i c_i . lambda_S(y - c_i)
        float v = 0.f;
        if (cx(k)) v += cx(k) * (cube_s[wv][0][c0 - o] - cube_s[wv][0][c0 + o]);
        if (cy(k)) v += cy(k) * (cube_s[wv][1][c0 - o] - cube_s[wv][1][c0 + o]);
        if (cz(k)) v += cz(k) * (cube_s[wv][2][c0 - o] - cube_s[wv][2][c0 + o]);
        lphi += wgt(k) * v;
        // S^np(y) = sum_i w_i rho^np(y + c_i) c_i
        const float dd = wgt(k) * (cube_r[wv][c0 + o] - cube_r[wv][c0 - o]);
        if (cx(k)) S[0] += cx(k) * dd;
        if (cy(k)) S[1] += cy(k) * dd;
        if (cz(k)) S[2] += cz(k) * dd;
    }
    float lFb[3], I[3];
    for (int a = 0; a < 3; ++a) {
        lFb[a] = wave_sum(w * lfib[a]);
        I[a] = wave_sum(w * S[a]);
    }
    const float la1 = wave_sum(w * lphi);
    const float lU[3] = {d.lam_X[3 * b], d.lam_X[3 * b + 1], d.lam_X[3 * b + 2]};
    const float Fb[3] = {d.node_F[3 * b], d.node_F[3 * b + 1], d.node_F[3 * b + 2]};
    const float val = lU[0] * uu[0] + lU[1] * uu[1] + lU[2] * uu[2] + lfib[0] * Fb[0] + lfib[1] * Fb[1] +
                      lfib[2] * Fb[2] + a_b * lphi - L.G * a_b * (lFb[0] * S[0] + lFb[1] * S[1] + lFb[2] * S[2]);
    float gX[3];
    for (int a = 0; a < 3; ++a) gX[a] = wave_sum(gw[a] * val);
    if (lane == 0) {
        const float lFI = lFb[0] * I[0] + lFb[1] * I[1] + lFb[2] * I[2];
        const float la = la1 - L.G * lFI;
        for (int a = 0; a < 3; ++a) {
            d.lam_Fb[3 * b + a] = lFb[a];
            d.lam_q[3 * b + a] = -L.G * a_b * lFb[a];
            d.lam_Xg[3 * b + a] = gX[a];
        }
        d.node_g[2 * b] = -(double)a_b * lFI;
        d.node_g[2 * b + 1] = (double)la * d.node_area[b] * C.drv;
    }
}

// FP64 directional derivative of each capsule volume along lambda_Fb.
__global__ __launch_bounds__(256) void k_adj_capdV(Dev d, int n_faces) {
    __shared__ double sh[256];
    __shared__ int cap_first, cap_last;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    const int f_last = min((int)(blockIdx.x * blockDim.x + blockDim.x), n_faces) - 1;
    double v = 0.0;
    int cap = -1;
    if (f < n_faces) {
        cap = d.face_cap[f];
        double X[3][3], l[3][3];
        for (int k = 0; k < 3; ++k) {
            const int bb = d.tri[3 * f + k];
            for (int j = 0; j < 3; ++j) {
                X[k][j] = (double)d.off_hi[3 * bb + j];
                l[k][j] = (double)d.lam_Fb[3 * bb + j];
            }
        }
        double c0[3], c1[3], c2[3];
        cross3<double>(X[1], X[2], c0);
        cross3<double>(X[2], X[0], c1);
        cross3<double>(X[0], X[1], c2);
        for (int j = 0; j < 3; ++j) v += c0[j] * l[0][j] + c1[j] * l[1][j] + c2[j] * l[2][j];
        v /= 6.0;
    }
    if (threadIdx.x == 0) {
        cap_first = d.face_cap[blockIdx.x * blockDim.x];
        cap_last = d.face_cap[f_last];
    }
    __syncthreads();
    if (cap_first != cap_last) {
        if (f < n_faces) unsafeAtomicAdd(&d.capdV[cap], v);
        return;
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) unsafeAtomicAdd(&d.capdV[cap_first], sh[0]);
}

// Tangent of the face forces along X + eps lambda_Fb (the Hessian-vector
// product of the elastic energy, written to face_F) and the kS derivative
// sum_corners lambda_Fb . F_skalak / kS.
__global__ __launch_bounds__(256) void k_adj_faces(Dev d, int n_faces) {
    __shared__ double sh[256];
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    double gk = 0.0;
    if (f < n_faces) {
        const int cap = d.face_cap[f];
        const CapDev& C = d.caps[cap];
        Dual X[3][3];
        float l[3][3];
        for (int k = 0; k < 3; ++k) {
            const int bb = d.tri[3 * f + k];
            for (int j = 0; j < 3; ++j) {
                l[k][j] = d.lam_Fb[3 * bb + j];
                X[k][j] = Dual{d.off_hi[3 * bb + j], l[k][j]};
            }
        }
        Dual vfac{0.0f, 0.0f};
        if (C.kV != 0.0f) {
            vfac.v = -(float)((double)C.kV * (d.capV[cap] - C.V0) / C.V0) * (1.0f / 6.0f);
            vfac.e = -(float)((double)C.kV * d.capdV[cap] / C.V0) * (1.0f / 6.0f);
        }
        Dual Fsk[3][3], F[3][3];
        face_forces<Dual>(X, d.fref[f], C.kS, C.C, vfac, Fsk, F);
        for (int k = 0; k < 3; ++k) {
            float* o = d.face_F + 3 * (int64_t)d.corner_slot[3 * f + k];
            for (int j = 0; j < 3; ++j) {
                o[j] = F[k][j].e;
                gk += (double)l[k][j] * Fsk[k][j].v;
            }
        }
        gk /= (double)C.kS;
    }
    sh[threadIdx.x] = gk;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && sh[0] != 0.0) unsafeAtomicAdd(&d.grads[1], sh[0]);
}

// lambda_X(step input) = lambda_X(step output) + delta-gradient terms +
// Hessian-vector product gathered over the node's triangles.
__global__ __launch_bounds__(256) void k_adj_node_update(Dev d, int n_nodes) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_nodes) return;
    float g[3] = {d.lam_Xg[3 * b], d.lam_Xg[3 * b + 1], d.lam_Xg[3 * b + 2]};
    for (int k = d.csr_ptr[b]; k < d.csr_ptr[b + 1]; ++k)
        for (int a = 0; a < 3; ++a) g[a] += d.face_F[3 * (int64_t)k + a];
    for (int a = 0; a < 3; ++a) d.lam_X[3 * b + a] += g[a];
}

// sum of the per-node G and theta parts in a fixed order
__global__ __launch_bounds__(1024) void k_adj_node_grads(Dev d, int n_nodes) {
    __shared__ double sh[2][1024];
    double g0 = 0.0, g1 = 0.0;
    for (int b = threadIdx.x; b < n_nodes; b += 1024) {
        g0 += d.node_g[2 * b];
        g1 += d.node_g[2 * b + 1];
    }
    sh[0][threadIdx.x] = g0;
    sh[1][threadIdx.x] = g1;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        d.grads[2] += sh[0][0];
        d.grads[0] += sh[1][0];
    }
}

__global__ __launch_bounds__(256) void k_debug_bins(Lattice L, Dev d, int n_nodes) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_nodes) return;
    const NodePos p = node_pos(d, b);
    d.dbg_bins[4 * b + 0] = bin_of(L, wrapi(p.fl[0], L.nx), wrapi(p.fl[1], L.ny), wrapi(p.fl[2], L.nz));
    d.dbg_bins[4 * b + 1] = p.fl[0] - 1;
    d.dbg_bins[4 * b + 2] = p.fl[1] - 1;
    d.dbg_bins[4 * b + 3] = p.fl[2] - 1;
}

}  // namespace

void launch_clear_tiles(const Lattice& L, Dev& d, int pp, int pc, int n_caps, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_tiles, dim3(CLEAR_GRID), dim3(256), 0, s, L, d, pp, pc, n_caps);
}
void launch_advect_clear(const Lattice& L, Dev& d, int n_nodes, int pp, int pc, int n_caps, hipStream_t s) {
    const int n_ib = (n_nodes + 15) / 16;
    hipLaunchKernelGGL(k_advect_clear, dim3(n_ib + CLEAR_GRID), dim3(256), 0, s, L, d, n_nodes, n_ib, pp, pc, n_caps);
}
void launch_cap_volume(const Dev& d, int n_faces, int n_caps, hipStream_t s) {
    if (n_faces <= 0) return;
    if (d.det)
        hipLaunchKernelGGL(k_cap_volume_det, dim3(n_caps), dim3(256), 0, s, d);
    else
        hipLaunchKernelGGL(k_cap_volume, dim3((n_faces + 255) / 256), dim3(256), 0, s, d, n_faces);
}
void launch_faces(const Dev& d, int n_faces, hipStream_t s) {
    if (n_faces > 0) hipLaunchKernelGGL(k_faces, dim3((n_faces + 255) / 256), dim3(256), 0, s, d, n_faces);
}
void launch_node_gather(const Lattice& L, const Dev& d, int n_nodes, int par, hipStream_t s) {
    if (n_nodes > 0) hipLaunchKernelGGL(k_node_gather, dim3((n_nodes + 15) / 16), dim3(256), 0, s, L, d, n_nodes, par);
}

void launch_bin_scan(const Dev& d, int n_nodes, int par, hipStream_t s) {
    if (n_nodes > 0) hipLaunchKernelGGL(k_bin_alloc, dim3((n_nodes + 255) / 256), dim3(256), 0, s, d, par);
}
void launch_bin_scatter(const Lattice& L, const Dev& d, int n_nodes, int par, hipStream_t s) {
    if (n_nodes <= 0) return;
    hipLaunchKernelGGL(k_bin_scatter, dim3((n_nodes + 255) / 256), dim3(256), 0, s, L, d, n_nodes, par);
    if (d.det) {
        hipLaunchKernelGGL(k_bin_rank_det, dim3((n_nodes + 255) / 256), dim3(256), 0, s, d, n_nodes);
        hipLaunchKernelGGL(k_bin_place_det, dim3((n_nodes + 255) / 256), dim3(256), 0, s, d, n_nodes);
    }
}
void launch_repulse(const Lattice& L, const Dev& d, int n_nodes, float eps, float d0, hipStream_t s) {
    if (n_nodes > 0)
        hipLaunchKernelGGL(k_repulse, dim3((n_nodes + 256 / REP_LANES - 1) / (256 / REP_LANES)), dim3(256), 0, s, L, d,
                           n_nodes, eps, d0);
}
void launch_adj_repulse(const Lattice& L, const Dev& d, int n_nodes, float eps, float d0, hipStream_t s) {
    if (n_nodes > 0)
        hipLaunchKernelGGL(k_adj_repulse, dim3((n_nodes + 255) / 256), dim3(256), 0, s, L, d, n_nodes, eps, d0);
}
void launch_bending(const Dev& d, int n_nodes, hipStream_t s) {
    if (n_nodes <= 0) return;
    const dim3 g((n_nodes + 255) / 256);
    hipLaunchKernelGGL(k_bend_geo, g, dim3(256), 0, s, d, n_nodes);
    hipLaunchKernelGGL(k_bend_force, g, dim3(256), 0, s, d, n_nodes);
}
void launch_reference_step(const Dev& d, int n_nodes, int n_faces, int n_caps, bool bend, float gamma, float w,
                           double z_interface, float mu, hipStream_t s) {
    if (n_faces <= 0) return;
    hipLaunchKernelGGL(k_ref_zero_volume, dim3((n_caps + 255) / 256), dim3(256), 0, s, d, n_caps);
    launch_cap_volume(d, n_faces, n_caps, s);
    launch_faces(d, n_faces, s);
    hipLaunchKernelGGL(k_ref_tension, dim3((n_faces + 255) / 256), dim3(256), 0, s, d, n_faces, gamma, w, z_interface);
    hipLaunchKernelGGL(k_ref_gather, dim3((n_nodes + 255) / 256), dim3(256), 0, s, d, n_nodes);
    if (bend) launch_bending(d, n_nodes, s);
    hipLaunchKernelGGL(k_ref_advance, dim3((n_nodes + 255) / 256), dim3(256), 0, s, d, n_nodes, mu);
}
void launch_gather_forces(const Dev& d, int n_nodes, hipStream_t s) {
    if (n_nodes > 0) hipLaunchKernelGGL(k_ref_gather, dim3((n_nodes + 255) / 256), dim3(256), 0, s, d, n_nodes);
}
void launch_spread(const Lattice& L, const Dev& d, int par, const float* rho_n, const float* cs, hipStream_t s) {
    if (L.psi_exp)
        hipLaunchKernelGGL(k_spread<true>, dim3(SPREAD_GRID), dim3(256), 0, s, L, d, par, rho_n, cs);
    else
        hipLaunchKernelGGL(k_spread<false>, dim3(SPREAD_GRID), dim3(256), 0, s, L, d, par, rho_n, cs);
    if (d.det) hipLaunchKernelGGL(k_spread_gather_det, dim3(SPREAD_GRID), dim3(256), 0, s, L, d, par);
}
void launch_interp_advect(const Lattice& L, const Dev& d, int n_nodes, hipStream_t s) {
    if (n_nodes > 0)
        hipLaunchKernelGGL(k_interp_advect, dim3((n_nodes + 15) / 16), dim3(256), 0, s, L, d, n_nodes);
}
void launch_cap_moments(const Dev& d, int n_caps, hipStream_t s) {
    if (n_caps > 0) hipLaunchKernelGGL(k_cap_moments, dim3(n_caps), dim3(256), 0, s, d);
}
void launch_spread_vec(const Lattice& L, const Dev& d, int par, const float* val, float* target, int mode,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_spread_vec, dim3(SPREAD_GRID), dim3(256), 0, s, L, d, par, val, target, mode);
}
void launch_adj_nodes(const Lattice& L, const Dev& d, const float* rho_n, int n_nodes, hipStream_t s) {
    if (n_nodes > 0)
        hipLaunchKernelGGL(k_adj_nodes, dim3((n_nodes + 3) / 4), dim3(256), 0, s, L, d, rho_n, n_nodes);
}
void launch_adj_membrane(const Dev& d, int n_nodes, int n_faces, hipStream_t s) {
    if (n_faces <= 0) return;
    const dim3 gf((n_faces + 255) / 256);
    hipLaunchKernelGGL(k_adj_capdV, gf, dim3(256), 0, s, d, n_faces);
    hipLaunchKernelGGL(k_adj_faces, gf, dim3(256), 0, s, d, n_faces);
    hipLaunchKernelGGL(k_adj_node_update, dim3((n_nodes + 255) / 256), dim3(256), 0, s, d, n_nodes);
    hipLaunchKernelGGL(k_adj_node_grads, dim3(1), dim3(1024), 0, s, d, n_nodes);
}
void launch_debug_bins(const Lattice& L, const Dev& d, int n_nodes, hipStream_t s) {
    if (n_nodes > 0)
        hipLaunchKernelGGL(k_debug_bins, dim3((n_nodes + 255) / 256), dim3(256), 0, s, L, d, n_nodes);
}

}  // namespace lbmx
