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
//   k_nodes         one wavefront per node: gather its triangles' corner
//                   forces, add the wettability reaction (64 lanes = the
//                   4x4x4 delta stencil, psi staged on a 6^3 LDS cube),
//                   count the node into its home bin (4^3), mark the 8^3
//                   tiles its stencil touches
//   k_bin_scan      exclusive scan of the home-tile counts
//   k_bin_scatter   counting-sort scatter of node ids into tile bins
//   k_spread        one workgroup per occupied bin: accumulate F_b delta and
//                   the virtual density in a 7^3 LDS box (LDS atomics,
//                   one lane per stencil point), then flush non-zero cells
//                   to HBM with global atomics
//   k_interp_advect one wavefront per node: U_b = sum u delta, X += U_b
#include "lbm_internal.h"

namespace lbmx {

namespace {

constexpr int CNT_TOUCHED = 0;   // counters[0..1]
constexpr int CNT_HOME = 2;      // counters[2..3]

__device__ __forceinline__ int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Peskin 4-point kernel
__device__ __forceinline__ float peskin(float r) {
    const float a = fabsf(r);
    if (a <= 1.0f) return (3.0f - 2.0f * a + sqrtf(1.0f + 4.0f * a - 4.0f * a * a)) * 0.125f;
    if (a <= 2.0f) return (5.0f - 2.0f * a - sqrtf(-7.0f + 12.0f * a - 4.0f * a * a)) * 0.125f;
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
    const CapDev& C = d.caps[d.node_cap[b]];
    NodePos p;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float o = d.off_hi[3 * b + k];
        const float fo = floorf(o);
        p.fl[k] = C.anchor[k] + (int)fo;
        p.r[k] = o - fo;
    }
    return p;
}

__device__ __forceinline__ int tile_of(const Lattice& L, int x, int y, int z) {
    return ((z >> 3) * L.nty + (y >> 3)) * L.ntx + (x >> 3);
}

__device__ __forceinline__ int bin_of(const Lattice& L, int x, int y, int z) {
    return ((z / BIN) * L.nby + (y / BIN)) * L.nbx + (x / BIN);
}

__global__ __launch_bounds__(256) void k_clear_tiles(Lattice L, Dev d, int pp, int pc, int n_caps) {
    const int nt = d.counters[CNT_TOUCHED + pp];
    const int nh = d.counters[CNT_HOME + pp];
    const int64_t N = L.n;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < (int64_t)nt * 512;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int e = (int)(k >> 9), c = (int)(k & 511);
        const int t = d.touched[pp][e];
        const int tx = t % L.ntx, ty = (t / L.ntx) % L.nty, tz = t / (L.ntx * L.nty);
        const int x = tx * TILE + (c & 7), y = ty * TILE + ((c >> 3) & 7), z = tz * TILE + (c >> 6);
        if (x < L.nx && y < L.ny && z < L.nz) {
            const int64_t node = ((int64_t)z * L.ny + y) * L.nx + x;
#pragma unroll
            for (int f = 0; f < 5; ++f) d.fib[f * N + node] = 0.0f;
        }
        if (c == 0) d.tile_flag[t] = 0;
    }
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nh;
         k += (int64_t)gridDim.x * blockDim.x)
        d.tile_count[d.home[pp][k]] = 0;
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            d.counters[CNT_TOUCHED + pc] = 0;
            d.counters[CNT_HOME + pc] = 0;
        }
        for (int k = threadIdx.x; k < n_caps; k += blockDim.x) d.capV[k] = 0.0;
    }
}

// FP64 enclosed volume per capsule, V = (1/6) sum_T X1 . (X2 x X3) over
// anchor-relative offsets: one thread per triangle, a block reduction when
// the block's triangles belong to one capsule, FP64 atomics otherwise.
__global__ __launch_bounds__(256) void k_cap_volume(Dev d, int n_faces) {
    __shared__ double sh[256];
    __shared__ int cap_first, cap_last;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    const int f_last = min((int)(blockIdx.x * blockDim.x + blockDim.x), n_faces) - 1;
    double v = 0.0;
    int cap = -1;
    if (f < n_faces) {
        cap = d.face_cap[f];
        double X[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int b = d.tri[3 * f + k];
#pragma unroll
            for (int j = 0; j < 3; ++j) X[k][j] = (double)d.off_hi[3 * b + j];
        }
        v = (X[0][0] * (X[1][1] * X[2][2] - X[1][2] * X[2][1])
           + X[0][1] * (X[1][2] * X[2][0] - X[1][0] * X[2][2])
           + X[0][2] * (X[1][0] * X[2][1] - X[1][1] * X[2][0])) / 6.0;
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

__device__ __forceinline__ void cross3(const float* a, const float* b, float* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

// Skalak energy per triangle, E_T = A0 (kS/4)(I1^2 + 2 I1 - 2 I2 + C I2^2),
// I1 = tr(M0^-1 M) - 2, I2 = det M / det M0 - 1, with its analytic
// gradient; and the volume penalty gradient kV (V - V0)/V0 dV/dX.
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
    const FaceRef R = d.fref[f];
    float e1[3], e2[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        e1[j] = X[1][j] - X[0][j];
        e2[j] = X[2][j] - X[0][j];
    }
    const float m11 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
    const float m12 = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
    const float m22 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
    const float I1 = R.q11 * m11 + 2.0f * R.q12 * m12 + R.q22 * m22 - 2.0f;
    const float I2 = (m11 * m22 - m12 * m12) * R.inv_det0 - 1.0f;
    const float W1 = 0.25f * C.kS * (2.0f * I1 + 2.0f);
    const float W2 = 0.25f * C.kS * (2.0f * C.C * I2 - 2.0f) * R.inv_det0;
    float g1[3], g2[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        // d tr/d e1 = 2 (q11 e1 + q12 e2), d det/d e1 = 2 (m22 e1 - m12 e2)
        g1[j] = R.A0 * (W1 * 2.0f * (R.q11 * e1[j] + R.q12 * e2[j]) + W2 * 2.0f * (m22 * e1[j] - m12 * e2[j]));
        g2[j] = R.A0 * (W1 * 2.0f * (R.q12 * e1[j] + R.q22 * e2[j]) + W2 * 2.0f * (m11 * e2[j] - m12 * e1[j]));
    }
    float F[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        F[0][j] = g1[j] + g2[j];
        F[1][j] = -g1[j];
        F[2][j] = -g2[j];
    }
    if (C.kV != 0.0f) {
        const float lam = -(float)((double)C.kV * (d.capV[cap] - C.V0) / C.V0) * (1.0f / 6.0f);
        float c0[3], c1[3], c2[3];
        cross3(X[1], X[2], c0);
        cross3(X[2], X[0], c1);
        cross3(X[0], X[1], c2);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            F[0][j] += lam * c0[j];
            F[1][j] += lam * c1[j];
            F[2][j] += lam * c2[j];
        }
    }
    float* o = d.face_F + 9 * (int64_t)f;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) o[3 * k + j] = F[k][j];
}

__global__ __launch_bounds__(256) void k_nodes(Lattice L, Dev d, const float* __restrict__ rho_n,
                                               const float* __restrict__ cs, int n_nodes, int par) {
    constexpr int CB = 6;                       // psi cube edge: stencil plus one-node halo
    __shared__ float cube[4][CB * CB * CB];
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= n_nodes) return;                   // whole wavefront; no block barrier below
    float* cb = cube[threadIdx.x >> 6];
    // corner forces of the incident triangles
    float gx = 0.f, gy = 0.f, gz = 0.f;
    const int beg = d.csr_ptr[b], end = d.csr_ptr[b + 1];
    for (int k = beg + lane; k < end; k += 64) {
        const int e = d.csr_idx[k];
        gx += d.face_F[3 * (int64_t)e + 0];
        gy += d.face_F[3 * (int64_t)e + 1];
        gz += d.face_F[3 * (int64_t)e + 2];
    }
    const NodePos p = node_pos(d, b);
    const float wet = d.node_wet[b];
    if (wet != 0.0f) {
        // reaction of the virtual density on the node:
        // -G |rho_v| A_b sum_y delta(y - X_b) sum_i w_i psi^np(y + c_i) c_i
        const int np = 1 - d.caps[d.node_cap[b]].pref;
        const float* rc = rho_n + (int64_t)np * L.n;
        const float sc = cs ? cs[np] : 1.0f;      // FP16 form: mass compensation of this step
        // the wavefront stages psi^np on the 6^3 cube floor(X)-2 .. floor(X)+3
        for (int j = lane; j < CB * CB * CB; j += 64) {
            const int qz = j / (CB * CB), qy = (j / CB) % CB, qx = j % CB;
            int gy = wrapi(p.fl[1] - 2 + qy, L.ny);
            if (L.walls) gy = gy == 0 ? 1 : (gy == L.ny - 1 ? L.ny - 2 : gy);
            cb[j] = sc * rc[((int64_t)wrapi(p.fl[2] - 2 + qz, L.nz) * L.ny + gy) * L.nx + wrapi(p.fl[0] - 2 + qx, L.nx)];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int kx = lane & 3, ky = (lane >> 2) & 3, kz = lane >> 4;
        const float w = peskin(p.r[0] + 1.0f - kx) * peskin(p.r[1] + 1.0f - ky) * peskin(p.r[2] + 1.0f - kz);
        const int c0 = ((kz + 1) * CB + (ky + 1)) * CB + (kx + 1);
        float S[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int k = 1; k < Q; k += 2) {
            const int o = (cz(k) * CB + cy(k)) * CB + cx(k);
            const float va = cb[c0 + o];
            const float vb = cb[c0 - o];
            const float dd = wgt(k) * (va - vb);
            if (cx(k)) S[0] += cx(k) * dd;
            if (cy(k)) S[1] += cy(k) * dd;
            if (cz(k)) S[2] += cz(k) * dd;
        }
        const float s = -L.G * wet * w;
        gx += s * S[0];
        gy += s * S[1];
        gz += s * S[2];
    }
    gx = wave_sum(gx);
    gy = wave_sum(gy);
    gz = wave_sum(gz);
    if (lane == 0) {
        d.node_F[3 * b + 0] = gx;
        d.node_F[3 * b + 1] = gy;
        d.node_F[3 * b + 2] = gz;
    } else if (lane == 1) {
        const int wx = wrapi(p.fl[0], L.nx), wy = wrapi(p.fl[1], L.ny), wz = wrapi(p.fl[2], L.nz);
        const int t = bin_of(L, wx, wy, wz);
        const int rank = atomicAdd(&d.tile_count[t], 1);
        d.node_tile[b] = t;
        d.node_rank[b] = rank;
        if (rank == 0) d.home[par][atomicAdd(&d.counters[CNT_HOME + par], 1)] = t;
    } else if (lane >= 8 && lane < 16) {
        // tiles touched by the stencil floor(X)-1 .. floor(X)+2: at most two
        // per axis; lane 8 + (i, j, k) takes one combination
        const int sel[3] = {(lane - 8) & 1, ((lane - 8) >> 1) & 1, ((lane - 8) >> 2) & 1};
        const int nn[3] = {L.nx, L.ny, L.nz};
        int tt[3];
        bool ok = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int t0 = wrapi(p.fl[a] - 1, nn[a]) >> 3;
            int t1 = -1;
            for (int k = 1; k < 4; ++k) {
                const int tk = wrapi(p.fl[a] - 1 + k, nn[a]) >> 3;
                if (tk != t0) t1 = tk;
            }
            tt[a] = sel[a] ? t1 : t0;
            ok = ok && tt[a] >= 0;
        }
        if (ok) {
            const int t2 = (tt[2] * L.nty + tt[1]) * L.ntx + tt[0];
            if (atomicExch(&d.tile_flag[t2], 1) == 0)
                d.touched[par][atomicAdd(&d.counters[CNT_TOUCHED + par], 1)] = t2;
        }
    }
}

__global__ __launch_bounds__(1024) void k_bin_scan(Dev d, int par) {
    __shared__ int sh[1024];
    const int nh = d.counters[CNT_HOME + par];
    int carry = 0;
    for (int base = 0; base < nh; base += 1024) {
        const int k = base + (int)threadIdx.x;
        const int v = k < nh ? d.tile_count[d.home[par][k]] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int add = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (k < nh) {
            const int start = carry + sh[threadIdx.x] - v;
            d.home_start[k] = start;
            d.tile_offset[d.home[par][k]] = start;
        }
        carry += sh[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_bin_scatter(Dev d, int n_nodes) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_nodes) return;
    d.sorted[d.tile_offset[d.node_tile[b]] + d.node_rank[b]] = b;
}

constexpr int SPREAD_GRID = 2048;

__global__ __launch_bounds__(256) void k_spread(Lattice L, Dev d, int par) {
    constexpr int B3 = BOX * BOX * BOX;
    __shared__ float box[5][B3];
    const int nh = d.counters[CNT_HOME + par];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kx = lane & 3, ky = (lane >> 2) & 3, kz = lane >> 4;
    const int64_t N = L.n;
    for (int e = blockIdx.x; e < nh; e += gridDim.x) {
        const int t = d.home[par][e];
        const int start = d.home_start[e], cnt = d.tile_count[t];
        const int ox = (t % L.nbx) * BIN, oy = ((t / L.nbx) % L.nby) * BIN, oz = (t / (L.nbx * L.nby)) * BIN;
        for (int k = threadIdx.x; k < 5 * B3; k += 256) (&box[0][0])[k] = 0.0f;
        __syncthreads();
        for (int j = wave; j < cnt; j += 4) {
            const int b = d.sorted[start + j];
            const NodePos p = node_pos(d, b);
            const float w = peskin(p.r[0] + 1.0f - kx) * peskin(p.r[1] + 1.0f - ky) * peskin(p.r[2] + 1.0f - kz);
            const int ix = wrapi(p.fl[0], L.nx) - ox + kx;
            const int iy = wrapi(p.fl[1], L.ny) - oy + ky;
            const int iz = wrapi(p.fl[2], L.nz) - oz + kz;
            const int cell = (iz * BOX + iy) * BOX + ix;
            atomicAdd(&box[0][cell], w * d.node_F[3 * b + 0]);
            atomicAdd(&box[1][cell], w * d.node_F[3 * b + 1]);
            atomicAdd(&box[2][cell], w * d.node_F[3 * b + 2]);
            const float wet = d.node_wet[b];
            if (wet != 0.0f) atomicAdd(&box[3 + d.caps[d.node_cap[b]].pref][cell], w * wet);
        }
        __syncthreads();
        for (int k = threadIdx.x; k < 5 * B3; k += 256) {
            const float v = (&box[0][0])[k];
            if (v != 0.0f) {
                const int f = k / B3, cell = k - f * B3;
                const int iz = cell / (BOX * BOX), iy = (cell / BOX) % BOX, ix = cell % BOX;
                const int gx = wrapi(ox - 1 + ix, L.nx), gy = wrapi(oy - 1 + iy, L.ny), gz = wrapi(oz - 1 + iz, L.nz);
                unsafeAtomicAdd(&d.fib[f * N + ((int64_t)gz * L.ny + gy) * L.nx + gx], v);
            }
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_interp_advect(Lattice L, Dev d, int n_nodes) {
    const int lane = threadIdx.x & 63;
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= n_nodes) return;
    const NodePos p = node_pos(d, b);
    const int kx = lane & 3, ky = (lane >> 2) & 3, kz = lane >> 4;
    const float w = peskin(p.r[0] + 1.0f - kx) * peskin(p.r[1] + 1.0f - ky) * peskin(p.r[2] + 1.0f - kz);
    const int64_t node = ((int64_t)wrapi(p.fl[2] - 1 + kz, L.nz) * L.ny + wrapi(p.fl[1] - 1 + ky, L.ny)) * L.nx
                       + wrapi(p.fl[0] - 1 + kx, L.nx);
    const float ux = wave_sum(w * d.u[node]);
    const float uy = wave_sum(w * d.u[L.n + node]);
    const float uz = wave_sum(w * d.u[2 * L.n + node]);
    if (lane == 0) {
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
    hipLaunchKernelGGL(k_clear_tiles, dim3(1024), dim3(256), 0, s, L, d, pp, pc, n_caps);
}
void launch_cap_volume(const Dev& d, int n_faces, hipStream_t s) {
    if (n_faces > 0) hipLaunchKernelGGL(k_cap_volume, dim3((n_faces + 255) / 256), dim3(256), 0, s, d, n_faces);
}
void launch_faces(const Dev& d, int n_faces, hipStream_t s) {
    if (n_faces > 0) hipLaunchKernelGGL(k_faces, dim3((n_faces + 255) / 256), dim3(256), 0, s, d, n_faces);
}
void launch_nodes(const Lattice& L, const Dev& d, const float* rho_n, const float* cs, int n_nodes, int par,
                  hipStream_t s) {
    if (n_nodes > 0)
        hipLaunchKernelGGL(k_nodes, dim3((n_nodes + 3) / 4), dim3(256), 0, s, L, d, rho_n, cs, n_nodes, par);
}
void launch_bin_scan(const Dev& d, int par, hipStream_t s) {
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, s, d, par);
}
void launch_bin_scatter(const Dev& d, int n_nodes, hipStream_t s) {
    if (n_nodes > 0) hipLaunchKernelGGL(k_bin_scatter, dim3((n_nodes + 255) / 256), dim3(256), 0, s, d, n_nodes);
}
void launch_spread(const Lattice& L, const Dev& d, int par, hipStream_t s) {
    hipLaunchKernelGGL(k_spread, dim3(SPREAD_GRID), dim3(256), 0, s, L, d, par);
}
void launch_interp_advect(const Lattice& L, const Dev& d, int n_nodes, hipStream_t s) {
    if (n_nodes > 0)
        hipLaunchKernelGGL(k_interp_advect, dim3((n_nodes + 3) / 4), dim3(256), 0, s, L, d, n_nodes);
}
void launch_cap_moments(const Dev& d, int n_caps, hipStream_t s) {
    if (n_caps > 0) hipLaunchKernelGGL(k_cap_moments, dim3(n_caps), dim3(256), 0, s, d);
}
void launch_debug_bins(const Lattice& L, const Dev& d, int n_nodes, hipStream_t s) {
    if (n_nodes > 0)
        hipLaunchKernelGGL(k_debug_bins, dim3((n_nodes + 255) / 256), dim3(256), 0, s, L, d, n_nodes);
}

}  // namespace lbmx
