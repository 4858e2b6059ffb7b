// Lattice kernels of the two-component Shan-Chen D3Q19 BGK step (gfx950).
//
// Storage: structure of arrays f[c][i][z][y][x], x fastest, holding the
// post-collision populations f* of the previous step.  Streaming is a pull:
// the population i of node x at the new time level is f*_i(x - c_i), read
// at the point of use, so every load and store of a wavefront (64 nodes
// along x) touches consecutive addresses.
//
// The Shan-Chen force (Sec. II.D, eq. method:shanchen) needs the density
// of the new time level at the 18 neighbours, which the pull cannot give a
// node by itself, so a step is two passes over the lattice:
//   k_density  rho^n(x) = sum_i f*_i(x - c_i)                (Sec. II.A)
//   k_collide  pull, Shan-Chen + wettability + immersed-boundary force,
//              equilibrium-velocity shift, BGK (Sec. II.A), store f*.
// k_collide marches a 64 x 4 column of nodes up z and keeps three planes of
// psi + phi (pseudo-potential plus virtual density) for the column and its
// one-node halo in LDS, so the 36 neighbour reads per node come from LDS.
#include "lbm_internal.h"

namespace lbmx {

namespace {

__device__ __forceinline__ int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// source of the pull for direction i at (x, y, z): x - c_i, with the
// neighbour coordinates precomputed (xm = x-1, xp = x+1 wrapped, ...).
template <int I>
__device__ __forceinline__ int64_t pull_index(int x, int xm, int xp, int y, int ym, int yp,
                                              int z, int zm, int zp, int nx, int ny) {
    const int sx = cx(I) == 1 ? xm : (cx(I) == -1 ? xp : x);
    const int sy = cy(I) == 1 ? ym : (cy(I) == -1 ? yp : y);
    const int sz = cz(I) == 1 ? zm : (cz(I) == -1 ? zp : z);
    return ((int64_t)sz * ny + sy) * nx + sx;
}

// Moving-wall half-way bounce-back (Sec. II.C, eq. method:SBB): the
// population entering a fluid node from a solid row is the node's own
// opposite post-collision population plus 2 w_i rho (c_i . u_w) / c_s^2.
template <int I>
__device__ __forceinline__ float wall_term(const Lattice& L, float rho_prev_node) {
    const float* uw = cy(I) == 1 ? L.uw_lo : L.uw_hi;
    const float cu = cx(I) * uw[0] + cy(I) * uw[1] + cz(I) * uw[2];
    return 2.0f * wgt(I) * rho_prev_node * cu * 3.0f;
}

struct Pulled {
    float f[Q];
};

template <bool WALLS, int I>
__device__ __forceinline__ void pull_one(const float* __restrict__ fc, const Lattice& L, int64_t node,
                                         int x, int xm, int xp, int y, int ym, int yp, int z, int zm,
                                         int zp, float rp, Pulled& P) {
    if (WALLS && ((cy(I) == 1 && y == 1) || (cy(I) == -1 && y == L.ny - 2))) {
        P.f[I] = fc[(int64_t)opp(I) * L.n + node] + wall_term<I>(L, rp);
    } else {
        P.f[I] = fc[(int64_t)I * L.n + pull_index<I>(x, xm, xp, y, ym, yp, z, zm, zp, L.nx, L.ny)];
    }
}

template <bool WALLS, int... Is>
__device__ __forceinline__ void pull_all(const float* __restrict__ fc, const Lattice& L, int64_t node,
                                         int x, int xm, int xp, int y, int ym, int yp, int z, int zm,
                                         int zp, float rp, Pulled& P,
                                         std::integer_sequence<int, Is...>) {
    (pull_one<WALLS, Is>(fc, L, node, x, xm, xp, y, ym, yp, z, zm, zp, rp, P), ...);
}

template <bool WALLS>
__device__ __forceinline__ void pull(const float* __restrict__ fc, const Lattice& L, int64_t node,
                                     int x, int y, int z, float rp, Pulled& P) {
    const int xm = x == 0 ? L.nx - 1 : x - 1, xp = x == L.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? L.ny - 1 : y - 1, yp = y == L.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? L.nz - 1 : z - 1, zp = z == L.nz - 1 ? 0 : z + 1;
    pull_all<WALLS>(fc, L, node, x, xm, xp, y, ym, yp, z, zm, zp, rp, P,
                    std::make_integer_sequence<int, Q>{});
}

__device__ __forceinline__ float sum_pop(const Pulled& P) {
    // rest first, then opposite pairs
    float s = P.f[0];
#pragma unroll
    for (int k = 1; k < Q; k += 2) s += P.f[k] + P.f[k + 1];
    return s;
}

// j = sum_i f_i c_i, accumulated as differences of opposite pairs
__device__ __forceinline__ void momentum(const Pulled& P, float& jx, float& jy, float& jz) {
    jx = jy = jz = 0.0f;
#pragma unroll
    for (int k = 1; k < Q; k += 2) {
        const float d = P.f[k] - P.f[k + 1];
        if (cx(k) != 0) jx += cx(k) * d;
        if (cy(k) != 0) jy += cy(k) * d;
        if (cz(k) != 0) jz += cz(k) * d;
    }
}

__global__ __launch_bounds__(256) void k_init_rest(float* __restrict__ f, const float* __restrict__ rhoA,
                                                   const float* __restrict__ rhoB, int64_t n) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const float ra = rhoA[k], rb = rhoB[k];
        float resta = ra, restb = rb;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const float fa = wgt(i) * ra, fb = wgt(i) * rb;
            resta -= fa;
            restb -= fb;
            f[(int64_t)i * n + k] = fa;
            f[(int64_t)(Q + i) * n + k] = fb;
        }
        // rest populations close each node's mass
        f[k] = resta;
        f[(int64_t)Q * n + k] = restb;
    }
}

template <bool WALLS>
__global__ __launch_bounds__(256) void k_density(const float* __restrict__ fin,
                                                 const float* __restrict__ rho_prev,
                                                 float* __restrict__ rho_out, Lattice L) {
    const int x = blockIdx.x * BX + threadIdx.x;
    const int y = blockIdx.y * BY + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= L.nx || y >= L.ny) return;
    if (WALLS && (y == 0 || y == L.ny - 1)) return;
    const int64_t node = ((int64_t)z * L.ny + y) * L.nx + x;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        Pulled P;
        const float rp = WALLS ? rho_prev[c * L.n + node] : 0.0f;
        pull<WALLS>(fin + (int64_t)c * Q * L.n, L, node, x, y, z, rp, P);
        rho_out[c * L.n + node] = sum_pop(P);
    }
}

// Fused pull + force + collide.  MACRO: recompute the macroscopic fields of
// this collision without storing populations (field read-back).
template <bool WALLS, bool IBM, bool MACRO>
__global__ __launch_bounds__(256) void k_collide(const float* __restrict__ fin, float* __restrict__ fout,
                                                 const float* __restrict__ rho_n,
                                                 const float* __restrict__ rho_p,
                                                 const float* __restrict__ fib,
                                                 const int* __restrict__ tile_flag,
                                                 float* __restrict__ u_out,
                                                 float* __restrict__ rho_macro, Lattice L) {
    constexpr int SW = BX + 2, SH = BY + 2;
    __shared__ float sp[3][2][SH][SW];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * BX + tx;
    const int x0 = blockIdx.x * BX, y0 = blockIdx.y * BY, z0 = blockIdx.z * ZC;
    const int z1 = min(z0 + ZC, L.nz);
    const int64_t N = L.n;

    auto stage = [&](int zz) {
        const int slot = (zz - z0 + 1) % 3;
        const int zw = wrapi(zz, L.nz);
        for (int k = tid; k < 2 * SH * SW; k += BX * BY) {
            const int c = k / (SH * SW);
            const int r = k - c * SH * SW;
            const int ly = r / SW, lx = r - ly * SW;
            const int gx = wrapi(x0 - 1 + lx, L.nx);
            int gy = wrapi(y0 - 1 + ly, L.ny);
            if (WALLS) {
                // solid rows take the pseudo-potential of the adjacent fluid row
                if (gy == 0) gy = 1;
                if (gy == L.ny - 1) gy = L.ny - 2;
            }
            const int64_t idx = ((int64_t)zw * L.ny + gy) * L.nx + gx;
            float v = rho_n[c * N + idx];
            if (IBM) {
                const int t = ((zw >> 3) * L.nty + (gy >> 3)) * L.ntx + (gx >> 3);
                if (tile_flag[t]) v += fib[(3 + c) * N + idx];
            }
            sp[slot][c][ly][lx] = v;
        }
    };

    stage(z0 - 1);
    stage(z0);
    const int x = x0 + tx, y = y0 + ty;
    const bool active = x < L.nx && y < L.ny && (!WALLS || (y > 0 && y < L.ny - 1));
    for (int z = z0; z < z1; ++z) {
        stage(z + 1);
        __syncthreads();
        if (active) {
            const int64_t node = ((int64_t)z * L.ny + y) * L.nx + x;
            Pulled A, B;
            const float rpa = WALLS ? rho_p[node] : 0.0f;
            const float rpb = WALLS ? rho_p[N + node] : 0.0f;
            pull<WALLS>(fin, L, node, x, y, z, rpa, A);
            pull<WALLS>(fin + (int64_t)Q * N, L, node, x, y, z, rpb, B);
            const float ra = sum_pop(A), rb = sum_pop(B);
            float jax, jay, jaz, jbx, jby, jbz;
            momentum(A, jax, jay, jaz);
            momentum(B, jbx, jby, jbz);

            // neighbour sums S^c = sum_i w_i (psi^c + phi^c)(x + c_i) c_i
            float sa[3] = {0.f, 0.f, 0.f}, sb[3] = {0.f, 0.f, 0.f};
            const int s0 = (z - z0 + 1) % 3;
#pragma unroll
            for (int k = 1; k < Q; k += 2) {
                const int sp_ = (s0 + cz(k) + 3) % 3, sm_ = (s0 - cz(k) + 3) % 3;
                const int ly = ty + 1, lx = tx + 1;
                const float da = sp[sp_][0][ly + cy(k)][lx + cx(k)] - sp[sm_][0][ly - cy(k)][lx - cx(k)];
                const float db = sp[sp_][1][ly + cy(k)][lx + cx(k)] - sp[sm_][1][ly - cy(k)][lx - cx(k)];
                const float w = wgt(k);
                if (cx(k) != 0) { sa[0] += w * cx(k) * da; sb[0] += w * cx(k) * db; }
                if (cy(k) != 0) { sa[1] += w * cy(k) * da; sb[1] += w * cy(k) * db; }
                if (cz(k) != 0) { sa[2] += w * cz(k) * da; sb[2] += w * cz(k) * db; }
            }
            const float rsum = ra + rb;
            float Fa[3], Fb[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                Fa[d] = -L.G * ra * sb[d];
                Fb[d] = -L.G * rb * sa[d];
            }
            bool flagged = false;
            if (IBM) {
                const int t = ((z >> 3) * L.nty + (y >> 3)) * L.ntx + (x >> 3);
                flagged = tile_flag[t] != 0;
                if (flagged) {
                    // immersed-boundary force shared by mass fraction
                    const float fa = ra / rsum, fb = rb / rsum;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const float Fi = fib[d * N + node];
                        Fa[d] += fa * Fi;
                        Fb[d] += fb * Fi;
                    }
                }
            }
            // common velocity u' and the shifted equilibrium velocities
            const float wa = L.omega[0], wb = L.omega[1];
            const float den = 1.0f / (ra * wa + rb * wb);
            const float upx = (jax * wa + jbx * wb) * den;
            const float upy = (jay * wa + jby * wb) * den;
            const float upz = (jaz * wa + jbz * wb) * den;
            if (MACRO || (IBM && flagged)) {
                const float ir = 1.0f / rsum;
                u_out[node] = (jax + jbx + 0.5f * (Fa[0] + Fb[0])) * ir;
                u_out[N + node] = (jay + jby + 0.5f * (Fa[1] + Fb[1])) * ir;
                u_out[2 * N + node] = (jaz + jbz + 0.5f * (Fa[2] + Fb[2])) * ir;
            }
            if (!MACRO) {
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const Pulled& P = c == 0 ? A : B;
                    const float r = c == 0 ? ra : rb;
                    const float* F = c == 0 ? Fa : Fb;
                    const float om = L.omega[c];
                    const float ts = L.tau[c] / r;
                    const float ux = upx + ts * F[0], uy = upy + ts * F[1], uz = upz + ts * F[2];
                    const float base = r * (1.0f - 1.5f * (ux * ux + uy * uy + uz * uz));
                    float* fo = fout + (int64_t)c * Q * N + node;
                    float rest = r;
#pragma unroll
                    for (int i = 1; i < Q; ++i) {
                        const float cu = cx(i) * ux + cy(i) * uy + cz(i) * uz;
                        const float feq = wgt(i) * (base + r * cu * (3.0f + 4.5f * cu));
                        const float fs = P.f[i] + om * (feq - P.f[i]);
                        rest -= fs;
                        fo[(int64_t)i * N] = fs;
                    }
                    // rest population closes the node's mass exactly
                    fo[0] = rest;
                }
            }
        } else if (MACRO && x < L.nx && y < L.ny) {
            const int64_t node = ((int64_t)z * L.ny + y) * L.nx + x;
            u_out[node] = u_out[N + node] = u_out[2 * N + node] = 0.f;
        }
        __syncthreads();
    }
}

// FP64 mass and momentum of the post-collision state over fluid nodes:
// per-block partial sums [mass A, mass B, px, py, pz].
__global__ __launch_bounds__(256) void k_reduce_fluid(const float* __restrict__ f, double* __restrict__ partial,
                                                      Lattice L) {
    __shared__ double sh[5][256];
    double acc[5] = {0, 0, 0, 0, 0};
    const int64_t plane = (int64_t)L.nx * L.ny;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < L.n;
         k += (int64_t)gridDim.x * blockDim.x) {
        if (L.walls) {
            const int y = (int)((k % plane) / L.nx);
            if (y == 0 || y == L.ny - 1) continue;
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const float* fc = f + (int64_t)c * Q * L.n + k;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const double v = fc[(int64_t)i * L.n];
                acc[c] += v;
                if (cx(i)) acc[2] += cx(i) * v;
                if (cy(i)) acc[3] += cy(i) * v;
                if (cz(i)) acc[4] += cz(i) * v;
            }
        }
    }
    for (int j = 0; j < 5; ++j) sh[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int j = 0; j < 5; ++j) sh[j][threadIdx.x] += sh[j][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int j = 0; j < 5; ++j) partial[blockIdx.x * 8 + j] = sh[j][0];
}

}  // namespace

void launch_init_rest(const Lattice& L, float* f, const float* rhoA, const float* rhoB, hipStream_t s) {
    const int64_t blocks = std::min<int64_t>((L.n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_init_rest, dim3((unsigned)blocks), dim3(256), 0, s, f, rhoA, rhoB, L.n);
}

void launch_density(const Lattice& L, const float* fin, const float* rho_prev, float* rho_out,
                    hipStream_t s) {
    dim3 grid((L.nx + BX - 1) / BX, (L.ny + BY - 1) / BY, L.nz);
    dim3 block(BX, BY);
    if (L.walls)
        hipLaunchKernelGGL(k_density<true>, grid, block, 0, s, fin, rho_prev, rho_out, L);
    else
        hipLaunchKernelGGL(k_density<false>, grid, block, 0, s, fin, rho_prev, rho_out, L);
}

template <bool W, bool I, bool M>
static void launch_collide_t(const Lattice& L, const float* fin, float* fout, const float* rho_n,
                             const float* rho_prev, const float* fib, const int* tile_flag, float* u,
                             float* rho_macro, hipStream_t s) {
    dim3 grid((L.nx + BX - 1) / BX, (L.ny + BY - 1) / BY, (L.nz + ZC - 1) / ZC);
    dim3 block(BX, BY);
    hipLaunchKernelGGL((k_collide<W, I, M>), grid, block, 0, s, fin, fout, rho_n, rho_prev, fib, tile_flag,
                       u, rho_macro, L);
}

void launch_collide(const Lattice& L, const float* fin, float* fout, const float* rho_n,
                    const float* rho_prev, const float* fib, const int* tile_flag, float* u,
                    float* rho_macro, bool has_ibm, bool macro, hipStream_t s) {
    const bool w = L.walls != 0;
#define LC(W, I, M) launch_collide_t<W, I, M>(L, fin, fout, rho_n, rho_prev, fib, tile_flag, u, rho_macro, s)
    if (macro) {
        if (w) { if (has_ibm) LC(true, true, true); else LC(true, false, true); }
        else { if (has_ibm) LC(false, true, true); else LC(false, false, true); }
    } else {
        if (w) { if (has_ibm) LC(true, true, false); else LC(true, false, false); }
        else { if (has_ibm) LC(false, true, false); else LC(false, false, false); }
    }
#undef LC
}

void launch_reduce_fluid(const Lattice& L, const float* fpost, double* partial, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_fluid, dim3(RED_BLOCKS), dim3(256), 0, s, fpost, partial, L);
}

}  // namespace lbmx
