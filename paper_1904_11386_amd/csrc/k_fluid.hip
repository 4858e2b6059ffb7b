// Lattice kernels of the two-component Shan-Chen D3Q19 BGK step (gfx950).
//
// Storage: f[i][z][y][x][c], x fastest with the two components c side by
// side (one vector per direction and node), holding the
// post-collision populations f* of the previous step.  Streaming is a pull:
// the population i of node x at the new time level is f*_i(x - c_i), read
// at the point of use, so every load and store of a wavefront (64 nodes
// along x) touches consecutive addresses.
//
// Two storage forms share the kernels (template HALF):
//   FP32   f_i itself;
//   FP16   g_i = f_i / rho_enc - w_i in binary16, rho_enc the density of the
//          node that wrote it (after the FP64 mass compensation of that
//          step).  Decoding needs rho_enc of the source node of each pull,
//          which the kernels stage in LDS next to psi.  Arithmetic is FP32.
//
// The Shan-Chen force (Sec. II.D, eq. method:shanchen) needs the density
// of the new time level at the 18 neighbours, which the pull cannot give a
// node by itself, so a step is two passes over the lattice:
//   k_density  rho^n(x) = sum_i f*_i(x - c_i)                (Sec. II.A)
//   k_collide  pull, Shan-Chen + wettability + immersed-boundary force,
//              equilibrium-velocity shift, BGK (Sec. II.A), store f*;
// or, in FP32 on periodic lattices, one: k_collide_one forms the densities
// of its block and a one-node halo from the populations it pulls (the
// same sums), and k_density_tiles gives the immersed boundary's tiles
// theirs for the wettability reaction that precedes the collide.
// k_collide marches a BX x BY column of nodes up z and keeps three planes
// of psi + phi (pseudo-potential plus virtual density) for the column and
// its one-node halo in LDS, so the 36 neighbour reads per node come from
// LDS.  In the FP16 form k_density marches the same way, and also leaves
// FP64 block sums of rho^n, from which k_compensate forms the per-component
// factor M0 / M^n that k_collide applies (global mass held at its initial
// FP64 value).
#include "lbm_internal.h"

namespace lbmx {

namespace {

__device__ __forceinline__ int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Block coordinates in an XCD-aware order.  Workgroups are dealt to the 8
// dies round-robin (linear id b runs on die b % 8).  With ystrips each die
// takes a contiguous strip of block rows in y through every z, so blocks that
// share halo rows share an L2 while every die still meets the capsules;
// without, the grid is walked in (x, y, z) order.
__device__ __forceinline__ void block_xyz(int& bx, int& by, int& bz, bool ystrips = true) {
    const int gx = gridDim.x, gy = gridDim.y;
    const int b = (blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x;
    if (ystrips && gy % NXCD == 0) {
        const int die = b % NXCD, slot = b / NXCD, R = gy / NXCD;
        bx = slot % gx;
        by = die * R + (slot / gx) % R;
        bz = slot / (gx * R);
        return;
    }
    bx = b % gx;
    by = (b / gx) % gy;
    bz = b / (gx * gy);
}

// Lattice addressing.  Blocks are BX x BY threads with BX a multiple of the
// wavefront, so all lanes of a wavefront share y (and z): the row offset
// (z * ny + y) * nx is wave-uniform and goes to scalar registers, and each
// lane adds only its x as a 32-bit byte offset (global accesses with a
// scalar base).  The host keeps every array below 2^32 bytes per component
// and direction.
static_assert(BX % 64 == 0, "a wavefront must lie within one row of the block");
__device__ __forceinline__ int uniform_ty() { return __builtin_amdgcn_readfirstlane((int)threadIdx.y); }

template <typename T>
__device__ __forceinline__ T ldx(const T* __restrict__ row, uint32_t x) {
    return *(const T*)((const char*)row + x * (uint32_t)sizeof(T));
}
// Cache policy of the population streams (every population is read once
// and written once per pass).  A lattice whose population buffer fits the
// caches' reach well (CACHED) loads populations non-temporally and stores
// them normally; a larger one does the opposite.  Each was measured the
// faster on its side (a 128^3 and a 512^3 lattice).
template <bool NT, typename T>
__device__ __forceinline__ T ldpop(const T* __restrict__ row, uint32_t x) {
    const T* p = (const T*)((const char*)row + x * (uint32_t)sizeof(T));
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <typename T>
__device__ __forceinline__ T* ptrx(T* row, uint32_t x) {
    return (T*)((char*)row + x * (uint32_t)sizeof(T));
}

// Quotients of the collision: correctly rounded, or (FAST, the FP16 form,
// whose storage rounding is far coarser) the hardware reciprocal, ~1 ulp.
template <bool FAST>
__device__ __forceinline__ float qdiv(float a, float b) {
    return FAST ? a * __builtin_amdgcn_rcpf(b) : a / b;
}

template <bool NT, typename T>
__device__ __forceinline__ void store_pop(T* p, T v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}
// A global-memory pointer kept in scalar registers: the population stores
// walk the 19 directions by adding the direction stride to it, so each
// store is this base plus the lane's 32-bit x offset.  The empty asm keeps
// LLVM from folding the x offset into a 64-bit per-lane address.
template <typename T>
using GPtr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ GPtr<T> gstep(GPtr<T> p, int64_t stride) {
    p += stride;
    asm volatile("" : "+s"(p));
    return p;
}
template <bool NT, typename T>
__device__ __forceinline__ void store_popx(GPtr<T> row, uint32_t x, T v) {
    GPtr<T> p = (GPtr<T>)((__attribute__((address_space(1))) char*)row + x * (uint32_t)sizeof(T));
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Populations of the two components for one direction and node sit side by
// side: f[i][z][y][x][c], so one pull is one 8-byte (FP32) or 4-byte (FP16)
// vector access.
typedef float pf2 __attribute__((ext_vector_type(2)));
typedef _Float16 ph2 __attribute__((ext_vector_type(2)));
template <bool HALF>
using PopT = typename std::conditional<HALF, ph2, pf2>::type;
template <bool HALF>
__device__ __forceinline__ PopT<HALF> pack(float a, float b) {
    PopT<HALF> v;
    v.x = a;
    v.y = b;
    return v;
}

// c_i . v with only the non-zero terms: IEEE rules keep a product by a zero
// coefficient (and the load feeding it), so the plain dot product would cost
// three operations for every direction.
__device__ __forceinline__ float cdot(int i, float vx, float vy, float vz) {
    if (cx(i) == 0 && cy(i) == 0 && cz(i) == 0) return 0.0f;
    float s = cx(i) > 0 ? vx : -vx;
    bool have = cx(i) != 0;
    if (cy(i) != 0) {
        const float t = cy(i) > 0 ? vy : -vy;
        s = have ? s + t : t;
        have = true;
    }
    if (cz(i) != 0) {
        const float t = cz(i) > 0 ? vz : -vz;
        s = have ? s + t : t;
    }
    return s;
}

// Moving-wall half-way bounce-back (Sec. II.C, eq. method:SBB): the
// population entering a fluid node from a solid row is the node's own
// opposite post-collision population plus 2 w_i rho (c_i . u_w) / c_s^2.
template <int I>
__device__ __forceinline__ float wall_term(const Lattice& L, float rho_prev_node) {
    const float* uw = cy(I) == 1 ? L.uw_lo : L.uw_hi;
    const float cu = cdot(I, uw[0], uw[1], uw[2]);
    return 2.0f * wgt(I) * rho_prev_node * cu * 3.0f;
}

struct Pulled {
    float f[Q];
};

struct PullCtx {
    int x, xm, xp, y, ym, yp, z, zm, zp;
    int64_t node;
    int64_t n;          // direction stride (a per-plane copy of L.n)
    uint32_t row;
};

// Pull of direction I for both components.  enc(cx, cy, cz, a, b) gives
// the decode densities of the source node x - c (FP16 form only); ra_prev,
// rb_prev are the node's own previous densities (wall term, and the decode
// density of its own reflected population).
template <bool WALLS, bool HALF, bool NTL, int I, typename EncAt>
__device__ __forceinline__ void pull_one(const PopT<HALF>* __restrict__ f, const Lattice& L, const PullCtx& c,
                                         float ra_prev, float rb_prev, const EncAt& enc, Pulled& A, Pulled& B) {
    if (WALLS && ((cy(I) == 1 && c.y == 1) || (cy(I) == -1 && c.y == L.ny - 2))) {
        const PopT<HALF> v = ldpop<NTL>(f + opp(I) * c.n + c.row, (uint32_t)c.x);
        A.f[I] = (HALF ? ra_prev * (wgt(opp(I)) + (float)v.x) : (float)v.x) + wall_term<I>(L, ra_prev);
        B.f[I] = (HALF ? rb_prev * (wgt(opp(I)) + (float)v.y) : (float)v.y) + wall_term<I>(L, rb_prev);
    } else {
        const int sx = cx(I) == 1 ? c.xm : (cx(I) == -1 ? c.xp : c.x);
        const int sy = cy(I) == 1 ? c.ym : (cy(I) == -1 ? c.yp : c.y);
        const int sz = cz(I) == 1 ? c.zm : (cz(I) == -1 ? c.zp : c.z);
        const uint32_t srow = (uint32_t)((sz * L.ny + sy) * L.nx);
        const PopT<HALF> v = ldpop<NTL>(f + I * c.n + srow, (uint32_t)sx);
        if (HALF) {
            float ea, eb;
            enc(cx(I), cy(I), cz(I), ea, eb);
            A.f[I] = ea * (wgt(I) + (float)v.x);
            B.f[I] = eb * (wgt(I) + (float)v.y);
        } else {
            A.f[I] = (float)v.x;
            B.f[I] = (float)v.y;
        }
    }
}

template <bool WALLS, bool HALF, bool NTL, typename EncAt, int... Is>
__device__ __forceinline__ void pull_all(const PopT<HALF>* __restrict__ f, const Lattice& L, const PullCtx& c,
                                         float ra_prev, float rb_prev, const EncAt& enc, Pulled& A, Pulled& B,
                                         std::integer_sequence<int, Is...>) {
    (pull_one<WALLS, HALF, NTL, Is>(f, L, c, ra_prev, rb_prev, enc, A, B), ...);
}

template <bool WALLS, bool HALF, bool NTL = false, typename EncAt>
__device__ __forceinline__ void pull(const PopT<HALF>* __restrict__ f, const Lattice& L, int64_t node, int x,
                                     int y, int z, float ra_prev, float rb_prev, const EncAt& enc, Pulled& A,
                                     Pulled& B) {
    PullCtx c;
    c.x = x; c.y = y; c.z = z; c.node = node; c.n = L.n;
    c.row = (uint32_t)((z * L.ny + y) * L.nx);
    c.xm = x == 0 ? L.nx - 1 : x - 1; c.xp = x == L.nx - 1 ? 0 : x + 1;
    c.ym = y == 0 ? L.ny - 1 : y - 1; c.yp = y == L.ny - 1 ? 0 : y + 1;
    c.zm = z == 0 ? L.nz - 1 : z - 1; c.zp = z == L.nz - 1 ? 0 : z + 1;
    pull_all<WALLS, HALF, NTL>(f, L, c, ra_prev, rb_prev, enc, A, B, std::make_integer_sequence<int, Q>{});
}

// The same pull in two phases, so that a z-marching kernel can issue the
// loads of the next plane before it computes the current one: load_raw
// only reads the 19 vectors (addresses depend on x, y, z and, at walls, on
// the row), decode turns them into populations.
template <bool HALF>
struct Raw {
    PopT<HALF> v[Q];
};

template <bool WALLS, bool HALF, bool NTL, int I>
__device__ __forceinline__ void load_raw_one(const PopT<HALF>* __restrict__ f, const Lattice& L, const PullCtx& c,
                                             Raw<HALF>& R) {
    if (WALLS && ((cy(I) == 1 && c.y == 1) || (cy(I) == -1 && c.y == L.ny - 2))) {
        R.v[I] = ldpop<NTL>(f + opp(I) * c.n + c.row, (uint32_t)c.x);
    } else {
        const int sx = cx(I) == 1 ? c.xm : (cx(I) == -1 ? c.xp : c.x);
        const int sy = cy(I) == 1 ? c.ym : (cy(I) == -1 ? c.yp : c.y);
        const int sz = cz(I) == 1 ? c.zm : (cz(I) == -1 ? c.zp : c.z);
        const uint32_t srow = (uint32_t)((sz * L.ny + sy) * L.nx);
        R.v[I] = ldpop<NTL>(f + I * c.n + srow, (uint32_t)sx);
    }
}

template <bool WALLS, bool HALF, bool NTL, int... Is>
__device__ __forceinline__ void load_raw_all(const PopT<HALF>* __restrict__ f, const Lattice& L, const PullCtx& c,
                                             Raw<HALF>& R, std::integer_sequence<int, Is...>) {
    (load_raw_one<WALLS, HALF, NTL, Is>(f, L, c, R), ...);
}

__device__ __forceinline__ PullCtx pull_ctx(const Lattice& L, int64_t node, int x, int y, int z) {
    PullCtx c;
    c.x = x; c.y = y; c.z = z; c.node = node;
    c.row = (uint32_t)((z * L.ny + y) * L.nx);
    c.xm = x == 0 ? L.nx - 1 : x - 1; c.xp = x == L.nx - 1 ? 0 : x + 1;
    c.ym = y == 0 ? L.ny - 1 : y - 1; c.yp = y == L.ny - 1 ? 0 : y + 1;
    c.zm = z == 0 ? L.nz - 1 : z - 1; c.zp = z == L.nz - 1 ? 0 : z + 1;
    // Fresh lane offsets and direction stride for every plane: each load is
    // then a scalar row base plus one of three 32-bit x offsets, rebuilt in a
    // few scalar instructions, instead of a pointer per direction held in
    // (vector, or spilled scalar) registers across the march.
    c.n = L.n;
    asm volatile("" : "+v"(c.xm), "+v"(c.x), "+v"(c.xp), "+s"(c.n));
    return c;
}

template <bool WALLS, bool HALF, bool NTL = false>
__device__ __forceinline__ void load_raw(const PopT<HALF>* __restrict__ f, const Lattice& L, int64_t node, int x,
                                         int y, int z, Raw<HALF>& R) {
    load_raw_all<WALLS, HALF, NTL>(f, L, pull_ctx(L, node, x, y, z), R, std::make_integer_sequence<int, Q>{});
}

template <bool WALLS, bool HALF, int I, typename EncAt>
__device__ __forceinline__ void decode_one(const Lattice& L, int y, const Raw<HALF>& R, float ra_prev, float rb_prev,
                                           const EncAt& enc, Pulled& A, Pulled& B) {
    const PopT<HALF> v = R.v[I];
    // FP16: f = rho_enc (w + g), as rho_enc g + rho_enc w (one mixed-precision
    // FMA that reads the binary16 value directly)
    if (WALLS && ((cy(I) == 1 && y == 1) || (cy(I) == -1 && y == L.ny - 2))) {
        A.f[I] = (HALF ? fmaf(ra_prev, (float)v.x, ra_prev * wgt(opp(I))) : (float)v.x) + wall_term<I>(L, ra_prev);
        B.f[I] = (HALF ? fmaf(rb_prev, (float)v.y, rb_prev * wgt(opp(I))) : (float)v.y) + wall_term<I>(L, rb_prev);
    } else if (HALF) {
        float ea, eb;
        enc(cx(I), cy(I), cz(I), ea, eb);
        A.f[I] = fmaf(ea, (float)v.x, ea * wgt(I));
        B.f[I] = fmaf(eb, (float)v.y, eb * wgt(I));
    } else {
        A.f[I] = (float)v.x;
        B.f[I] = (float)v.y;
    }
}

template <bool WALLS, bool HALF, typename EncAt, int... Is>
__device__ __forceinline__ void decode_all(const Lattice& L, int y, const Raw<HALF>& R, float ra_prev, float rb_prev,
                                           const EncAt& enc, Pulled& A, Pulled& B, std::integer_sequence<int, Is...>) {
    (decode_one<WALLS, HALF, Is>(L, y, R, ra_prev, rb_prev, enc, A, B), ...);
}

template <bool WALLS, bool HALF, typename EncAt>
__device__ __forceinline__ void decode(const Lattice& L, int y, const Raw<HALF>& R, float ra_prev, float rb_prev,
                                       const EncAt& enc, Pulled& A, Pulled& B) {
    decode_all<WALLS, HALF>(L, y, R, ra_prev, rb_prev, enc, A, B, std::make_integer_sequence<int, Q>{});
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

// Rest equilibrium f_i = w_i rho (u = 0), the rest population closing the
// mass; in the FP16 form that is g_i = 0 with rho_enc = rho.
template <bool HALF>
__global__ __launch_bounds__(256) void k_init_rest(PopT<HALF>* __restrict__ f, const float* __restrict__ rhoA,
                                                   const float* __restrict__ rhoB, int64_t n) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        if (HALF) {
            for (int i = 0; i < Q; ++i) f[(int64_t)i * n + k] = pack<HALF>(0.0f, 0.0f);
            continue;
        }
        const float ra = rhoA[k], rb = rhoB[k];
        float resta = ra, restb = rb;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const float fa = wgt(i) * ra, fb = wgt(i) * rb;
            resta -= fa;
            restb -= fb;
            f[(int64_t)i * n + k] = pack<HALF>(fa, fb);
        }
        f[k] = pack<HALF>(resta, restb);
    }
}

// Three-plane LDS ring over the column and its halo: slot(zz) = (zz - z0 + 1) % 3.
template <int NC>
struct Ring {
    static constexpr int SW = BX + 2, SH = BY + 2;
    float v[3][NC][SH][SW];
};
// The same for a pair of components read together (both fluid components
// at one cell): one 8-byte LDS access per neighbour instead of two.
struct Ring2 {
    static constexpr int SW = BX + 2, SH = BY + 2;
    float2 v[3][SH][SW];
};

// Staging a plane of the ring.  stage_positions fixes, once per block, the
// plane positions a thread stages (they do not depend on z; with WALLS the
// solid rows take the value of the adjacent fluid row); stage_load reads
// one plane zz at those positions into registers (per component, optionally
// times a per-component scale, optionally plus the virtual density where
// tiles are flagged) and stage_store writes them into the ring.
struct StagePos {
    static constexpr int SW = BX + 2, SH = BY + 2;
    static constexpr int POS = SH * SW;
    static constexpr int NIT = (POS + BX * BY - 1) / (BX * BY);
    uint32_t xy[NIT];    // gy * nx + gx of the position
    uint32_t txy[NIT];   // its tile within a plane of tiles
};

template <int NC>
struct StageRegs {
    float v[StagePos::NIT][NC];
};

// Position k = ly * SW + lx of the plane is also its offset within one
// component plane of the ring (and its cell in a Ring2 plane).
__device__ __forceinline__ bool stage_has(int tid, int it) { return tid + it * BX * BY < StagePos::POS; }

__device__ __forceinline__ void stage_store2(Ring2& R, const StageRegs<2>& S, int zz, int z0, int tid) {
    const int slot = (zz - z0 + 1) % 3;
#pragma unroll
    for (int it = 0; it < StagePos::NIT; ++it)
        if (stage_has(tid, it)) (&R.v[slot][0][0])[tid + it * BX * BY] = make_float2(S.v[it][0], S.v[it][1]);
}

template <bool WALLS>
__device__ __forceinline__ StagePos stage_positions(int x0, int y0, int tid, const Lattice& L) {
    StagePos P;
#pragma unroll
    for (int it = 0; it < StagePos::NIT; ++it) {
        const int k = min(tid + it * BX * BY, StagePos::POS - 1);
        const int ly = k / StagePos::SW, lx = k - ly * StagePos::SW;
        const int gx = wrapi(x0 - 1 + lx, L.nx);
        int gy = wrapi(y0 - 1 + ly, L.ny);
        // on-site boundaries: a neighbour beyond the box is the boundary row
        if (!WALLS && L.onsite) gy = min(max(y0 - 1 + ly, 0), L.ny - 1);
        if (WALLS) {
            // solid rows take the value of the adjacent fluid row
            if (gy == 0) gy = 1;
            if (gy == L.ny - 1) gy = L.ny - 2;
        }
        P.xy[it] = (uint32_t)(gy * L.nx + gx);
        P.txy[it] = (uint32_t)((gy >> 3) * L.ntx + (gx >> 3));
    }
    return P;
}

// PSI: the staged densities become the exponential Shan-Chen pseudo-potential
// 1 - exp(-rho) before the virtual density field is added (a compile-time
// choice: a runtime flag made the compiler specialise the whole z march).
template <bool ADD_PHI, int NC, bool PSI = false>
__device__ __forceinline__ void stage_load(StageRegs<NC>& S, const StagePos& P, int zz, int tid,
                                           const float* __restrict__ src, const float* scale,
                                           const float* __restrict__ fib, const int* __restrict__ tile_flag,
                                           const Lattice& L) {
    const int zw = wrapi(zz, L.nz);
    const int64_t zoff = (int64_t)zw * L.ny * L.nx;
    const int tz = (zw >> 3) * L.nty * L.ntx;
#pragma unroll
    for (int it = 0; it < StagePos::NIT; ++it) {
        if (stage_has(tid, it)) {
            bool flag = false;
            if (ADD_PHI) flag = tile_flag[tz + P.txy[it]] != 0;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                float v = ldx(src + c * L.n + zoff, P.xy[it]);
                if (scale) v *= scale[c];
                if constexpr (PSI) v = psi_exp(v);
                if (ADD_PHI) {
                    // the load goes out unconditionally so that no wait on
                    // the flag sits between the loads in flight
                    const float phi = ldx(fib + (3 + c) * L.n + zoff, P.xy[it]);
                    v += flag ? phi : 0.0f;
                }
                S.v[it][c] = v;
            }
        }
    }
}

// (components c of the registers go to ring fields C0 + c)
template <int NC, int NR, int C0 = 0>
__device__ __forceinline__ void stage_store(Ring<NR>& R, const StageRegs<NC>& S, int zz, int z0, int tid) {
    static_assert(C0 + NC <= NR, "ring too small");
    const int slot = (zz - z0 + 1) % 3;
#pragma unroll
    for (int it = 0; it < StagePos::NIT; ++it) {
        if (stage_has(tid, it)) {
#pragma unroll
            for (int c = 0; c < NC; ++c) (&R.v[slot][C0 + c][0][0])[tid + it * BX * BY] = S.v[it][c];
        }
    }
}

// ---------------------------------------------------------------------------
// Density pass, FP32: one thread per node.
template <bool WALLS, bool CACHED>
__global__ __launch_bounds__(BX * BY) void k_density(const pf2* __restrict__ fin,
                                                 const float* __restrict__ rho_prev,
                                                 float* __restrict__ rho_out, Lattice L) {
    int bx, by, bz;
    block_xyz(bx, by, bz);
    const int x = bx * BX + threadIdx.x;
    const int y = by * BY + uniform_ty();
    const int z = bz;
    if (x >= L.nx || y >= L.ny) return;
    if (WALLS && (y == 0 || y == L.ny - 1)) return;
    const int64_t node = ((int64_t)z * L.ny + y) * L.nx + x;
    const uint32_t row = (uint32_t)((z * L.ny + y) * L.nx);
    auto none = [](int, int, int, float&, float&) {};
    Pulled A, B;
    const float rpa = WALLS ? ldx(rho_prev + row, (uint32_t)x) : 0.0f;
    const float rpb = WALLS ? ldx(rho_prev + L.n + row, (uint32_t)x) : 0.0f;
    pull<WALLS, false, CACHED>(fin, L, node, x, y, z, rpa, rpb, none, A, B);
    *ptrx(rho_out + row, (uint32_t)x) = sum_pop(A);
    *ptrx(rho_out + L.n + row, (uint32_t)x) = sum_pop(B);
}

// Density pass, FP16: z-marching column with the decode densities
// cscale(prev) * rho^{n-1} staged in LDS, plus FP64 block sums of rho^n.
template <bool WALLS, bool CACHED>
__global__ __launch_bounds__(BX * BY) void k_density_half(const ph2* __restrict__ fin,
                                                      const float* __restrict__ rho_prev,
                                                      const float* __restrict__ cscale, int par_prev,
                                                      float* __restrict__ rho_out, double* __restrict__ partial,
                                                      Lattice L) {
    __shared__ Ring2 ring;
    __shared__ double red[2][BX * BY];
    const int tx = threadIdx.x, ty = uniform_ty(), tid = ty * BX + tx;
    int bx, by, bz;
    block_xyz(bx, by, bz);
    const int x0 = bx * BX, y0 = by * BY, z0 = bz * L.zc;
    const int z1 = min(z0 + L.zc, L.nz);
    const float cp[2] = {cscale[2 * par_prev], cscale[2 * par_prev + 1]};
    const StagePos P = stage_positions<WALLS>(x0, y0, tid, L);
    StageRegs<2> st;
    stage_load<false, 2>(st, P, z0 - 1, tid, rho_prev, cp, nullptr, nullptr, L);
    stage_store2(ring, st, z0 - 1, z0, tid);
    stage_load<false, 2>(st, P, z0, tid, rho_prev, cp, nullptr, nullptr, L);
    stage_store2(ring, st, z0, z0, tid);
    const int x = x0 + tx, y = y0 + ty;
    const bool active = x < L.nx && y < L.ny && (!WALLS || (y > 0 && y < L.ny - 1));
    double acc[2] = {0.0, 0.0};
    Raw<true> rcur;
#pragma unroll 1
    for (int z = z0; z < z1; ++z) {
        stage_load<false, 2>(st, P, z + 1, tid, rho_prev, cp, nullptr, nullptr, L);
        stage_store2(ring, st, z + 1, z0, tid);
        __syncthreads();
        if (active) load_raw<WALLS, true, CACHED>(fin, L, ((int64_t)z * L.ny + y) * L.nx + x, x, y, z, rcur);
        if (active) {
            const uint32_t row = (uint32_t)((z * L.ny + y) * L.nx);
            const int s0 = (z - z0 + 1) % 3;
            auto enc = [&](int ex, int ey, int ez, float& a, float& b) {
                const int sl = (s0 - ez + 3) % 3;
                const float2 e = ring.v[sl][ty + 1 - ey][tx + 1 - ex];
                a = e.x;
                b = e.y;
            };
            Pulled A, B;
            const float2 e0 = ring.v[s0][ty + 1][tx + 1];
            decode<WALLS, true>(L, y, rcur, e0.x, e0.y, enc, A, B);
            const float ra = sum_pop(A), rb = sum_pop(B);
            *ptrx(rho_out + row, (uint32_t)x) = ra;
            *ptrx(rho_out + L.n + row, (uint32_t)x) = rb;
            acc[0] += (double)ra;
            acc[1] += (double)rb;
        }
        __syncthreads();
    }
    red[0][tid] = acc[0];
    red[1][tid] = acc[1];
    __syncthreads();
    for (int s = BX * BY / 2; s > 0; s >>= 1) {
        if (tid < s) {
            red[0][tid] += red[0][tid + s];
            red[1][tid] += red[1][tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const int64_t b = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        partial[2 * b] = red[0][0];
        partial[2 * b + 1] = red[1][0];
    }
}

// Per-component compensation factor M0 / M^n from the FP64 block sums, in a
// fixed summation order.
__global__ __launch_bounds__(1024) void k_compensate(const double* __restrict__ partial, int nblocks,
                                                     double m0a, double m0b, float* __restrict__ cscale,
                                                     int par_cur, double* __restrict__ mass_out) {
    __shared__ double sh[2][1024];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nblocks; k += 1024) {
        a += partial[2 * k];
        b += partial[2 * k + 1];
    }
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cscale[2 * par_cur] = (float)(m0a / sh[0][0]);
        cscale[2 * par_cur + 1] = (float)(m0b / sh[1][0]);
        mass_out[0] = sh[0][0];
        mass_out[1] = sh[1][0];
    }
}

// ---------------------------------------------------------------------------
// Fused pull + force + collide.  MACRO: recompute the velocity of this
// collision without storing populations (field read-back).  SHARP (the
// bounce-back coupling): flagged tiles carry, instead of the immersed
// boundary's force and virtual densities, corrections dS^A, dS^B to the
// Shan-Chen neighbour sums from neighbours across a membrane (fib fields
// 0..2 and 3..5), added before the force is formed.
//
// ONE (one lattice pass): the densities of the ring are formed here from
// pulled populations instead of read from the density pass.  Per plane
// each thread pulls its own node (kept in registers for its collide one
// plane later) and one halo cell: thread row 0 the row below the block,
// row 1 the row above, twelve lanes of row 2 the corners and the x-halo;
// the ring values are the same bit for bit as the two-pass ones.
template <bool WALLS, bool IBM, bool MACRO, bool HALF, bool CACHED, bool PSI, bool SHARP, bool ONE>
__device__ __forceinline__ void collide_body(const PopT<HALF>* __restrict__ fin, PopT<HALF>* __restrict__ fout,
                                                 const float* __restrict__ rho_n,
                                                 const float* __restrict__ rho_p,
                                                 const float* __restrict__ fib,
                                                 const int* __restrict__ tile_flag,
                                                 float* __restrict__ u_out, const float* __restrict__ cscale,
                                                 int par_prev, int par_cur, Lattice L) {
    __shared__ Ring2 sp;                         // psi + phi at time n (A, B)
    __shared__ Ring2 se;                         // decode densities rho_enc^{n-1} (FP16)
    static_assert(!ONE || (!WALLS && !HALF && !MACRO && !SHARP), "one pass: FP32, periodic, stepping only");
    const int tx = threadIdx.x, ty = uniform_ty();
    const int tid = ty * BX + tx;
    int bx, by, bz;
    // y-strips on cache-sized lattices; on larger ones the plain order
    // measured faster for this kernel (the density passes gain either way);
    // the one-pass form re-reads its halo rows from the neighbouring blocks'
    // reads, which y-strips keep on one die (10% faster at 512^3)
    block_xyz(bx, by, bz, CACHED || ONE);
    const int x0 = bx * BX, y0 = by * BY, z0 = bz * L.zc;
    const int z1 = min(z0 + L.zc, L.nz);
    const int64_t N = L.n;
    // FP16: cpv scales the stored densities to the decode densities of the
    // writing step; ccu is this step's FP64 mass compensation, applied to
    // the decoded populations through the staged decode densities
    // (cdec = cpv ccu; decoding is linear in them, the wall term included)
    float cpv[2] = {1.0f, 1.0f}, ccu[2] = {1.0f, 1.0f}, cdec[2] = {1.0f, 1.0f};
    if (HALF) {
        cpv[0] = cscale[2 * par_prev];
        cpv[1] = cscale[2 * par_prev + 1];
        ccu[0] = cscale[2 * par_cur];
        ccu[1] = cscale[2 * par_cur + 1];
        cdec[0] = cpv[0] * ccu[0];
        cdec[1] = cpv[1] * ccu[1];
    }

    // Does any tile that the block's column or its halo overlaps carry
    // immersed-boundary fields this step?  Most blocks lie away from every
    // membrane and then skip all per-node tile lookups.
    bool near_ibm = false;
    if (IBM) {
        const int tx0 = wrapi(x0 - 1, L.nx) >> 3, ntx_b = (BX + 2 + 7) / 8 + 1;
        const int ty0 = wrapi(y0 - 1, L.ny) >> 3, nty_b = (BY + 2 + 7) / 8 + 1;
        const int tz0 = wrapi(z0 - 1, L.nz) >> 3, ntz_b = (L.zc + 2 + 7) / 8 + 1;
        bool hit = false;
        for (int k = tid; k < ntx_b * nty_b * ntz_b; k += BX * BY) {
            const int i = k % ntx_b, j = (k / ntx_b) % nty_b, l = k / (ntx_b * nty_b);
            const int t = (((tz0 + l) % L.ntz) * L.nty + (ty0 + j) % L.nty) * L.ntx + (tx0 + i) % L.ntx;
            hit = hit || tile_flag[t] != 0;
        }
        near_ibm = __syncthreads_or(hit) != 0;
    }
    const StagePos P = stage_positions<WALLS>(x0, y0, tid, L);
    StageRegs<2> np;
    StageRegs<2> ne;
    auto load_plane = [&](int zz) {
        if (IBM && !SHARP && near_ibm)
            stage_load<true, 2, PSI>(np, P, zz, tid, rho_n, HALF ? ccu : nullptr, fib, tile_flag, L);
        else
            stage_load<false, 2, PSI>(np, P, zz, tid, rho_n, HALF ? ccu : nullptr, nullptr, nullptr, L);
        if constexpr (HALF) stage_load<false, 2>(ne, P, zz, tid, rho_p, cdec, nullptr, nullptr, L);
    };
    auto store_plane = [&](int zz) {
        stage_store2(sp, np, zz, z0, tid);
        if constexpr (HALF) stage_store2(se, ne, zz, z0, tid);
    };

    const int x = x0 + tx, y = y0 + ty;
    const bool active = x < L.nx && y < L.ny && (!WALLS || (y > 0 && y < L.ny - 1));
    // one pass: the ring cell of a pulled node, psi(rho) plus the virtual
    // density where its tile is flagged (as stage_load forms it)
    auto none = [](int, int, int, float&, float&) {};
    auto ring_cell = [&](const auto& R, int gx, int gy, int zw) {   // (generic: built for ONE only)
        Pulled A, B;
        decode<false, false>(L, gy, R, 0.f, 0.f, none, A, B);
        float va = sum_pop(A), vb = sum_pop(B);
        if constexpr (PSI) { va = psi_exp(va); vb = psi_exp(vb); }
        if (IBM && near_ibm) {
            const uint32_t pos = (uint32_t)((zw * L.ny + gy) * L.nx + gx);
            const bool flag = tile_flag[((zw >> 3) * L.nty + (gy >> 3)) * L.ntx + (gx >> 3)] != 0;
            const float pa = ldx(fib + 3 * N, pos), pb = ldx(fib + 4 * N, pos);
            va += flag ? pa : 0.0f;
            vb += flag ? pb : 0.0f;
        }
        return make_float2(va, vb);
    };
    // (the node itself wraps, so that a partial block still fills the ring
    // cells its active neighbours read)
    const int ix = wrapi(x, L.nx), iy = wrapi(y, L.ny);
    const int hrow = ty == 0 ? 0 : BY + 1;                  // thread rows 0, 1: a halo row each
    const int hy = wrapi(y0 - 1 + hrow, L.ny);
    // the two edge cells (x0 - 1, x0 + BX) of the BY + 2 ring rows: ring row
    // r by wavefront 2 BX / 64 + r % (waves left), one row per pass, so that
    // every load of a pass has one row
    constexpr int WV = BX * BY / 64, W0 = 2 * BX / 64, WR = WV - W0;
    static_assert(BY >= 3 && WR >= 1, "halo rows per wavefront");
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int ehx = wrapi(lane == 0 ? x0 - 1 : x0 + BX, L.nx), elx = lane == 0 ? 0 : BX + 1;
    auto one_plane = [&](int zz, auto& R) {
        const int zw = wrapi(zz, L.nz), sl = (zz - z0 + 1) % 3;
        load_raw<false, false, CACHED>(fin, L, ((int64_t)zw * L.ny + iy) * L.nx + ix, ix, iy, zw, R);
        sp.v[sl][ty + 1][tx + 1] = ring_cell(R, ix, iy, zw);
        __builtin_amdgcn_sched_barrier(0);
        if (ty < 2) {
            std::remove_reference_t<decltype(R)> H;
            load_raw<false, false, CACHED>(fin, L, ((int64_t)zw * L.ny + hy) * L.nx + ix, ix, hy, zw, H);
            sp.v[sl][hrow][tx + 1] = ring_cell(H, ix, hy, zw);
        }
        if (wv >= W0) {
            for (int r = wv - W0; r < BY + 2; r += WR) {
                const int ey = wrapi(y0 - 1 + r, L.ny);
                std::remove_reference_t<decltype(R)> H;
                if (lane < 2) {
                    load_raw<false, false, CACHED>(fin, L, ((int64_t)zw * L.ny + ey) * L.nx + ehx, ehx, ey, zw, H);
                    sp.v[sl][r][elx] = ring_cell(H, ehx, ey, zw);
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    Raw<HALF> rcur, rnext;
    if constexpr (ONE) {
        one_plane(z0 - 1, rnext);
        one_plane(z0, rcur);
    } else {
        load_plane(z0 - 1);
        store_plane(z0 - 1);
        load_plane(z0);
        store_plane(z0);
    }
#pragma unroll 1
    for (int z = z0; z < z1; ++z) {
        if constexpr (ONE) {
            one_plane(z + 1, rnext);
        } else {
            load_plane(z + 1);
            store_plane(z + 1);
        }
        __syncthreads();
        if (!ONE && active) load_raw<WALLS, HALF, CACHED>(fin, L, ((int64_t)z * L.ny + y) * L.nx + x, x, y, z, rcur);
        if (active) {
            const uint32_t row = (uint32_t)((z * L.ny + y) * L.nx), xo = (uint32_t)x;
            const int s0 = (z - z0 + 1) % 3;
            Pulled A, B;
            if constexpr (HALF) {
                auto enc = [&](int ex, int ey, int ez, float& a, float& b) {
                    const int sl = (s0 - ez + 3) % 3;
                    const float2 e = se.v[sl][ty + 1 - ey][tx + 1 - ex];
                    a = e.x;
                    b = e.y;
                };
                const float2 e0 = se.v[s0][ty + 1][tx + 1];
                decode<WALLS, true>(L, y, rcur, e0.x, e0.y, enc, A, B);
            } else {
                auto none = [](int, int, int, float&, float&) {};
                const float rpa = WALLS ? ldx(rho_p + row, xo) : 0.0f;
                const float rpb = WALLS ? ldx(rho_p + N + row, xo) : 0.0f;
                decode<WALLS, false>(L, y, rcur, rpa, rpb, none, A, B);
            }
            const float ra = sum_pop(A), rb = sum_pop(B);
            float jax, jay, jaz, jbx, jby, jbz;
            momentum(A, jax, jay, jaz);
            momentum(B, jbx, jby, jbz);

            // neighbour sums S^c = sum_i w_i (psi^c + phi^c)(x + c_i) c_i
            float sa[3] = {0.f, 0.f, 0.f}, sb[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 1; k < Q; k += 2) {
                const int sP = (s0 + cz(k) + 3) % 3, sM = (s0 - cz(k) + 3) % 3;
                const int ly = ty + 1, lx = tx + 1;
                const float2 vp = sp.v[sP][ly + cy(k)][lx + cx(k)], vm = sp.v[sM][ly - cy(k)][lx - cx(k)];
                const float da = vp.x - vm.x, db = vp.y - vm.y;
                const float w = wgt(k);
                if (cx(k) != 0) { sa[0] += w * cx(k) * da; sb[0] += w * cx(k) * db; }
                if (cy(k) != 0) { sa[1] += w * cy(k) * da; sb[1] += w * cy(k) * db; }
                if (cz(k) != 0) { sa[2] += w * cz(k) * da; sb[2] += w * cz(k) * db; }
            }
            const float rsum = ra + rb;
            // the node's own pseudo-potential
            const float pa = PSI ? psi_exp(ra) : ra, pb = PSI ? psi_exp(rb) : rb;
            bool flagged = false;
            if (SHARP && near_ibm) {
                const int t = ((z >> 3) * L.nty + (y >> 3)) * L.ntx + (x >> 3);
                flagged = tile_flag[t] != 0;
                if (flagged) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        sa[d] += ldx(fib + d * N + row, xo);
                        sb[d] += ldx(fib + (3 + d) * N + row, xo);
                    }
                }
            }
            float Fa[3], Fb[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                Fa[d] = -L.G * pa * sb[d];
                Fb[d] = -L.G * pb * sa[d];
            }
            if (IBM && !SHARP && near_ibm) {
                const int t = ((z >> 3) * L.nty + (y >> 3)) * L.ntx + (x >> 3);
                flagged = tile_flag[t] != 0;
                if (flagged) {
                    // immersed-boundary force shared by mass fraction
                    const float fa = qdiv<HALF>(ra, rsum), fb = qdiv<HALF>(rb, rsum);
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const float Fi = ldx(fib + d * N + row, xo);
                        Fa[d] += fa * Fi;
                        Fb[d] += fb * Fi;
                    }
                }
            }
            // common velocity u' and the shifted equilibrium velocities
            const float wa = L.omega[0], wb = L.omega[1];
            const float den = qdiv<HALF>(1.0f, ra * wa + rb * wb);
            const float upx = (jax * wa + jbx * wb) * den;
            const float upy = (jay * wa + jby * wb) * den;
            const float upz = (jaz * wa + jbz * wb) * den;
            if (MACRO || (IBM && flagged)) {
                const float ir = qdiv<HALF>(1.0f, rsum);
                *ptrx(u_out + row, xo) = (jax + jbx + 0.5f * (Fa[0] + Fb[0])) * ir;
                *ptrx(u_out + N + row, xo) = (jay + jby + 0.5f * (Fa[1] + Fb[1])) * ir;
                *ptrx(u_out + 2 * N + row, xo) = (jaz + jbz + 0.5f * (Fa[2] + Fb[2])) * ir;
            }
            if (!MACRO) {
                float ux[2], uy[2], uz[2], base[2], inv[2];
                const float r2[2] = {ra, rb};
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const float* F = c == 0 ? Fa : Fb;
                    const float ts = qdiv<HALF>(L.tau[c], r2[c]);
                    ux[c] = upx + ts * F[0];
                    uy[c] = upy + ts * F[1];
                    uz[c] = upz + ts * F[2];
                    base[c] = r2[c] * (1.0f - 1.5f * (ux[c] * ux[c] + uy[c] * uy[c] + uz[c] * uz[c]));
                    // FP16: encode relative to this node's compensated density,
                    // bit-identical to what the next step's decoder stages
                    inv[c] = HALF ? qdiv<true>(1.0f, ccu[c] * ldx(rho_n + c * N + row, xo)) : 1.0f;
                }
                // direction bases advance by the stride in scalar registers,
                // so each store is a scalar base plus the lane's x offset
                // (row is wave-uniform; the one-pass form says so explicitly,
                // or the backend fails to keep the store bases in scalars)
                const GPtr<PopT<HALF>> fo =
                    (GPtr<PopT<HALF>>)(fout + (ONE ? (uint32_t)__builtin_amdgcn_readfirstlane(row) : row));
                GPtr<PopT<HALF>> fi = fo;
                int64_t Ns = N;                    // direction stride, rebuilt per plane
                uint32_t xs = xo;                  // 32-bit lane offset, per plane
                asm volatile("" : "+s"(Ns), "+v"(xs));
                if constexpr (HALF) {
                    // BGK and the encode in one step, per opposite pair
                    // (c_{k+1} = -c_k, equal weights).  With feq_i = w_i t_i,
                    // t_i = base + rho (c.u)(3 + 4.5 c.u), the stored
                    // g_i = f*_i / rho_enc - w_i = a1 f_i + bo w_i t_i - w_i
                    // (a1 = (1 - omega) inv, bo = omega inv, inv = 1/rho_enc)
                    // splits into a part even in c.u,
                    // P = bo w (base + 4.5 rho (c.u)^2) - w, and an odd part,
                    // H = 3 bo w rho (c.u):
                    //   g_k = a1 f_k + P + H,  g_{k+1} = a1 f_{k+1} + P - H.
                    // The rest population closes the mass in g units,
                    // g_0 = rho inv - 1 - sum_{i>0} g_i, with
                    // sum_{i>0} g_i = a1 (rho - f_0) + 2 sum P.  Constants of the
                    // diagonal class (w = 1/36) are half the axis class's (1/18).
                    float a1[2], B1[2][2], K45[2][2], K3[2][2], sumP[2] = {0.f, 0.f};
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        a1[c] = (1.0f - L.omega[c]) * inv[c];
                        const float bw = L.omega[c] * inv[c] * (1.0f / 18.0f);
                        B1[0][c] = fmaf(bw, base[c], -1.0f / 18.0f);
                        K3[0][c] = (3.0f * bw) * r2[c];
                        K45[0][c] = 1.5f * K3[0][c];
                        B1[1][c] = 0.5f * B1[0][c];
                        K3[1][c] = 0.5f * K3[0][c];
                        K45[1][c] = 0.5f * K45[0][c];
                    }
#pragma unroll
                    for (int k = 1; k < Q; k += 2) {
                        const int cls = k <= 6 ? 0 : 1;
                        float g1[2], g2[2];
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const Pulled& Pp = c == 0 ? A : B;
                            const float cu = cdot(k, ux[c], uy[c], uz[c]);
                            const float Pe = fmaf(K45[cls][c], cu * cu, B1[cls][c]);
                            const float Ho = K3[cls][c] * cu;
                            g1[c] = fmaf(a1[c], Pp.f[k], Pe + Ho);
                            g2[c] = fmaf(a1[c], Pp.f[k + 1], Pe - Ho);
                            sumP[c] += Pe;
                        }
                        fi = gstep(fi, Ns);
                        store_popx<!CACHED>(fi, xs, pack<HALF>(g1[0], g1[1]));
                        fi = gstep(fi, Ns);
                        store_popx<!CACHED>(fi, xs, pack<HALF>(g2[0], g2[1]));
                    }
                    float g0[2];
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const Pulled& Pp = c == 0 ? A : B;
                        g0[c] = fmaf(r2[c], inv[c], -1.0f) - fmaf(a1[c], r2[c] - Pp.f[0], 2.0f * sumP[c]);
                    }
                    store_popx<!CACHED>(fo, xs, pack<HALF>(g0[0], g0[1]));
                } else {
                    // (per direction: the pairwise form above costs this
                    // HBM-bound path a wave of occupancy)
                    float rest[2] = {r2[0], r2[1]};
#pragma unroll
                    for (int i = 1; i < Q; ++i) {
                        float fs[2];
#pragma unroll
                        for (int c = 0; c < 2; ++c) {
                            const Pulled& P = c == 0 ? A : B;
                            const float cu = cdot(i, ux[c], uy[c], uz[c]);
                            const float feq = wgt(i) * (base[c] + r2[c] * cu * (3.0f + 4.5f * cu));
                            fs[c] = P.f[i] + L.omega[c] * (feq - P.f[i]);
                            rest[c] -= fs[c];
                        }
                        fi = gstep(fi, Ns);
                        store_popx<!CACHED>(fi, xs, pack<HALF>(fs[0], fs[1]));
                    }
                    // rest populations close the node's mass
                    store_popx<!CACHED>(fo, xs, pack<HALF>(rest[0], rest[1]));
                }
            }
        } else if (MACRO && x < L.nx && y < L.ny) {
            const int64_t node = ((int64_t)z * L.ny + y) * L.nx + x;
            u_out[node] = u_out[N + node] = u_out[2 * N + node] = 0.f;
        }
        if constexpr (ONE) rcur = rnext;
        __syncthreads();
    }
}

#define COLLIDE_ARGS                                                                                        \
    const PopT<HALF>* __restrict__ fin, PopT<HALF>* __restrict__ fout, const float* __restrict__ rho_n,     \
        const float* __restrict__ rho_p, const float* __restrict__ fib, const int* __restrict__ tile_flag, \
        float* __restrict__ u_out, const float* __restrict__ cscale, int par_prev, int par_cur, Lattice L
template <bool WALLS, bool IBM, bool MACRO, bool HALF, bool CACHED, bool PSI, bool SHARP = false>
__global__ __launch_bounds__(BX * BY) LBM_COLLIDE_ATTR void k_collide(COLLIDE_ARGS) {
    collide_body<WALLS, IBM, MACRO, HALF, CACHED, PSI, SHARP, false>(fin, fout, rho_n, rho_p, fib, tile_flag, u_out,
                                                                     cscale, par_prev, par_cur, L);
}
// The one-pass form at four waves per SIMD (at most 128 VGPRs: two blocks per
// compute unit, so one block's barrier wait overlaps the other's work);
// left to itself the compiler takes 145 and fits one block (10.5 against
// 9.2 ms at 512^3).
template <bool IBM, bool CACHED, bool PSI>
__global__ __launch_bounds__(BX * BY) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_collide_one(
    const pf2* __restrict__ fin, pf2* __restrict__ fout, const float* __restrict__ rho_n,
    const float* __restrict__ rho_p, const float* __restrict__ fib, const int* __restrict__ tile_flag,
    float* __restrict__ u_out, const float* __restrict__ cscale, int par_prev, int par_cur, Lattice L) {
    collide_body<false, IBM, false, false, CACHED, PSI, false, true>(fin, fout, rho_n, rho_p, fib, tile_flag, u_out,
                                                                     cscale, par_prev, par_cur, L);
}
#undef COLLIDE_ARGS

// One lattice pass with capsules: this step's densities on the tiles the
// immersed boundary touches, which the spreading's wettability reaction
// reads before the collide forms them again (the same sums, so the same
// values).  A bin's reaction reads cells -2 .. +6 around it and its
// stencils flag the tiles of cells -1 .. +5; with every lattice edge a
// multiple of the tile both lie in the same tiles, else (dil) each tile is
// widened by one cell, wrapped.
// Without widening, a touched tile is handled with its x partner (tiles 2k
// and 2k + 1): rows of 16 cells read whole 128-byte lines of each direction
// (an 8-cell row reads half of one); a pair whose even tile is touched is
// handled from that tile only.
__global__ __launch_bounds__(256) void k_density_tiles(const pf2* __restrict__ fin, float* __restrict__ rho_out,
                                                       const int* __restrict__ touched, const int* __restrict__ count,
                                                       const int* __restrict__ tile_flag, int dil, Lattice L) {
    const int nt = *count;
    const int E = TILE + 2 * dil, EX = dil ? E : 2 * TILE, N3 = EX * E * E;
    auto none = [](int, int, int, float&, float&) {};
    for (int e = blockIdx.x; e < nt; e += gridDim.x) {
        const int t = touched[e];
        int tx = t % L.ntx;
        const int ty = (t / L.ntx) % L.nty, tz = t / (L.ntx * L.nty);
        if (!dil) {
            if ((tx & 1) && tile_flag[t - 1] != 0) continue;      // (block-uniform)
            tx &= ~1;
        }
        for (int c = threadIdx.x; c < N3; c += blockDim.x) {
            int x = tx * TILE - dil + c % EX, y = ty * TILE - dil + (c / EX) % E, z = tz * TILE - dil + c / (EX * E);
            if (!dil && (x >= L.nx || y >= L.ny || z >= L.nz)) continue;
            x = wrapi(x, L.nx);
            y = wrapi(y, L.ny);
            z = wrapi(z, L.nz);
            const int64_t node = ((int64_t)z * L.ny + y) * L.nx + x;
            Pulled A, B;
            pull<false, false>(fin, L, node, x, y, z, 0.f, 0.f, none, A, B);
            rho_out[node] = sum_pop(A);
            rho_out[L.n + node] = sum_pop(B);
        }
    }
}

// FP32 storage, mass compensation at a mass check: each population of
// component c at the fluid nodes times s_c, the ratio of the intended to
// the stored FP64 mass of the component.
__global__ __launch_bounds__(256) void k_scale_pops(pf2* __restrict__ f, float sa, float sb, Lattice L) {
    const int64_t plane = (int64_t)L.nx * L.ny;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < L.n;
         k += (int64_t)gridDim.x * blockDim.x) {
        if (L.walls) {
            const int y = (int)((k % plane) / L.nx);
            if (y == 0 || y == L.ny - 1) continue;
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            pf2 p = f[(int64_t)i * L.n + k];
            p.x *= sa;
            p.y *= sb;
            f[(int64_t)i * L.n + k] = p;
        }
    }
}

// FP64 mass and momentum of the post-collision state over fluid nodes:
// per-block partial sums [mass A, mass B, px, py, pz].  FP16: decoded with
// rho_enc = cscale * rho of the writing step.
template <bool HALF>
__global__ __launch_bounds__(256) void k_reduce_fluid(const PopT<HALF>* __restrict__ f, const float* __restrict__ renc,
                                                      const float* __restrict__ cscale, int par,
                                                      double* __restrict__ partial, Lattice L) {
    __shared__ double sh[5][256];
    double acc[5] = {0, 0, 0, 0, 0};
    const int64_t plane = (int64_t)L.nx * L.ny;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < L.n;
         k += (int64_t)gridDim.x * blockDim.x) {
        if (L.walls) {
            const int y = (int)((k % plane) / L.nx);
            if (y == 0 || y == L.ny - 1) continue;
        }
        const double r[2] = {HALF ? (double)(cscale[2 * par] * renc[k]) : 1.0,
                             HALF ? (double)(cscale[2 * par + 1] * renc[L.n + k]) : 1.0};
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const PopT<HALF> p = f[(int64_t)i * L.n + k];
            const double g[2] = {(double)(float)p.x, (double)(float)p.y};
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const double v = HALF ? r[c] * ((double)wgt(i) + g[c]) : g[c];
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


// ---------------------------------------------------------------------------
// Discrete adjoint of the lattice part of one step (FP32 storage).  Given
// lambda* (adjoint of this step's output f*^n) and lambda_u (adjoint of u^n
// where the immersed boundary reads it), the three kernels below produce
// lambda* of the step's input f*^{n-1}:
//   k_adj_collide  per node: adjoint of u = (sum j + F/2)/rho, of the BGK
//                  collision with the shifted equilibrium, of the common
//                  velocity, and of F^c = -G rho^c S^c' + (rho^c/rho) F_ib;
//                  leaves lambda_rho (local part), lambda_j, lambda_S and
//                  lambda_Fib, and the G derivative of the Shan-Chen force;
//   k_adj_gather   transpose of S^c(x) = sum_i w_i psi^c(x + c_i) c_i:
//                  lambda_rho^c(y) += sum_i w_i c_i . lambda_S^c(y - c_i);
//   k_adj_push     transpose of the pull (with the wall bounce-back and its
//                  density term): lambda*_old_k(y) = lambda_f_k(y + c_k),
//                  lambda_f_i = (1 - omega) lambda*_i + lambda_rho + lambda_j . c_i.

__device__ __forceinline__ double block_sum_d(double v, double* sh, int tid, int nt) {
    sh[tid] = v;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
        if (tid < s) sh[tid] += sh[tid + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

template <bool WALLS, bool IBM, bool PSI>
__global__ __launch_bounds__(BX * BY) void k_adj_collide(const pf2* __restrict__ fin, const float* __restrict__ rho_n,
                                                     const float* __restrict__ rho_p, const float* __restrict__ fib,
                                                     const int* __restrict__ tile_flag, const pf2* __restrict__ lam_in,
                                                     const float* __restrict__ lam_u, float* __restrict__ lam_rho,
                                                     float* __restrict__ lam_j, float* __restrict__ lam_S,
                                                     float* __restrict__ lam_Fib, float* __restrict__ u_out,
                                                     double* __restrict__ grads, Lattice L) {
    __shared__ Ring2 sp;
    __shared__ double red[BX * BY];
    const int tx = threadIdx.x, ty = uniform_ty(), tid = ty * BX + tx;
    int bx, by, bz;
    block_xyz(bx, by, bz);
    const int x0 = bx * BX, y0 = by * BY, z0 = bz * L.zc;
    const int z1 = min(z0 + L.zc, L.nz);
    const int64_t N = L.n;
    bool near_ibm = false;
    if (IBM) {
        const int tx0 = wrapi(x0 - 1, L.nx) >> 3, ntx_b = (BX + 2 + 7) / 8 + 1;
        const int ty0 = wrapi(y0 - 1, L.ny) >> 3, nty_b = (BY + 2 + 7) / 8 + 1;
        const int tz0 = wrapi(z0 - 1, L.nz) >> 3, ntz_b = (L.zc + 2 + 7) / 8 + 1;
        bool hit = false;
        for (int k = tid; k < ntx_b * nty_b * ntz_b; k += BX * BY) {
            const int i = k % ntx_b, j = (k / ntx_b) % nty_b, l = k / (ntx_b * nty_b);
            const int t = (((tz0 + l) % L.ntz) * L.nty + (ty0 + j) % L.nty) * L.ntx + (tx0 + i) % L.ntx;
            hit = hit || tile_flag[t] != 0;
        }
        near_ibm = __syncthreads_or(hit) != 0;
    }
    const StagePos P = stage_positions<WALLS>(x0, y0, tid, L);
    StageRegs<2> np;
    auto stage = [&](int zz) {
        if (IBM && near_ibm)
            stage_load<true, 2, PSI>(np, P, zz, tid, rho_n, nullptr, fib, tile_flag, L);
        else
            stage_load<false, 2, PSI>(np, P, zz, tid, rho_n, nullptr, nullptr, nullptr, L);
        stage_store2(sp, np, zz, z0, tid);
    };
    stage(z0 - 1);
    stage(z0);
    const int x = x0 + tx, y = y0 + ty;
    const bool active = x < L.nx && y < L.ny && (!WALLS || (y > 0 && y < L.ny - 1));
    double gG = 0.0;
    Raw<false> rcur;
#pragma unroll 1
    for (int z = z0; z < z1; ++z) {
        stage(z + 1);
        __syncthreads();
        if (active) load_raw<WALLS, false>(fin, L, 0, x, y, z, rcur);
        if (active) {
            const uint32_t row = (uint32_t)((z * L.ny + y) * L.nx), xo = (uint32_t)x;
            const int s0 = (z - z0 + 1) % 3;
            Pulled A, B;
            auto none = [](int, int, int, float&, float&) {};
            decode<WALLS, false>(L, y, rcur, WALLS ? ldx(rho_p + row, xo) : 0.0f,
                                 WALLS ? ldx(rho_p + N + row, xo) : 0.0f, none, A, B);
            const float ra = sum_pop(A), rb = sum_pop(B);
            float ja[3], jb[3];
            momentum(A, ja[0], ja[1], ja[2]);
            momentum(B, jb[0], jb[1], jb[2]);
            float sa[3] = {0.f, 0.f, 0.f}, sb[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 1; k < Q; k += 2) {
                const int sP = (s0 + cz(k) + 3) % 3, sM = (s0 - cz(k) + 3) % 3;
                const int ly = ty + 1, lx = tx + 1;
                const float2 vp = sp.v[sP][ly + cy(k)][lx + cx(k)], vm = sp.v[sM][ly - cy(k)][lx - cx(k)];
                const float da = vp.x - vm.x, db = vp.y - vm.y;
                const float w = wgt(k);
                if (cx(k) != 0) { sa[0] += w * cx(k) * da; sb[0] += w * cx(k) * db; }
                if (cy(k) != 0) { sa[1] += w * cy(k) * da; sb[1] += w * cy(k) * db; }
                if (cz(k) != 0) { sa[2] += w * cz(k) * da; sb[2] += w * cz(k) * db; }
            }
            const float rs = ra + rb, ir = 1.0f / rs;
            float Fib[3] = {0.f, 0.f, 0.f};
            bool flagged = false;
            if (IBM && near_ibm) {
                const int t = ((z >> 3) * L.nty + (y >> 3)) * L.ntx + (x >> 3);
                flagged = tile_flag[t] != 0;
                if (flagged)
                    for (int d = 0; d < 3; ++d) Fib[d] = ldx(fib + d * N + row, xo);
            }
            const float ma = ra * ir, mb = rb * ir;
            // pseudo-potentials and their slopes (exp form: d psi / d rho = 1 - psi)
            const float pa = PSI ? psi_exp(ra) : ra, pb = PSI ? psi_exp(rb) : rb;
            const float dpa = PSI ? 1.0f - pa : 1.0f, dpb = PSI ? 1.0f - pb : 1.0f;
            float Fa[3], Fb[3];
            for (int d = 0; d < 3; ++d) {
                Fa[d] = -L.G * pa * sb[d] + ma * Fib[d];
                Fb[d] = -L.G * pb * sa[d] + mb * Fib[d];
            }
            const float wa = L.omega[0], wb = L.omega[1];
            const float Dn = ra * wa + rb * wb, iD = 1.0f / Dn;
            float up[3], u[3], ue[2][3];
            for (int d = 0; d < 3; ++d) {
                up[d] = (ja[d] * wa + jb[d] * wb) * iD;
                u[d] = (ja[d] + jb[d] + 0.5f * (Fa[d] + Fb[d])) * ir;
                ue[0][d] = up[d] + L.tau[0] * Fa[d] / ra;
                ue[1][d] = up[d] + L.tau[1] * Fb[d] / rb;
            }
            // adjoint of u = (sum j + F/2) / rho; u itself is left where the
            // membrane adjoint reads it
            float lu[3] = {0.f, 0.f, 0.f};
            if (flagged)
                for (int d = 0; d < 3; ++d) {
                    lu[d] = ldx(lam_u + d * N + row, xo);
                    *ptrx(u_out + d * N + row, xo) = u[d];
                }
            float lj[2][3], lF[2][3], lr[2];
            const float luu = (lu[0] * u[0] + lu[1] * u[1] + lu[2] * u[2]) * ir;
            for (int c = 0; c < 2; ++c) {
                lr[c] = -luu;
                for (int d = 0; d < 3; ++d) {
                    lj[c][d] = lu[d] * ir;
                    lF[c][d] = 0.5f * lu[d] * ir;
                }
            }
            // adjoint of the collision f* = f + omega (feq(rho, u_eq) - f)
            float lup[3] = {0.f, 0.f, 0.f};
            const float r2[2] = {ra, rb};
            for (int c = 0; c < 2; ++c) {
                const float om = L.omega[c], r = r2[c];
                const float usq = ue[c][0] * ue[c][0] + ue[c][1] * ue[c][1] + ue[c][2] * ue[c][2];
                float lrf = 0.f, lue[3] = {0.f, 0.f, 0.f};
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    const pf2 lv = ldx(lam_in + (int64_t)i * N + row, xo);
                    const float mu = om * (c == 0 ? lv.x : lv.y);
                    const float eu = cdot(i, ue[c][0], ue[c][1], ue[c][2]);
                    lrf += mu * wgt(i) * (1.0f + 3.0f * eu + 4.5f * eu * eu - 1.5f * usq);
                    const float co = mu * wgt(i) * r;
                    const float ce = co * (3.0f + 9.0f * eu);
                    if (cx(i)) lue[0] += ce * cx(i);
                    if (cy(i)) lue[1] += ce * cy(i);
                    if (cz(i)) lue[2] += ce * cz(i);
                    lue[0] -= 3.0f * co * ue[c][0];
                    lue[1] -= 3.0f * co * ue[c][1];
                    lue[2] -= 3.0f * co * ue[c][2];
                }
                lr[c] += lrf;
                const float* F = c == 0 ? Fa : Fb;
                float lueF = 0.f;
                for (int d = 0; d < 3; ++d) {
                    lup[d] += lue[d];
                    lF[c][d] += L.tau[c] * lue[d] / r;
                    lueF += lue[d] * F[d];
                }
                lr[c] -= L.tau[c] * lueF / (r * r);
            }
            // adjoint of the common velocity u' = sum_c omega_c j^c / sum_c omega_c rho^c
            const float lupu = (lup[0] * up[0] + lup[1] * up[1] + lup[2] * up[2]) * iD;
            for (int c = 0; c < 2; ++c) {
                const float om = L.omega[c];
                for (int d = 0; d < 3; ++d) lj[c][d] += om * lup[d] * iD;
                lr[c] -= om * lupu;
            }
            // adjoint of F^c = -G rho^c S^c' + m^c F_ib
            float lSa[3], lSb[3];
            for (int d = 0; d < 3; ++d) {
                lSb[d] = -L.G * pa * lF[0][d];     // S of B enters the force on A
                lSa[d] = -L.G * pb * lF[1][d];
            }
            lr[0] += -L.G * dpa * (lF[0][0] * sb[0] + lF[0][1] * sb[1] + lF[0][2] * sb[2]);
            lr[1] += -L.G * dpb * (lF[1][0] * sa[0] + lF[1][1] * sa[1] + lF[1][2] * sa[2]);
            gG += -(double)pa * (lF[0][0] * sb[0] + lF[0][1] * sb[1] + lF[0][2] * sb[2])
                  - (double)pb * (lF[1][0] * sa[0] + lF[1][1] * sa[1] + lF[1][2] * sa[2]);
            if (flagged) {
                float lma = 0.f, lmb = 0.f;
                for (int d = 0; d < 3; ++d) {
                    *ptrx(lam_Fib + d * N + row, xo) = ma * lF[0][d] + mb * lF[1][d];
                    lma += lF[0][d] * Fib[d];
                    lmb += lF[1][d] * Fib[d];
                }
                const float ir2 = ir * ir;
                lr[0] += (lma - lmb) * rb * ir2;
                lr[1] += (lmb - lma) * ra * ir2;
            }
            *ptrx(lam_rho + row, xo) = lr[0];
            *ptrx(lam_rho + N + row, xo) = lr[1];
            for (int d = 0; d < 3; ++d) {
                *ptrx(lam_j + d * N + row, xo) = lj[0][d];
                *ptrx(lam_j + (3 + d) * N + row, xo) = lj[1][d];
                *ptrx(lam_S + d * N + row, xo) = lSa[d];
                *ptrx(lam_S + (3 + d) * N + row, xo) = lSb[d];
            }
        }
        __syncthreads();
    }
    const double tot = block_sum_d(gG, red, tid, BX * BY);
    if (tid == 0 && tot != 0.0) unsafeAtomicAdd(&grads[2], tot);
}

// lambda_rho^c(y) += sum_i w_i c_i . lambda_S^c(y - c_i); with walls, the
// first and last fluid rows also collect what their solid-row copies
// received.
template <bool WALLS, bool PSI>
__global__ __launch_bounds__(BX * BY) void k_adj_gather(const float* __restrict__ lam_S, float* __restrict__ lam_rho,
                                                    const float* __restrict__ rho_n, Lattice L) {
    __shared__ Ring<6> sr;
    const int tx = threadIdx.x, ty = uniform_ty(), tid = ty * BX + tx;
    int bx, by, bz;
    block_xyz(bx, by, bz);
    const int x0 = bx * BX, y0 = by * BY, z0 = bz * L.zc;
    const int z1 = min(z0 + L.zc, L.nz);
    const int64_t N = L.n;
    const StagePos P = stage_positions<false>(x0, y0, tid, L);
    StageRegs<6> st;
    auto stage = [&](int zz) {
        stage_load<false, 6>(st, P, zz, tid, lam_S, nullptr, nullptr, nullptr, L);
        stage_store<6>(sr, st, zz, z0, tid);
    };
    stage(z0 - 1);
    stage(z0);
    const int x = x0 + tx, y = y0 + ty;
    const bool active = x < L.nx && y < L.ny && (!WALLS || (y > 0 && y < L.ny - 1));
#pragma unroll 1
    for (int z = z0; z < z1; ++z) {
        stage(z + 1);
        __syncthreads();
        if (active) {
            const uint32_t row = (uint32_t)((z * L.ny + y) * L.nx), xo = (uint32_t)x;
            const int s0 = (z - z0 + 1) % 3;
            const int ly = ty + 1, lx = tx + 1;
            float acc[2] = {0.f, 0.f};
#pragma unroll
            for (int k = 1; k < Q; k += 2) {
                const int sM = (s0 - cz(k) + 3) % 3, sP = (s0 + cz(k) + 3) % 3;
                for (int c = 0; c < 2; ++c) {
                    float v = 0.f;
                    for (int d = 0; d < 3; ++d) {
                        const int e = d == 0 ? cx(k) : (d == 1 ? cy(k) : cz(k));
                        if (e == 0) continue;
                        v += e * (sr.v[sM][3 * c + d][ly - cy(k)][lx - cx(k)] - sr.v[sP][3 * c + d][ly + cy(k)][lx + cx(k)]);
                    }
                    acc[c] += wgt(k) * v;
                }
            }
            if (WALLS && (y == 1 || y == L.ny - 2)) {
                // sources x = s - c_i of the solid neighbour s, for the directions
                // that pointed from the fluid row into the solid row
                const int sgn = y == 1 ? -1 : 1;
#pragma unroll
                for (int i = 1; i < Q; ++i) {
                    if (cy(i) != sgn) continue;
                    const int sl = (s0 - cz(i) + 3) % 3;
                    for (int c = 0; c < 2; ++c) {
                        float v = 0.f;
                        for (int d = 0; d < 3; ++d) {
                            const int e = d == 0 ? cx(i) : (d == 1 ? cy(i) : cz(i));
                            if (e) v += e * sr.v[sl][3 * c + d][ly][lx - cx(i)];
                        }
                        acc[c] += wgt(i) * v;
                    }
                }
            }
            if constexpr (PSI) {
                // the gathered sum is the adjoint of the pseudo-potential; its
                // density part carries d psi / d rho = exp(-rho) = 1 - psi
                acc[0] *= 1.0f - psi_exp(ldx(rho_n + row, xo));
                acc[1] *= 1.0f - psi_exp(ldx(rho_n + N + row, xo));
            }
            *ptrx(lam_rho + row, xo) += acc[0];
            *ptrx(lam_rho + N + row, xo) += acc[1];
        }
        __syncthreads();
    }
}

template <bool WALLS>
__global__ __launch_bounds__(BX * BY) void k_adj_push(const pf2* __restrict__ lam_in, const float* __restrict__ lam_rho,
                                                  const float* __restrict__ lam_j, pf2* __restrict__ lam_out,
                                                  Lattice L) {
    __shared__ Ring<8> rj;
    const int tx = threadIdx.x, ty = uniform_ty(), tid = ty * BX + tx;
    int bx, by, bz;
    block_xyz(bx, by, bz);
    const int x0 = bx * BX, y0 = by * BY, z0 = bz * L.zc;
    const int z1 = min(z0 + L.zc, L.nz);
    const int64_t N = L.n;
    // lambda_rho and lambda_j share one 8-field ring (fields 0-1 and 2-7);
    // the positions wrap periodically in y as the push reads them
    const StagePos P = stage_positions<false>(x0, y0, tid, L);
    StageRegs<2> sr2;
    StageRegs<6> sr6;
    auto stage = [&](int zz) {
        stage_load<false, 2>(sr2, P, zz, tid, lam_rho, nullptr, nullptr, nullptr, L);
        stage_load<false, 6>(sr6, P, zz, tid, lam_j, nullptr, nullptr, nullptr, L);
        stage_store<2, 8, 0>(rj, sr2, zz, z0, tid);
        stage_store<6, 8, 2>(rj, sr6, zz, z0, tid);
    };
    stage(z0 - 1);
    stage(z0);
    const int x = x0 + tx, y = y0 + ty;
    const bool inside = x < L.nx && y < L.ny;
    const bool active = inside && (!WALLS || (y > 0 && y < L.ny - 1));
#pragma unroll 1
    for (int z = z0; z < z1; ++z) {
        stage(z + 1);
        __syncthreads();
        if (active) {
            const uint32_t row = (uint32_t)((z * L.ny + y) * L.nx), xo = (uint32_t)x;
            const int s0 = (z - z0 + 1) % 3;
            const int ly = ty + 1, lx = tx + 1;
            int xm = x == 0 ? L.nx - 1 : x - 1, xp = x == L.nx - 1 ? 0 : x + 1, xc = x;
            // fresh lane offsets per plane (scalar row base plus 32-bit x)
            asm volatile("" : "+v"(xm), "+v"(xc), "+v"(xp));
            const int ym = y == 0 ? L.ny - 1 : y - 1, yp = y == L.ny - 1 ? 0 : y + 1;
            const int zm = z == 0 ? L.nz - 1 : z - 1, zp = z == L.nz - 1 ? 0 : z + 1;
            // own lambda_f_i for the bounced directions and the wall density term
            auto own_lf = [&](int i, int c) {
                const pf2 lv = ldx(lam_in + (int64_t)i * N + row, xo);
                const float ls = c == 0 ? lv.x : lv.y;
                const float lj = cdot(i, rj.v[s0][2 + 3 * c][ly][lx], rj.v[s0][3 + 3 * c][ly][lx],
                                      rj.v[s0][4 + 3 * c][ly][lx]);
                return (1.0f - L.omega[c]) * ls + rj.v[s0][c][ly][lx] + lj;
            };
            float wall_extra[2] = {0.f, 0.f};
            if (WALLS && (y == 1 || y == L.ny - 2)) {
                const int sgn = y == 1 ? 1 : -1;      // directions pulled from the solid row
                for (int i = 1; i < Q; ++i) {
                    if (cy(i) != sgn) continue;
                    const float* uw = sgn == 1 ? L.uw_lo : L.uw_hi;
                    const float cu = cdot(i, uw[0], uw[1], uw[2]);
                    for (int c = 0; c < 2; ++c) wall_extra[c] += own_lf(i, c) * 2.0f * wgt(i) * cu * 3.0f;
                }
            }
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                float out[2];
                const bool into_wall = WALLS && ((cy(k) == -1 && y == 1) || (cy(k) == 1 && y == L.ny - 2));
                if (into_wall) {
                    out[0] = own_lf(opp(k), 0);
                    out[1] = own_lf(opp(k), 1);
                } else {
                    const int sx = cx(k) == 1 ? xp : (cx(k) == -1 ? xm : xc);
                    const int sy = cy(k) == 1 ? yp : (cy(k) == -1 ? ym : y);
                    const int sz = cz(k) == 1 ? zp : (cz(k) == -1 ? zm : z);
                    const pf2 lv = ldx(lam_in + (int64_t)k * N + (uint32_t)((sz * L.ny + sy) * L.nx), (uint32_t)sx);
                    const int sl = (s0 + cz(k) + 3) % 3, qy = ly + cy(k), qx = lx + cx(k);
                    for (int c = 0; c < 2; ++c) {
                        const float lj = cdot(k, rj.v[sl][2 + 3 * c][qy][qx], rj.v[sl][3 + 3 * c][qy][qx],
                                              rj.v[sl][4 + 3 * c][qy][qx]);
                        out[c] = (1.0f - L.omega[c]) * (c == 0 ? lv.x : lv.y) + rj.v[sl][c][qy][qx] + lj;
                    }
                }
                *ptrx(lam_out + (int64_t)k * N + row, xo) = pack<false>(out[0] + wall_extra[0], out[1] + wall_extra[1]);
            }
        } else if (inside) {
            const uint32_t row = (uint32_t)((z * L.ny + y) * L.nx);
            for (int k = 0; k < Q; ++k) *ptrx(lam_out + (int64_t)k * N + row, (uint32_t)x) = pack<false>(0.f, 0.f);
        }
        __syncthreads();
    }
}

}  // namespace

// On-site velocity boundaries on the rows y = 0 and y = ny - 1 (Zou and He,
// in the D3Q19 form of Hecht and Harting).  One thread per boundary node,
// after the collide (and once after initialisation).  The next pull brings
// each boundary node its unknown populations (c_y = +1 at y = 0, c_y = -1 at
// y = ny - 1) from the opposite boundary row through the periodic
// addressing; those slots hold populations that leave the box and that
// nothing else reads, so the closure is stored there:
//   rho = (Z + 2 O) / (1 - s u_y),   s = c_y of the unknowns,
//   f_i = f_opp(i) + 6 w_i rho (c_i . u) - c_ix N_x - c_iz N_z,
//   N_x = (1/2) sum_{c_y = 0} f c_x - rho u_x / 3 (N_z alike),
// Z the sum of the known populations with c_y = 0 and O of those with
// c_y = -s, all as the pull will deliver them.  The slots read (rows 0 and 1,
// ny - 2 and ny - 1, directions with c_y != s) and the slots written (c_y =
// +1 in row ny - 1, c_y = -1 in row 0) are disjoint.
// FP16 form: a pulled value decodes with its source node's compensated
// density cs * rho_enc, as in the lattice kernels; the decoders stage the
// densities of a source beyond the box from the boundary row itself (the
// clamp that also serves the Shan-Chen neighbours), so the unknowns are
// encoded with the density of the boundary node x - c at the same row.
template <bool HALF>
__global__ __launch_bounds__(256) void k_onsite(PopT<HALF>* __restrict__ f, const float* __restrict__ rho_enc,
                                                const float* __restrict__ cs, Lattice L) {
    const int64_t per = (int64_t)L.nx * L.nz;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= 2 * per) return;
    const int top = t >= per ? 1 : 0;
    const int rem = (int)(t - top * per);
    const int z = rem / L.nx, x = rem - z * L.nx;
    const int yb = top ? L.ny - 1 : 0;
    const int s = top ? -1 : 1;
    const float uw[3] = {top ? L.uw_hi[0] : L.uw_lo[0], top ? L.uw_hi[1] : L.uw_lo[1],
                         top ? L.uw_hi[2] : L.uw_lo[2]};
    const float sca = HALF ? cs[0] : 1.0f, scb = HALF ? cs[1] : 1.0f;
    float fa[Q], fb[Q];
    float Za = 0.f, Zb = 0.f, Oa = 0.f, Ob = 0.f, Xa = 0.f, Xb = 0.f, Wa = 0.f, Wb = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        fa[i] = fb[i] = 0.0f;
        if (cy(i) == s) continue;
        const int sx = wrapi(x - cx(i), L.nx), sy = yb - cy(i), sz = wrapi(z - cz(i), L.nz);
        const int64_t node = ((int64_t)sz * L.ny + sy) * L.nx + sx;
        const PopT<HALF> v = f[i * L.n + node];
        if (HALF) {
            const float ea = sca * rho_enc[node], eb = scb * rho_enc[L.n + node];
            fa[i] = fmaf(ea, (float)v.x, ea * wgt(i));
            fb[i] = fmaf(eb, (float)v.y, eb * wgt(i));
        } else {
            fa[i] = (float)v.x;
            fb[i] = (float)v.y;
        }
        if (cy(i) == 0) {
            Za += fa[i]; Zb += fb[i];
            Xa += cx(i) * fa[i]; Xb += cx(i) * fb[i];
            Wa += cz(i) * fa[i]; Wb += cz(i) * fb[i];
        } else {
            Oa += fa[i]; Ob += fb[i];
        }
    }
    const float inv = 1.0f / (1.0f - s * uw[1]);
    const float ra = (Za + 2.0f * Oa) * inv, rb = (Zb + 2.0f * Ob) * inv;
    const float nxa = 0.5f * Xa - ra * uw[0] / 3.0f, nxb = 0.5f * Xb - rb * uw[0] / 3.0f;
    const float nza = 0.5f * Wa - ra * uw[2] / 3.0f, nzb = 0.5f * Wb - rb * uw[2] / 3.0f;
    const int yd = top ? 0 : L.ny - 1;          // the row the unknowns are pulled from
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (cy(i) != s) continue;
        const float cu = cx(i) * uw[0] + cy(i) * uw[1] + cz(i) * uw[2];
        float va = fa[opp(i)] + 6.0f * wgt(i) * ra * cu - cx(i) * nxa - cz(i) * nza;
        float vb = fb[opp(i)] + 6.0f * wgt(i) * rb * cu - cx(i) * nxb - cz(i) * nzb;
        const int sx = wrapi(x - cx(i), L.nx), sz = wrapi(z - cz(i), L.nz);
        if (HALF) {
            const int64_t enc = ((int64_t)sz * L.ny + yb) * L.nx + sx;
            va = va / (sca * rho_enc[enc]) - wgt(i);
            vb = vb / (scb * rho_enc[L.n + enc]) - wgt(i);
        }
        f[i * L.n + ((int64_t)sz * L.ny + yd) * L.nx + sx] = pack<HALF>(va, vb);
    }
}

void launch_onsite(const Lattice& L, void* f, bool half, const float* rho_enc, const float* cs, hipStream_t s) {
    const int64_t n = 2 * (int64_t)L.nx * L.nz;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (half)
        hipLaunchKernelGGL(k_onsite<true>, grid, block, 0, s, (ph2*)f, rho_enc, cs, L);
    else
        hipLaunchKernelGGL(k_onsite<false>, grid, block, 0, s, (pf2*)f, rho_enc, cs, L);
}

void launch_init_rest(const Lattice& L, void* f, const float* rhoA, const float* rhoB, bool half,
                      hipStream_t s) {
    const int64_t blocks = std::min<int64_t>((L.n + 255) / 256, 65536);
    if (half)
        hipLaunchKernelGGL(k_init_rest<true>, dim3((unsigned)blocks), dim3(256), 0, s, (ph2*)f, rhoA, rhoB, L.n);
    else
        hipLaunchKernelGGL(k_init_rest<false>, dim3((unsigned)blocks), dim3(256), 0, s, (pf2*)f, rhoA, rhoB, L.n);
}

int64_t density_blocks(const Lattice& L, bool half) {
    return (int64_t)((L.nx + BX - 1) / BX) * ((L.ny + BY - 1) / BY) * (half ? (L.nz + L.zc - 1) / L.zc : L.nz);
}

void launch_density(const Lattice& L, const void* fin, const float* rho_prev, float* rho_out, bool half,
                    const float* cscale, int par_prev, double* partial, hipStream_t s) {
    const dim3 grid((L.nx + BX - 1) / BX, (L.ny + BY - 1) / BY, half ? (L.nz + L.zc - 1) / L.zc : L.nz);
    const dim3 block(BX, BY);
#define LD_H(W, C)                                                                                            \
    hipLaunchKernelGGL((k_density_half<W, C>), grid, block, 0, s, (const ph2*)fin, rho_prev, cscale, par_prev, \
                       rho_out, partial, L)
#define LD_F(W, C) hipLaunchKernelGGL((k_density<W, C>), grid, block, 0, s, (const pf2*)fin, rho_prev, rho_out, L)
    const bool w = L.walls != 0, c = L.cached != 0;
    if (half) {
        if (w) { if (c) LD_H(true, true); else LD_H(true, false); }
        else { if (c) LD_H(false, true); else LD_H(false, false); }
    } else {
        if (w) { if (c) LD_F(true, true); else LD_F(true, false); }
        else { if (c) LD_F(false, true); else LD_F(false, false); }
    }
#undef LD_F
#undef LD_H
}

void launch_density_tiles(const Lattice& L, const void* fin, float* rho_out, const int* touched, const int* count,
                          const int* tile_flag, hipStream_t s) {
    const int dil = (L.nx % TILE || L.ny % TILE || L.nz % TILE) ? 1 : 0;
    hipLaunchKernelGGL(k_density_tiles, dim3(2048), dim3(256), 0, s, (const pf2*)fin, rho_out, touched, count,
                       tile_flag, dil, L);
}

void launch_compensate(const Lattice& L, const double* partial, double m0a, double m0b, float* cscale, int par_cur,
                       double* mass_out, hipStream_t s) {
    const int nb = (int)density_blocks(L, true);
    hipLaunchKernelGGL(k_compensate, dim3(1), dim3(1024), 0, s, partial, nb, m0a, m0b, cscale, par_cur, mass_out);
}

template <bool W, bool I, bool M, bool H, bool P, bool S = false>
static void launch_collide_t(const Lattice& L, const void* fin, void* fout, const float* rho_n,
                             const float* rho_prev, const float* fib, const int* tile_flag, float* u,
                             const float* cscale, int par_prev, int par_cur, hipStream_t s) {
    dim3 grid((L.nx + BX - 1) / BX, (L.ny + BY - 1) / BY, (L.nz + L.zc - 1) / L.zc);
    dim3 block(BX, BY);
    if constexpr (!W && !M && !H && !S) {
        if (L.one) {
            if (L.cached)
                hipLaunchKernelGGL((k_collide_one<I, true, P>), grid, block, 0, s, (const pf2*)fin, (pf2*)fout, rho_n,
                                   rho_prev, fib, tile_flag, u, cscale, par_prev, par_cur, L);
            else
                hipLaunchKernelGGL((k_collide_one<I, false, P>), grid, block, 0, s, (const pf2*)fin, (pf2*)fout, rho_n,
                                   rho_prev, fib, tile_flag, u, cscale, par_prev, par_cur, L);
            return;
        }
    }
    // the velocity read-back (M) writes no populations; it runs in one policy
    if constexpr (!M) {
        if (L.cached) {
            hipLaunchKernelGGL((k_collide<W, I, M, H, true, P, S>), grid, block, 0, s, (const PopT<H>*)fin,
                               (PopT<H>*)fout, rho_n, rho_prev, fib, tile_flag, u, cscale, par_prev, par_cur, L);
            return;
        }
    }
    hipLaunchKernelGGL((k_collide<W, I, M, H, false, P, S>), grid, block, 0, s, (const PopT<H>*)fin,
                       (PopT<H>*)fout, rho_n, rho_prev, fib, tile_flag, u, cscale, par_prev, par_cur, L);
}

void launch_collide(const Lattice& L, const void* fin, void* fout, const float* rho_n, const float* rho_prev,
                    const float* fib, const int* tile_flag, float* u, bool has_ibm, bool macro, bool half,
                    const float* cscale, int par_prev, int par_cur, hipStream_t s) {
    const bool w = L.walls != 0;
    if (L.sharp) {
        // the bounce-back coupling: periodic, FP32 storage
#define LS(M, P) launch_collide_t<false, true, M, false, P, true>(L, fin, fout, rho_n, rho_prev, fib, tile_flag, u, \
                                                                  cscale, par_prev, par_cur, s)
        if (macro) {
            if (L.psi_exp) LS(true, true); else LS(true, false);
        } else {
            if (L.psi_exp) LS(false, true); else LS(false, false);
        }
#undef LS
        return;
    }
#define LC(W, I, M, H, P) \
    launch_collide_t<W, I, M, H, P>(L, fin, fout, rho_n, rho_prev, fib, tile_flag, u, cscale, par_prev, par_cur, s)
#define LC_P(W, I, M, H) \
    do { if (L.psi_exp) LC(W, I, M, H, true); else LC(W, I, M, H, false); } while (0)
#define LC_H(W, I, M) \
    do { if (half) LC_P(W, I, M, true); else LC_P(W, I, M, false); } while (0)
#define LC_I(W, M) \
    do { if (has_ibm) LC_H(W, true, M); else LC_H(W, false, M); } while (0)
    if (macro) {
        if (w) LC_I(true, true); else LC_I(false, true);
    } else {
        if (w) LC_I(true, false); else LC_I(false, false);
    }
#undef LC_I
#undef LC_H
#undef LC_P
#undef LC
}

void launch_reduce_fluid(const Lattice& L, const void* fpost, bool half, const float* renc, const float* cscale,
                         int par, double* partial, hipStream_t s) {
    if (half)
        hipLaunchKernelGGL(k_reduce_fluid<true>, dim3(RED_BLOCKS), dim3(256), 0, s, (const ph2*)fpost, renc,
                           cscale, par, partial, L);
    else
        hipLaunchKernelGGL(k_reduce_fluid<false>, dim3(RED_BLOCKS), dim3(256), 0, s, (const pf2*)fpost, renc,
                           cscale, par, partial, L);
}

void launch_scale_pops(const Lattice& L, void* f, float sa, float sb, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_pops, dim3(RED_BLOCKS), dim3(256), 0, s, (pf2*)f, sa, sb, L);
}

template <bool W, bool P>
static void launch_adj_collide_t(const Lattice& L, const void* fin, const float* rho_n, const float* rho_p,
                                 const float* fib, const int* tile_flag, const void* lam_in, const float* lam_u,
                                 float* lam_rho, float* lam_j, float* lam_S, float* lam_Fib, float* u_out,
                                 double* grads, hipStream_t s) {
    dim3 grid((L.nx + BX - 1) / BX, (L.ny + BY - 1) / BY, (L.nz + L.zc - 1) / L.zc), block(BX, BY);
    hipLaunchKernelGGL((k_adj_collide<W, true, P>), grid, block, 0, s, (const pf2*)fin, rho_n, rho_p, fib,
                       tile_flag, (const pf2*)lam_in, lam_u, lam_rho, lam_j, lam_S, lam_Fib, u_out, grads, L);
}
void launch_adj_collide(const Lattice& L, const void* fin, const float* rho_n, const float* rho_p, const float* fib,
                        const int* tile_flag, const void* lam_in, const float* lam_u, float* lam_rho, float* lam_j,
                        float* lam_S, float* lam_Fib, float* u_out, double* grads, hipStream_t s) {
#define AC(W, P) launch_adj_collide_t<W, P>(L, fin, rho_n, rho_p, fib, tile_flag, lam_in, lam_u, lam_rho, lam_j, \
                                            lam_S, lam_Fib, u_out, grads, s)
    if (L.walls) {
        if (L.psi_exp) AC(true, true); else AC(true, false);
    } else {
        if (L.psi_exp) AC(false, true); else AC(false, false);
    }
#undef AC
}
void launch_adj_gather(const Lattice& L, const float* lam_S, float* lam_rho, const float* rho_n, hipStream_t s) {
    dim3 grid((L.nx + BX - 1) / BX, (L.ny + BY - 1) / BY, (L.nz + L.zc - 1) / L.zc), block(BX, BY);
#define AG(W, P) hipLaunchKernelGGL((k_adj_gather<W, P>), grid, block, 0, s, lam_S, lam_rho, rho_n, L)
    if (L.walls) {
        if (L.psi_exp) AG(true, true); else AG(true, false);
    } else {
        if (L.psi_exp) AG(false, true); else AG(false, false);
    }
#undef AG
}

void launch_adj_push(const Lattice& L, const void* lam_in, const float* lam_rho, const float* lam_j, void* lam_out,
                     hipStream_t s) {
    dim3 grid((L.nx + BX - 1) / BX, (L.ny + BY - 1) / BY, (L.nz + L.zc - 1) / L.zc), block(BX, BY);
    if (L.walls)
        hipLaunchKernelGGL(k_adj_push<true>, grid, block, 0, s, (const pf2*)lam_in, lam_rho, lam_j, (pf2*)lam_out, L);
    else
        hipLaunchKernelGGL(k_adj_push<false>, grid, block, 0, s, (const pf2*)lam_in, lam_rho, lam_j, (pf2*)lam_out, L);
}

}  // namespace lbmx
