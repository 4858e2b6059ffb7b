// The paper's own fluid-structure coupling (gfx950): half-way bounce-back on
// the moving membrane (Sec. II.C, eqs. method:SBB and
// method:momentumtransfer), the Shan-Chen sum across it with densities
// interpolated from the viewer's side and the colour offset (Sec. II.D,
// eq. method:interpolateshanchen), fresh nodes with the adaptive mass
// correction (Sec. II.E, eqs. method:freshnodes and method:masscorrection)
// and the inertial node update (Sec. II.B, first-order Euler; node mass of
// Sec. III).  The lattice kernels are the immersed boundary's; the coupling
// works on the few lattice nodes next to each membrane.
//
// Head of step n (nodes at X^n, V^n; populations f*^{n-1}):
//   k_bb_box      per capsule: the anchor-relative box of its nodes widened by
//                 MARGIN, the mean node offset; counters and volumes zeroed
//   k_bb_overlap  per pair of capsules of one parity colour: their boxes
//                 must not meet (reported)
//   k_bb_clear    per box: new labels -1, parity bits 0, link keys empty
//   k_bb_links    per triangle and half-direction: the lattice links it
//                 pierces (FP64 Moeller-Trumbore over its bounding box, after
//                 a plane-side test); its centroid; for each link, its
//                 element is the triangle pierced nearest the
//                 link's start node (the end from which it points along a
//                 positive half-direction; lowest index among ties at single
//                 precision), for both of its ends; the parity of the
//                 crossings of each +z link, one bit per capsule colour
//   k_bb_list     per box cell: the links crossed there, listed once each
//                 (by the box of their element's capsule)
//   k_bb_label    per box column: inside where the +z crossings below by the
//                 capsule's own membrane (its colour's bit) are odd
//   k_bb_detect   per box: fresh nodes (label changed) listed, once each
//   k_bb_refill   per fresh node (a block each): the density
//                 interpolated from its side's non-fresh neighbours,
//                 mass-corrected and clamped to their range; the velocity of
//                 the nearest element (the threads share the search); the
//                 equilibrium populations; removed minus created momentum to
//                 the element
//   k_bb_commit   per box: labels := new labels
//   k_bb_link_density  per listed link: the densities of both ends, before
//                 any population is bounced
//   k_bb_fixup    per listed link whose ends differ in label: each end gets
//                 its own outgoing population back with the moving-element
//                 term, stored where its next pull reads; the exchanged
//                 momentum to the element's nodes
//   k_bb_ledger   the mass the step's refills and bounce-backs added, into
//                 the FP64 ledger the mass correction reads
// The mass correction needs each component's mass change since the start.
// Collision and streaming conserve mass exactly; only the moving-element
// bounce-back term and the fresh-node refills change it, so the library
// keeps that change as an FP64 ledger of those events (the same quantity in
// exact arithmetic).  A sum over the FP32 lattice would carry the storage's
// rounding, which the correction's gain (C0 sum rho_init / rho_init^c / V_sys,
// about 0.5 per unit of mass here) would turn into density changes of 1e-4
// at fresh nodes.
//   k_bb_unflag, k_bb_flag  tile flags reset; per box: Shan-Chen corrections
//                 zeroed, its tiles flagged for the collide
// In the step, after the density pass:
//   k_bb_sc       per listed crossing: the corrections dS of both ends'
//                 Shan-Chen sums for the neighbour across, the force those
//                 pairs would put on the far side to the element's nodes
//   (the collide adds dS inside flagged tiles)
//   k_bb_advance  per node: F = elastic + half this and half the last
//                 exchanged momentum + reactions; V += F / m (or the
//                 prescribed V); X += V
// Every element quantity goes to its three nodes in equal thirds (Sec. II.C).
#include "lbm_internal.h"

namespace lbmx {

namespace {

constexpr int MARGIN = 3;       // box margin around a capsule's nodes, lattice units
// Node offsets from a capsule's anchor beyond this (or not finite) mean the
// membrane has diverged: it is reported and its box left empty.
constexpr double COORD_MAX = 1048576.0;
constexpr int CNT_LINKS = 0, CNT_FRESH = 1, CNT_FLAGS = 2;
// overflow and consistency flags in bb_count[CNT_FLAGS]
constexpr int FLAG_BOX = 1, FLAG_LINKS = 2, FLAG_FRESH = 4, FLAG_PARITY = 8, FLAG_OVERLAP = 16;

__device__ __forceinline__ int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

__device__ __forceinline__ int64_t lat(const Lattice& L, int x, int y, int z) {
    return ((int64_t)wrapi(z, L.nz) * L.ny + wrapi(y, L.ny)) * L.nx + wrapi(x, L.nx);
}

// the same for coordinates within one cell of the lattice (-1 .. n)
__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
__device__ __forceinline__ int64_t lat1(const Lattice& L, int x, int y, int z) {
    return ((int64_t)wrap1(z, L.nz) * L.ny + wrap1(y, L.ny)) * L.nx + wrap1(x, L.nx);
}

// the D3Q19 direction of half-direction d = 0..8: +x, +y, +z and the six
// diagonals with a positive first non-zero component
__device__ __forceinline__ int half_dir(int d) { return 2 * d + 1; }

__device__ __forceinline__ void node_rel(const Dev& d, int b, double p[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) p[k] = (double)d.off_hi[3 * b + k] + (double)d.off_lo[3 * b + k];
}

__device__ __forceinline__ double psi_of(double r, int kind) { return kind ? 1.0 - exp(-r) : r; }

// A box cell of capsule `cap` for the linear cell index c, or false.
__device__ __forceinline__ bool box_cell(const Dev& d, int cap, int c, int q[3]) {
    const int* bx = d.bbox + 8 * cap;
    const int ex = bx[3] - bx[0] + 1, ey = bx[4] - bx[1] + 1, ez = bx[5] - bx[2] + 1;
    if (c >= ex * ey * ez) return false;
    q[0] = bx[0] + c % ex;
    q[1] = bx[1] + (c / ex) % ey;
    q[2] = bx[2] + c / (ex * ey);
    return true;
}

__device__ __forceinline__ void add3(double* a, const double v[3], double s) {
    unsafeAtomicAdd(a + 0, v[0] * s);
    unsafeAtomicAdd(a + 1, v[1] * s);
    unsafeAtomicAdd(a + 2, v[2] * s);
}

// ---- head of the step ----------------------------------------------------

__global__ __launch_bounds__(256) void k_bb_box(Dev d, int ext) {
    __shared__ double sh[7][256];
    const int cap = blockIdx.x;
    const CapDev& C = d.caps[cap];
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300}, sm[3] = {0, 0, 0};
    for (int b = C.node_start + threadIdx.x; b < C.node_start + C.node_count; b += blockDim.x) {
        double p[3];
        node_rel(d, b, p);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            mn[k] = fmin(mn[k], p[k]);
            mx[k] = fmax(mx[k], p[k]);
            sm[k] += p[k];
        }
    }
    for (int k = 0; k < 3; ++k) {
        sh[k][threadIdx.x] = mn[k];
        sh[3 + k][threadIdx.x] = mx[k];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int k = 0; k < 3; ++k) {
                sh[k][threadIdx.x] = fmin(sh[k][threadIdx.x], sh[k][threadIdx.x + s]);
                sh[3 + k][threadIdx.x] = fmax(sh[3 + k][threadIdx.x], sh[3 + k][threadIdx.x + s]);
            }
        __syncthreads();
    }
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = sh[k][0];
        hi[k] = sh[3 + k][0];
    }
    __syncthreads();
    for (int k = 0; k < 3; ++k) {
        sh[k][threadIdx.x] = sm[k];
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        int* bx = d.bbox + 8 * cap;
        // a diverged membrane (offsets not finite or beyond COORD_MAX) gets
        // an empty box, so that no loop runs over its coordinates
        bool sane = true;
        for (int k = 0; k < 3; ++k) sane = sane && fabs(lo[k]) <= COORD_MAX && fabs(hi[k]) <= COORD_MAX;
        if (!sane) atomicOr(&d.bb_count[CNT_FLAGS], FLAG_BOX);
        for (int k = 0; k < 3; ++k) {
            bx[k] = sane ? (int)floor(lo[k]) - MARGIN : 0;
            bx[3 + k] = sane ? (int)ceil(hi[k]) + MARGIN : -1;
            if (bx[3 + k] - bx[k] + 1 > ext) {
                atomicOr(&d.bb_count[CNT_FLAGS], FLAG_BOX);
                bx[3 + k] = bx[k] + ext - 1;
            }
            d.bb_com[3 * cap + k] = sane ? sh[k][0] / C.node_count : 0.0;
        }
        d.capV[cap] = 0.0;
        if (cap == 0) {
            d.bb_count[CNT_LINKS] = 0;
            d.bb_count[CNT_FRESH] = 0;
        }
    }
}

// Pairs of capsules of one parity colour whose boxes meet (periodic): their
// labels would count each other's crossings, so the step reports it.
__global__ __launch_bounds__(256) void k_bb_overlap(Lattice L, Dev d, int n_caps) {
    const int a = blockIdx.y, b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b <= a || b >= n_caps) return;
    const CapDev& A = d.caps[a];
    const CapDev& B = d.caps[b];
    if (A.colour != B.colour) return;
    const int* ba = d.bbox + 8 * a;
    const int* bb = d.bbox + 8 * b;
    const int nn[3] = {L.nx, L.ny, L.nz};
    bool meet = true;
    for (int k = 0; k < 3; ++k) {
        const int la = wrapi(A.anchor[k] + ba[k], nn[k]), ha = la + (ba[3 + k] - ba[k]);
        const int lb = wrapi(B.anchor[k] + bb[k], nn[k]), hb = lb + (bb[3 + k] - bb[k]);
        bool m = false;
        for (int sh = -1; sh <= 1; ++sh) m = m || (la <= hb + sh * nn[k] && lb + sh * nn[k] <= ha);
        meet = meet && m;
    }
    if (meet) atomicOr(&d.bb_count[CNT_FLAGS], FLAG_OVERLAP);
}

__global__ __launch_bounds__(256) void k_bb_clear(Lattice L, Dev d) {
    const int cap = blockIdx.y;
    int q[3];
    if (!box_cell(d, cap, blockIdx.x * blockDim.x + threadIdx.x, q)) return;
    const CapDev& C = d.caps[cap];
    const int64_t node = lat(L, C.anchor[0] + q[0], C.anchor[1] + q[1], C.anchor[2] + q[2]);
    d.lab_new[node] = -1;
    d.lpar[node] = 0u;      // (every box is cleared before any capsule's links are found)
    for (int k = 0; k < 9; ++k) d.lkey[k * L.n + node] = ~0ull;
}

// Segment p -> p + c against triangle (a, b, c): Moeller and Trumbore, FP64,
// the crossing parameter t in [0, 1) and the closed triangle.
__device__ __forceinline__ bool seg_hits(const double p[3], int cx_, int cy_, int cz_, const double a[3],
                                         const double e1[3], const double e2[3], double& tout) {
    const double dir[3] = {(double)cx_, (double)cy_, (double)cz_};
    const double pv[3] = {dir[1] * e2[2] - dir[2] * e2[1], dir[2] * e2[0] - dir[0] * e2[2],
                          dir[0] * e2[1] - dir[1] * e2[0]};
    const double det = e1[0] * pv[0] + e1[1] * pv[1] + e1[2] * pv[2];
    if (det == 0.0) return false;
    const double inv = 1.0 / det;
    const double tv[3] = {p[0] - a[0], p[1] - a[1], p[2] - a[2]};
    const double u = (tv[0] * pv[0] + tv[1] * pv[1] + tv[2] * pv[2]) * inv;
    if (u < 0.0 || u > 1.0) return false;
    const double qv[3] = {tv[1] * e1[2] - tv[2] * e1[1], tv[2] * e1[0] - tv[0] * e1[2], tv[0] * e1[1] - tv[1] * e1[0]};
    const double v = (dir[0] * qv[0] + dir[1] * qv[1] + dir[2] * qv[2]) * inv;
    if (v < 0.0 || u + v > 1.0) return false;
    const double t = (e2[0] * qv[0] + e2[1] * qv[1] + e2[2] * qv[2]) * inv;
    tout = t;
    return t >= 0.0 && t < 1.0;
}

// One thread per (triangle, half-direction).  Only start points from which
// the segment can reach the triangle's bounding box are visited, and those
// whose segment stays strictly on one side of the triangle's plane (both
// signed distances beyond a margin far above their FP64 rounding) are
// skipped before the full test; neither skips a segment the full test would
// accept.
__global__ __launch_bounds__(256) void k_bb_links(Lattice L, Dev d, int n_faces, int link_cap) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 9 * n_faces) return;
    const int f = gid / 9, dh = gid - 9 * f;
    const CapDev& C = d.caps[d.face_cap[f]];
    double V[3][3];
    for (int k = 0; k < 3; ++k) node_rel(d, d.tri[3 * f + k], V[k]);
    if (dh == 0)
        for (int j = 0; j < 3; ++j) d.face_cen[3 * f + j] = V[0][j] + V[1][j] + V[2][j];
    double e1[3], e2[3];
    int lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        // a diverged membrane: report, do not scan (the loop bounds below
        // stay far inside the int range)
        for (int j = 0; j < 3; ++j)
            if (!(fabs(V[j][k]) <= COORD_MAX)) {
                atomicOr(&d.bb_count[CNT_FLAGS], FLAG_BOX);
                return;
            }
        e1[k] = V[1][k] - V[0][k];
        e2[k] = V[2][k] - V[0][k];
        lo[k] = (int)floor(fmin(V[0][k], fmin(V[1][k], V[2][k]))) - 1;
        hi[k] = (int)floor(fmax(V[0][k], fmax(V[1][k], V[2][k]))) + 1;
        if (hi[k] - lo[k] > 16) {    // a torn mesh: report, do not scan
            atomicOr(&d.bb_count[CNT_FLAGS], FLAG_BOX);
            return;
        }
    }
    const int i = half_dir(dh);
    // a hit p + t c (0 <= t < 1) lies in the triangle's bounding box, so p
    // lies in that box moved back by t c: per axis [min - max(c, 0), max -
    // min(c, 0)], widened by far more than the test's FP64 rounding
    const int ci[3] = {cx(i), cy(i), cz(i)};
    for (int k = 0; k < 3; ++k) {
        const double mn = fmin(V[0][k], fmin(V[1][k], V[2][k])), mx = fmax(V[0][k], fmax(V[1][k], V[2][k]));
        lo[k] = max(lo[k], (int)ceil(mn - (double)max(ci[k], 0) - 1e-9));
        hi[k] = min(hi[k], (int)floor(mx - (double)min(ci[k], 0) + 1e-9));
    }
    const double nrm[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double nc = nrm[0] * ci[0] + nrm[1] * ci[1] + nrm[2] * ci[2];
    const double margin = 1e-9 * (fabs(nrm[0]) + fabs(nrm[1]) + fabs(nrm[2]));
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) {
                const double p[3] = {(double)x, (double)y, (double)z};
                const double d0 = nrm[0] * (p[0] - V[0][0]) + nrm[1] * (p[1] - V[0][1]) + nrm[2] * (p[2] - V[0][2]);
                const double d1 = d0 + nc;
                if ((d0 > margin && d1 > margin) || (d0 < -margin && d1 < -margin)) continue;
                double t;
                if (!seg_hits(p, cx(i), cy(i), cz(i), V[0], e1, e2, t)) continue;
                const int64_t node = lat(L, C.anchor[0] + x, C.anchor[1] + y, C.anchor[2] + z);
                if (i == 5) atomicXor(&d.lpar[node], 1u << C.colour);
                // the link's element: nearest crossing, then lowest index
                // (k_bb_list lists the links from these keys)
                const unsigned long long key =
                    ((unsigned long long)__float_as_uint((float)t) << 32) | (unsigned long long)(unsigned)f;
                atomicMin(&d.lkey[dh * L.n + node], key);
            }
}

// Start of this thread's run of c slots in the list whose length is *count:
// one atomic per block (every thread of the block calls it).
__device__ __forceinline__ int block_append(int c, int* count) {
    __shared__ int wsum[4];
    __shared__ int base;
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    int inc = c;                                   // inclusive scan within the wavefront
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    int before = 0, total = 0;
    for (int w = 0; w < 4; ++w) {
        before += w < wave ? wsum[w] : 0;
        total += wsum[w];
    }
    if (threadIdx.x == 0) base = total > 0 ? atomicAdd(count, total) : 0;
    __syncthreads();
    return base + before + inc - c;
}

// Per box cell: the links from the node that a triangle crosses, each listed
// once, by the box of the capsule its element belongs to.
__global__ __launch_bounds__(256) void k_bb_list(Lattice L, Dev d, int link_cap) {
    const int cap = blockIdx.y;
    int q[3];
    const bool in = box_cell(d, cap, blockIdx.x * blockDim.x + threadIdx.x, q);
    if (__syncthreads_or(in) == 0) return;     // (block-uniform)
    int64_t node = 0;
    unsigned mine = 0u;
    if (in) {
        const CapDev& C = d.caps[cap];
        node = lat(L, C.anchor[0] + q[0], C.anchor[1] + q[1], C.anchor[2] + q[2]);
        for (int dh = 0; dh < 9; ++dh) {
            const unsigned long long key = d.lkey[dh * L.n + node];
            if (key != ~0ull && d.face_cap[(unsigned)(key & 0xffffffffull)] == cap) mine |= 1u << dh;
        }
    }
    int k = block_append(__popc(mine), &d.bb_count[CNT_LINKS]);
    for (int dh = 0; dh < 9; ++dh) {
        if (!(mine & (1u << dh))) continue;
        if (k < link_cap)
            d.links[k] = make_int4((int)node, dh, 0, 0);
        else
            atomicOr(&d.bb_count[CNT_FLAGS], FLAG_LINKS);
        ++k;
    }
}

__global__ __launch_bounds__(256) void k_bb_label(Lattice L, Dev d) {
    const int cap = blockIdx.y;
    const int* bx = d.bbox + 8 * cap;
    const int ex = bx[3] - bx[0] + 1, ey = bx[4] - bx[1] + 1;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ex * ey) return;
    const CapDev& C = d.caps[cap];
    const int x = C.anchor[0] + bx[0] + c % ex, y = C.anchor[1] + bx[1] + c / ex;
    bool inside = false;    // the box bottom lies outside (margin)
    const unsigned bit = 1u << C.colour;      // crossings of this capsule's membrane only
    for (int z = bx[2]; z <= bx[5]; ++z) {
        const int64_t node = lat(L, x, y, C.anchor[2] + z);
        if (inside) d.lab_new[node] = cap;
        inside = inside != ((d.lpar[node] & bit) != 0);
    }
    if (inside) atomicOr(&d.bb_count[CNT_FLAGS], FLAG_PARITY);
}

__global__ __launch_bounds__(256) void k_bb_detect(Lattice L, Dev d, int fresh_cap) {
    const int cap = blockIdx.y;
    int q[3];
    if (!box_cell(d, cap, blockIdx.x * blockDim.x + threadIdx.x, q)) return;
    const CapDev& C = d.caps[cap];
    const int64_t node = lat(L, C.anchor[0] + q[0], C.anchor[1] + q[1], C.anchor[2] + q[2]);
    const int a = d.lab_new[node], b = d.lab[node];
    // each changed node is listed by one capsule: its new one, or its old one when it left
    if (a != b && (a == cap || (a == -1 && b == cap))) {
        const int k = atomicAdd(&d.bb_count[CNT_FRESH], 1);
        if (k < fresh_cap)
            d.fresh[k] = (int)node;
        else
            atomicOr(&d.bb_count[CNT_FLAGS], FLAG_FRESH);
    }
}

// committed ledger [0..1] += the pending changes [2..3] of this head
__global__ void k_bb_ledger(Dev d) {
    if (threadIdx.x < 2) {
        d.bb_mass[threadIdx.x] += d.bb_mass[2 + threadIdx.x];
        d.bb_mass[2 + threadIdx.x] = 0.0;
    }
}

// One block per fresh node: thread 0 forms the interpolated density, the
// 256 threads share the nearest-element search over the centroids
// k_bb_links left (faces t, t + 256, ...; the least distance, then the
// lowest index, as a scan in face order finds it), thread 0 writes.
__global__ __launch_bounds__(256) void k_bb_refill(Lattice L, Dev d, BBConst K, float2* __restrict__ f,
                                                  const float* __restrict__ rho, int fresh_cap) {
    __shared__ double sbd[4];
    __shared__ int sbest[4];
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    const int n_fresh = min(d.bb_count[CNT_FRESH], fresh_cap);
    const int64_t N = L.n;
    for (int e = blockIdx.x; e < n_fresh; e += gridDim.x) {
        const int64_t node = d.fresh[e];
        const int x = (int)(node % L.nx), y = (int)((node / L.nx) % L.ny), z = (int)(node / ((int64_t)L.nx * L.ny));
        const int ell = d.lab_new[node];
        double rf[2] = {0.0, 0.0};
        if (threadIdx.x == 0) {
            // the density interpolated from the non-fresh neighbours on the node's side
            double sum[2] = {0, 0}, mn[2] = {1e300, 1e300}, mx[2] = {-1e300, -1e300};
            int cnt = 0;
            for (int i = 1; i < Q; ++i) {
                const int64_t nb = lat1(L, x + cx(i), y + cy(i), z + cz(i));
                const int ln = d.lab_new[nb];
                if (ln != ell || ln != d.lab[nb]) continue;
                ++cnt;
                for (int c = 0; c < 2; ++c) {
                    const double r = rho[c * N + nb];
                    sum[c] += r;
                    mn[c] = fmin(mn[c], r);
                    mx[c] = fmax(mx[c], r);
                }
            }
            for (int c = 0; c < 2; ++c) {
                if (cnt == 0) {
                    rf[c] = rho[c * N + node];
                } else {
                    const double corr = 1.0 - K.c0 * ((K.rho_init[0] + K.rho_init[1]) / K.rho_init[c]) *
                                                  d.bb_mass[c] / K.vsys;
                    rf[c] = fmin(fmax(sum[c] / cnt * corr, mn[c]), mx[c]);
                }
            }
        }
        // the nearest element (nearest centroid) of the capsule whose membrane passed
        const int cap = ell >= 0 ? ell : d.lab[node];
        const CapDev& C = d.caps[cap];
        double p[3] = {(double)(x - C.anchor[0]), (double)(y - C.anchor[1]), (double)(z - C.anchor[2])};
        const int nn[3] = {L.nx, L.ny, L.nz};
        for (int k = 0; k < 3; ++k) p[k] -= nn[k] * rint((p[k] - d.bb_com[3 * cap + k]) / nn[k]);
        int best = 0x7fffffff;
        double bd = 1e300;
        const int fend = C.face_start + C.face_count;
        for (int f0 = C.face_start + (int)threadIdx.x; f0 < fend; f0 += 4 * 256) {
            double cen[4][3];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int ff = min(f0 + 256 * u, fend - 1);
#pragma unroll
                for (int j = 0; j < 3; ++j) cen[u][j] = d.face_cen[3 * ff + j];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int ff = f0 + 256 * u;
                double dd = 0.0;
                for (int j = 0; j < 3; ++j) {
                    const double t = cen[u][j] / 3.0 - p[j];
                    dd += t * t;
                }
                if (ff < fend && dd < bd) {      // (a thread's faces come in increasing order)
                    bd = dd;
                    best = ff;
                }
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double obd = __shfl_xor(bd, o, 64);
            const int ob = __shfl_xor(best, o, 64);
            if (obd < bd || (obd == bd && ob < best)) {
                bd = obd;
                best = ob;
            }
        }
        if (lane == 0) {
            sbd[wave] = bd;
            sbest[wave] = best;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int w = 1; w < 4; ++w)
                if (sbd[w] < bd || (sbd[w] == bd && sbest[w] < best)) {
                    bd = sbd[w];
                    best = sbest[w];
                }
            if (best == 0x7fffffff) best = C.face_start;      // (no finite distance: a torn membrane)
            double v[3] = {0, 0, 0};
            for (int k = 0; k < 3; ++k)
                for (int j = 0; j < 3; ++j) v[j] += d.node_V[3 * d.tri[3 * best + k] + j] / 3.0;
            // removed momentum, new populations, created momentum
            double old[3] = {0, 0, 0}, dm[2] = {0, 0};
            const float uu = (float)(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            for (int i = 0; i < Q; ++i) {
                const float2 g = f[i * N + node];
                const double sg = (double)g.x + (double)g.y;
                old[0] += sg * cx(i);
                old[1] += sg * cy(i);
                old[2] += sg * cz(i);
                const float cu = (float)(cx(i) * v[0] + cy(i) * v[1] + cz(i) * v[2]);
                const float t = wgt(i) * (1.0f + 3.0f * cu + 4.5f * cu * cu - 1.5f * uu);
                const float2 nf = make_float2((float)rf[0] * t, (float)rf[1] * t);
                f[i * N + node] = nf;
                dm[0] += (double)nf.x - (double)g.x;
                dm[1] += (double)nf.y - (double)g.y;
            }
            unsafeAtomicAdd(&d.bb_mass[2], dm[0]);
            unsafeAtomicAdd(&d.bb_mass[3], dm[1]);
            double q[3];
            for (int j = 0; j < 3; ++j) q[j] = (old[j] - (rf[0] + rf[1]) * v[j]) / 3.0;
            for (int k = 0; k < 3; ++k) add3(d.QR + 3 * d.tri[3 * best + k], q, 1.0);
        }
        __syncthreads();      // (sbd, sbest are reused by the next fresh node)
    }
}

__global__ __launch_bounds__(256) void k_bb_commit(Lattice L, Dev d) {
    const int cap = blockIdx.y;
    int q[3];
    if (!box_cell(d, cap, blockIdx.x * blockDim.x + threadIdx.x, q)) return;
    const CapDev& C = d.caps[cap];
    const int64_t node = lat(L, C.anchor[0] + q[0], C.anchor[1] + q[1], C.anchor[2] + q[2]);
    d.lab[node] = d.lab_new[node];
}

__device__ __forceinline__ void node_density(const float2* __restrict__ f, int64_t N, int64_t node, double r[2]) {
    r[0] = r[1] = 0.0;
    for (int i = 0; i < Q; ++i) {
        const float2 g = f[i * N + node];
        r[0] += g.x;
        r[1] += g.y;
    }
}

// The densities of both ends of each listed link, before any population is
// bounced (a node with several crossing links has them all rewritten).
__global__ __launch_bounds__(256) void k_bb_link_density(Lattice L, Dev d, const float2* __restrict__ f,
                                                         int link_cap) {
    const int n = min(d.bb_count[CNT_LINKS], link_cap);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int4 rec = d.links[e];
        const int64_t xn = rec.x;
        const int i = half_dir(rec.y);
        const int x = (int)(xn % L.nx), y = (int)((xn / L.nx) % L.ny), z = (int)(xn / ((int64_t)L.nx * L.ny));
        const int64_t yn = lat1(L, x + cx(i), y + cy(i), z + cz(i));
        double rx[2], ry[2];
        node_density(f, L.n, xn, rx);
        node_density(f, L.n, yn, ry);
        d.link_rho[e] = make_double4(rx[0], rx[1], ry[0], ry[1]);
    }
}

__global__ __launch_bounds__(256) void k_bb_fixup(Lattice L, Dev d, float2* __restrict__ f, int link_cap) {
    const int n = min(d.bb_count[CNT_LINKS], link_cap);
    const int64_t N = L.n;
    // (the loop is wave-uniform: every lane of a wavefront reaches the reduction)
    for (int base = blockIdx.x * blockDim.x + (int)(threadIdx.x & ~63u); base < n; base += gridDim.x * blockDim.x) {
        const int e = base + (int)(threadIdx.x & 63);
        double dmA = 0.0, dmB = 0.0;      // this lane's change of each component's stored mass
        if (e < n) {
            const int4 rec = d.links[e];
            const int64_t xn = rec.x;
            const int i = half_dir(rec.y), j = opp(i);
            const int x = (int)(xn % L.nx), y = (int)((xn / L.nx) % L.ny), z = (int)(xn / ((int64_t)L.nx * L.ny));
            const int64_t yn = lat1(L, x + cx(i), y + cy(i), z + cz(i));
            if (d.lab[xn] != d.lab[yn]) {       // (equal: the link crosses the membrane twice, or not)
                const int face = (int)(unsigned)(d.lkey[rec.y * N + xn] & 0xffffffffull);
                double v0[3] = {0, 0, 0};
                for (int k = 0; k < 3; ++k)
                    for (int a = 0; a < 3; ++a) v0[a] += d.node_V[3 * d.tri[3 * face + k] + a] / 3.0;
                const double4 lr = d.link_rho[e];
                const double rx[2] = {lr.x, lr.y}, ry[2] = {lr.z, lr.w};
                const double ci[3] = {(double)cx(i), (double)cy(i), (double)cz(i)};
                const double cv = ci[0] * v0[0] + ci[1] * v0[1] + ci[2] * v0[2];      // c_i . v0 = -(c_j . v0)
                const double w = wgt(i);
                // the slot (x, i) is what the pull at y reads along c_i, the slot (y, j)
                // what the pull at x reads along c_j
                const float2 a = f[i * N + xn];      // x's outgoing population towards y
                const float2 b = f[j * N + yn];      // y's outgoing population towards x
                const float2 back_x = make_float2((float)((double)a.x - 6.0 * w * rx[0] * cv),
                                                  (float)((double)a.y - 6.0 * w * rx[1] * cv));     // to x along c_j
                const float2 back_y = make_float2((float)((double)b.x + 6.0 * w * ry[0] * cv),
                                                  (float)((double)b.y + 6.0 * w * ry[1] * cv));     // to y along c_i
                f[j * N + yn] = back_x;
                f[i * N + xn] = back_y;
                // the moving-element terms change each side's mass (as stored)
                dmA = ((double)back_x.x - a.x) + ((double)back_y.x - b.x);
                dmB = ((double)back_x.y - a.y) + ((double)back_y.y - b.y);
                // momentum to the element: [out + back] c_out at each end
                const double sx = (double)a.x + a.y + back_x.x + back_x.y;
                const double sy = (double)b.x + b.y + back_y.x + back_y.y;
                double dp[3];
                for (int k = 0; k < 3; ++k) dp[k] = (sx - sy) * ci[k] / 3.0;
                for (int k = 0; k < 3; ++k) add3(d.P_cur + 3 * d.tri[3 * face + k], dp, 1.0);
            }
        }
        // the ledger: one pair of atomics per wavefront
        for (int o = 32; o > 0; o >>= 1) {
            dmA += __shfl_xor(dmA, o, 64);
            dmB += __shfl_xor(dmB, o, 64);
        }
        if ((threadIdx.x & 63) == 0 && (dmA != 0.0 || dmB != 0.0)) {
            unsafeAtomicAdd(&d.bb_mass[2], dmA);
            unsafeAtomicAdd(&d.bb_mass[3], dmB);
        }
    }
}

__global__ __launch_bounds__(256) void k_bb_unflag(Lattice L, Dev d, int n_tiles) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n_tiles; t += gridDim.x * blockDim.x) d.tile_flag[t] = 0;
}

__global__ __launch_bounds__(256) void k_bb_flag(Lattice L, Dev d) {
    const int cap = blockIdx.y;
    int q[3];
    if (!box_cell(d, cap, blockIdx.x * blockDim.x + threadIdx.x, q)) return;
    const CapDev& C = d.caps[cap];
    const int x = wrapi(C.anchor[0] + q[0], L.nx), y = wrapi(C.anchor[1] + q[1], L.ny),
              z = wrapi(C.anchor[2] + q[2], L.nz);
    const int64_t node = ((int64_t)z * L.ny + y) * L.nx + x;
    for (int k = 0; k < 6; ++k) d.fib[k * L.n + node] = 0.0f;
    d.tile_flag[((z >> 3) * L.nty + (y >> 3)) * L.ntx + (x >> 3)] = 1;
}

// ---- the Shan-Chen sum across the membrane ---------------------------------

// The densities of node `of`'s neighbours with label `side`, averaged
// (eq. method:interpolateshanchen); `of` has at least one such neighbour,
// the node across from which it is seen.
__device__ __forceinline__ void bound_density(const Lattice& L, const Dev& d, const float* __restrict__ rho,
                                              int64_t of, int side, double r[2]) {
    const int x = (int)(of % L.nx), y = (int)((of / L.nx) % L.ny), z = (int)(of / ((int64_t)L.nx * L.ny));
    int lb[Q];
    float ra[Q], rb[Q];
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        const int64_t nb = lat1(L, x + cx(q), y + cy(q), z + cz(q));
        lb[q] = d.lab[nb];
        ra[q] = rho[nb];
        rb[q] = rho[L.n + nb];
    }
    double s[2] = {0, 0};
    int cnt = 0;
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        if (lb[q] != side) continue;
        ++cnt;
        s[0] += ra[q];
        s[1] += rb[q];
    }
    r[0] = s[0] / cnt;
    r[1] = s[1] / cnt;
}

__global__ __launch_bounds__(256) void k_bb_sc(Lattice L, Dev d, BBConst K, const float* __restrict__ rho,
                                              int link_cap) {
    const int n = min(d.bb_count[CNT_LINKS], link_cap);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        const int4 rec = d.links[e];
        const int64_t N = L.n;
        const int64_t xn = rec.x;
        const int i = half_dir(rec.y);
        const int x = (int)(xn % L.nx), y = (int)((xn / L.nx) % L.ny), z = (int)(xn / ((int64_t)L.nx * L.ny));
        const int64_t yn = lat1(L, x + cx(i), y + cy(i), z + cz(i));
        const int lx = d.lab[xn], ly = d.lab[yn];
        if (lx == ly) continue;
        const int face = (int)(unsigned)(d.lkey[rec.y * N + xn] & 0xffffffffull);
        const CapDev& C = d.caps[d.face_cap[face]];
        const double w = wgt(i), G = L.G;
        const double ci[3] = {(double)cx(i), (double)cy(i), (double)cz(i)};
        double react[3] = {0, 0, 0};
        // end 0: x sees y along +c_i; end 1: y sees x along -c_i
        for (int end = 0; end < 2; ++end) {
            const int64_t self = end == 0 ? xn : yn, other = end == 0 ? yn : xn;
            const double sg = end == 0 ? 1.0 : -1.0;
            double rb[2];
            bound_density(L, d, rho, other, end == 0 ? lx : ly, rb);
            rb[C.pref] += C.rv_abs;
            double pv[2], po[2], ps[2];
            for (int c = 0; c < 2; ++c) {
                pv[c] = psi_of(rb[c], K.psi_exp);
                po[c] = psi_of(rho[c * N + other], K.psi_exp);
                ps[c] = psi_of(rho[c * N + self], K.psi_exp);
            }
            // dS^c(self) += w (psi_virtual^c - psi^c(other)) c; the collide forms
            // F^A = -G psi^A (S^B + dS^B) and F^B alike
            for (int c = 0; c < 2; ++c)
                for (int k = 0; k < 3; ++k)
                    if (ci[k] != 0.0)
                        atomicAdd(&d.fib[(3 * c + k) * N + self], (float)(w * (pv[c] - po[c]) * sg * ci[k]));
            // minus the force on self from the virtual neighbour
            const double fr = G * w * (ps[0] * pv[1] + ps[1] * pv[0]) * sg;
            for (int k = 0; k < 3; ++k) react[k] += fr * ci[k] / 3.0;
        }
        for (int k = 0; k < 3; ++k) add3(d.QR + 3 * d.tri[3 * face + k], react, 1.0);
    }
}

// ---- node update ---------------------------------------------------------

__global__ __launch_bounds__(256) void k_bb_advance(Dev d, BBConst K, int n_nodes) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_nodes) return;
    const CapDev& C = d.caps[d.node_cap[b]];
    for (int k = 0; k < 3; ++k) {
        const double F = (double)d.node_F[3 * b + k] + 0.5 * (d.P_cur[3 * b + k] + d.P_prev[3 * b + k]) +
                         d.QR[3 * b + k];
        d.node_F[3 * b + k] = (float)F;
        const float V = C.prescribed ? C.vp[k] : (float)((double)d.node_V[3 * b + k] + F * K.inv_mass);
        d.node_V[3 * b + k] = V;
        // compensated (hi, lo) += V, as in the immersed-boundary advection
        const float a = d.off_hi[3 * b + k];
        const float bb = d.off_lo[3 * b + k] + V;
        const float s = a + bb;
        const float bv = s - a;
        const float err = (a - (s - bv)) + (bb - bv);
        d.off_hi[3 * b + k] = s;
        d.off_lo[3 * b + k] = err;
        d.P_prev[3 * b + k] = d.P_cur[3 * b + k];
        d.P_cur[3 * b + k] = 0.0;
        d.QR[3 * b + k] = 0.0;
    }
}

__global__ __launch_bounds__(256) void k_bb_init(Lattice L, Dev d) {
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < L.n; k += (int64_t)gridDim.x * blockDim.x) {
        d.lab[k] = -1;
        d.lab_new[k] = -1;
        d.lpar[k] = 0u;
    }
}

}  // namespace

void launch_bb_init(const Lattice& L, Dev& d, hipStream_t s) {
    hipLaunchKernelGGL(k_bb_init, dim3(2048), dim3(256), 0, s, L, d);
}

void launch_bb_geometry(const Lattice& L, Dev& d, const BBSizes& z, int n_caps, int n_faces, bool detect_fresh,
                        hipStream_t s) {
    if (n_caps <= 0) return;
    const int cells = z.ext * z.ext * z.ext;
    const dim3 gbox((cells + 255) / 256, n_caps), gcol((z.ext * z.ext + 255) / 256, n_caps);
    hipLaunchKernelGGL(k_bb_box, dim3(n_caps), dim3(256), 0, s, d, z.ext);
    if (n_caps > 1) hipLaunchKernelGGL(k_bb_overlap, dim3((n_caps + 255) / 256, n_caps), dim3(256), 0, s, L, d, n_caps);
    hipLaunchKernelGGL(k_bb_clear, gbox, dim3(256), 0, s, L, d);
    hipLaunchKernelGGL(k_bb_links, dim3((9 * n_faces + 255) / 256), dim3(256), 0, s, L, d, n_faces, z.link_cap);
    hipLaunchKernelGGL(k_bb_list, gbox, dim3(256), 0, s, L, d, z.link_cap);
    hipLaunchKernelGGL(k_bb_label, gcol, dim3(256), 0, s, L, d);
    if (detect_fresh) hipLaunchKernelGGL(k_bb_detect, gbox, dim3(256), 0, s, L, d, z.fresh_cap);
}

void launch_bb_refill(const Lattice& L, Dev& d, const BBSizes& z, const BBConst& k, void* fpost, const float* rho,
                      int n_caps, hipStream_t s) {
    if (n_caps <= 0) return;
    const int cells = z.ext * z.ext * z.ext;
    hipLaunchKernelGGL(k_bb_refill, dim3(std::min(z.fresh_cap, 512)), dim3(256), 0, s, L, d, k,
                       (float2*)fpost, rho, z.fresh_cap);
    hipLaunchKernelGGL(k_bb_commit, dim3((cells + 255) / 256, n_caps), dim3(256), 0, s, L, d);
}

void launch_bb_fixup(const Lattice& L, Dev& d, const BBSizes& z, void* fpost, int n_caps, hipStream_t s) {
    if (n_caps <= 0) return;
    const dim3 g(std::min((z.link_cap + 255) / 256, 1024));
    hipLaunchKernelGGL(k_bb_link_density, g, dim3(256), 0, s, L, d, (const float2*)fpost, z.link_cap);
    hipLaunchKernelGGL(k_bb_fixup, g, dim3(256), 0, s, L, d, (float2*)fpost, z.link_cap);
    hipLaunchKernelGGL(k_bb_ledger, dim3(1), dim3(64), 0, s, d);
}

void launch_bb_flags(const Lattice& L, Dev& d, const BBSizes& z, int n_caps, hipStream_t s) {
    const int nt = L.ntx * L.nty * L.ntz;
    hipLaunchKernelGGL(k_bb_unflag, dim3(std::min((nt + 255) / 256, 1024)), dim3(256), 0, s, L, d, nt);
    if (n_caps <= 0) return;
    const int cells = z.ext * z.ext * z.ext;
    hipLaunchKernelGGL(k_bb_flag, dim3((cells + 255) / 256, n_caps), dim3(256), 0, s, L, d);
}

void launch_bb_shan_chen(const Lattice& L, Dev& d, const BBSizes& z, const BBConst& k, const float* rho,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_bb_sc, dim3(std::min((z.link_cap + 255) / 256, 1024)), dim3(256), 0, s, L, d, k, rho,
                       z.link_cap);
}

void launch_bb_advance(Dev& d, const BBConst& k, int n_nodes, hipStream_t s) {
    if (n_nodes > 0) hipLaunchKernelGGL(k_bb_advance, dim3((n_nodes + 255) / 256), dim3(256), 0, s, d, k, n_nodes);
}

}  // namespace lbmx
