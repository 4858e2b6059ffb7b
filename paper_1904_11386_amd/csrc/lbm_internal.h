// Internal declarations shared by the HIP kernels and the host side of the
// library.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmx {

// ---- D3Q19 (Sec. II.A, eq. lbm:weights) -------------------------------
// 0 rest; 1..6 = +x -x +y -y +z -z; 7..18 = (+-1,+-1,0), (+-1,0,+-1),
// (0,+-1,+-1), opposites adjacent.
constexpr int Q = 19;
__host__ __device__ constexpr int cx(int i) {
    constexpr int v[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[i];
}
__host__ __device__ constexpr int cy(int i) {
    constexpr int v[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int cz(int i) {
    constexpr int v[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return v[i];
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr float wgt(int i) {
    return i == 0 ? 1.0f / 3.0f : (i <= 6 ? 1.0f / 18.0f : 1.0f / 36.0f);
}

constexpr int TILE = 8;        // edge of the tiles flagged as touched by a stencil
constexpr int BIN = 4;         // edge of the spreading bins (a node's home bin holds floor(X))
constexpr int BOX = BIN + 3;   // spreading box edge: stencil reach of one bin's nodes
#ifndef LBM_BX
#define LBM_BX 128
#endif
#ifndef LBM_BY
#define LBM_BY 4
#endif
#ifndef LBM_ZC
#define LBM_ZC 8
#endif
#ifndef LBM_COLLIDE_ATTR
#define LBM_COLLIDE_ATTR
#endif
constexpr int BX = LBM_BX;     // lattice blocks: x extent (a multiple of the wavefront)
constexpr int BY = LBM_BY;     // lattice blocks: y extent
constexpr int ZC = LBM_ZC;     // lattice blocks: fewest z planes marched per block
constexpr int NXCD = 8;        // accelerator dies; workgroups are dealt round-robin to them

struct Lattice {
    int nx, ny, nz;
    int ntx, nty, ntz;     // tile counts (TILE)
    int nbx, nby, nbz;     // bin counts (BIN)
    int zc;                // z planes marched per lattice block (a multiple of ZC)
    int cached;            // population streams: non-temporal loads, cached stores (1) or the reverse
    int psi_exp;           // Shan-Chen pseudo-potential 1 - exp(-rho) (1) or rho (0)
    int64_t n;             // nx*ny*nz
    int walls;             // half-way bounce-back walls: solid rows y = 0 and ny - 1
    int onsite;            // on-site velocity boundaries on the fluid rows y = 0 and ny - 1
    int sharp;             // the bounce-back coupling: flagged tiles carry Shan-Chen sum corrections
    int one;               // one lattice pass: k_collide forms the step's densities itself
    float G;
    float tau[2];
    float omega[2];        // 1/tau
    float uw_lo[3], uw_hi[3];
};

// The exponential Shan-Chen pseudo-potential 1 - exp(-v) (Sec. II.D, rho0 = 1),
// branch-free: below 0.5 a degree-7 Taylor polynomial (truncation below 2e-7
// relative), above it the direct form (the subtraction loses below 2e-7).
__device__ __forceinline__ float psi_exp(float v) {
    const float p = v * (1.0f + v * (-0.5f + v * (1.0f / 6.0f + v * (-1.0f / 24.0f + v * (1.0f / 120.0f +
                    v * (-1.0f / 720.0f + v * (1.0f / 5040.0f)))))));
    const float q = 1.0f - __expf(-v);
    return v < 0.5f ? p : q;
}

struct CapDev {
    int anchor[3];
    int node_start, node_count, face_start, face_count;
    int pref;           // preferred component of the virtual density (0 A, 1 B)
    float rv_abs;       // |rho_v|
    float drv;          // d|rho_v| / d theta (per radian)
    float kS, C, kV;
    float kB;           // Helfrich bending modulus (0 = none)
    double V0;
    float vp[3];        // bounce-back coupling: the prescribed node velocity
    int prescribed;     // 1: the nodes keep vp (rigid translation)
    int colour;         // bounce-back coupling: its bit (0..31) in the crossing-parity words; capsules whose
                        // label boxes meet have different colours
};

struct FaceRef {        // rest metric of a triangle
    float q11, q12, q22; // inverse of the rest metric [e_a . e_b]
    float inv_det0;      // 1 / det of the rest metric
    float A0;            // rest area
};

// Device-side pointers of one context (all inside the caller's workspace).
struct Dev {
    void* f[2];           // populations [2 comps][19][N]: float (FP32) or g in _Float16 (FP16)
    float* cscale;        // [2 parities][2 comps] FP64-derived mass compensation factors (FP16)
    double* dpart;        // [density blocks][2] FP64 block sums of rho (FP16)
    double* dmass;        // [2] FP64 component masses of the last density pass (FP16)
    float* rho[2];        // [2][N] density buffers, ping-pong by step parity
    float* fib;           // [5][N]: F_ib x, y, z, phi_A, phi_B
    float* u;             // [3][N] velocity where the immersed boundary needs it
    int* tile_flag;       // [tiles] 1 when touched by a stencil this step
    int* tile_count;      // [bins] nodes whose home bin it is
    int* tile_offset;     // [bins] start of the bin in `sorted`
    int* touched[2];      // lists of touched tiles (step parity)
    int* home[2];         // lists of occupied bins (step parity)
    int* home_start;      // [bins] bin start per home-list entry
    int* counters;        // [8]: touched count[2], home count[2]
    // nodes
    float* off_hi;        // [nodes][3]
    float* off_lo;        // [nodes][3]
    int* node_cap;        // [nodes]
    int4* node_anc;       // [nodes] the capsule's anchor (x, y, z) and preferred component (w)
    float* node_wet;      // [nodes] |rho_v| A_b
    float* node_F;        // [nodes][3]
    int* node_tile;       // [nodes]
    int* node_rank;       // [nodes]
    int* sorted;          // [nodes]
    int* csr_ptr;         // [nodes + 1] corners of node b: slots csr_ptr[b] .. csr_ptr[b+1]-1
    int* corner_slot;     // [faces][3] slot of corner (face, k), in node order
    int* slot_corner;     // [3 faces] the inverse: 3 * face + k of each slot
    float* node_bend;     // [nodes][6] bending geometry: H, K, mixed area, outward normal
    int* dbg_bins;        // [nodes][4] debug binning output
    // faces
    int* tri;             // [faces][3] global node indices
    FaceRef* fref;        // [faces]
    int* face_cap;        // [faces]
    float* face_F;        // [3 faces][3] corner forces, stored at the corners' slots
    // capsules
    CapDev* caps;         // [max caps]
    double* capV;         // [max caps]
    double* cap_mom;      // [max caps][16] observables moments
    double* red;          // [RED_BLOCKS][8] reduction partials
    // adjoint (allocated when the recompute ring is requested)
    void* lam[2];         // adjoint populations, [Q][N] component pairs (FP32)
    float* lam_rho;       // [2][N]
    float* lam_j;         // [6][N]  (component * 3 + axis)
    float* lam_S;         // [6][N]  adjoint of the Shan-Chen neighbour sums
    float* lam_u;         // [3][N]  touched tiles only
    float* lam_Fib;       // [3][N]  touched tiles only
    float* lam_X;         // [nodes][3] adjoint of the node positions
    float* lam_Fb;        // [nodes][3] adjoint of the node forces
    float* lam_q;         // [nodes][3] -G a_b lam_Fb, spread into lam_S
    float* lam_Xg;        // [nodes][3] delta-gradient terms
    double* node_g;       // [nodes][2] per-node dJ/dG, dJ/dtheta parts
    float* node_area;     // [nodes] rest area A_b
    double* capdV;        // [max caps] directional derivative of V
    double* grads;        // [4] dJ/dtheta, dJ/dkS, dJ/dG
    // bounce-back coupling (allocated when it is chosen)
    int* lab;             // [N] label of the current membranes: capsule inside, or -1
    int* lab_new;         // [N] labels being computed (scratch, valid in the capsules' boxes)
    unsigned* lpar;       // [N] bit k: parity of the crossings of the node's +z link by the membranes of
                          //     colour k
    int4* links;          // [link capacity] (node, half-direction, -, -)
    unsigned long long* lkey; // [9][N] per link: (FP32 crossing parameter, triangle), the least wins;
                              //     all ones where no triangle crosses it
    double4* link_rho;    // [link capacity] densities of the link's ends (A, B at the start; A, B at the end)
    double* face_cen;     // [faces][3] sum of each triangle's three anchor-relative node positions (FP64), this step
    int* fresh;           // [fresh capacity] nodes whose label changed
    int* bb_count;        // [8]: links, fresh nodes, overflow flags
    int* bbox;            // [max caps][8]: box lo (x, y, z), hi (x, y, z), anchor-relative
    double* bb_com;       // [max caps][3] mean node offset (anchor-relative)
    double* bb_mass;      // [4] FP64 ledger of the mass the coupling added per component: committed [0..1],
                          //     this step's head [2..3]
    float* node_V;        // [nodes][3] node velocities
    double* P_cur;        // [nodes][3] momentum exchanged at the last streaming
    double* P_prev;       // [nodes][3] the one before
    double* QR;           // [nodes][3] fresh-node and Shan-Chen reactions of the step
    int det;              // 1: the immersed boundary's sums in a fixed order (deterministic mode)
};

// sizes of the bounce-back coupling's lists and boxes
struct BBSizes {
    int link_cap, fresh_cap;
    int ext;              // edge of the largest capsule box the launches cover
};

constexpr int RED_BLOCKS = 1024;
constexpr int MOM_STRIDE = 16;

// ---- launchers (k_fluid.hip) -------------------------------------------
void launch_init_rest(const Lattice& L, void* f, const float* rhoA, const float* rhoB, bool half,
                      hipStream_t s);
int64_t density_blocks(const Lattice& L, bool half);
void launch_density(const Lattice& L, const void* fin, const float* rho_prev, float* rho_out, bool half,
                    const float* cscale, int par_prev, double* partial, hipStream_t s);
void launch_density_tiles(const Lattice& L, const void* fin, float* rho_out, const int* touched, const int* count,
                          const int* tile_flag, hipStream_t s);
void launch_compensate(const Lattice& L, const double* partial, double m0a, double m0b, float* cscale,
                       int par_cur, double* mass_out, hipStream_t s);
void launch_collide(const Lattice& L, const void* fin, void* fout, const float* rho_n, const float* rho_prev,
                    const float* fib, const int* tile_flag, float* u, bool has_ibm, bool macro, bool half,
                    const float* cscale, int par_prev, int par_cur, hipStream_t s);
void launch_onsite(const Lattice& L, void* f, bool half, const float* rho_enc, const float* cs, hipStream_t s);
void launch_scale_pops(const Lattice& L, void* f, float sa, float sb, hipStream_t s);
void launch_reduce_fluid(const Lattice& L, const void* fpost, bool half, const float* renc,
                         const float* cscale, int par, double* partial, hipStream_t s);

// ---- launchers (k_ibm.hip) ---------------------------------------------
void launch_clear_tiles(const Lattice& L, Dev& d, int parity_prev, int parity_cur, int n_caps,
                        hipStream_t s);
void launch_advect_clear(const Lattice& L, Dev& d, int n_nodes, int parity_prev, int parity_cur, int n_caps,
                         hipStream_t s);
void launch_cap_volume(const Dev& d, int n_faces, int n_caps, hipStream_t s);
void launch_faces(const Dev& d, int n_faces, hipStream_t s);
void launch_node_gather(const Lattice& L, const Dev& d, int n_nodes, int parity, hipStream_t s);
void launch_bin_scan(const Dev& d, int n_nodes, int parity, hipStream_t s);
void launch_bin_scatter(const Lattice& L, const Dev& d, int n_nodes, int par, hipStream_t s);
void launch_repulse(const Lattice& L, const Dev& d, int n_nodes, float eps, float d0, hipStream_t s);
void launch_bending(const Dev& d, int n_nodes, hipStream_t s);
void launch_reference_step(const Dev& d, int n_nodes, int n_faces, int n_caps, bool bend, float gamma, float w,
                           double z_interface, float mu, hipStream_t s);
void launch_spread(const Lattice& L, const Dev& d, int parity, const float* rho_n, const float* cs, hipStream_t s);
void launch_interp_advect(const Lattice& L, const Dev& d, int n_nodes, hipStream_t s);
void launch_cap_moments(const Dev& d, int n_caps, hipStream_t s);
void launch_debug_bins(const Lattice& L, const Dev& d, int n_nodes, hipStream_t s);
void launch_gather_forces(const Dev& d, int n_nodes, hipStream_t s);
// the bounce-back coupling (k_bb.hip)
struct BBConst {
    double m0[2];         // initial component masses
    double rho_init[2];   // their per-node averages
    double vsys;          // fluid node count
    double c0;            // strength of the adaptive mass correction
    float inv_mass;       // 1 / node mass
    int psi_exp;
};
void launch_bb_init(const Lattice& L, Dev& d, hipStream_t s);
void launch_bb_geometry(const Lattice& L, Dev& d, const BBSizes& z, int n_caps, int n_faces, bool detect_fresh,
                        hipStream_t s);
void launch_bb_refill(const Lattice& L, Dev& d, const BBSizes& z, const BBConst& k, void* fpost, const float* rho,
                      int n_caps, hipStream_t s);
void launch_bb_fixup(const Lattice& L, Dev& d, const BBSizes& z, void* fpost, int n_caps, hipStream_t s);
void launch_bb_flags(const Lattice& L, Dev& d, const BBSizes& z, int n_caps, hipStream_t s);
void launch_bb_shan_chen(const Lattice& L, Dev& d, const BBSizes& z, const BBConst& k, const float* rho,
                         hipStream_t s);
void launch_bb_advance(Dev& d, const BBConst& k, int n_nodes, hipStream_t s);
// adjoint (k_ibm.hip)
void launch_spread_vec(const Lattice& L, const Dev& d, int parity, const float* val, float* target, int mode,
                       hipStream_t s);
void launch_adj_nodes(const Lattice& L, const Dev& d, const float* rho_n, int n_nodes, hipStream_t s);
void launch_adj_membrane(const Dev& d, int n_nodes, int n_faces, hipStream_t s);
void launch_adj_repulse(const Lattice& L, const Dev& d, int n_nodes, float eps, float d0, hipStream_t s);
// adjoint (k_fluid.hip)
void launch_adj_collide(const Lattice& L, const void* fin, const float* rho_n, const float* rho_p, const float* fib,
                        const int* tile_flag, const void* lam_in, const float* lam_u, float* lam_rho, float* lam_j,
                        float* lam_S, float* lam_Fib, float* u_out, double* grads, hipStream_t s);
void launch_adj_gather(const Lattice& L, const float* lam_S, float* lam_rho, const float* rho_n, hipStream_t s);
void launch_adj_push(const Lattice& L, const void* lam_in, const float* lam_rho, const float* lam_j, void* lam_out,
                     hipStream_t s);

}  // namespace lbmx
