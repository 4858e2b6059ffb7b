// Host side of the C ABI declared in include/lbm.h: validation, workspace
// carving, capsule set-up (reference metric, rest areas and volume in FP64),
// the per-step launch sequence on the caller's stream, and the FP64
// observables.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <mutex>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"

using namespace lbmx;

// lbm_observables_noalloc keeps its FP64 reduction partials and the
// per-capsule moments in a fixed device array instead of the workspace:
// at most NOALLOC_MAX_CAPS capsules (about 576 KiB per device)
constexpr int NOALLOC_MAX_CAPS = 4096;
constexpr size_t NOALLOC_DOUBLES = (size_t)RED_BLOCKS * 8 + (size_t)NOALLOC_MAX_CAPS * MOM_STRIDE;
constexpr int NOALLOC_MAX_DEVICES = 64;

// Static scratch of lbm_observables_noalloc: the FP64 reduction partials and
// the per-capsule moments, per device (each device holds its own copy until
// the process ends).  Host code uses only the device address resolved at
// lbm_init, never this name.
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

static std::mutex g_scratch_mu;
static double* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The address of `scratch` on device `dev` (current), resolved once per device.
static hipError_t resolve_scratch(int dev, double** out) {
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = (double*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}


namespace {

thread_local std::string g_init_error;

struct Layout {
    size_t total = 0;
    size_t f[2], rho[2], fib, u;
    size_t tile_flag, tile_count, tile_offset, home_start, touched[2], home[2], counters;
    int64_t bins;
    size_t off_hi, off_lo, node_cap, node_anc, node_wet, node_F, node_tile, node_rank, sorted, csr_ptr, corner_slot,
        slot_corner, node_bend, dbg_bins;
    size_t tri, fref, face_cap, face_F;
    size_t caps, capV, cap_mom, red, cscale, dpart, dmass;
    size_t slot0, slot_bytes, fbytes;
    size_t slot_f, slot_rho, slot_off, slot_cs;   // offsets inside a slot
    bool adjoint = false;
    size_t lam[2], lam_rho, lam_j, lam_S, lam_u, lam_Fib, lam_X, lam_Fb, lam_q, lam_Xg, node_g, node_area, capdV,
        grads;
    size_t ring0, ring_bytes, ring_f, ring_rho, ring_off;
    int64_t tiles, max_caps;
    // the bounce-back coupling
    bool bb = false;
    size_t lab, lab_new, lpar, lkey, links, link_rho, face_cen, fresh, bb_count, bbox, bb_com, bb_mass, node_V, P_cur, P_prev, QR;
    int link_cap = 0, fresh_cap = 0;
};

size_t take(size_t& cur, size_t bytes) {
    const size_t at = (cur + 255) & ~size_t(255);
    cur = at + bytes;
    return at;
}

Layout make_layout(const lbm_params* p, int64_t max_nodes, int64_t max_faces) {
    Layout l;
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    const int64_t T = (int64_t)((p->nx + TILE - 1) / TILE) * ((p->ny + TILE - 1) / TILE) * ((p->nz + TILE - 1) / TILE);
    const int64_t nb = std::max<int64_t>(max_nodes, 1), nf = std::max<int64_t>(max_faces, 1);
    l.tiles = T;
    const int64_t NB = (int64_t)((p->nx + BIN - 1) / BIN) * ((p->ny + BIN - 1) / BIN) * ((p->nz + BIN - 1) / BIN);
    l.bins = NB;
    l.max_caps = nb / 12 + 1;
    size_t c = 0;
    const bool half = p->precision == LBM_FP16;
    const size_t fbytes = (size_t)2 * Q * N * (half ? 2 : 4);
    l.fbytes = fbytes;
    const int64_t dblocks = (int64_t)((p->nx + BX - 1) / BX) * ((p->ny + BY - 1) / BY) * ((p->nz + ZC - 1) / ZC);
    l.f[0] = take(c, fbytes);
    l.f[1] = take(c, fbytes);
    l.rho[0] = take(c, 2 * N * sizeof(float));
    l.rho[1] = take(c, 2 * N * sizeof(float));
    l.bb = p->coupling == 1;
    // (the bounce-back coupling keeps six Shan-Chen sum corrections there)
    l.fib = take(c, (l.bb ? 6 : 5) * N * sizeof(float));
    l.u = take(c, 3 * N * sizeof(float));
    l.tile_flag = take(c, T * 4);
    l.tile_count = take(c, NB * 4);
    l.tile_offset = take(c, NB * 4);
    l.home_start = take(c, NB * 4);
    l.touched[0] = take(c, T * 4);
    l.touched[1] = take(c, T * 4);
    l.home[0] = take(c, NB * 4);
    l.home[1] = take(c, NB * 4);
    l.counters = take(c, 8 * 4);
    l.off_hi = take(c, 3 * nb * 4);
    l.off_lo = take(c, 3 * nb * 4);
    l.node_cap = take(c, nb * 4);
    l.node_anc = take(c, nb * 16);
    l.node_wet = take(c, nb * 4);
    l.node_F = take(c, 3 * nb * 4);
    l.node_tile = take(c, nb * 4);
    l.node_rank = take(c, nb * 4);
    l.sorted = take(c, nb * 4);
    l.csr_ptr = take(c, (nb + 1) * 4);
    l.corner_slot = take(c, 3 * nf * 4);
    l.slot_corner = take(c, 3 * nf * 4);
    l.node_bend = take(c, 6 * nb * 4);
    l.dbg_bins = take(c, 4 * nb * 4);
    l.tri = take(c, 3 * nf * 4);
    l.fref = take(c, nf * sizeof(FaceRef));
    l.face_cap = take(c, nf * 4);
    l.face_F = take(c, 9 * nf * 4);
    l.caps = take(c, l.max_caps * sizeof(CapDev));
    l.capV = take(c, l.max_caps * 8);
    l.cap_mom = take(c, l.max_caps * MOM_STRIDE * 8);
    l.red = take(c, RED_BLOCKS * 8 * 8);
    l.cscale = take(c, 4 * sizeof(float));
    l.dpart = take(c, (size_t)dblocks * 2 * 8);
    l.dmass = take(c, 2 * 8);
    size_t s = 0;
    l.slot_f = take(s, fbytes);
    l.slot_rho = take(s, 4 * N * sizeof(float));
    l.slot_off = take(s, 6 * nb * 4);
    l.slot_cs = take(s, 4 * sizeof(float));
    l.slot_bytes = (s + 255) & ~size_t(255);
    l.slot0 = take(c, (size_t)std::max(p->n_slots, 0) * l.slot_bytes);
    l.adjoint = p->ring_len > 0 && !half && max_nodes > 0;
    l.node_area = take(c, nb * 4);
    if (l.adjoint) {
        l.lam[0] = take(c, fbytes);
        l.lam[1] = take(c, fbytes);
        l.lam_rho = take(c, 2 * N * 4);
        l.lam_j = take(c, 6 * N * 4);
        l.lam_S = take(c, 6 * N * 4);
        l.lam_u = take(c, 3 * N * 4);
        l.lam_Fib = take(c, 3 * N * 4);
        l.lam_X = take(c, 3 * nb * 4);
        l.lam_Fb = take(c, 3 * nb * 4);
        l.lam_q = take(c, 3 * nb * 4);
        l.lam_Xg = take(c, 3 * nb * 4);
        l.node_g = take(c, 2 * nb * 8);
        l.capdV = take(c, l.max_caps * 8);
        l.grads = take(c, 4 * 8);
        size_t r = 0;
        l.ring_f = take(r, fbytes);
        l.ring_rho = take(r, 2 * N * 4);
        l.ring_off = take(r, 6 * nb * 4);
        l.ring_bytes = (r + 255) & ~size_t(255);
        l.ring0 = take(c, (size_t)p->ring_len * l.ring_bytes);
    }
    if (l.bb) {
        // links: a triangle of these meshes is pierced by a few links; 64 per
        // triangle is far above what a membrane moving under 1 lu per step
        // produces (overflow is reported as LBM_EUNSTABLE)
        l.link_cap = (int)std::min<int64_t>(64 * nf + 1024, (int64_t)1 << 30);
        l.fresh_cap = (int)std::min<int64_t>(std::max<int64_t>(4 * nb, 4096), (int64_t)1 << 30);
        l.lab = take(c, N * 4);
        l.lab_new = take(c, N * 4);
        l.lpar = take(c, N * 4);
        l.lkey = take(c, (size_t)9 * N * 8);
        l.links = take(c, (size_t)l.link_cap * 16);
        l.link_rho = take(c, (size_t)l.link_cap * 32);
        l.face_cen = take(c, (size_t)nf * 3 * 8);
        l.fresh = take(c, (size_t)l.fresh_cap * 4);
        l.bb_count = take(c, 8 * 4);
        l.bbox = take(c, l.max_caps * 8 * 4);
        l.bb_com = take(c, l.max_caps * 3 * 8);
        l.bb_mass = take(c, 4 * 8);
        l.node_V = take(c, 3 * nb * 4);
        l.P_cur = take(c, 3 * nb * 8);
        l.P_prev = take(c, 3 * nb * 8);
        l.QR = take(c, 3 * nb * 8);
    }
    l.total = (c + 255) & ~size_t(255);
    return l;
}

// z planes per lattice block.  A longer march amortises the two halo planes
// of the ring; the FP16 form gains from it when the grid still holds at
// least 8192 blocks (32 per compute unit), the FP32 form does not.
// Population streams: a buffer of at most 512 MiB (128^3 in FP32) streams
// with non-temporal loads and cached stores, a larger one the other way round.
bool lattice_cached(const lbm_params* p) {
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    if (p->stream_policy == 0) return N * 2 * Q * (p->precision == LBM_FP16 ? 2 : 4) <= ((int64_t)512 << 20);
    return p->stream_policy == 1;
}

bool one_pass_allowed(const lbm_params* p) {
    return p->precision == LBM_FP32 && p->walls == 0 && p->coupling == 0 && p->ring_len == 0;
}

// One lattice pass where allowed and the populations exceed the caches'
// reach: at 256^3 and 512^3 it is 1.24x the two passes' speed on the
// lattice, at 128^3 0.98x.
bool one_pass_for(const lbm_params* p) {
    if (p->lattice_passes == 1) return true;
    return p->lattice_passes == 0 && one_pass_allowed(p) && !lattice_cached(p);
}

// z planes per lattice block.  Sixteen where the grid keeps enough blocks:
// the FP16 collide with 8192 or more (+5% at 512^3), the one-pass collide
// with 2048 or more (each chunk pulls two ring planes it does not collide:
// +4% at 256^3, 32 and 64 planes within 1% at 512^3).
int zc_for(const lbm_params* p) {
    const int64_t cols = (int64_t)((p->nx + BX - 1) / BX) * ((p->ny + BY - 1) / BY);
    const int64_t blocks16 = cols * ((p->nz + 2 * ZC - 1) / (2 * ZC));
    if (p->precision == LBM_FP16 && blocks16 >= 8192) return 2 * ZC;
    if (one_pass_for(p) && blocks16 >= 2048) return 2 * ZC;
    return ZC;
}

std::string validate(const lbm_params* p) {
    if (!p) return "params is NULL";
    if (p->nx < 4 || p->ny < 4 || p->nz < 4) return "lattice sizes must be >= 4";
    // kernels address one component of one direction with 32-bit offsets
    if ((int64_t)p->nx * p->ny * p->nz > ((int64_t)1 << 30)) return "lattice too large (more than 2^30 nodes)";
    if (p->precision != LBM_FP32 && p->precision != LBM_FP16) return "precision must be LBM_FP32 or LBM_FP16";
    if (p->walls < 0 || p->walls > 2) return "walls must be 0, 1 or 2";
    if (p->walls == 1 && p->ny < 5) return "walls need ny >= 5";
    if (p->walls == 2 && p->ring_len > 0) return "the adjoint does not cover on-site velocity boundaries (walls = 2)";
    for (int c = 0; c < 2; ++c)
        if (!(p->tau[c] > 0.5) || !isfinite(p->tau[c])) return "tau must be finite and > 0.5";
    if (!(p->G >= 0.0) || !isfinite(p->G)) return "G must be finite and >= 0";
    for (int k = 0; k < 3; ++k)
        if (!isfinite(p->wall_u_lo[k]) || !isfinite(p->wall_u_hi[k])) return "wall velocities must be finite";
    if (!isfinite(p->rho_maj) || !isfinite(p->rho_min)) return "rho_maj / rho_min must be finite";
    if (!(p->wet_scale >= 0.0) || !isfinite(p->wet_scale)) return "wet_scale must be finite and >= 0";
    if (p->n_slots < 0 || p->n_slots > 4096) return "n_slots out of range";
    if (p->check_every < 0) return "check_every must be >= 0";
    if (p->use_graphs != 0 && p->use_graphs != 1) return "use_graphs must be 0 or 1";
    if (p->ring_len < 0 || p->ring_len > 100000) return "ring_len out of range";
    if (p->ring_len > 0 && p->precision != LBM_FP32) return "the adjoint needs FP32 storage";
    if (p->stream_policy < 0 || p->stream_policy > 2) return "stream_policy must be 0, 1 or 2";
    if (p->zchunk != 0 && (p->zchunk % ZC != 0 || p->zchunk > 8 * ZC)) return "zchunk must be 0 or a multiple of 8 up to 64";
    if (p->psi_kind != 0 && p->psi_kind != 1) return "psi_kind must be 0 or 1";
    if (!(p->rep_eps >= 0.0) || !isfinite(p->rep_eps)) return "rep_eps must be finite and >= 0";
    if (p->rep_eps > 0.0 && !(p->rep_d0 > 0.0 && p->rep_d0 <= 2.0)) return "rep_d0 must be in (0, 2]";
    if (p->coupling != 0 && p->coupling != 1) return "coupling must be 0 (immersed boundary) or 1 (bounce-back)";
    if (p->deterministic != 0 && p->deterministic != 1) return "deterministic must be 0 or 1";
    if (p->lattice_passes < 0 || p->lattice_passes > 2) return "lattice_passes must be 0, 1 or 2";
    if (p->lattice_passes == 1 && !one_pass_allowed(p))
        return "lattice_passes 1 needs FP32 storage, walls 0, coupling 0 and ring_len 0";
    if (p->mass_fix != 0 && p->mass_fix != 1) return "mass_fix must be 0 or 1";
    if (p->mass_fix && (p->precision != LBM_FP32 || p->check_every <= 0 || p->walls == 2))
        return "mass_fix needs FP32 storage, check_every > 0 and walls 0 or 1";
    if (p->deterministic && p->coupling == 1)
        return "deterministic mode covers the immersed boundary (coupling 0) only";
    if (p->coupling == 1) {
        if (p->precision != LBM_FP32) return "the bounce-back coupling needs FP32 storage";
        if (p->walls != 0) return "the bounce-back coupling runs in a periodic box (walls = 0)";
        if (p->n_slots != 0 || p->ring_len != 0) return "the bounce-back coupling has no checkpoints or adjoint";
        if (p->rep_eps != 0.0) return "the bounce-back coupling has no particle-particle repulsion";
        if (!(p->node_mass > 0.0) || !isfinite(p->node_mass)) return "node_mass must be finite and > 0";
        if (!(p->mass_c0 >= 0.0) || !isfinite(p->mass_c0)) return "mass_c0 must be finite and >= 0";
    }
    return "";
}

double cos_deg(double t) { return t == 90.0 ? 0.0 : cos(t * (M_PI / 180.0)); }

}  // namespace

struct lbm_ctx {
    lbm_params p;
    Lattice L;
    Dev d;
    Layout lay;
    char* ws = nullptr;
    hipStream_t stream = nullptr;
    // the membrane kernels that read no density of the step run on a second
    // stream beside the density pass, forked from and joined to `stream`
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool interp_pending = false;   // the last step's advection is still to launch
    unsigned group_used = 0;       // bit k: kernel group k launched something in an event-timed step of the call
    int64_t max_nodes = 0, max_faces = 0;
    int64_t step = 0;
    int device = -1;               // the device current at lbm_init
    double* scratch = nullptr;     // that device's address of the static scratch (lbm_observables_noalloc)
    int flip = 0;                  // parity of the immersed-boundary tile lists
    double mass0[2] = {0, 0};
    std::vector<int64_t> slot_step;
    // host copies of the capsule set
    std::vector<CapDev> caps;
    std::vector<float> off;        // [nodes][3]
    std::vector<int> node_cap;
    std::vector<float> node_wet;
    std::vector<float> node_area;
    // adjoint run description
    int adj_nsteps = 0, adj_every = 0, adj_obj = 0, adj_cap = 0;
    int64_t adj_step0 = -1;
    // reverse sweep driven step by step (lbm_adjoint_seed / _record / _step)
    bool adj_seeded = false;
    int adj_p = 0;                 // parity of the adjoint population buffers
    int rec_len = 0, rec_next = -1;
    int64_t rec_step0 = 0;
    bool launched = false;         // a step (or its graph) has been enqueued
    std::vector<int> tri_global;
    std::vector<FaceRef> fref;
    std::vector<int> face_cap;
    int n_nodes = 0, n_faces = 0;
    hipGraphExec_t graph[2][2][2] = {};  // [step parity][flip][advection pending at the start]
    bool graphs_failed = false;
    bool bending = false;          // some capsule has a bending modulus
    // the bounce-back coupling
    BBSizes bbz{};
    BBConst bbk{};
    bool bb_primed = false;        // the first step detects no fresh nodes
    std::string err;

    bool half() const { return p.precision == LBM_FP16; }

    ~lbm_ctx() {
        for (auto& plane : graph)
            for (auto& row : plane)
                for (auto& g : row)
                    if (g) (void)hipGraphExecDestroy(g);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (side) (void)hipStreamDestroy(side);
    }

    int fail(int code, const char* fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
};

#define HIPCHK(ctx, call)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) return (ctx)->fail(LBM_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Node and face ids are 32-bit, and the node and face arrays hold three
// entries per id, so both counts stay below 2^29.
constexpr int64_t MAX_IDS = (int64_t)1 << 29;

extern "C" {

int lbm_workspace_bytes(const lbm_params* p, int64_t max_nodes, int64_t max_faces, int64_t* bytes) {
    const std::string e = validate(p);
    if (!e.empty()) { g_init_error = e; return LBM_EINVAL; }
    if (max_nodes < 0 || max_faces < 0 || max_nodes > MAX_IDS || max_faces > MAX_IDS || !bytes) {
        g_init_error = "bad sizes (max_nodes, max_faces in [0, 2^29]) or NULL output";
        return LBM_EINVAL;
    }
    *bytes = (int64_t)make_layout(p, max_nodes, max_faces).total;
    return LBM_OK;
}

int lbm_init(const lbm_params* p, const float* rhoA, const float* rhoB, void* workspace, int64_t ws_bytes,
             int64_t max_nodes, int64_t max_faces, void* hip_stream, lbm_ctx** out) {
    if (out) *out = nullptr;
    const std::string e = validate(p);
    if (!e.empty()) { g_init_error = e; return LBM_EINVAL; }
    if (!out || !rhoA || !rhoB || !workspace || max_nodes < 0 || max_faces < 0 || max_nodes > MAX_IDS ||
        max_faces > MAX_IDS) {
        g_init_error = "NULL argument, or max_nodes / max_faces outside [0, 2^29]";
        return LBM_EINVAL;
    }
    if (((uintptr_t)workspace & 255) != 0) { g_init_error = "workspace must be 256-byte aligned"; return LBM_EINVAL; }
    const Layout lay = make_layout(p, max_nodes, max_faces);
    if (ws_bytes < (int64_t)lay.total) {
        g_init_error = "workspace too small: need " + std::to_string(lay.total) + " bytes";
        return LBM_ENOMEM;
    }
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    double m[2] = {0, 0};
    for (int64_t k = 0; k < N; ++k) {
        const int y = (int)((k / p->nx) % p->ny);
        const bool fluid = p->walls != 1 || (y > 0 && y < p->ny - 1);
        if (!fluid) continue;
        if (!(rhoA[k] > 0.0f) || !(rhoB[k] > 0.0f) || !isfinite(rhoA[k]) || !isfinite(rhoB[k])) {
            g_init_error = "initial densities must be finite and > 0 on fluid nodes";
            return LBM_EINVAL;
        }
        m[0] += rhoA[k];
        m[1] += rhoB[k];
    }
    lbm_ctx* c = new lbm_ctx();
    c->p = *p;
    // the static scratch of lbm_observables_noalloc on this device (once per device)
    {
        hipError_t er0 = hipGetDevice(&c->device);
        if (er0 == hipSuccess) er0 = resolve_scratch(c->device, &c->scratch);
        if (er0 != hipSuccess) {
            g_init_error = std::string("device scratch address: ") + hipGetErrorString(er0);
            delete c;
            return LBM_EHIP;
        }
    }
    c->lay = lay;
    c->ws = (char*)workspace;
    c->stream = (hipStream_t)hip_stream;
    c->max_nodes = max_nodes;
    c->max_faces = max_faces;
    c->mass0[0] = m[0];
    c->mass0[1] = m[1];
    c->slot_step.assign(std::max(p->n_slots, 0), -1);
    Lattice& L = c->L;
    L.nx = p->nx; L.ny = p->ny; L.nz = p->nz;
    L.ntx = (p->nx + TILE - 1) / TILE; L.nty = (p->ny + TILE - 1) / TILE; L.ntz = (p->nz + TILE - 1) / TILE;
    L.nbx = (p->nx + BIN - 1) / BIN; L.nby = (p->ny + BIN - 1) / BIN; L.nbz = (p->nz + BIN - 1) / BIN;
    L.n = N;
    L.psi_exp = p->psi_kind;
    L.zc = p->zchunk ? p->zchunk : zc_for(p);
    L.cached = lattice_cached(p) ? 1 : 0;
    L.one = one_pass_for(p) ? 1 : 0;
    L.walls = p->walls == 1 ? 1 : 0;
    L.onsite = p->walls == 2 ? 1 : 0;
    L.G = (float)p->G;
    for (int k = 0; k < 2; ++k) { L.tau[k] = (float)p->tau[k]; L.omega[k] = (float)(1.0 / p->tau[k]); }
    for (int k = 0; k < 3; ++k) { L.uw_lo[k] = (float)p->wall_u_lo[k]; L.uw_hi[k] = (float)p->wall_u_hi[k]; }
    Dev& d = c->d;
    d.det = p->deterministic ? 1 : 0;
    char* w = c->ws;
    d.f[0] = (void*)(w + lay.f[0]);
    d.f[1] = (void*)(w + lay.f[1]);
    d.cscale = (float*)(w + lay.cscale);
    d.dpart = (double*)(w + lay.dpart);
    d.dmass = (double*)(w + lay.dmass);
    d.rho[0] = (float*)(w + lay.rho[0]);
    d.rho[1] = (float*)(w + lay.rho[1]);
    d.fib = (float*)(w + lay.fib);
    d.u = (float*)(w + lay.u);
    d.tile_flag = (int*)(w + lay.tile_flag);
    d.tile_count = (int*)(w + lay.tile_count);
    d.tile_offset = (int*)(w + lay.tile_offset);
    d.home_start = (int*)(w + lay.home_start);
    for (int k = 0; k < 2; ++k) { d.touched[k] = (int*)(w + lay.touched[k]); d.home[k] = (int*)(w + lay.home[k]); }
    d.counters = (int*)(w + lay.counters);
    d.off_hi = (float*)(w + lay.off_hi);
    d.off_lo = (float*)(w + lay.off_lo);
    d.node_cap = (int*)(w + lay.node_cap);
    d.node_anc = (int4*)(w + lay.node_anc);
    d.node_wet = (float*)(w + lay.node_wet);
    d.node_F = (float*)(w + lay.node_F);
    d.node_tile = (int*)(w + lay.node_tile);
    d.node_rank = (int*)(w + lay.node_rank);
    d.sorted = (int*)(w + lay.sorted);
    d.csr_ptr = (int*)(w + lay.csr_ptr);
    d.corner_slot = (int*)(w + lay.corner_slot);
    d.slot_corner = (int*)(w + lay.slot_corner);
    d.node_bend = (float*)(w + lay.node_bend);
    d.dbg_bins = (int*)(w + lay.dbg_bins);
    d.tri = (int*)(w + lay.tri);
    d.fref = (FaceRef*)(w + lay.fref);
    d.face_cap = (int*)(w + lay.face_cap);
    d.face_F = (float*)(w + lay.face_F);
    d.caps = (CapDev*)(w + lay.caps);
    d.capV = (double*)(w + lay.capV);
    d.cap_mom = (double*)(w + lay.cap_mom);
    d.red = (double*)(w + lay.red);
    d.node_area = (float*)(w + lay.node_area);
    L.sharp = lay.bb ? 1 : 0;
    if (lay.bb) {
        d.lab = (int*)(w + lay.lab);
        d.lab_new = (int*)(w + lay.lab_new);
        d.lpar = (unsigned*)(w + lay.lpar);
        d.lkey = (unsigned long long*)(w + lay.lkey);
        d.links = (int4*)(w + lay.links);
        d.link_rho = (double4*)(w + lay.link_rho);
        d.face_cen = (double*)(w + lay.face_cen);
        d.fresh = (int*)(w + lay.fresh);
        d.bb_count = (int*)(w + lay.bb_count);
        d.bbox = (int*)(w + lay.bbox);
        d.bb_com = (double*)(w + lay.bb_com);
        d.bb_mass = (double*)(w + lay.bb_mass);
        d.node_V = (float*)(w + lay.node_V);
        d.P_cur = (double*)(w + lay.P_cur);
        d.P_prev = (double*)(w + lay.P_prev);
        d.QR = (double*)(w + lay.QR);
        c->bbz.link_cap = lay.link_cap;
        c->bbz.fresh_cap = lay.fresh_cap;
        c->bbz.ext = 0;
        BBConst& k = c->bbk;
        for (int j = 0; j < 2; ++j) {
            k.m0[j] = m[j];
            k.rho_init[j] = m[j] / (double)N;
        }
        k.vsys = (double)N;
        k.c0 = p->mass_c0;
        k.inv_mass = (float)(1.0 / p->node_mass);
        k.psi_exp = p->psi_kind;
    }
    if (lay.adjoint) {
        d.lam[0] = (void*)(w + lay.lam[0]);
        d.lam[1] = (void*)(w + lay.lam[1]);
        d.lam_rho = (float*)(w + lay.lam_rho);
        d.lam_j = (float*)(w + lay.lam_j);
        d.lam_S = (float*)(w + lay.lam_S);
        d.lam_u = (float*)(w + lay.lam_u);
        d.lam_Fib = (float*)(w + lay.lam_Fib);
        d.lam_X = (float*)(w + lay.lam_X);
        d.lam_Fb = (float*)(w + lay.lam_Fb);
        d.lam_q = (float*)(w + lay.lam_q);
        d.lam_Xg = (float*)(w + lay.lam_Xg);
        d.node_g = (double*)(w + lay.node_g);
        d.capdV = (double*)(w + lay.capdV);
        d.grads = (double*)(w + lay.grads);
    }

    hipStream_t s = c->stream;
    // initial densities into both density buffers (the previous-step buffer
    // feeds the wall bounce-back of the first step), rest populations in f[0]
    auto bad = [&](hipError_t er, const char* what) {
        g_init_error = std::string(what) + ": " + hipGetErrorString(er);
        delete c;
        return LBM_EHIP;
    };
    hipError_t er;
    for (int b = 0; b < 2; ++b) {
        if ((er = hipMemcpyAsync(d.rho[b], rhoA, N * sizeof(float), hipMemcpyHostToDevice, s)) != hipSuccess)
            return bad(er, "hipMemcpyAsync");
        if ((er = hipMemcpyAsync(d.rho[b] + N, rhoB, N * sizeof(float), hipMemcpyHostToDevice, s)) != hipSuccess)
            return bad(er, "hipMemcpyAsync");
    }
    const bool half = p->precision == LBM_FP16;
    launch_init_rest(L, d.f[0], d.rho[0], d.rho[0] + N, half, s);
    static const float ones[4] = {1.0f, 1.0f, 1.0f, 1.0f};
    if ((er = hipMemcpyAsync(d.cscale, ones, sizeof ones, hipMemcpyHostToDevice, s)) != hipSuccess)
        return bad(er, "hipMemcpyAsync");
    // (the first step decodes with the initial densities and unit compensation)
    if (L.onsite) launch_onsite(L, d.f[0], half, d.rho[1], d.cscale + 2, s);
    if ((er = hipMemsetAsync(d.fib, 0, (lay.bb ? 6 : 5) * N * sizeof(float), s)) != hipSuccess)
        return bad(er, "hipMemsetAsync");
    if ((er = hipMemsetAsync(d.tile_flag, 0, lay.tiles * 4, s)) != hipSuccess) return bad(er, "hipMemsetAsync");
    if ((er = hipMemsetAsync(d.tile_count, 0, lay.bins * 4, s)) != hipSuccess) return bad(er, "hipMemsetAsync");
    if ((er = hipMemsetAsync(d.counters, 0, 8 * 4, s)) != hipSuccess) return bad(er, "hipMemsetAsync");
    if (lay.bb) {
        const size_t nb3 = 3 * (size_t)std::max<int64_t>(max_nodes, 1);
        launch_bb_init(L, d, s);
        if ((er = hipMemsetAsync(d.bb_count, 0, 8 * 4, s)) != hipSuccess) return bad(er, "hipMemsetAsync");
        if ((er = hipMemsetAsync(d.bb_mass, 0, 4 * 8, s)) != hipSuccess) return bad(er, "hipMemsetAsync");
        if ((er = hipMemsetAsync(d.node_V, 0, nb3 * 4, s)) != hipSuccess) return bad(er, "hipMemsetAsync");
        if ((er = hipMemsetAsync(d.P_cur, 0, nb3 * 8, s)) != hipSuccess) return bad(er, "hipMemsetAsync");
        if ((er = hipMemsetAsync(d.P_prev, 0, nb3 * 8, s)) != hipSuccess) return bad(er, "hipMemsetAsync");
        if ((er = hipMemsetAsync(d.QR, 0, nb3 * 8, s)) != hipSuccess) return bad(er, "hipMemsetAsync");
    }
    if ((er = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking)) != hipSuccess)
        return bad(er, "hipStreamCreateWithFlags");
    if ((er = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming)) != hipSuccess)
        return bad(er, "hipEventCreateWithFlags");
    if ((er = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming)) != hipSuccess)
        return bad(er, "hipEventCreateWithFlags");
    if (lay.adjoint) {
        if ((er = hipMemsetAsync(d.lam_u, 0, 3 * N * 4, s)) != hipSuccess) return bad(er, "hipMemsetAsync");
        if ((er = hipMemsetAsync(d.capdV, 0, lay.max_caps * 8, s)) != hipSuccess) return bad(er, "hipMemsetAsync");
    }
    if ((er = hipGetLastError()) != hipSuccess) return bad(er, "init kernel launch");
    // the host arrays may be freed once the copies are done
    if ((er = hipStreamSynchronize(s)) != hipSuccess) return bad(er, "hipStreamSynchronize");
    *out = c;
    return LBM_OK;
}

int lbm_capsules_add(lbm_ctx* c, int32_t n_caps, const int32_t* nodes_per_cap, const int32_t* faces_per_cap,
                     const double* xyz_rest, const int32_t* tri, const double* kS, const double* C,
                     const double* kV, const double* theta_deg, int32_t* first_id) {
    if (!c) return LBM_EINVAL;
    // (sticky: a state loaded back to step 0 still has graphs and tile lists
    // built for the capsules present at the first step)
    if (c->step != 0 || c->launched) return c->fail(LBM_ESTATE, "capsules must be added before the first step");
    if (n_caps < 0) return c->fail(LBM_EINVAL, "n_caps < 0");
    if (n_caps == 0) { if (first_id) *first_id = (int32_t)c->caps.size(); return LBM_OK; }
    if (!nodes_per_cap || !faces_per_cap || !xyz_rest || !tri || !kS || !C || !kV || !theta_deg)
        return c->fail(LBM_EINVAL, "NULL capsule array");
    int64_t add_nodes = 0, add_faces = 0;
    for (int k = 0; k < n_caps; ++k) {
        if (nodes_per_cap[k] < 4 || faces_per_cap[k] < 4) return c->fail(LBM_EINVAL, "capsule %d: too few nodes/faces", k);
        if (!(kS[k] > 0.0) || !(C[k] > -0.5) || !(kV[k] >= 0.0) || !isfinite(kS[k]) || !isfinite(C[k]) || !isfinite(kV[k]))
            return c->fail(LBM_EINVAL, "capsule %d: need kS > 0, C > -1/2, kV >= 0", k);
        if (!(theta_deg[k] >= 0.0 && theta_deg[k] <= 180.0)) return c->fail(LBM_EINVAL, "capsule %d: theta outside [0, 180]", k);
        add_nodes += nodes_per_cap[k];
        add_faces += faces_per_cap[k];
    }
    if (c->n_nodes + add_nodes > c->max_nodes || c->n_faces + add_faces > c->max_faces ||
        (int64_t)c->caps.size() + n_caps > c->lay.max_caps)
        return c->fail(LBM_ENOMEM, "capsules exceed the workspace sizes given to lbm_init");
    const double rv_scale = 2.0 * (c->p.rho_maj - c->p.rho_min) * c->p.wet_scale;
    int64_t nofs = 0, fofs = 0;
    // validate the whole batch before touching the context: indices,
    // positions, every node on some triangle, no degenerate triangle, and a
    // positive rest volume (outward triangles)
    for (int k = 0; k < n_caps; ++k) {
        const int nn = nodes_per_cap[k], nf = faces_per_cap[k];
        const double* X = xyz_rest + 3 * nofs;
        const int32_t* T = tri + 3 * fofs;
        std::vector<char> used(nn, 0);
        for (int f = 0; f < nf; ++f)
            for (int j = 0; j < 3; ++j) {
                const int v = T[3 * f + j];
                if (v < 0 || v >= nn) return c->fail(LBM_EINVAL, "capsule %d: triangle index out of range", k);
                used[v] = 1;
            }
        for (int64_t b = 0; b < 3 * (int64_t)nn; ++b)
            if (!isfinite(X[b])) return c->fail(LBM_EINVAL, "capsule %d: non-finite position", k);
        for (int b = 0; b < nn; ++b)
            if (!used[b]) return c->fail(LBM_EINVAL, "capsule %d: node %d is on no triangle", k, b);
        double V = 0.0;
        for (int f = 0; f < nf; ++f) {
            const double* a = X + 3 * T[3 * f];
            const double* bq = X + 3 * T[3 * f + 1];
            const double* cc = X + 3 * T[3 * f + 2];
            double e1[3], e2[3];
            for (int j = 0; j < 3; ++j) { e1[j] = bq[j] - a[j]; e2[j] = cc[j] - a[j]; }
            const double n0 = e1[1] * e2[2] - e1[2] * e2[1], n1 = e1[2] * e2[0] - e1[0] * e2[2],
                         n2 = e1[0] * e2[1] - e1[1] * e2[0];
            if (!(n0 * n0 + n1 * n1 + n2 * n2 > 0.0)) return c->fail(LBM_EINVAL, "capsule %d: degenerate triangle %d", k, f);
            // (1/6) a . (b x c) summed: the enclosed volume, relative to the first node
            double r1[3], r2[3], r0[3];
            for (int j = 0; j < 3; ++j) { r0[j] = a[j] - X[j]; r1[j] = bq[j] - X[j]; r2[j] = cc[j] - X[j]; }
            V += (r0[0] * (r1[1] * r2[2] - r1[2] * r2[1]) + r0[1] * (r1[2] * r2[0] - r1[0] * r2[2]) +
                  r0[2] * (r1[0] * r2[1] - r1[1] * r2[0])) / 6.0;
        }
        if (!(V > 0.0)) return c->fail(LBM_EINVAL, "capsule %d: rest volume not positive (triangles must face outward)", k);
        if (c->lay.bb) {
            // the bounce-back coupling labels the lattice nodes in a box around
            // each capsule: room for it to deform by half its size again plus
            // the box margin, without wrapping onto itself
            for (int j = 0; j < 3; ++j) {
                double lo = X[j], hi = X[j];
                for (int b = 1; b < nn; ++b) {
                    lo = std::min(lo, X[3 * b + j]);
                    hi = std::max(hi, X[3 * b + j]);
                }
                const int need = (int)ceil(1.5 * (hi - lo)) + 9;
                if (need > std::min(c->p.nx, std::min(c->p.ny, c->p.nz)))
                    return c->fail(LBM_EINVAL, "capsule %d: too large for the lattice under the bounce-back coupling", k);
            }
        }
        nofs += nn;
        fofs += nf;
    }
    if (c->lay.bb) {
        for (int k = 0, o = 0; k < n_caps; o += nodes_per_cap[k], ++k)
            for (int j = 0; j < 3; ++j) {
                const double* X = xyz_rest + 3 * (size_t)o;
                double lo = X[j], hi = X[j];
                for (int b = 1; b < nodes_per_cap[k]; ++b) {
                    lo = std::min(lo, X[3 * b + j]);
                    hi = std::max(hi, X[3 * b + j]);
                }
                c->bbz.ext = std::max(c->bbz.ext, (int)ceil(1.5 * (hi - lo)) + 9);
            }
    }
    // Parity colours of the bounce-back labels: each capsule counts only the
    // crossings of its own colour, so capsules whose boxes may meet (anchors
    // within one box capacity on every axis, periodic) get different colours;
    // the step reports two boxes of one colour that do meet.
    std::vector<int> colour(n_caps, 0);
    if (c->lay.bb) {
        std::vector<std::array<int, 3>> anc;
        std::vector<int> col;
        for (const CapDev& e : c->caps) {
            anc.push_back({e.anchor[0], e.anchor[1], e.anchor[2]});
            col.push_back(e.colour);
        }
        const int nn3[3] = {c->p.nx, c->p.ny, c->p.nz};
        for (int k = 0, o = 0; k < n_caps; o += nodes_per_cap[k], ++k) {
            std::array<int, 3> a;
            for (int j = 0; j < 3; ++j) {
                double m = 0.0;
                for (int b = 0; b < nodes_per_cap[k]; ++b) m += xyz_rest[3 * ((size_t)o + b) + j];
                a[j] = (int)floor(m / nodes_per_cap[k] + 0.5);
            }
            unsigned used = 0u;
            for (size_t e = 0; e < anc.size(); ++e) {
                bool near = true;
                for (int j = 0; j < 3; ++j) {
                    int dd = (a[j] - anc[e][j]) % nn3[j];
                    if (dd < 0) dd += nn3[j];
                    dd = std::min(dd, nn3[j] - dd);
                    near = near && dd < c->bbz.ext;
                }
                if (near) used |= 1u << col[e];
            }
            if (used == 0xffffffffu)
                return c->fail(LBM_EINVAL, "capsule %d: more than 32 capsules within one label box of each other "
                                           "under the bounce-back coupling", k);
            int q = 0;
            while (used & (1u << q)) ++q;
            colour[k] = q;
            anc.push_back(a);
            col.push_back(q);
        }
    }
    if (first_id) *first_id = (int32_t)c->caps.size();
    nofs = fofs = 0;
    for (int k = 0; k < n_caps; ++k) {
        const int nn = nodes_per_cap[k], nf = faces_per_cap[k];
        const double* X = xyz_rest + 3 * nofs;
        const int32_t* T = tri + 3 * fofs;
        CapDev cd;
        double mean[3] = {0, 0, 0};
        for (int b = 0; b < nn; ++b)
            for (int j = 0; j < 3; ++j) mean[j] += X[3 * b + j];
        for (int j = 0; j < 3; ++j) cd.anchor[j] = (int)floor(mean[j] / nn + 0.5);
        cd.node_start = c->n_nodes;
        cd.node_count = nn;
        cd.face_start = c->n_faces;
        cd.face_count = nf;
        const double dr = cos_deg(theta_deg[k]);
        const double rv = dr * rv_scale;
        cd.pref = rv >= 0.0 ? 0 : 1;
        cd.rv_abs = (float)fabs(rv);
        // d|rho_v|/dtheta per radian for the preferred component chosen here
        cd.drv = (float)((cd.pref == 0 ? 1.0 : -1.0) * (-sin(theta_deg[k] * (M_PI / 180.0))) * rv_scale);
        cd.kS = (float)kS[k];
        cd.C = (float)C[k];
        cd.kV = (float)kV[k];
        cd.kB = 0.0f;
        cd.vp[0] = cd.vp[1] = cd.vp[2] = 0.0f;
        cd.prescribed = 0;
        cd.colour = colour[k];
        // rest geometry in FP64, relative to the anchor
        std::vector<double> R(3 * (size_t)nn);
        for (int b = 0; b < nn; ++b)
            for (int j = 0; j < 3; ++j) R[3 * b + j] = X[3 * b + j] - cd.anchor[j];
        std::vector<double> narea(nn, 0.0);
        double V0 = 0.0;
        const int cap_id = (int)c->caps.size();
        for (int f = 0; f < nf; ++f) {
            const double* a = &R[3 * T[3 * f + 0]];
            const double* b = &R[3 * T[3 * f + 1]];
            const double* cc = &R[3 * T[3 * f + 2]];
            double e1[3], e2[3];
            for (int j = 0; j < 3; ++j) { e1[j] = b[j] - a[j]; e2[j] = cc[j] - a[j]; }
            const double m11 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
            const double m12 = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
            const double m22 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
            const double det = m11 * m22 - m12 * m12;
            if (!(det > 0.0)) return c->fail(LBM_EINVAL, "capsule %d: degenerate triangle %d", k, f);
            FaceRef fr;
            fr.q11 = (float)(m22 / det);
            fr.q12 = (float)(-m12 / det);
            fr.q22 = (float)(m11 / det);
            fr.inv_det0 = (float)(1.0 / det);
            const double A0 = 0.5 * sqrt(det);
            fr.A0 = (float)A0;
            for (int j = 0; j < 3; ++j) narea[T[3 * f + j]] += A0 / 3.0;
            V0 += (a[0] * (b[1] * cc[2] - b[2] * cc[1]) + a[1] * (b[2] * cc[0] - b[0] * cc[2])
                   + a[2] * (b[0] * cc[1] - b[1] * cc[0])) / 6.0;
            c->fref.push_back(fr);
            c->face_cap.push_back(cap_id);
            for (int j = 0; j < 3; ++j) c->tri_global.push_back(cd.node_start + T[3 * f + j]);
        }
        if (!(V0 > 0.0)) return c->fail(LBM_EINVAL, "capsule %d: rest volume not positive (triangles must face outward)", k);
        cd.V0 = V0;
        for (int b = 0; b < nn; ++b) {
            for (int j = 0; j < 3; ++j) c->off.push_back((float)R[3 * b + j]);
            c->node_cap.push_back(cap_id);
            c->node_wet.push_back((float)(fabs(rv) * narea[b]));
            c->node_area.push_back((float)narea[b]);
        }
        c->caps.push_back(cd);
        c->n_nodes += nn;
        c->n_faces += nf;
        nofs += nn;
        fofs += nf;
    }
    // node -> (face, corner) adjacency: the corners of node b, in face
    // order, own slots ptr[b] .. ptr[b+1]-1, where the face kernels store
    // their corner forces
    std::vector<int> ptr(c->n_nodes + 1, 0), slot(3 * (size_t)c->n_faces);
    for (int f = 0; f < c->n_faces; ++f)
        for (int j = 0; j < 3; ++j) ptr[c->tri_global[3 * f + j] + 1]++;
    for (int b = 0; b < c->n_nodes; ++b) ptr[b + 1] += ptr[b];
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (int f = 0; f < c->n_faces; ++f)
        for (int j = 0; j < 3; ++j) slot[3 * f + j] = fill[c->tri_global[3 * f + j]]++;
    std::vector<int> slot_corner(3 * (size_t)c->n_faces);
    for (int64_t q = 0; q < 3 * (int64_t)c->n_faces; ++q) slot_corner[slot[q]] = (int)q;
    std::vector<int> anc(4 * (size_t)c->n_nodes);
    for (int b = 0; b < c->n_nodes; ++b) {
        const CapDev& cd = c->caps[c->node_cap[b]];
        for (int j = 0; j < 3; ++j) anc[4 * b + j] = cd.anchor[j];
        anc[4 * b + 3] = cd.pref;
    }
    Dev& d = c->d;
    hipStream_t s = c->stream;
    const size_t nb = c->n_nodes, nf = c->n_faces;
    std::vector<float> zeros(3 * nb, 0.0f);
    HIPCHK(c, hipMemcpyAsync(d.off_hi, c->off.data(), 3 * nb * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(d.off_lo, zeros.data(), 3 * nb * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(d.node_cap, c->node_cap.data(), nb * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(d.node_wet, c->node_wet.data(), nb * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(d.node_area, c->node_area.data(), nb * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(d.csr_ptr, ptr.data(), (nb + 1) * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(d.corner_slot, slot.data(), 3 * nf * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(d.slot_corner, slot_corner.data(), 3 * nf * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(d.node_anc, anc.data(), nb * 16, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(d.tri, c->tri_global.data(), 3 * nf * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(d.fref, c->fref.data(), nf * sizeof(FaceRef), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(d.face_cap, c->face_cap.data(), nf * 4, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(d.caps, c->caps.data(), c->caps.size() * sizeof(CapDev), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return LBM_OK;
}

static int check_mass(lbm_ctx* c) {
    Dev& d = c->d;
    const int pw = (int)((c->step & 1) ^ 1);   // parity of the step that wrote the state
    launch_reduce_fluid(c->L, d.f[c->step & 1], c->half(), d.rho[pw], d.cscale, pw, d.red, c->stream);
    std::vector<double> part(RED_BLOCKS * 8);
    HIPCHK(c, hipMemcpyAsync(part.data(), d.red, part.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // the intended masses: the start, plus the bounce-back coupling's own change when the storage is compensated
    double target[2] = {c->mass0[0], c->mass0[1]};
    if (c->p.mass_fix && c->lay.bb) {
        double led[2];
        HIPCHK(c, hipMemcpyAsync(led, d.bb_mass, sizeof led, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        target[0] += led[0];
        target[1] += led[1];
    }
    double m[2] = {0.0, 0.0};
    for (int comp = 0; comp < 2; ++comp) {
        for (int b = 0; b < RED_BLOCKS; ++b) m[comp] += part[b * 8 + comp];
        // (on-site boundaries exchange mass with the outside: finiteness only)
        if (!isfinite(m[comp]) ||
            (!c->L.onsite && fabs(m[comp] - target[comp]) > c->p.mass_tol * fabs(c->mass0[comp])))
            return c->fail(LBM_EUNSTABLE, "step %lld: mass of component %d is %.17g (start %.17g, intended %.17g)",
                           (long long)c->step, comp, m[comp], c->mass0[comp], target[comp]);
    }
    if (c->p.mass_fix && m[0] > 0.0 && m[1] > 0.0) {
        launch_scale_pops(c->L, d.f[c->step & 1], (float)(target[0] / m[0]), (float)(target[1] / m[1]),
                          c->stream);
        HIPCHK(c, hipGetLastError());
    }
    return LBM_OK;
}

// Enqueue one time step from fin / rho_p into fout / rho_n.  ev (may be
// NULL) receives LBM_NK + 1 events: ev[k] is recorded before kernel group k
// and ev[LBM_NK] after the last.  advect = false leaves the nodes in place
// (the adjoint's recompute of a step's intermediates).
// With `ev` the kernels run in order on one stream with an event before
// each group (the per-kernel timing), and so they do without `overlap` (the
// adjoint's recompute).  Otherwise the membrane kernels
// that read no density of this step (the previous step's advection when it
// was deferred, tile clearing, volumes, triangle forces, the node gather and
// the bin sort) run on the side stream beside the density pass and join
// before the optional node terms and the spreading, which adds the
// wettability reaction (the one membrane term that reads the step's
// densities).  With `defer_interp` this step's
// advection is left to the next step's side branch; the caller launches the
// last one pending before it returns.
static void enqueue_core(lbm_ctx* c, const void* fin, void* fout, float* rho_n, const float* rho_p, bool advect,
                         hipEvent_t* ev, bool overlap = false, bool defer_interp = false) {
    const Lattice& L = c->L;
    Dev& d = c->d;
    hipStream_t s = c->stream;
    const bool ibm = c->n_nodes > 0;
    const int ncap = (int)c->caps.size();
    const int cur = (int)(c->step & 1), nxt = cur ^ 1;
    const int par = c->flip;
    const bool half = c->half();
    const float* cs = half ? d.cscale + 2 * cur : nullptr;
    auto mark = [&](int k) { if (ev) (void)hipEventRecord(ev[k], s); };
    const bool fork = overlap && !ev && fout && ibm;
    c->launched = true;
    if (ev) {
        // the groups this step launches kernels in (the others read 0 in lbm_step_timed)
        unsigned u = 0;
        auto use = [&](int k, bool on) { if (on) u |= 1u << k; };
        use(LBM_K_CLEAR, c->interp_pending || ibm);
        use(LBM_K_DENSITY, fout != nullptr && !L.one);
        for (int k : {LBM_K_VOLUME, LBM_K_FACES, LBM_K_NODES, LBM_K_SCAN, LBM_K_SCATTER, LBM_K_SPREAD}) use(k, ibm);
        use(LBM_K_REPULSE, ibm && c->p.rep_eps > 0.0 && ncap > 1);
        use(LBM_K_BEND, ibm && c->bending);
        use(LBM_K_COLLIDE, fout != nullptr);
        use(LBM_K_INTERP, fout != nullptr && ibm && advect);
        c->group_used |= u;
    }
    hipStream_t m = fork ? c->side : s;       // the membrane kernels' stream up to the join
    if (fork) {
        (void)hipEventRecord(c->ev_fork, s);
        (void)hipStreamWaitEvent(c->side, c->ev_fork, 0);
    }
    mark(LBM_K_CLEAR);
    if (c->interp_pending) {
        // the previous step's advection and this step's clearing, one launch
        launch_advect_clear(L, d, c->n_nodes, par ^ 1, par, ncap, m);
        c->interp_pending = false;
    } else if (ibm) {
        launch_clear_tiles(L, d, par ^ 1, par, ncap, m);
    }
    if (fork) {
        launch_cap_volume(d, c->n_faces, ncap, m);
        launch_faces(d, c->n_faces, m);
        launch_node_gather(L, d, c->n_nodes, par, m);
        launch_bin_scan(d, c->n_nodes, par, m);
        launch_bin_scatter(L, d, c->n_nodes, par, m);
        (void)hipEventRecord(c->ev_join, m);
    }
    mark(LBM_K_DENSITY);
    // (one pass: the collide forms the densities; an adjoint recompute,
    // fout NULL, never runs in that form)
    if (fout && !L.one) launch_density(L, fin, rho_p, rho_n, half, d.cscale, nxt, d.dpart, s);
    // (on-site boundaries exchange mass with the outside, so there is no
    // fixed total to restore: their FP16 form keeps unit compensation)
    if (half && fout && !L.onsite)
        launch_compensate(L, d.dpart, c->mass0[0], c->mass0[1], d.cscale, cur, d.dmass, s);
    if (fork) {
        (void)hipStreamWaitEvent(s, c->ev_join, 0);
    } else {
        mark(LBM_K_VOLUME);
        if (ibm) launch_cap_volume(d, c->n_faces, ncap, s);
        mark(LBM_K_FACES);
        if (ibm) launch_faces(d, c->n_faces, s);
        mark(LBM_K_NODES);
        if (ibm) launch_node_gather(L, d, c->n_nodes, par, s);
        mark(LBM_K_SCAN);
        if (ibm) launch_bin_scan(d, c->n_nodes, par, s);
        mark(LBM_K_SCATTER);
        if (ibm) launch_bin_scatter(L, d, c->n_nodes, par, s);
    }
    mark(LBM_K_REPULSE);
    if (ibm && c->p.rep_eps > 0.0 && ncap > 1)
        launch_repulse(L, d, c->n_nodes, (float)c->p.rep_eps, (float)c->p.rep_d0, s);
    mark(LBM_K_BEND);
    if (ibm && c->bending) launch_bending(d, c->n_nodes, s);
    mark(LBM_K_SPREAD);
    // one pass: the densities of the touched tiles, for the wettability
    // reaction (timed with the spreading)
    // (counters[par] counts the touched tiles of list par)
    if (ibm && L.one && fout) launch_density_tiles(L, fin, rho_n, d.touched[par], d.counters + par, d.tile_flag, s);
    if (ibm) launch_spread(L, d, par, rho_n, cs, s);
    mark(LBM_K_COLLIDE);
    if (!fout) {
        // the adjoint's recompute stops here: intermediates of the step only
        c->flip ^= 1;
        return;
    }
    launch_collide(L, fin, fout, rho_n, rho_p, d.fib, d.tile_flag, d.u, ibm, false, half, d.cscale, nxt, cur, s);
    if (L.onsite) launch_onsite(L, fout, half, rho_n, d.cscale + 2 * cur, s);
    mark(LBM_K_INTERP);
    if (ibm && advect) {
        if (defer_interp && fork)
            c->interp_pending = true;
        else
            launch_interp_advect(L, d, c->n_nodes, s);
    }
    mark(LBM_NK);
    c->step++;
    c->flip ^= 1;
}

// One step of the bounce-back coupling (see k_bb.hip), on one stream:
// the head (labels of the membranes at X^n, fresh nodes, the bounce-back of
// the populations that cross them, tile flags), the density pass, the
// membrane forces, the Shan-Chen sum across the membranes, the collide and
// the node update.
static void enqueue_bb_step(lbm_ctx* c, hipEvent_t* ev) {
    const Lattice& L = c->L;
    Dev& d = c->d;
    hipStream_t s = c->stream;
    const int ncap = (int)c->caps.size();
    const int cur = (int)(c->step & 1), nxt = cur ^ 1;
    void* fin = d.f[cur];
    void* fout = d.f[nxt];
    float* rho_n = d.rho[cur];
    const float* rho_p = d.rho[nxt];
    auto mark = [&](int k) { if (ev) (void)hipEventRecord(ev[k], s); };
    c->launched = true;
    if (ev) {
        unsigned u = (1u << LBM_K_CLEAR) | (1u << LBM_K_DENSITY) | (1u << LBM_K_COLLIDE);
        if (c->n_faces > 0) u |= (1u << LBM_K_VOLUME) | (1u << LBM_K_FACES);
        if (c->n_nodes > 0) u |= (1u << LBM_K_NODES) | (1u << LBM_K_INTERP);
        if (c->bending) u |= 1u << LBM_K_BEND;
        if (ncap) u |= 1u << LBM_K_SPREAD;
        c->group_used |= u;
    }
    mark(LBM_K_CLEAR);
    launch_bb_geometry(L, d, c->bbz, ncap, c->n_faces, c->bb_primed, s);
    launch_bb_refill(L, d, c->bbz, c->bbk, fin, rho_p, ncap, s);
    launch_bb_fixup(L, d, c->bbz, fin, ncap, s);
    launch_bb_flags(L, d, c->bbz, ncap, s);
    c->bb_primed = true;
    mark(LBM_K_DENSITY);
    launch_density(L, fin, rho_p, rho_n, false, d.cscale, nxt, d.dpart, s);
    mark(LBM_K_VOLUME);
    launch_cap_volume(d, c->n_faces, ncap, s);
    mark(LBM_K_FACES);
    launch_faces(d, c->n_faces, s);
    mark(LBM_K_NODES);
    launch_gather_forces(d, c->n_nodes, s);
    mark(LBM_K_SCAN);
    mark(LBM_K_SCATTER);
    mark(LBM_K_REPULSE);
    mark(LBM_K_BEND);
    if (c->bending) launch_bending(d, c->n_nodes, s);
    mark(LBM_K_SPREAD);
    if (ncap) launch_bb_shan_chen(L, d, c->bbz, c->bbk, rho_n, s);
    mark(LBM_K_COLLIDE);
    launch_collide(L, fin, fout, rho_n, rho_p, d.fib, d.tile_flag, d.u, ncap > 0, false, false, d.cscale, nxt, cur,
                   s);
    mark(LBM_K_INTERP);
    launch_bb_advance(d, c->bbk, c->n_nodes, s);
    mark(LBM_NK);
    c->step++;
}

// The overflow and consistency flags of the bounce-back coupling's lists
// (synchronises).
static int check_bb(lbm_ctx* c) {
    int cnt[8];
    HIPCHK(c, hipMemcpyAsync(cnt, c->d.bb_count, sizeof cnt, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int f = cnt[2];
    if (f & 1) return c->fail(LBM_EUNSTABLE, "step %lld: a capsule outgrew its label box", (long long)c->step);
    if (f & 2) return c->fail(LBM_EUNSTABLE, "step %lld: more membrane links than the list holds", (long long)c->step);
    if (f & 4) return c->fail(LBM_EUNSTABLE, "step %lld: more fresh nodes than the list holds", (long long)c->step);
    if (f & 8) return c->fail(LBM_EUNSTABLE, "step %lld: a membrane is not closed (odd crossings)", (long long)c->step);
    if (f & 16)
        return c->fail(LBM_EUNSTABLE, "step %lld: the label boxes of two capsules of one parity colour met",
                       (long long)c->step);
    return LBM_OK;
}

static void enqueue_step(lbm_ctx* c, hipEvent_t* ev, bool defer_interp = false) {
    if (c->lay.bb) {
        enqueue_bb_step(c, ev);
        return;
    }
    const int cur = (int)(c->step & 1), nxt = cur ^ 1;
    enqueue_core(c, c->d.f[cur], c->d.f[nxt], c->d.rho[cur], c->d.rho[nxt], true, ev, true, defer_interp);
}

// Two steps captured as one graph; both leave their advection to the next
// step, so a graph ends with one pending, and its first step takes over the
// one pending before it, if any.  The launch arguments depend only on the
// step parity, the tile-list parity and that pending advection, so eight
// graphs cover every state.
static hipGraphExec_t two_step_graph(lbm_ctx* c) {
    const int sp = (int)(c->step & 1), fp = c->flip, pin = c->interp_pending ? 1 : 0;
    if (c->graph[sp][fp][pin]) return c->graph[sp][fp][pin];
    if (c->graphs_failed || c->stream == nullptr) return nullptr;
    const int64_t step0 = c->step;
    const int flip0 = c->flip;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        c->graphs_failed = true;
        (void)hipGetLastError();
        return nullptr;
    }
    enqueue_step(c, nullptr, true);
    enqueue_step(c, nullptr, true);
    const hipError_t e = hipStreamEndCapture(c->stream, &g);
    c->step = step0;
    c->flip = flip0;
    c->interp_pending = pin != 0;
    hipGraphExec_t ex = nullptr;
    if (e != hipSuccess || !g || hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        c->graphs_failed = true;
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return nullptr;
    }
    (void)hipGraphDestroy(g);
    c->graph[sp][fp][pin] = ex;
    return ex;
}


int lbm_capsules_velocity(lbm_ctx* c, int32_t first_id, int32_t n_caps, const double* v, int32_t prescribed) {
    if (!c) return LBM_EINVAL;
    if (!c->lay.bb) return c->fail(LBM_EINVAL, "node velocities need the bounce-back coupling (coupling = 1)");
    if (n_caps < 0 || first_id < 0 || (int64_t)first_id + n_caps > (int64_t)c->caps.size())
        return c->fail(LBM_EINVAL, "capsule range outside the capsules added");
    if (n_caps == 0) return LBM_OK;
    if (!v) return c->fail(LBM_EINVAL, "NULL v");
    for (int k = 0; k < 3 * n_caps; ++k)
        if (!isfinite(v[k]) || !(fabs(v[k]) < 0.5)) return c->fail(LBM_EINVAL, "velocities must be finite and below 0.5");
    std::vector<float> V;
    const int b0 = c->caps[first_id].node_start;
    for (int k = 0; k < n_caps; ++k) {
        CapDev& cd = c->caps[first_id + k];
        for (int j = 0; j < 3; ++j) cd.vp[j] = (float)v[3 * k + j];
        cd.prescribed = prescribed != 0;
        for (int b = 0; b < cd.node_count; ++b)
            for (int j = 0; j < 3; ++j) V.push_back(cd.vp[j]);
    }
    // (stream-ordered after the steps already enqueued)
    HIPCHK(c, hipMemcpyAsync(c->d.node_V + 3 * (size_t)b0, V.data(), V.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d.caps, c->caps.data(), c->caps.size() * sizeof(CapDev), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm_capsules_bending(lbm_ctx* c, int32_t first_id, int32_t n_caps, const double* kB) {
    if (!c) return LBM_EINVAL;
    if (c->step != 0 || c->launched) return c->fail(LBM_ESTATE, "bending moduli must be set before the first step");
    if (n_caps < 0 || first_id < 0 || (int64_t)first_id + n_caps > (int64_t)c->caps.size())
        return c->fail(LBM_EINVAL, "capsule range outside the capsules added");
    if (n_caps == 0) return LBM_OK;
    if (!kB) return c->fail(LBM_EINVAL, "NULL kB");
    bool any = false;
    for (int k = 0; k < n_caps; ++k) {
        if (!(kB[k] >= 0.0) || !isfinite(kB[k])) return c->fail(LBM_EINVAL, "capsule %d: kB must be finite and >= 0", first_id + k);
        any = any || kB[k] > 0.0;
    }
    if (any && c->p.ring_len > 0) return c->fail(LBM_EINVAL, "the adjoint does not differentiate bending: kB must be 0");
    for (int k = 0; k < n_caps; ++k) c->caps[first_id + k].kB = (float)kB[k];
    bool on = false;
    for (const CapDev& cd : c->caps) on = on || cd.kB > 0.0f;
    c->bending = on;
    for (auto& plane : c->graph)
        for (auto& row : plane)
            for (auto& e : row)
                if (e) { (void)hipGraphExecDestroy(e); e = nullptr; }
    HIPCHK(c, hipMemcpyAsync(c->d.caps, c->caps.data(), c->caps.size() * sizeof(CapDev), hipMemcpyHostToDevice, c->stream));
    return LBM_OK;
}

int lbm_reference_relax(lbm_ctx* c, int32_t nsteps, double gamma, double w, double z_interface, double mobility) {
    if (!c) return LBM_EINVAL;
    if (nsteps < 0) return c->fail(LBM_EINVAL, "nsteps < 0");
    if (!(gamma >= 0.0) || !isfinite(gamma)) return c->fail(LBM_EINVAL, "gamma must be finite and >= 0");
    if (!(w > 0.0) || !isfinite(w)) return c->fail(LBM_EINVAL, "w must be finite and > 0");
    if (!isfinite(z_interface)) return c->fail(LBM_EINVAL, "z_interface must be finite");
    if (!(mobility > 0.0) || !isfinite(mobility)) return c->fail(LBM_EINVAL, "mobility must be finite and > 0");
    if (c->caps.empty() || nsteps == 0) return LBM_OK;
    Dev& d = c->d;
    // the axes: each capsule's centre of mass now
    launch_cap_moments(d, (int)c->caps.size(), c->stream);
    for (int k = 0; k < nsteps; ++k)
        launch_reference_step(d, c->n_nodes, c->n_faces, (int)c->caps.size(), c->bending, (float)gamma, (float)w,
                              z_interface, (float)mobility, c->stream);
    HIPCHK(c, hipGetLastError());
    return LBM_OK;
}
int lbm_step(lbm_ctx* c, int32_t nsteps) {
    if (!c) return LBM_EINVAL;
    if (nsteps < 0) return c->fail(LBM_EINVAL, "nsteps < 0");
    if (c->lay.bb) {
        // After the first step (which lists no fresh nodes) a step's launches
        // depend only on its parity: pairs of steps are replayed from the
        // same two-step graphs, never across a check.
        int left = nsteps;
        while (left > 0) {
            const int ce = c->p.check_every;
            hipGraphExec_t ex = nullptr;
            if (c->p.use_graphs && c->bb_primed && left >= 2 && (ce == 0 || c->step % ce + 2 <= ce))
                ex = two_step_graph(c);
            if (ex) {
                HIPCHK(c, hipGraphLaunch(ex, c->stream));
                c->step += 2;
                left -= 2;
            } else {
                enqueue_bb_step(c, nullptr);
                --left;
            }
            if (ce > 0 && c->step % ce == 0) {
                HIPCHK(c, hipGetLastError());
                int r = check_bb(c);
                if (r == LBM_OK) r = check_mass(c);
                if (r != LBM_OK) return r;
            }
        }
        HIPCHK(c, hipGetLastError());
        return nsteps > 0 ? check_bb(c) : LBM_OK;
    }
    int left = nsteps;
    while (left > 0) {
        int chunk = left;
        if (c->p.check_every > 0) chunk = std::min<int64_t>(chunk, c->p.check_every - c->step % c->p.check_every);
        left -= chunk;
        while (chunk >= 2 && c->p.use_graphs) {
            hipGraphExec_t ex = two_step_graph(c);
            if (!ex) break;
            HIPCHK(c, hipGraphLaunch(ex, c->stream));
            c->step += 2;
            c->interp_pending = c->n_nodes > 0;
            chunk -= 2;
        }
        for (; chunk > 0; --chunk) enqueue_step(c, nullptr, true);
        // the last advection, so that the call leaves the nodes moved
        if (c->interp_pending) {
            launch_interp_advect(c->L, c->d, c->n_nodes, c->stream);
            c->interp_pending = false;
        }
        HIPCHK(c, hipGetLastError());
        if (c->p.check_every > 0 && c->step % c->p.check_every == 0) {
            const int r = check_mass(c);
            if (r != LBM_OK) return r;
        }
    }
    return LBM_OK;
}

int lbm_step_timed(lbm_ctx* c, int32_t nsteps, double* kernel_ms) {
    if (!c || !kernel_ms) return c ? c->fail(LBM_EINVAL, "NULL output") : LBM_EINVAL;
    if (nsteps < 1) return c->fail(LBM_EINVAL, "nsteps < 1");
    std::vector<hipEvent_t> ev((size_t)nsteps * (LBM_NK + 1));
    for (auto& e : ev) HIPCHK(c, hipEventCreate(&e));
    c->group_used = 0;
    for (int k = 0; k < nsteps; ++k) enqueue_step(c, &ev[(size_t)k * (LBM_NK + 1)]);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->lay.bb) {
        const int r = check_bb(c);
        if (r != LBM_OK) {
            for (auto& e : ev) (void)hipEventDestroy(e);
            return r;
        }
    }
    for (int j = 0; j < LBM_NK; ++j) kernel_ms[j] = 0.0;
    for (int k = 0; k < nsteps; ++k)
        for (int j = 0; j < LBM_NK; ++j) {
            if (!(c->group_used >> j & 1u)) continue;     // (a group with no launch reads 0)
            float ms = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms, ev[(size_t)k * (LBM_NK + 1) + j], ev[(size_t)k * (LBM_NK + 1) + j + 1]));
            kernel_ms[j] += ms;
        }
    for (auto& e : ev) (void)hipEventDestroy(e);
    return LBM_OK;
}

// eigenvalues of a symmetric 3x3 matrix (cyclic Jacobi), ascending
static void eig3(double A[3][3], double ev[3]) {
    for (int sweep = 0; sweep < 50; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        if (off < 1e-300) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (A[p][q] == 0.0) continue;
                const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < 3; ++k) {
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = cs * akp - sn * akq;
                    A[k][q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = cs * apk - sn * aqk;
                    A[q][k] = sn * apk + cs * aqk;
                }
            }
    }
    ev[0] = A[0][0]; ev[1] = A[1][1]; ev[2] = A[2][2];
    std::sort(ev, ev + 3);
}

// Per-capsule observables from its FP64 shape moments m[MOM_STRIDE] (origin at
// the anchor): [0] V, [1] A, [2..4] sum of node offsets, [5..7] int x dV,
// [8..13] int x x^T dV.
static void cap_obs_from_moments(const CapDev& cd, const double* m, double z_interface, lbm_capsule_obs& o) {
    const double V = m[0];
    o.volume = V;
    o.area = m[1];
    for (int j = 0; j < 3; ++j) o.com[j] = cd.anchor[j] + m[2 + j] / cd.node_count;
    const double xc[3] = {m[5] / V, m[6] / V, m[7] / V};
    double M[3][3];
    M[0][0] = m[8]; M[1][1] = m[9]; M[2][2] = m[10];
    M[0][1] = M[1][0] = m[11];
    M[0][2] = M[2][0] = m[12];
    M[1][2] = M[2][1] = m[13];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i][j] -= V * xc[i] * xc[j];
    double ev[3];
    eig3(M, ev);
    for (int j = 0; j < 3; ++j) o.axes[j] = sqrt(5.0 * std::max(ev[j], 0.0) / V);
    o.taylor_D = (o.axes[2] - o.axes[0]) / (o.axes[2] + o.axes[0]);
    o.height = o.com[2] - z_interface;
}

int lbm_observables(lbm_ctx* c, lbm_obs* out, lbm_capsule_obs* caps) {
    if (!c || !out) return c ? c->fail(LBM_EINVAL, "NULL output") : LBM_EINVAL;
    Dev& d = c->d;
    hipStream_t s = c->stream;
    const int pw = (int)((c->step & 1) ^ 1);   // parity of the step that wrote the state
    launch_reduce_fluid(c->L, d.f[c->step & 1], c->half(), d.rho[pw], d.cscale, pw, d.red, s);
    const int ncap = (int)c->caps.size();
    if (caps && ncap) launch_cap_moments(d, ncap, s);
    HIPCHK(c, hipGetLastError());
    std::vector<double> part(RED_BLOCKS * 8), mom((size_t)std::max(ncap, 1) * MOM_STRIDE);
    HIPCHK(c, hipMemcpyAsync(part.data(), d.red, part.size() * 8, hipMemcpyDeviceToHost, s));
    if (caps && ncap)
        HIPCHK(c, hipMemcpyAsync(mom.data(), d.cap_mom, (size_t)ncap * MOM_STRIDE * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    double acc[5] = {0, 0, 0, 0, 0};
    for (int b = 0; b < RED_BLOCKS; ++b)
        for (int j = 0; j < 5; ++j) acc[j] += part[b * 8 + j];
    out->mass[0] = acc[0];
    out->mass[1] = acc[1];
    for (int j = 0; j < 3; ++j) out->momentum[j] = acc[2 + j];
    out->step = c->step;
    for (int j = 0; j < 3; ++j) out->particle_momentum[j] = out->pending_momentum[j] = 0.0;
    if (c->lay.bb && c->n_nodes) {
        const size_t nb = c->n_nodes;
        std::vector<float> V(3 * nb);
        std::vector<double> P(3 * nb);
        HIPCHK(c, hipMemcpyAsync(V.data(), d.node_V, 3 * nb * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(P.data(), d.P_prev, 3 * nb * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        for (size_t b = 0; b < nb; ++b)
            for (int j = 0; j < 3; ++j) {
                out->particle_momentum[j] += c->p.node_mass * V[3 * b + j];
                out->pending_momentum[j] += 0.5 * P[3 * b + j];
            }
    }
    out->mass_ledger[0] = out->mass_ledger[1] = 0.0;
    if (c->lay.bb) {
        HIPCHK(c, hipMemcpyAsync(out->mass_ledger, d.bb_mass, 2 * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    if (caps)
        for (int k = 0; k < ncap; ++k) cap_obs_from_moments(c->caps[k], &mom[(size_t)k * MOM_STRIDE], c->p.z_interface,
                                                            caps[k]);
    return LBM_OK;
}

int lbm_observables_noalloc(lbm_ctx* c, lbm_obs* out, lbm_capsule_obs* caps) {
    if (!c || !out) return c ? c->fail(LBM_EINVAL, "NULL output") : LBM_EINVAL;
    if (!c->scratch) return c->fail(LBM_EHIP, "the static scratch was not resolved on this context's device");
    const int ncap = (int)c->caps.size();
    if (caps && ncap > NOALLOC_MAX_CAPS)
        return c->fail(LBM_EINVAL, "lbm_observables_noalloc handles at most %d capsules (%d here)", NOALLOC_MAX_CAPS, ncap);
    Dev& d = c->d;
    hipStream_t s = c->stream;
    double* part = c->scratch;                               // [RED_BLOCKS][8]
    double* mom = c->scratch + (size_t)RED_BLOCKS * 8;       // [caps][MOM_STRIDE]
    const int pw = (int)((c->step & 1) ^ 1);
    // (every partial and moment is stored, none accumulated: nothing to clear)
    launch_reduce_fluid(c->L, d.f[c->step & 1], c->half(), d.rho[pw], d.cscale, pw, part, s);
    if (caps && ncap) {
        Dev dm = d;
        dm.cap_mom = mom;
        launch_cap_moments(dm, ncap, s);
    }
    HIPCHK(c, hipGetLastError());
    // host side in fixed stack chunks, in the order lbm_observables sums
    constexpr int CH = 64;
    double buf[CH * 8];
    double acc[5] = {0, 0, 0, 0, 0};
    for (int b0 = 0; b0 < RED_BLOCKS; b0 += CH) {
        HIPCHK(c, hipMemcpyAsync(buf, part + (size_t)b0 * 8, sizeof buf, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        for (int b = 0; b < CH; ++b)
            for (int j = 0; j < 5; ++j) acc[j] += buf[b * 8 + j];
    }
    out->mass[0] = acc[0];
    out->mass[1] = acc[1];
    for (int j = 0; j < 3; ++j) out->momentum[j] = acc[2 + j];
    out->step = c->step;
    for (int j = 0; j < 3; ++j) out->particle_momentum[j] = out->pending_momentum[j] = 0.0;
    if (c->lay.bb && c->n_nodes) {
        float vb[3 * CH];
        double pb[3 * CH];
        for (int b0 = 0; b0 < c->n_nodes; b0 += CH) {
            const int n = std::min(CH, c->n_nodes - b0);
            HIPCHK(c, hipMemcpyAsync(vb, d.node_V + 3 * (size_t)b0, 3 * (size_t)n * 4, hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipMemcpyAsync(pb, d.P_prev + 3 * (size_t)b0, 3 * (size_t)n * 8, hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipStreamSynchronize(s));
            for (int b = 0; b < n; ++b)
                for (int j = 0; j < 3; ++j) {
                    out->particle_momentum[j] += c->p.node_mass * vb[3 * b + j];
                    out->pending_momentum[j] += 0.5 * pb[3 * b + j];
                }
        }
    }
    out->mass_ledger[0] = out->mass_ledger[1] = 0.0;
    if (c->lay.bb) {
        HIPCHK(c, hipMemcpyAsync(out->mass_ledger, d.bb_mass, 2 * 8, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    if (caps) {
        double mb[MOM_STRIDE];
        for (int k = 0; k < ncap; ++k) {
            HIPCHK(c, hipMemcpyAsync(mb, mom + (size_t)k * MOM_STRIDE, sizeof mb, hipMemcpyDeviceToHost, s));
            HIPCHK(c, hipStreamSynchronize(s));
            cap_obs_from_moments(c->caps[k], mb, c->p.z_interface, caps[k]);
        }
    }
    return LBM_OK;
}

int lbm_get_fields(lbm_ctx* c, float* rhoA, float* rhoB, float* u) {
    if (!c) return LBM_EINVAL;
    if (c->step < 1) return c->fail(LBM_ESTATE, "no step has been taken");
    Dev& d = c->d;
    hipStream_t s = c->stream;
    const int last = (int)((c->step - 1) & 1);
    const int64_t N = c->L.n;
    // one pass leaves the density field written on the touched tiles only:
    // form it everywhere (the same sums) before it is read back
    if (c->L.one) launch_density(c->L, d.f[last], d.rho[last ^ 1], d.rho[last], false, d.cscale, last ^ 1, d.dpart, s);
    if (u) {
        launch_collide(c->L, d.f[last], nullptr, d.rho[last], d.rho[last ^ 1], d.fib, d.tile_flag, d.u,
                       c->n_nodes > 0, true, c->half(), d.cscale, last ^ 1, last, s);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(u, d.u, 3 * N * sizeof(float), hipMemcpyDeviceToHost, s));
    }
    float cs[4] = {1.0f, 1.0f, 1.0f, 1.0f};
    if (c->half()) HIPCHK(c, hipMemcpyAsync(cs, d.cscale, sizeof cs, hipMemcpyDeviceToHost, s));
    if (rhoA) HIPCHK(c, hipMemcpyAsync(rhoA, d.rho[last], N * sizeof(float), hipMemcpyDeviceToHost, s));
    if (rhoB) HIPCHK(c, hipMemcpyAsync(rhoB, d.rho[last] + N, N * sizeof(float), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (c->half()) {
        // the collision used the compensated density
        for (int64_t k = 0; k < N; ++k) {
            if (rhoA) rhoA[k] *= cs[2 * last];
            if (rhoB) rhoB[k] *= cs[2 * last + 1];
        }
    }
    return LBM_OK;
}

int lbm_get_nodes(lbm_ctx* c, double* xyz) {
    if (!c || !xyz) return c ? c->fail(LBM_EINVAL, "NULL output") : LBM_EINVAL;
    const size_t nb = c->n_nodes;
    if (!nb) return LBM_OK;
    std::vector<float> hi(3 * nb), lo(3 * nb);
    HIPCHK(c, hipMemcpyAsync(hi.data(), c->d.off_hi, 3 * nb * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(lo.data(), c->d.off_lo, 3 * nb * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t b = 0; b < nb; ++b) {
        const CapDev& cd = c->caps[c->node_cap[b]];
        for (int j = 0; j < 3; ++j) xyz[3 * b + j] = cd.anchor[j] + (double)hi[3 * b + j] + (double)lo[3 * b + j];
    }
    return LBM_OK;
}

int lbm_get_node_forces(lbm_ctx* c, float* F) {
    if (!c || !F) return c ? c->fail(LBM_EINVAL, "NULL output") : LBM_EINVAL;
    if (c->step < 1) return c->fail(LBM_ESTATE, "no step has been taken");
    if (!c->n_nodes) return LBM_OK;
    HIPCHK(c, hipMemcpyAsync(F, c->d.node_F, 3 * (size_t)c->n_nodes * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm_get_spread(lbm_ctx* c, float* Fib, float* phi) {
    if (!c) return LBM_EINVAL;
    if (c->step < 1) return c->fail(LBM_ESTATE, "no step has been taken");
    const int64_t N = c->L.n;
    if (Fib) HIPCHK(c, hipMemcpyAsync(Fib, c->d.fib, 3 * N * 4, hipMemcpyDeviceToHost, c->stream));
    if (phi) HIPCHK(c, hipMemcpyAsync(phi, c->d.fib + 3 * N, 2 * N * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm_debug_labels(lbm_ctx* c, int32_t* labels) {
    if (!c || !labels) return c ? c->fail(LBM_EINVAL, "NULL output") : LBM_EINVAL;
    if (!c->lay.bb) return c->fail(LBM_EINVAL, "labels need the bounce-back coupling (coupling = 1)");
    Dev& d = c->d;
    hipStream_t s = c->stream;
    // the labels of the current positions, computed as the next step's head
    // does; the fresh-node list is not touched
    launch_bb_geometry(c->L, d, c->bbz, (int)c->caps.size(), c->n_faces, false, s);
    std::vector<int> box(8 * std::max<size_t>(c->caps.size(), 1));
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(labels, d.lab, c->L.n * 4, hipMemcpyDeviceToHost, s));
    std::vector<int> nw(c->L.n);
    HIPCHK(c, hipMemcpyAsync(nw.data(), d.lab_new, c->L.n * 4, hipMemcpyDeviceToHost, s));
    if (!c->caps.empty())
        HIPCHK(c, hipMemcpyAsync(box.data(), d.bbox, box.size() * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    // the new labels are valid inside the capsules' boxes; elsewhere the
    // committed ones (-1 away from every membrane)
    const Lattice& L = c->L;
    for (size_t k = 0; k < c->caps.size(); ++k) {
        const CapDev& cd = c->caps[k];
        const int* bx = &box[8 * k];
        for (int z = bx[2]; z <= bx[5]; ++z)
            for (int y = bx[1]; y <= bx[4]; ++y)
                for (int x = bx[0]; x <= bx[3]; ++x) {
                    auto wr = [](int v, int n) { v %= n; return v < 0 ? v + n : v; };
                    const int64_t node = ((int64_t)wr(cd.anchor[2] + z, L.nz) * L.ny + wr(cd.anchor[1] + y, L.ny)) * L.nx +
                                         wr(cd.anchor[0] + x, L.nx);
                    labels[node] = nw[node];
                }
    }
    return check_bb(c);
}

int lbm_get_node_velocities(lbm_ctx* c, float* V) {
    if (!c || !V) return c ? c->fail(LBM_EINVAL, "NULL output") : LBM_EINVAL;
    const size_t nb = c->n_nodes;
    if (!nb) return LBM_OK;
    if (!c->lay.bb) {
        for (size_t k = 0; k < 3 * nb; ++k) V[k] = 0.0f;
        return LBM_OK;
    }
    HIPCHK(c, hipMemcpyAsync(V, c->d.node_V, 3 * nb * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm_debug_bins(lbm_ctx* c, int32_t* tile_of_node, int32_t* base_idx) {
    if (!c) return LBM_EINVAL;
    const size_t nb = c->n_nodes;
    if (!nb) return LBM_OK;
    launch_debug_bins(c->L, c->d, (int)nb, c->stream);
    HIPCHK(c, hipGetLastError());
    std::vector<int> v(4 * nb);
    HIPCHK(c, hipMemcpyAsync(v.data(), c->d.dbg_bins, 4 * nb * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (size_t b = 0; b < nb; ++b) {
        if (tile_of_node) tile_of_node[b] = v[4 * b];
        if (base_idx)
            for (int j = 0; j < 3; ++j) base_idx[3 * b + j] = v[4 * b + 1 + j];
    }
    return LBM_OK;
}

int lbm_state_save(lbm_ctx* c, int32_t slot) {
    if (!c) return LBM_EINVAL;
    if (slot < 0 || slot >= c->p.n_slots) return c->fail(LBM_EINVAL, "slot %d out of range", slot);
    char* base = c->ws + c->lay.slot0 + (size_t)slot * c->lay.slot_bytes;
    const int64_t N = c->L.n;
    const int cur = (int)(c->step & 1);
    hipStream_t s = c->stream;
    HIPCHK(c, hipMemcpyAsync(base + c->lay.slot_f, c->d.f[cur], c->lay.fbytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(base + c->lay.slot_cs, c->d.cscale, 4 * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(base + c->lay.slot_rho, c->d.rho[0], 2 * N * 4, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(base + c->lay.slot_rho + 2 * N * 4, c->d.rho[1], 2 * N * 4, hipMemcpyDeviceToDevice, s));
    if (c->n_nodes) {
        HIPCHK(c, hipMemcpyAsync(base + c->lay.slot_off, c->d.off_hi, 3 * (size_t)c->n_nodes * 4, hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipMemcpyAsync(base + c->lay.slot_off + 3 * (size_t)c->n_nodes * 4, c->d.off_lo,
                                 3 * (size_t)c->n_nodes * 4, hipMemcpyDeviceToDevice, s));
    }
    c->slot_step[slot] = c->step;
    return LBM_OK;
}

int lbm_state_load(lbm_ctx* c, int32_t slot) {
    if (!c) return LBM_EINVAL;
    if (slot < 0 || slot >= c->p.n_slots) return c->fail(LBM_EINVAL, "slot %d out of range", slot);
    if (c->slot_step[slot] < 0) return c->fail(LBM_ESTATE, "slot %d is empty", slot);
    char* base = c->ws + c->lay.slot0 + (size_t)slot * c->lay.slot_bytes;
    const int64_t N = c->L.n;
    c->step = c->slot_step[slot];
    const int cur = (int)(c->step & 1);
    hipStream_t s = c->stream;
    HIPCHK(c, hipMemcpyAsync(c->d.f[cur], base + c->lay.slot_f, c->lay.fbytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->d.cscale, base + c->lay.slot_cs, 4 * sizeof(float), hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->d.rho[0], base + c->lay.slot_rho, 2 * N * 4, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->d.rho[1], base + c->lay.slot_rho + 2 * N * 4, 2 * N * 4, hipMemcpyDeviceToDevice, s));
    if (c->n_nodes) {
        HIPCHK(c, hipMemcpyAsync(c->d.off_hi, base + c->lay.slot_off, 3 * (size_t)c->n_nodes * 4, hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipMemcpyAsync(c->d.off_lo, base + c->lay.slot_off + 3 * (size_t)c->n_nodes * 4,
                                 3 * (size_t)c->n_nodes * 4, hipMemcpyDeviceToDevice, s));
    }
    return LBM_OK;
}

// ---- adjoint ---------------------------------------------------------------

// eigen-decomposition of a symmetric 3x3 matrix (cyclic Jacobi): values and
// column eigenvectors
static void eig3v(double A[3][3], double ev[3], double V[3][3]) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        if (off < 1e-300) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (A[p][q] == 0.0) continue;
                const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < 3; ++k) {
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = cs * akp - sn * akq;
                    A[k][q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = cs * apk - sn * aqk;
                    A[q][k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = cs * vkp - sn * vkq;
                    V[k][q] = sn * vkp + cs * vkq;
                }
            }
    }
    for (int k = 0; k < 3; ++k) ev[k] = A[k][k];
}

// Taylor deformation D of a closed triangulated surface and its gradient with
// respect to the node positions, in FP64.  V, m1 = int x dV and
// m2 = int x x^T dV are sums over the tetrahedra (origin, a, b, c); the
// central moment is M = m2 - m1 m1^T / V, its eigenvalues mu_k give the
// half-axes a_k = sqrt(5 mu_k / V), D = (a_max - a_min) / (a_max + a_min).
// The gradient runs the same chain backwards (eigenvalue derivative
// v_k^T dM v_k for distinct eigenvalues).
static double taylor_D_grad(const std::vector<double>& X, const int* tri, int nf, std::vector<double>& g) {
    double V = 0, m1[3] = {0, 0, 0}, m2[3][3] = {{0}};
    for (int f = 0; f < nf; ++f) {
        const double* a = &X[3 * tri[3 * f]];
        const double* b = &X[3 * tri[3 * f + 1]];
        const double* cc = &X[3 * tri[3 * f + 2]];
        const double v = (a[0] * (b[1] * cc[2] - b[2] * cc[1]) + a[1] * (b[2] * cc[0] - b[0] * cc[2]) +
                          a[2] * (b[0] * cc[1] - b[1] * cc[0])) / 6.0;
        double s[3];
        for (int j = 0; j < 3; ++j) s[j] = a[j] + b[j] + cc[j];
        V += v;
        for (int i = 0; i < 3; ++i) {
            m1[i] += v * s[i] / 4.0;
            for (int j = 0; j < 3; ++j) m2[i][j] += v / 20.0 * (a[i] * a[j] + b[i] * b[j] + cc[i] * cc[j] + s[i] * s[j]);
        }
    }
    double M[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[i][j] = m2[i][j] - m1[i] * m1[j] / V;
    double ev[3], EV[3][3], Mc[3][3];
    memcpy(Mc, M, sizeof M);
    eig3v(Mc, ev, EV);
    int kmin = 0, kmax = 0;
    for (int k = 1; k < 3; ++k) {
        if (ev[k] < ev[kmin]) kmin = k;
        if (ev[k] > ev[kmax]) kmax = k;
    }
    const double a1 = sqrt(5.0 * ev[kmin] / V), a3 = sqrt(5.0 * ev[kmax] / V);
    const double D = (a3 - a1) / (a3 + a1);
    // backwards: D -> a_k -> (mu_k, V) -> (M, V) -> (m2, m1, V)
    const double den = (a1 + a3) * (a1 + a3);
    const double c3 = 2.0 * a1 / den, c1 = -2.0 * a3 / den;
    double lV = 0.0, lmu[3] = {0, 0, 0};
    lmu[kmax] += c3 * 5.0 / (2.0 * a3 * V);
    lmu[kmin] += c1 * 5.0 / (2.0 * a1 * V);
    lV += -c3 * 5.0 * ev[kmax] / (2.0 * a3 * V * V) - c1 * 5.0 * ev[kmin] / (2.0 * a1 * V * V);
    double lM[3][3] = {{0}};
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) lM[i][j] += lmu[k] * EV[i][k] * EV[j][k];
    double lm1[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) lm1[i] += -2.0 * lM[i][j] * m1[j] / V;
    double m1Lm1 = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) m1Lm1 += m1[i] * lM[i][j] * m1[j];
    lV += m1Lm1 / (V * V);
    g.assign(X.size(), 0.0);
    for (int f = 0; f < nf; ++f) {
        const int id[3] = {tri[3 * f], tri[3 * f + 1], tri[3 * f + 2]};
        const double* P[3] = {&X[3 * id[0]], &X[3 * id[1]], &X[3 * id[2]]};
        const double v = (P[0][0] * (P[1][1] * P[2][2] - P[1][2] * P[2][1]) +
                          P[0][1] * (P[1][2] * P[2][0] - P[1][0] * P[2][2]) +
                          P[0][2] * (P[1][0] * P[2][1] - P[1][1] * P[2][0])) / 6.0;
        double s[3];
        for (int j = 0; j < 3; ++j) s[j] = P[0][j] + P[1][j] + P[2][j];
        double ls = 0.0, Ls[3] = {0, 0, 0}, quad = 0.0;
        for (int i = 0; i < 3; ++i) {
            ls += lm1[i] * s[i];
            for (int j = 0; j < 3; ++j) Ls[i] += lM[i][j] * s[j];
        }
        for (int q = 0; q < 3; ++q)
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) quad += P[q][i] * lM[i][j] * P[q][j];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) quad += 0.0 * s[i] * s[j];
        double sLs = 0.0;
        for (int i = 0; i < 3; ++i) sLs += s[i] * Ls[i];
        // adjoint weight of v for this face
        const double lv = lV + ls / 4.0 + (quad + sLs) / 20.0;
        for (int q = 0; q < 3; ++q) {
            const double* u1 = P[(q + 1) % 3];
            const double* u2 = P[(q + 2) % 3];
            const double dv[3] = {(u1[1] * u2[2] - u1[2] * u2[1]) / 6.0, (u1[2] * u2[0] - u1[0] * u2[2]) / 6.0,
                                  (u1[0] * u2[1] - u1[1] * u2[0]) / 6.0};
            double LP[3] = {0, 0, 0};
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) LP[i] += lM[i][j] * P[q][j];
            for (int j = 0; j < 3; ++j)
                g[3 * id[q] + j] += lv * dv[j] + v * lm1[j] / 4.0 + v / 20.0 * (2.0 * LP[j] + 2.0 * Ls[j]);
        }
    }
    return D;
}

static bool adjoint_ready(lbm_ctx* c) { return c->lay.adjoint && c->n_nodes > 0; }

// ring entry k: populations, previous densities, node offsets (hi, lo)
static char* ring_at(lbm_ctx* c, int k) { return c->ws + c->lay.ring0 + (size_t)k * c->lay.ring_bytes; }

int lbm_adjoint_forward(lbm_ctx* c, int32_t nsteps, int32_t every, int32_t objective, int32_t capsule, double* J) {
    if (!c || !J) return c ? c->fail(LBM_EINVAL, "NULL output") : LBM_EINVAL;
    if (!adjoint_ready(c)) return c->fail(LBM_ESTATE, "the adjoint needs ring_len > 0, FP32 storage and capsules");
    if (nsteps < 1 || every < 1 || every > c->p.ring_len) return c->fail(LBM_EINVAL, "need 1 <= every <= ring_len");
    const int nseg = (nsteps + every - 1) / every;
    if (nseg > c->p.n_slots) return c->fail(LBM_EINVAL, "need n_slots >= ceil(nsteps / every) = %d", nseg);
    if (objective != LBM_OBJ_COM_Z && objective != LBM_OBJ_TAYLOR_D) return c->fail(LBM_EINVAL, "unknown objective");
    if (capsule < 0 || capsule >= (int)c->caps.size()) return c->fail(LBM_EINVAL, "capsule index out of range");
    c->adj_step0 = c->step;
    for (int sgm = 0; sgm < nseg; ++sgm) {
        const int r = lbm_state_save(c, sgm);
        if (r != LBM_OK) return r;
        const int n = std::min(every, nsteps - sgm * every);
        const int r2 = lbm_step(c, n);
        if (r2 != LBM_OK) return r2;
    }
    c->adj_nsteps = nsteps;
    c->adj_every = every;
    c->adj_obj = objective;
    c->adj_cap = capsule;
    std::vector<lbm_capsule_obs> co(c->caps.size());
    lbm_obs o;
    const int r = lbm_observables(c, &o, co.data());
    if (r != LBM_OK) return r;
    *J = objective == LBM_OBJ_COM_Z ? co[capsule].height : co[capsule].taylor_D;
    return LBM_OK;
}

// Seed of the reverse sweep: lambda_X = dJ/dX at the current node positions
// (FP64 on the host), every other adjoint field and the parameter gradients
// zero.
int lbm_adjoint_seed(lbm_ctx* c, int32_t objective, int32_t capsule) {
    if (!c) return LBM_EINVAL;
    if (!adjoint_ready(c)) return c->fail(LBM_ESTATE, "the adjoint needs ring_len > 0, FP32 storage and capsules");
    if (objective != LBM_OBJ_COM_Z && objective != LBM_OBJ_TAYLOR_D) return c->fail(LBM_EINVAL, "unknown objective");
    if (capsule < 0 || capsule >= (int)c->caps.size()) return c->fail(LBM_EINVAL, "capsule index out of range");
    Dev& d = c->d;
    hipStream_t s = c->stream;
    const int64_t N = c->L.n;
    const size_t nb = c->n_nodes;
    std::vector<float> hi(3 * nb), lo(3 * nb), seed(3 * nb, 0.0f);
    HIPCHK(c, hipMemcpyAsync(hi.data(), d.off_hi, 3 * nb * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(lo.data(), d.off_lo, 3 * nb * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const CapDev& cd = c->caps[capsule];
    if (objective == LBM_OBJ_COM_Z) {
        for (int b = 0; b < cd.node_count; ++b) seed[3 * (cd.node_start + b) + 2] = (float)(1.0 / cd.node_count);
    } else {
        std::vector<double> X(3 * (size_t)cd.node_count), gD;
        for (int b = 0; b < cd.node_count; ++b)
            for (int j = 0; j < 3; ++j)
                X[3 * b + j] = (double)hi[3 * (cd.node_start + b) + j] + (double)lo[3 * (cd.node_start + b) + j];
        std::vector<int> tl(3 * (size_t)cd.face_count);
        for (int f = 0; f < 3 * cd.face_count; ++f) tl[f] = c->tri_global[3 * (size_t)cd.face_start + f] - cd.node_start;
        taylor_D_grad(X, tl.data(), cd.face_count, gD);
        for (int b = 0; b < cd.node_count; ++b)
            for (int j = 0; j < 3; ++j) seed[3 * (cd.node_start + b) + j] = (float)gD[3 * b + j];
    }
    HIPCHK(c, hipMemcpyAsync(d.lam_X, seed.data(), 3 * nb * 4, hipMemcpyHostToDevice, s));
    c->adj_p = 0;
    HIPCHK(c, hipMemsetAsync(d.lam[0], 0, c->lay.fbytes, s));
    HIPCHK(c, hipMemsetAsync(d.lam_S, 0, 6 * N * 4, s));
    HIPCHK(c, hipMemsetAsync(d.lam_rho, 0, 2 * N * 4, s));
    HIPCHK(c, hipMemsetAsync(d.lam_j, 0, 6 * N * 4, s));
    HIPCHK(c, hipMemsetAsync(d.grads, 0, 4 * 8, s));
    // (the copy above reads a host vector that goes out of scope)
    HIPCHK(c, hipStreamSynchronize(s));
    c->adj_seeded = true;
    c->rec_len = 0;
    c->rec_next = -1;
    return LBM_OK;
}

// Ring entry 0 = the current state; entries 1 .. nsteps-1 the states after
// each of the next nsteps - 1 recomputed steps.  The context's step counter
// and state are left as they were at the call (node offsets aside, which
// lbm_adjoint_step reloads from the ring).
int lbm_adjoint_record(lbm_ctx* c, int32_t nsteps) {
    if (!c) return LBM_EINVAL;
    if (!adjoint_ready(c)) return c->fail(LBM_ESTATE, "the adjoint needs ring_len > 0, FP32 storage and capsules");
    if (nsteps < 1 || nsteps > c->p.ring_len) return c->fail(LBM_EINVAL, "need 1 <= nsteps <= ring_len");
    Dev& d = c->d;
    hipStream_t s = c->stream;
    const int64_t N = c->L.n;
    const size_t offb = 3 * (size_t)c->n_nodes * 4;
    {
        const int cur = (int)(c->step & 1);
        char* e0 = ring_at(c, 0);
        HIPCHK(c, hipMemcpyAsync(e0 + c->lay.ring_f, d.f[cur], c->lay.fbytes, hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipMemcpyAsync(e0 + c->lay.ring_rho, d.rho[cur ^ 1], 2 * N * 4, hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipMemcpyAsync(e0 + c->lay.ring_off, d.off_hi, offb, hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipMemcpyAsync(e0 + c->lay.ring_off + offb, d.off_lo, offb, hipMemcpyDeviceToDevice, s));
    }
    const int64_t step0 = c->step;
    for (int k = 0; k + 1 < nsteps; ++k) {
        char* ek = ring_at(c, k);
        char* en = ring_at(c, k + 1);
        enqueue_core(c, ek + c->lay.ring_f, en + c->lay.ring_f, (float*)(en + c->lay.ring_rho),
                     (const float*)(ek + c->lay.ring_rho), true, nullptr);
        HIPCHK(c, hipMemcpyAsync(en + c->lay.ring_off, d.off_hi, offb, hipMemcpyDeviceToDevice, s));
        HIPCHK(c, hipMemcpyAsync(en + c->lay.ring_off + offb, d.off_lo, offb, hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(c, hipGetLastError());
    c->step = step0;
    c->rec_step0 = step0;
    c->rec_len = nsteps;
    c->rec_next = nsteps - 1;
    return LBM_OK;
}

// The adjoint of step `ring_index` of the recorded segment, applied to the
// adjoint state; the steps must come in reverse order, last first.
int lbm_adjoint_step(lbm_ctx* c, int32_t ring_index) {
    if (!c) return LBM_EINVAL;
    if (!adjoint_ready(c) || !c->adj_seeded) return c->fail(LBM_ESTATE, "lbm_adjoint_step needs lbm_adjoint_seed first");
    if (c->rec_len < 1) return c->fail(LBM_ESTATE, "lbm_adjoint_step needs lbm_adjoint_record first");
    if (ring_index < 0 || ring_index >= c->rec_len) return c->fail(LBM_EINVAL, "ring_index outside the recorded segment");
    if (ring_index != c->rec_next)
        return c->fail(LBM_ESTATE, "adjoint steps run in reverse order: expected ring_index %d", c->rec_next);
    Dev& d = c->d;
    const Lattice& L = c->L;
    hipStream_t s = c->stream;
    const size_t offb = 3 * (size_t)c->n_nodes * 4;
    const int k = ring_index;
    const int len = c->rec_len;
    char* ek = ring_at(c, k);
    HIPCHK(c, hipMemcpyAsync(d.off_hi, ek + c->lay.ring_off, offb, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(d.off_lo, ek + c->lay.ring_off + offb, offb, hipMemcpyDeviceToDevice, s));
    c->step = c->rec_step0 + k;
    // (the tile-list parity alternates with each enqueued step, recorded or
    // adjoint, so the lists the previous launch flagged are cleared next)
    const int par = c->flip;
    int& p = c->adj_p;
    const void* fin = ek + c->lay.ring_f;
    const float* rho_p = (const float*)(ek + c->lay.ring_rho);
    // the densities of step k are the next ring entry's previous densities;
    // only the segment's last step computes them again
    float* rho_n = k + 1 < len ? (float*)(ring_at(c, k + 1) + c->lay.ring_rho) : d.rho[0];
    if (k + 1 >= len) launch_density(L, fin, rho_p, rho_n, false, d.cscale, 0, d.dpart, s);
    // membrane intermediates of step k: node forces, bins, spread fields
    enqueue_core(c, fin, nullptr, rho_n, rho_p, false, nullptr);
    launch_spread_vec(L, d, par, d.lam_X, d.lam_u, 0, s);
    launch_adj_collide(L, fin, rho_n, rho_p, d.fib, d.tile_flag, d.lam[p], d.lam_u, d.lam_rho, d.lam_j,
                       d.lam_S, d.lam_Fib, d.u, d.grads, s);
    launch_adj_nodes(L, d, rho_n, c->n_nodes, s);
    if (c->p.rep_eps > 0.0 && c->caps.size() > 1)
        launch_adj_repulse(L, d, c->n_nodes, (float)c->p.rep_eps, (float)c->p.rep_d0, s);
    launch_adj_membrane(d, c->n_nodes, c->n_faces, s);
    launch_spread_vec(L, d, par, d.lam_q, d.lam_S, 1, s);
    launch_adj_gather(L, d.lam_S, d.lam_rho, rho_n, s);
    launch_adj_push(L, d.lam[p], d.lam_rho, d.lam_j, d.lam[p ^ 1], s);
    p ^= 1;
    HIPCHK(c, hipGetLastError());
    c->step = c->rec_step0;
    c->rec_next = k - 1;
    return LBM_OK;
}

int lbm_adjoint_grads(lbm_ctx* c, double* grads) {
    if (!c || !grads) return c ? c->fail(LBM_EINVAL, "NULL output") : LBM_EINVAL;
    if (!adjoint_ready(c) || !c->adj_seeded) return c->fail(LBM_ESTATE, "lbm_adjoint_grads needs lbm_adjoint_seed first");
    double g[4];
    HIPCHK(c, hipMemcpyAsync(g, c->d.grads, sizeof g, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    grads[0] = g[0];
    grads[1] = g[1];
    grads[2] = g[2];
    return LBM_OK;
}

int lbm_adjoint_backward(lbm_ctx* c, double* grads) {
    if (!c || !grads) return c ? c->fail(LBM_EINVAL, "NULL output") : LBM_EINVAL;
    if (!adjoint_ready(c) || c->adj_step0 < 0 || c->step != c->adj_step0 + c->adj_nsteps)
        return c->fail(LBM_ESTATE, "lbm_adjoint_backward must follow lbm_adjoint_forward");
    int r = lbm_adjoint_seed(c, c->adj_obj, c->adj_cap);
    if (r != LBM_OK) return r;
    const int nseg = (c->adj_nsteps + c->adj_every - 1) / c->adj_every;
    for (int sgm = nseg - 1; sgm >= 0; --sgm) {
        const int len = std::min(c->adj_every, c->adj_nsteps - sgm * c->adj_every);
        if ((r = lbm_state_load(c, sgm)) != LBM_OK) return r;
        if ((r = lbm_adjoint_record(c, len)) != LBM_OK) return r;
        for (int k = len - 1; k >= 0; --k)
            if ((r = lbm_adjoint_step(c, k)) != LBM_OK) return r;
    }
    // leave the state at the start of the run
    if ((r = lbm_state_load(c, 0)) != LBM_OK) return r;
    if ((r = lbm_adjoint_grads(c, grads)) != LBM_OK) return r;
    c->adj_step0 = -1;
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) { delete c; }

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

}  // extern "C"
