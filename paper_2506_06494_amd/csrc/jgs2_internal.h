// Internal declarations shared by the libjgs2 translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/jgs2.h"

namespace jgs2 {

// Displacement record in FP64 (x, y, z; w spare or m/h^2): positions and the
// inertial target are stored to FP64 so that the iterate can move by less than
// an FP32 ulp of the displacement; every stress and Hessian evaluation is FP32
// on differences taken in FP64.
struct alignas(32) d4 {
    double x, y, z, w;
};
__host__ __device__ inline d4 make_d4(double x, double y, double z, double w) {
    d4 r;
    r.x = x; r.y = y; r.z = z; r.w = w;
    return r;
}

constexpr int LPV = 32;          // lanes per vertex sub-problem
constexpr int VPB = 8;           // vertices per 256-thread block
constexpr int BLOCK = LPV * VPB;
constexpr int KMAX = 32;         // max free one-ring size held in LDS
constexpr int SMAX = 8;          // max cubature samples per vertex
constexpr int SREC = 41;         // floats per sample: w, 4 gcoef, 4 x 9 U-bar
constexpr uint8_t SLOT_SELF = 0xFE;
constexpr uint8_t SLOT_NONE = 0xFF;

// Tet record: 5 x float4 = ids(bitcast) | Dm^-1 (9) | vol | V mu | V lam | rho V / (4 h^2)
constexpr int TET_F4 = 5;
// Incidence record of the plain and linear sweeps, one per (free vertex, incident tet):
// Dm^-1 (9) | V mu | V lam | own corner c (bitcast) | the tet's 4 corner ids (bitcast),
// as 4 float4 planes; rows in colour order, padded with zero records to maxi entries.
// Plane k of entry j of row q is at [(q * IREC_F4 + k) * maxi + j].
constexpr int IREC_F4 = 4;

struct SweepArgs {
    int nV, nVf, maxi, K, S;
    int nT;
    unsigned long long* bounds;  // bounds-checked build: first failed index check (line, index,
                                 // extent); nullptr otherwise
    const int* free_ids;    // [nVf]
    const int* list;        // optional subset of free indices (colour), or nullptr
    int n_list;
    const float4* tet;      // [nT * TET_F4]
    const int* inc;         // [nVf * maxi] packed (tet << 2 | corner), -1 pad
    const int4* inc4;       // [nVf * maxi] (tet << 2 | corner c, ids of corners c+1, c+2, c+3 mod 4)
    // the plain sweep's rows in colour order (position q = rank in the colour permutation)
    const float4* irec_c;   // [nVf * IREC_F4 * maxi] incidence records
    int nt_records;         // stream the records (non-temporal loads): they outgrow the cache
    const int* incn_c;      // [nVf]
    const int* vid_c;       // [nVf] vertex id
    const int* free_c;      // [nVf] free index (row of the correction tables)
    const int* fbody_c;     // [nVf] body
    int cbase;              // first row of the launched colour (0 for a whole sweep)
    const uint32_t* incslot;// [nVf * maxi] one-ring slot byte per corner
    const int* inc_n;       // [nVf]
    const int* ring;        // [nVf * K] vertex ids
    const int* ring_n;      // [nVf]
    const float* Uring;     // [(nVf * 9 + comp) * K + k]
    const int* samp_e;      // [nVf * S]
    const float* samp;      // [(nVf * SREC + field) * S + s]
    const float4* X;        // [nV] rest positions (w unused)
    const d4* u;            // [nV] current displacement x - X (w unused)
    d4* unext;              // [nV]
    const d4* zu;           // [nV] inertial target displacement, w = m_a / h^2 (0 if pinned)
    float4* g;              // [nV] assembled gradient (w unused)
    float4* R;              // [nV] per-vertex rotation as a unit quaternion (x, y, z, w)
    double* partial;        // [gridDim] per-block partial sums of |g|^2
    float omega;
    int in_place;           // write the update into u (coloured GS, plain variant)
    // planes
    int n_planes;
    float planes[JGS2_MAX_PLANES][4];
    float d_hat, kappa;
    double planes_d[JGS2_MAX_PLANES][4];  // the same planes in FP64 (feasibility test)
    // linear (adjoint) sweeps on H(u) y = rhs
    const float4* ly;       // [nV] current y
    float4* lynext;         // [nV] Jacobi output
    const float4* lrhs;     // [nV] right-hand side
    const float* mh2;       // [nV] m_a / h^2 (0 if pinned)
    int no_write;           // residual partials only, no update
    float4* lres;           // [nV] optional: the linear residual H y - rhs per free vertex
    // bodies: a free vertex of a body whose residual reached rel_tol is skipped
    const int* fbody;       // [nVf] body of each free vertex
    const int* body_on;     // [n_bodies] 1 while the body iterates (nullptr: all; the
                            // plain forward sweep requires it)
    int one_body;           // every free vertex is in body 0 (its flag is read once per wave)
    // exact variant: the rest Hessian's inverse in the lower triangle of
    // 64 x 64-vertex tiles over the permuted positions q of the free vertices
    // (tile (I, J), I >= J, at I (I + 1) / 2 + J, laid out [q % 64][3 r + c][q' % 64]),
    // B_q^-1 = ((H-bar^-1)_{q,q})^-1 per position, and per-sweep vectors
    const float* Mt;        // [n_tiles * 64 * 9 * 64]
    const _Float16* Mh;     // the same tiles in FP16, entry / tscale[tile] (after jgs2_exact_tiles_fp16)
    const float* tscale;    // [n_tiles] FP16 tile scale
    const float* Binv;      // [nVf * 9]
    const int* qpos;        // [nV] permuted position of a free vertex, -1 if pinned
    const int* qvert;       // [nVf] vertex id at position q
    const int* qfree;       // [nVf] free index at position q
    float4* hvec;           // [nVf rounded up to 64] R_a^T g_a at position q, zero past nVf
    float4* prow;           // [n_super * ntq * 64] row partials of H-bar^-1 h per super-tile column
    float4* pcol;           // [n_super * ntq * 64] column partials per super-tile row
    float4* yq;             // [nVf] (H-bar^-1 h)_q
    const uint64_t* smask;  // [n_super] bit w MT_SG + j: tile (MT_SG SI + w, MT_SG SJ + j) is streamed (nullptr: all)
    const int2* srange;     // [ns] per super-row SX: live row partials from super-column .x, column
                            // partials up to super-row .y; the rest are zero (nullptr: all)
    const int* slist;       // [n_slive] super-tiles holding a live tile, longest first (nullptr: all)
    int n_slive;
    const int* nactive;     // bodies still iterating (device count; nullptr: always run the product)
};

}  // namespace jgs2

struct jgs2_solver {
    jgs2_params p;
    hipStream_t stream = nullptr;
    std::string err;
    int device = 0;

    // mesh (host)
    int nV = 0, nT = 0, nVf = 0, maxi = 0, K = 0;
    std::vector<double> X;
    std::vector<int> tets;
    std::vector<uint8_t> pinned;
    std::vector<int> free_ids, free_index;
    std::vector<int> inc, inc_n, ring, ring_n;
    std::vector<int4> inc4;
    std::vector<uint32_t> incslot;
    std::vector<int> color, col_perm, col_off;  // colour per vertex, free idx sorted by colour
    int n_colors = 0;
    std::vector<int> valence;
    std::vector<double> vol, Dm_inv;  // per tet (FP64 host copies)
    std::vector<double> E, nu, rho;
    std::vector<double> mass;

    bool have_mesh = false, have_material = false, have_corr = false, have_state = false;
    // body tables (stop flags, chunked residual sums, readback slots) are
    // complete: cleared on entry to set_bodies, set after its last upload
    bool have_bodies = false;
    double corr_dt = 0.0;             // time step the correction was built for
    bool in_step = false, phase1_valid = false;
    int S = 0;
    std::vector<double> fit;          // per free vertex NNLS residual
    std::vector<double> pose_eigs;    // training-pose eigenvalues
    int n_poses = 0;
    double r0 = 0.0;
    int sweeps_in_step = 0;
    int ls_halvings = 0;

    // device
    float4* d_tet = nullptr;
    float4 *d_X = nullptr, *d_vhat = nullptr, *d_g = nullptr, *d_R = nullptr;
    jgs2::d4 *d_u = nullptr, *d_unext = nullptr, *d_uhat = nullptr, *d_zu = nullptr;
    float* d_mh2 = nullptr;
    int *d_free = nullptr, *d_inc = nullptr, *d_inc_n = nullptr, *d_ring = nullptr, *d_ring_n = nullptr;
    int4* d_inc4 = nullptr;
    float4* d_irec_c = nullptr;
    int *d_incn_c = nullptr, *d_vid_c = nullptr, *d_fbody_c = nullptr;
    uint32_t* d_incslot = nullptr;
    int* d_colperm = nullptr;
    float* d_Uring = nullptr;
    float* d_Mt = nullptr;                 // exact variant: H-bar^-1 tiles (see SweepArgs)
    _Float16* d_Mh = nullptr;              // the tiles in FP16 once converted (d_Mt then freed)
    float* d_tscale = nullptr;             // [n_tiles] their scales
    bool tiles_fp16 = false;
    float* d_Binv = nullptr;               // [nVf * 9]
    int* d_qpos = nullptr;                 // [nV]
    int* d_qvert = nullptr;                // [nVf]
    int* d_qfree = nullptr;                // [nVf]
    float4* d_hvec = nullptr;              // [nVf]
    float4* d_part = nullptr;              // [2 * n_super * ntq * 64]: row, then column partials
    float4* d_yq = nullptr;                // [nVf]
    uint64_t* d_smask = nullptr;           // [n_super] live-tile bits per super-tile under p.exact_drop
    int2* d_srange = nullptr;              // [ns] partial ranges per super-row
    int* d_slist = nullptr;                // [n_super] live super-tiles, longest first
    int n_slive = -1;                      // -1: every super-tile
    std::vector<float> tile_max;           // largest |entry| per tile, from the precompute
    int64_t n_live = 0;
    double live_bytes = 0.0;
    double part_bytes = 0.0;
    bool have_full = false;
    double* d_X64 = nullptr;               // device state I/O: FP64 rest positions [nV * 3]
    uint8_t* d_pin8 = nullptr;             // [nV]
    int* d_flag = nullptr;                 // [1]
    int* d_samp_e = nullptr;
    float* d_samp = nullptr;
    double* d_partial = nullptr;
    double* d_red = nullptr;
    int n_partial = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // per-kernel event timing
    bool prof = false;
    double kt_ms[JGS2_NKERNELS] = {};
    int64_t kt_n[JGS2_NKERNELS] = {};
    struct Pending { int k; hipEvent_t a, b; };
    std::vector<Pending> kt_pending;
    std::vector<hipEvent_t> ev_pool;
    // differentiable rollout: checkpoints [n_ck + 1][nV] (last = end state),
    // recomputed segment states [ckpt_every][nV], adjoint vectors
    int ro_steps = 0, ro_every = 0, ro_nck = 0;
    bool ro_valid = false;
    jgs2::d4 *d_ck_u = nullptr, *d_seg = nullptr;
    float4* d_ck_v = nullptr;
    float4 *d_y = nullptr, *d_ynext = nullptr, *d_xbar = nullptr, *d_vbar = nullptr, *d_rhs = nullptr;
    double* d_thbar = nullptr;
    // bodies (disjoint meshes solved together; per-body residuals and masks)
    int n_bodies = 1;
    std::vector<int> body_of_vertex;       // [nV]
    std::vector<int> seg_off, seg_idx;     // free indices grouped by body
    int* d_fbody = nullptr;                // [nVf]
    int* d_seg_idx = nullptr;
    int n_chunks = 0;                      // fixed chunks of the per-body residual sums
    int *d_chunk_lo = nullptr, *d_chunk_hi = nullptr, *d_body_chunk_off = nullptr;
    double* d_r2c = nullptr;
    jgs2::d4* d_uprev = nullptr;           // iterate before the last sweep of a group
    double *d_dx2c = nullptr, *d_dx2 = nullptr;
    double dx_norm = 0.0;
    int* d_body_on = nullptr;              // [n_bodies]
    int* d_body_sweeps = nullptr;          // [n_bodies]
    // one block read back after a check: [0] |u - u_prev|^2, [1] bodies still on
    // (an int in its first 4 bytes), [2..) per-body |g_b|^2; d_dx2, d_nactive and
    // d_r2 point into it
    double* d_rb = nullptr;
    int* d_nactive = nullptr;              // [1]
    unsigned long long* d_bounds = nullptr;  // bounds-checked build: [4] first failed index check
    double *d_r2 = nullptr, *d_r0sq = nullptr;  // [n_bodies]
    std::vector<double> r2_host, r0sq_host;
    int n_active = 0;
    // launch shape of the plain / linear sweep kernels
    int tune_lpv = 32, tune_block = 256;
    int stream_mode = -1;  // incidence records: -1 auto (> 128 MiB), 0 cached, 1 streamed
    bool persistent = false;               // plain GS groups as one cooperative launch
    int* d_coloff = nullptr;               // [n_colors + 1] colour offsets of the colour-ordered rows
    int n_cus = 0;                         // compute units of the device
    // captured sweep groups (k sweeps + residual check) per Jacobi parity
    hipStream_t own_stream = nullptr;
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
    int graph_k[2] = {0, 0};
    jgs2::d4* graph_u[2] = {nullptr, nullptr};
    int graph_next = 0;
    // pinned residual readback slots (two sweep groups in flight)
    // pinned readback slots, each one block laid out like d_rb (aliases into h_rb)
    double* h_rb[2] = {nullptr, nullptr};
    double* h_r2[2] = {nullptr, nullptr};
    int* h_nact[2] = {nullptr, nullptr};
    double* h_dx2[2] = {nullptr, nullptr};
    hipEvent_t rb_ev[2] = {nullptr, nullptr};

    int fail(int code, const std::string& msg) {
        err = msg;
        return code;
    }
};

namespace jgs2 {
int hip_check(jgs2_solver* s, hipError_t e, const char* what);
void free_device(jgs2_solver* s);
void drop_graphs(jgs2_solver* s);
void free_readback(jgs2_solver* s);
void build_sweep_args(jgs2_solver* s, SweepArgs& a);
// kernels launched from the host driver (sweep.hip)
// gate: skip the rows of stopped bodies (only inside a step's sweeps, after
// the stop flags were set for this step)
void launch_phase1(jgs2_solver* s, const SweepArgs& a, bool want_R, bool gate = false);
void launch_phase2_cubature(jgs2_solver* s, const SweepArgs& a);
void launch_plain(jgs2_solver* s, const SweepArgs& a);
// damper reading of the correction, fused with the plain gather (rows in
// colour order; rotations from the last phase-1 launch)
void launch_damper(jgs2_solver* s, const SweepArgs& a);
void launch_reduce_into(jgs2_solver* s, const double* in, int n, double* out);
void launch_rotations(jgs2_solver* s, const SweepArgs& a);  // every free row (a.list unused)
// y = H-bar^-1 (R^T g) in position order, from a.g and a.R (three launches)
void launch_reduced_gradient(jgs2_solver* s, const SweepArgs& a);
// bounds-checked build: one record of a failed check, written without any access
void launch_bounds_selftest(jgs2_solver* s);
// FP32 tiles -> FP16 tiles scaled per tile (entry x inv[tile])
void launch_tiles_to_fp16(jgs2_solver* s, const float* Mt, _Float16* Mh, const float* inv, size_t n_tiles);
void launch_exact(jgs2_solver* s, const SweepArgs& a);
void launch_exact_linear(jgs2_solver* s, const SweepArgs& a);
void launch_commit(jgs2_solver* s, const SweepArgs& a);
void launch_linear(jgs2_solver* s, const SweepArgs& a);
// k coloured GS sweeps of the plain variant in one cooperative launch (the
// iterate kept in uprev before the last one); returns the launch's status
int launch_plain_persistent(jgs2_solver* s, const SweepArgs& a, int k);
void launch_param_grad(jgs2_solver* s, const d4* u, const float4* y, double* thbar);
void launch_adj_vec(jgs2_solver* s, const float4* y, float4* xbar, float4* vbar, float4* rhs);
void launch_norm2(jgs2_solver* s, const float4* w);
void launch_seg_norm2(jgs2_solver* s);
int seg_chunk_size();
void launch_mask_init(jgs2_solver* s);
// residual check after k sweeps inside a step: per-body |g_b|^2, stop flags,
// sweep counts, bodies still on and |u - u_prev|^2 (two launches)
void launch_check(jgs2_solver* s, int k);
void launch_blend(jgs2_solver* s, const SweepArgs& a, float t);
void launch_reduce(jgs2_solver* s, int n);
void launch_predict(jgs2_solver* s, float h, const float* grav);
void launch_velocity(jgs2_solver* s, float h);
void launch_energy(jgs2_solver* s, const SweepArgs& a, int nT);
int precompute_device(jgs2_solver* s, int S, int n_cand, uint64_t seed);
int alloc_tables(jgs2_solver* s, int S);
int alloc_full_tables(jgs2_solver* s);
// live-tile flags from tile_max and p.exact_drop (host, then one upload)
int update_tile_mask(jgs2_solver* s);
// tiles of the exact variant's H-bar^-1: side, tiles per super-tile side,
// count over nVf positions
constexpr int MT_Q = 64;
constexpr int MT_SG = 4;
static_assert(MT_SG * MT_SG <= 64, "one 64-bit live mask per super-tile");
inline size_t mt_tiles(int nVf) {
    const size_t n = (size_t)(nVf + MT_Q - 1) / MT_Q;
    return n * (n + 1) / 2;
}
void prof_collect(jgs2_solver* s);
hipEvent_t pool_event(jgs2_solver* s);
}  // namespace jgs2
