// Host side of libjgs2: handle, mesh/material upload, device layout, the
// time-step driver and the C ABI declared in include/jgs2.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <mutex>
#include <numeric>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "jgs2_internal.h"
#include "jgs2_math.h"

using jgs2::KMAX;
using jgs2::SMAX;
using jgs2::SREC;

// roctx range over a host call (visible with rocprofv3 --marker-trace; a
// no-op without a tool attached)
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

namespace jgs2 {

int hip_check(jgs2_solver* s, hipError_t e, const char* what) {
    if (e == hipSuccess) return JGS2_OK;
    if (s) s->err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? JGS2_E_OOM : JGS2_E_HIP;
}

template <typename T> static void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

void free_device(jgs2_solver* s) {
    dfree(s->d_tet); dfree(s->d_X); dfree(s->d_u); dfree(s->d_unext); dfree(s->d_uhat); dfree(s->d_vhat);
    dfree(s->d_zu); dfree(s->d_mh2); dfree(s->d_g); dfree(s->d_R); dfree(s->d_free); dfree(s->d_inc);
    dfree(s->d_inc_n); dfree(s->d_ring); dfree(s->d_ring_n); dfree(s->d_incslot); dfree(s->d_colperm); dfree(s->d_coloff);
    dfree(s->d_inc4); dfree(s->d_irec_c); dfree(s->d_incn_c); dfree(s->d_vid_c); dfree(s->d_fbody_c);
    dfree(s->d_Uring); dfree(s->d_samp_e); dfree(s->d_samp); dfree(s->d_partial); dfree(s->d_red);
    dfree(s->d_Mt); dfree(s->d_Mh); dfree(s->d_tscale); s->tiles_fp16 = false; dfree(s->d_Binv); dfree(s->d_qpos); dfree(s->d_qvert); dfree(s->d_qfree); dfree(s->d_hvec);
    dfree(s->d_part); dfree(s->d_yq); dfree(s->d_smask); dfree(s->d_srange); dfree(s->d_slist); s->n_slive = -1;
    s->have_full = false;
    dfree(s->d_X64); dfree(s->d_pin8); dfree(s->d_flag);
    dfree(s->d_ck_u); dfree(s->d_ck_v); dfree(s->d_seg); dfree(s->d_y); dfree(s->d_ynext); dfree(s->d_xbar);
    dfree(s->d_vbar); dfree(s->d_rhs); dfree(s->d_thbar);
    dfree(s->d_fbody); dfree(s->d_seg_idx); dfree(s->d_body_on); dfree(s->d_body_sweeps);
    dfree(s->d_rb); s->d_nactive = nullptr; s->d_r2 = nullptr; s->d_dx2 = nullptr; dfree(s->d_r0sq);
    dfree(s->d_chunk_lo); dfree(s->d_chunk_hi); dfree(s->d_body_chunk_off); dfree(s->d_r2c);
    dfree(s->d_uprev); dfree(s->d_dx2c);
    s->ro_valid = false;
    drop_graphs(s);
    free_readback(s);
}

void free_readback(jgs2_solver* s) {
    for (int i = 0; i < 2; ++i) {
        if (s->h_rb[i]) (void)hipHostFree(s->h_rb[i]);
        s->h_rb[i] = nullptr;
        s->h_r2[i] = nullptr;
        s->h_nact[i] = nullptr;
        s->h_dx2[i] = nullptr;
    }
}

void drop_graphs(jgs2_solver* s) {
    for (int i = 0; i < 2; ++i) {
        if (s->graph_exec[i]) (void)hipGraphExecDestroy(s->graph_exec[i]);
        s->graph_exec[i] = nullptr;
        s->graph_k[i] = 0;
        s->graph_u[i] = nullptr;
    }
}

void build_sweep_args(jgs2_solver* s, SweepArgs& a) {
    std::memset(&a, 0, sizeof(a));
    a.nV = s->nV; a.nVf = s->nVf; a.maxi = s->maxi; a.K = s->K; a.S = s->have_corr ? s->S : 0;
    a.nT = s->nT; a.bounds = s->d_bounds;
    a.free_ids = s->d_free; a.list = nullptr; a.n_list = 0;
    a.tet = s->d_tet; a.inc = s->d_inc; a.inc4 = s->d_inc4; a.incslot = s->d_incslot; a.inc_n = s->d_inc_n;
    // records beyond half of the 256 MB last-level cache are streamed
    a.nt_records = s->stream_mode >= 0
                       ? s->stream_mode
                       : (double)s->nVf * s->maxi * IREC_F4 * sizeof(float4) > 128.0 * 1024 * 1024;
    a.irec_c = s->d_irec_c; a.incn_c = s->d_incn_c; a.vid_c = s->d_vid_c; a.fbody_c = s->d_fbody_c; a.cbase = 0;
    a.free_c = s->d_colperm;
    a.ring = s->d_ring; a.ring_n = s->d_ring_n; a.Uring = s->d_Uring; a.samp_e = s->d_samp_e; a.samp = s->d_samp;
    a.X = s->d_X; a.u = s->d_u; a.unext = s->d_unext; a.zu = s->d_zu; a.g = s->d_g; a.R = s->d_R;
    a.partial = s->d_partial; a.omega = (float)s->p.omega; a.in_place = 0;
    a.n_planes = s->p.n_planes;
    for (int i = 0; i < s->p.n_planes; ++i)
        for (int k = 0; k < 4; ++k) a.planes[i][k] = (float)s->p.planes[i][k];
    a.d_hat = (float)s->p.d_hat; a.kappa = (float)s->p.kappa;
    a.fbody = s->d_fbody; a.body_on = s->d_body_on; a.one_body = s->n_bodies == 1;
    a.Mt = s->d_Mt; a.Mh = s->d_Mh; a.tscale = s->d_tscale; a.Binv = s->d_Binv; a.qpos = s->d_qpos; a.qvert = s->d_qvert; a.qfree = s->d_qfree;
    a.hvec = s->d_hvec; a.yq = s->d_yq; a.nactive = s->d_nactive; a.smask = s->d_smask;
    a.srange = s->d_srange;
    a.slist = s->n_slive >= 0 ? s->d_slist : nullptr;
    a.n_slive = s->n_slive;
    const size_t ntq_ = ((size_t)s->nVf + MT_Q - 1) / MT_Q;
    a.prow = s->d_part;
    a.pcol = s->d_part ? s->d_part + (ntq_ + MT_SG - 1) / MT_SG * ntq_ * MT_Q : nullptr;
    for (int i = 0; i < s->p.n_planes; ++i)
        for (int k = 0; k < 4; ++k) a.planes_d[i][k] = s->p.planes[i][k];
}

}  // namespace jgs2

using namespace jgs2;

namespace jgs2 {
hipEvent_t pool_event(jgs2_solver* s) {
    if (!s->ev_pool.empty()) {
        hipEvent_t e = s->ev_pool.back();
        s->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// Accumulates finished event pairs (call after the stream is synchronised).
// Pairs whose end event has not completed yet (work still queued behind a
// partial synchronisation) stay pending.
void prof_collect(jgs2_solver* s) {
    std::vector<jgs2_solver::Pending> keep;
    for (auto& p : s->kt_pending) {
        if (hipEventQuery(p.b) == hipErrorNotReady) {
            keep.push_back(p);
            continue;
        }
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            s->kt_ms[p.k] += ms;
            s->kt_n[p.k] += 1;
        }
        s->ev_pool.push_back(p.a);
        s->ev_pool.push_back(p.b);
    }
    s->kt_pending.swap(keep);
}
}  // namespace jgs2

namespace jgs2 {
// Device correction tables for S samples per free vertex (zero-filled).
// The exact variant's H-bar^-1 tiles and h (zero-filled: the padding past
// nVf, in the last tile row and column and at the end of h, must read as
// zero), B^-1 per position, the position tables and the per-sweep vectors
// (freed first).
int alloc_full_tables(jgs2_solver* s) {
    const size_t nf = s->nVf, nt = mt_tiles(s->nVf);
    const size_t nfp = (nf + MT_Q - 1) / MT_Q * MT_Q;  // h padded to whole tiles, zero past nVf
    const size_t ntq = nfp / MT_Q, ns = (ntq + MT_SG - 1) / MT_SG, npart = ns * ntq * MT_Q;
    const size_t nsup = ns * (ns + 1) / 2;
    for (void** p : {(void**)&s->d_Mt, (void**)&s->d_Mh, (void**)&s->d_tscale, (void**)&s->d_Binv,
                     (void**)&s->d_qpos, (void**)&s->d_qvert,
                     (void**)&s->d_qfree, (void**)&s->d_hvec, (void**)&s->d_part, (void**)&s->d_yq,
                     (void**)&s->d_smask, (void**)&s->d_srange, (void**)&s->d_slist}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    s->have_full = false;
    s->tiles_fp16 = false;
    s->n_slive = -1;
    int r;
    const size_t mt_bytes = nt * MT_Q * 9 * MT_Q * sizeof(float);
    if ((r = hip_check(s, hipMalloc((void**)&s->d_Mt, mt_bytes), "hipMalloc H-bar^-1 tiles")) ||
        (r = hip_check(s, hipMalloc((void**)&s->d_Binv, nf * 9 * sizeof(float)), "hipMalloc tables")) ||
        (r = hip_check(s, hipMalloc((void**)&s->d_qpos, (size_t)s->nV * sizeof(int)), "hipMalloc tables")) ||
        (r = hip_check(s, hipMalloc((void**)&s->d_qvert, nf * sizeof(int)), "hipMalloc tables")) ||
        (r = hip_check(s, hipMalloc((void**)&s->d_qfree, nf * sizeof(int)), "hipMalloc tables")) ||
        (r = hip_check(s, hipMalloc((void**)&s->d_hvec, nfp * sizeof(float4)), "hipMalloc tables")) ||
        (r = hip_check(s, hipMalloc((void**)&s->d_part, 2 * npart * sizeof(float4)), "hipMalloc tables")) ||
        (r = hip_check(s, hipMalloc((void**)&s->d_yq, nf * sizeof(float4)), "hipMalloc tables")) ||
        (r = hip_check(s, hipMalloc((void**)&s->d_smask, nsup * sizeof(uint64_t)), "hipMalloc tables")) ||
        (r = hip_check(s, hipMalloc((void**)&s->d_srange, ns * sizeof(int2)), "hipMalloc tables")) ||
        (r = hip_check(s, hipMalloc((void**)&s->d_slist, nsup * sizeof(int)), "hipMalloc tables")) ||
        (r = hip_check(s, hipMemsetAsync(s->d_Mt, 0, mt_bytes, s->stream), "hipMemsetAsync tiles")) ||
        (r = hip_check(s, hipMemsetAsync(s->d_hvec, 0, nfp * sizeof(float4), s->stream), "hipMemsetAsync h")))
        return r;
    return JGS2_OK;
}

// A tile is live unless its largest |entry| is at most p.exact_drop times the
// largest entry of H-bar^-1; its bytes are those of its rows below nVf.
int update_tile_mask(jgs2_solver* s) {
    const size_t nt = s->tile_max.size();
    if (nt == 0 || !s->d_smask) return JGS2_OK;
    float gmax = 0.0f;
    for (float m : s->tile_max) gmax = std::max(gmax, m);
    const double cut = s->p.exact_drop * (double)gmax;
    std::vector<uint8_t> live(nt);
    s->n_live = 0;
    s->live_bytes = 0.0;
    const int ntq = (s->nVf + MT_Q - 1) / MT_Q;
    for (int I = 0; I < ntq; ++I) {
        const int rows = std::min(MT_Q, s->nVf - I * MT_Q);
        for (int J = 0; J <= I; ++J) {
            const size_t t = (size_t)I * (I + 1) / 2 + J;
            live[t] = (double)s->tile_max[t] > cut ? 1 : 0;
            if (live[t]) {
                ++s->n_live;
                s->live_bytes += (double)rows * 9 * MT_Q * (s->tiles_fp16 ? sizeof(_Float16) : sizeof(float));
            }
        }
    }
    // super-tiles with at least one live tile; the partials of the others are
    // never written, so they are cleared here once.  Launch order: longest
    // first (a super-tile's time is that of its wave with the most live
    // tiles), so that the short ones fill the last round of blocks.
    // Per super-tile the live tiles as bits; per super-row SX the range of
    // partials that can be non-zero: row partials of super-columns
    // srange.x .. SX, column partials of super-rows SX .. srange.y.
    const int ns = (ntq + MT_SG - 1) / MT_SG;
    std::vector<int> slist, work;
    std::vector<uint64_t> smask((size_t)ns * (ns + 1) / 2, 0);
    std::vector<int2> srange(ns);
    for (int SX = 0; SX < ns; ++SX) srange[SX] = make_int2(SX + 1, SX - 1);
    for (int SI = 0; SI < ns; ++SI)
        for (int SJ = 0; SJ <= SI; ++SJ) {
            int most = 0;
            uint64_t bits = 0;
            for (int I = MT_SG * SI; I < std::min(ntq, MT_SG * SI + MT_SG); ++I) {
                int n = 0;
                for (int J = MT_SG * SJ; J <= std::min(I, MT_SG * SJ + MT_SG - 1); ++J)
                    if (live[(size_t)I * (I + 1) / 2 + J]) {
                        ++n;
                        bits |= 1ull << ((I - MT_SG * SI) * MT_SG + (J - MT_SG * SJ));
                    }
                most = std::max(most, n);
            }
            if (most > 0) {
                slist.push_back(SI * (SI + 1) / 2 + SJ);
                work.push_back(most);
                smask[(size_t)SI * (SI + 1) / 2 + SJ] = bits;
                srange[SI].x = std::min(srange[SI].x, SJ);
                srange[SJ].y = std::max(srange[SJ].y, SI);
            }
        }
    {
        std::vector<int> order(slist.size());
        for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
        std::vector<int> sorted(slist.size());
        for (size_t k = 0; k < order.size(); ++k) sorted[k] = slist[order[k]];
        slist.swap(sorted);
    }
    s->part_bytes = 0.0;
    for (int b : slist) {
        int SI = 0;
        while ((SI + 1) * (SI + 2) / 2 <= b) ++SI;
        const int SJ = b - SI * (SI + 1) / 2;
        const int rows = std::min(MT_SG, ntq - MT_SG * SI), cols = std::min(MT_SG, ntq - MT_SG * SJ);
        s->part_bytes += (double)(rows + cols) * MT_Q * sizeof(float4);
    }
    drop_graphs(s);
    int r;
    const size_t npart = (size_t)ns * ntq * MT_Q;
    if ((r = hip_check(s, hipMemcpy(s->d_smask, smask.data(), smask.size() * sizeof(uint64_t),
                                    hipMemcpyHostToDevice), "upload tile masks")) ||
        (r = hip_check(s, hipMemcpy(s->d_srange, srange.data(), srange.size() * sizeof(int2),
                                    hipMemcpyHostToDevice), "upload partial ranges")) ||
        (r = hip_check(s, hipMemcpy(s->d_slist, slist.data(), slist.size() * sizeof(int), hipMemcpyHostToDevice),
                       "upload super-tile list")) ||
        (r = hip_check(s, hipMemset(s->d_part, 0, 2 * npart * sizeof(float4)), "clear partials")))
        return r;
    s->n_slive = (int)slist.size();
    return JGS2_OK;
}

int alloc_tables(jgs2_solver* s, int S) {
    const size_t nf = s->nVf, K = s->K;
    const size_t Sd = S > 0 ? S : 1;
    for (void** p : {(void**)&s->d_Uring, (void**)&s->d_samp_e, (void**)&s->d_samp}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    int r;
    if ((r = hip_check(s, hipMalloc((void**)&s->d_Uring, nf * 9 * K * sizeof(float)), "hipMalloc tables")) ||
        (r = hip_check(s, hipMalloc((void**)&s->d_samp_e, nf * Sd * sizeof(int)), "hipMalloc tables")) ||
        (r = hip_check(s, hipMalloc((void**)&s->d_samp, nf * SREC * Sd * sizeof(float)), "hipMalloc tables")))
        return r;
    if ((r = hip_check(s, hipMemsetAsync(s->d_Uring, 0, nf * 9 * K * sizeof(float), s->stream), "memset")) ||
        (r = hip_check(s, hipMemsetAsync(s->d_samp_e, 0xFF, nf * Sd * sizeof(int), s->stream), "memset")) ||
        (r = hip_check(s, hipMemsetAsync(s->d_samp, 0, nf * SREC * Sd * sizeof(float), s->stream), "memset")))
        return r;
    return JGS2_OK;
}
}  // namespace jgs2

// Scratch of jgs2_energy_noalloc: per-block partial sums of the incremental
// potential and, in the last slot, their total.  Every GPU the library runs
// on holds its own copy until the process ends; host code reaches it only
// through the per-device address taken once by hipGetSymbolAddress (the
// array's name is a host-side stand-in, not a device address).
static __device__ __align__(256) double scratch[JGS2_NOALLOC_MAX_PARTIALS + 1];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// Takes the scratch address on the current device (s->device) once.
static int setup_scratch(jgs2_solver* s) {
    if (s->device < 0 || s->device >= kMaxDevices) {
        s->err = "device ordinal beyond the scratch table";
        return JGS2_E_HIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[s->device]) return JGS2_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
        s->err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return JGS2_E_HIP;
    }
    g_scratch_ptr[s->device] = static_cast<double*>(p);
    return JGS2_OK;
}

#define HIPCHK(expr)                                               \
    do {                                                           \
        int _r = jgs2::hip_check(s, (expr), #expr);                \
        if (_r != JGS2_OK) return _r;                              \
    } while (0)

template <typename T> static int dalloc(jgs2_solver* s, T*& p, size_t n) {
    dfree(p);
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)&p, n * sizeof(T));
    if (e != hipSuccess) {
        p = nullptr;
        return jgs2::hip_check(s, e, "hipMalloc");
    }
    return JGS2_OK;
}

template <typename T> static int upload(jgs2_solver* s, T* d, const T* h, size_t n) {
    return jgs2::hip_check(s, hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, s->stream), "upload");
}

static int validate_params(const jgs2_params* p, std::string& why) {
    if (!p) { why = "params is NULL"; return JGS2_E_INVALID; }
    if (!(p->dt > 0) || !std::isfinite(p->dt)) { why = "dt must be positive"; return JGS2_E_INVALID; }
    if (p->variant != JGS2_PLAIN && p->variant != JGS2_CUBATURE && p->variant != JGS2_DAMPER &&
        p->variant != JGS2_EXACT) {
        why = "unknown variant";
        return JGS2_E_INVALID;
    }
    if (p->order != JGS2_JACOBI && p->order != JGS2_GS) { why = "unknown order"; return JGS2_E_INVALID; }
    if (!(p->omega > 0) || !std::isfinite(p->omega)) { why = "omega must be positive"; return JGS2_E_INVALID; }
    if (p->max_sweeps < 0 || p->check_every < 1) { why = "bad sweep limits"; return JGS2_E_INVALID; }
    if (p->n_planes < 0 || p->n_planes > JGS2_MAX_PLANES) { why = "bad plane count"; return JGS2_E_INVALID; }
    if (p->n_planes > 0 && !(p->d_hat > 0 && p->kappa >= 0)) { why = "bad barrier parameters"; return JGS2_E_INVALID; }
    if (p->line_search && p->order != JGS2_JACOBI) { why = "the energy line search supports the Jacobi order"; return JGS2_E_INVALID; }
    if (!(p->adj_rel_tol > 0) || p->adj_max_sweeps < 0) { why = "bad adjoint solve limits"; return JGS2_E_INVALID; }
    if (!(p->exact_drop >= 0.0 && p->exact_drop <= 1e-3)) { why = "exact_drop must be in [0, 1e-3]"; return JGS2_E_INVALID; }
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(p->gravity[i])) { why = "gravity must be finite"; return JGS2_E_INVALID; }
    return JGS2_OK;
}

static float bits_as_float(int i) {
    float f;
    std::memcpy(&f, &i, sizeof(f));
    return f;
}

// Incidence records of the plain and linear sweeps (rows in colour order,
// zero-padded to maxi entries) from the current material.
static int upload_incidence_records(jgs2_solver* s) {
    const size_t nf = s->nVf, mi = s->maxi;
    std::vector<float4> rec(nf * IREC_F4 * mi, make_float4(0.f, 0.f, 0.f, 0.f));
    for (size_t q = 0; q < nf; ++q) {
        const int f = s->col_perm[q];
        for (int j = 0; j < s->inc_n[f]; ++j) {
            const int pk = s->inc[(size_t)f * mi + j];
            const int t = pk >> 2;
            const double E = s->E[t], nu = s->nu[t];
            const double mu_l = E / (2.0 * (1.0 + nu));
            const double lam_l = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
            const double mu = mu_l, lam = lam_l + mu_l;
            const double V = s->vol[t];
            const double* D = &s->Dm_inv[9 * (size_t)t];
            float4* r = &rec[q * IREC_F4 * mi + j];
            r[0] = make_float4((float)D[0], (float)D[1], (float)D[2], (float)D[3]);
            r[mi] = make_float4((float)D[4], (float)D[5], (float)D[6], (float)D[7]);
            r[2 * mi] = make_float4((float)D[8], (float)(V * mu), (float)(V * lam), (float)V);
            r[3 * mi] = make_float4(bits_as_float(s->tets[4 * t]), bits_as_float(s->tets[4 * t + 1]),
                                    bits_as_float(s->tets[4 * t + 2]), bits_as_float(s->tets[4 * t + 3]));
        }
    }
    int r = upload(s, s->d_irec_c, rec.data(), rec.size());
    if (r != JGS2_OK) return r;
    return jgs2::hip_check(s, hipStreamSynchronize(s->stream), "upload incidence records");
}

// Per-tet device record and per-vertex m/h^2 from the current material and dt.
static int upload_material_records(jgs2_solver* s) {
    const double h = s->p.dt;
    std::vector<float4> rec((size_t)s->nT * TET_F4);
    for (int t = 0; t < s->nT; ++t) {
        const double E = s->E[t], nu = s->nu[t];
        const double mu_l = E / (2.0 * (1.0 + nu));
        const double lam_l = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
        const double mu = mu_l, lam = lam_l + mu_l;
        const double V = s->vol[t];
        const double* D = &s->Dm_inv[9 * (size_t)t];
        float4* r = &rec[(size_t)t * TET_F4];
        r[0] = make_float4(bits_as_float(s->tets[4 * t]), bits_as_float(s->tets[4 * t + 1]),
                           bits_as_float(s->tets[4 * t + 2]), bits_as_float(s->tets[4 * t + 3]));
        r[1] = make_float4((float)D[0], (float)D[1], (float)D[2], (float)D[3]);
        r[2] = make_float4((float)D[4], (float)D[5], (float)D[6], (float)D[7]);
        r[3] = make_float4((float)D[8], (float)V, (float)(V * mu), (float)(V * lam));
        r[4] = make_float4((float)(s->rho[t] * V / (4.0 * h * h)), 0.f, 0.f, 0.f);
    }
    std::vector<float> mh2(s->nV, 0.0f);
    for (int v = 0; v < s->nV; ++v)
        if (!s->pinned[v]) mh2[v] = (float)(s->mass[v] / (h * h));
    int r;
    if ((r = upload(s, s->d_tet, rec.data(), rec.size())) != JGS2_OK) return r;
    if ((r = upload(s, s->d_mh2, mh2.data(), mh2.size())) != JGS2_OK) return r;
    return jgs2::hip_check(s, hipStreamSynchronize(s->stream), "upload material");
}

extern "C" {

void jgs2_default_params(jgs2_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->dt = 1.0 / 120.0;
    p->gravity[1] = -9.8;
    p->variant = JGS2_PLAIN;
    p->order = JGS2_JACOBI;
    p->omega = 1.0;
    p->rel_tol = 1e-5;
    p->max_sweeps = 20000;
    p->check_every = 8;
    p->d_hat = 1e-3;
    p->kappa = 1e4;
    p->adj_rel_tol = 1e-5;
    p->adj_max_sweeps = 20000;
    p->exact_drop = 1e-10;
}

int32_t jgs2_create(const jgs2_params* p, jgs2_solver** out) {
    if (!out) return JGS2_E_INVALID;
    *out = nullptr;
    std::string why;
    int r = validate_params(p, why);
    if (r != JGS2_OK) return r;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return JGS2_E_HIP;
    jgs2_solver* s = new jgs2_solver();
    s->p = *p;
    (void)hipGetDevice(&s->device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, s->device) != hipSuccess) { delete s; return JGS2_E_HIP; }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) { delete s; return JGS2_E_HIP; }
    if (hipEventCreate(&s->ev0) != hipSuccess || hipEventCreate(&s->ev1) != hipSuccess) { delete s; return JGS2_E_HIP; }
    if (setup_scratch(s) != JGS2_OK) { delete s; return JGS2_E_HIP; }
#ifdef JGS2_BOUNDS_CHECK
    if (hipMalloc((void**)&s->d_bounds, 4 * sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(s->d_bounds, 0, 4 * sizeof(unsigned long long)) != hipSuccess) {
        jgs2_destroy(s);
        return JGS2_E_HIP;
    }
#endif
    *out = s;
    return JGS2_OK;
}

void jgs2_destroy(jgs2_solver* s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    free_device(s);
    prof_collect(s);
    if (s->own_stream) (void)hipStreamDestroy(s->own_stream);
    for (hipEvent_t e : s->rb_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    if (s->ev0) (void)hipEventDestroy(s->ev0);
    if (s->ev1) (void)hipEventDestroy(s->ev1);
    if (s->d_bounds) (void)hipFree(s->d_bounds);
    delete s;
}

int32_t jgs2_bounds_report(jgs2_solver* s, int32_t* line, int64_t* index, int64_t* extent, int32_t clear) {
    if (!s) return JGS2_E_INVALID;
    if (!s->d_bounds) return s->fail(JGS2_E_INVALID, "not a bounds-checked build");
    unsigned long long rec[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(rec, s->d_bounds, sizeof(rec), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (line) *line = (int32_t)rec[0];
    if (index) *index = (int64_t)rec[1];
    if (extent) *extent = (int64_t)rec[2];
    if (clear) {
        HIPCHK(hipMemsetAsync(s->d_bounds, 0, sizeof(rec), s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    return JGS2_OK;
}

int32_t jgs2_bounds_selftest(jgs2_solver* s) {
    if (!s) return JGS2_E_INVALID;
    if (!s->d_bounds) return s->fail(JGS2_E_INVALID, "not a bounds-checked build");
    jgs2::launch_bounds_selftest(s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->stream));
    return JGS2_OK;
}

const char* jgs2_last_error(const jgs2_solver* s) { return s ? s->err.c_str() : "null handle"; }

int32_t jgs2_set_params(jgs2_solver* s, const jgs2_params* p) {
    if (!s) return JGS2_E_INVALID;
    std::string why;
    int r = validate_params(p, why);
    if (r != JGS2_OK) return s->fail(r, why);
    if (s->in_step && (p->dt != s->p.dt || std::memcmp(p->gravity, s->p.gravity, sizeof(p->gravity)) != 0))
        return s->fail(JGS2_E_INVALID, "dt and gravity cannot change inside a step");
    const bool dt_changed = p->dt != s->p.dt;
    const bool drop_changed = p->exact_drop != s->p.exact_drop;
    if (p->line_search && s->n_bodies > 1)
        return s->fail(JGS2_E_INVALID, "the energy line search needs a single body");
    s->p = *p;
    if (drop_changed && s->have_full && !dt_changed) {
        if ((r = jgs2::update_tile_mask(s)) != JGS2_OK) return r;
    }
    s->ro_valid = false;
    drop_graphs(s);
    // the correction's rest Hessian carries M / h^2: it belongs to the old step
    if (dt_changed) s->have_corr = s->have_full = false;
    if (dt_changed && s->have_material) {
        if ((r = upload_material_records(s)) != JGS2_OK) return r;
    }
    return JGS2_OK;
}

int32_t jgs2_exact_tiles(jgs2_solver* s, int64_t* n_tiles, int64_t* n_live, double* live_bytes,
                         double* part_bytes) {
    if (!s) return JGS2_E_INVALID;
    if (!s->have_full) return s->fail(JGS2_E_NOT_READY, "no H-bar^-1 tiles (precompute with the JGS2_EXACT variant)");
    if (n_tiles) *n_tiles = (int64_t)s->tile_max.size();
    if (n_live) *n_live = s->n_live;
    if (live_bytes) *live_bytes = s->live_bytes;
    if (part_bytes) *part_bytes = s->part_bytes;
    return JGS2_OK;
}

int32_t jgs2_exact_tiles_fp16(jgs2_solver* s) {
    if (!s) return JGS2_E_INVALID;
    if (!s->have_full) return s->fail(JGS2_E_NOT_READY, "no H-bar^-1 tiles (precompute with the JGS2_EXACT variant)");
    if (s->in_step) return s->fail(JGS2_E_INVALID, "inside a step");
    if (s->tiles_fp16) return JGS2_OK;
    TraceRange trace_range("jgs2_exact_tiles_fp16");
    const size_t nt = s->tile_max.size(), n = nt * jgs2::MT_Q * 9 * jgs2::MT_Q;
    // the largest |entry| of a tile maps to 2^15 (below the FP16 maximum 65504)
    std::vector<float> scale(nt), inv(nt);
    for (size_t t = 0; t < nt; ++t) {
        const float m = s->tile_max[t];
        scale[t] = m > 0.0f ? m / 32768.0f : 1.0f;
        inv[t] = m > 0.0f ? 32768.0f / m : 1.0f;
    }
    float* dinv = nullptr;
    int r;
    if ((r = jgs2::hip_check(s, hipMalloc((void**)&s->d_Mh, n * sizeof(_Float16)), "hipMalloc FP16 tiles")) ||
        (r = jgs2::hip_check(s, hipMalloc((void**)&s->d_tscale, nt * sizeof(float)), "hipMalloc tile scales")) ||
        (r = jgs2::hip_check(s, hipMalloc((void**)&dinv, nt * sizeof(float)), "hipMalloc tile scales"))) {
        if (dinv) (void)hipFree(dinv);
        if (s->d_Mh) (void)hipFree(s->d_Mh);
        if (s->d_tscale) (void)hipFree(s->d_tscale);
        s->d_Mh = nullptr;
        s->d_tscale = nullptr;
        return r;
    }
    if ((r = jgs2::hip_check(s, hipMemcpyAsync(s->d_tscale, scale.data(), nt * sizeof(float), hipMemcpyHostToDevice,
                                               s->stream), "upload tile scales")) == JGS2_OK &&
        (r = jgs2::hip_check(s, hipMemcpyAsync(dinv, inv.data(), nt * sizeof(float), hipMemcpyHostToDevice, s->stream),
                             "upload tile scales")) == JGS2_OK) {
        jgs2::launch_tiles_to_fp16(s, s->d_Mt, s->d_Mh, dinv, nt);
        if ((r = jgs2::hip_check(s, hipGetLastError(), "FP16 tile conversion")) == JGS2_OK)
            r = jgs2::hip_check(s, hipStreamSynchronize(s->stream), "FP16 tile conversion");
    }
    (void)hipStreamSynchronize(s->stream);  // the host arrays above are read by queued copies
    (void)hipFree(dinv);
    if (r != JGS2_OK) {  // the FP32 tiles stay in use
        (void)hipFree(s->d_Mh);
        (void)hipFree(s->d_tscale);
        s->d_Mh = nullptr;
        s->d_tscale = nullptr;
        return r;
    }
    (void)hipFree(s->d_Mt);
    s->d_Mt = nullptr;
    s->tiles_fp16 = true;
    return jgs2::update_tile_mask(s);  // bytes per live tile halve; captured graphs are dropped
}

int32_t jgs2_set_stream(jgs2_solver* s, void* stream) {
    if (!s) return JGS2_E_INVALID;
    s->stream = (hipStream_t)stream;
    return JGS2_OK;
}

int32_t jgs2_upload_mesh(jgs2_solver* s, int32_t nV, const double* X, int32_t nT, const int32_t* tets,
                         const uint8_t* pinned) {
    if (!s) return JGS2_E_INVALID;
    if (nV <= 0 || nT <= 0 || !X || !tets || !pinned) return s->fail(JGS2_E_INVALID, "empty or NULL mesh");
    for (int64_t i = 0; i < 3LL * nV; ++i)
        if (!std::isfinite(X[i])) return s->fail(JGS2_E_INVALID, "non-finite rest position");
    for (int64_t i = 0; i < 4LL * nT; ++i)
        if (tets[i] < 0 || tets[i] >= nV) return s->fail(JGS2_E_INVALID, "tet vertex id out of range");
    free_device(s);
    s->have_mesh = s->have_material = s->have_corr = s->have_state = s->in_step = s->have_bodies = false;
    s->nV = nV; s->nT = nT;
    s->X.assign(X, X + 3 * (size_t)nV);
    s->tets.assign(tets, tets + 4 * (size_t)nT);
    s->pinned.assign(pinned, pinned + nV);
    // rest-shape geometry
    s->vol.resize(nT);
    s->Dm_inv.resize(9 * (size_t)nT);
    for (int t = 0; t < nT; ++t) {
        const int* c = &tets[4 * t];
        double Dm[9];
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) Dm[3 * i + k] = X[3 * c[k + 1] + i] - X[3 * c[0] + i];
        const double det = Dm[0] * (Dm[4] * Dm[8] - Dm[5] * Dm[7]) - Dm[1] * (Dm[3] * Dm[8] - Dm[5] * Dm[6]) +
                           Dm[2] * (Dm[3] * Dm[7] - Dm[4] * Dm[6]);
        if (!(det > 0)) return s->fail(JGS2_E_INVALID, "tet with non-positive orientation");
        s->vol[t] = det / 6.0;
        double* I = &s->Dm_inv[9 * (size_t)t];
        I[0] = (Dm[4] * Dm[8] - Dm[5] * Dm[7]) / det; I[1] = (Dm[2] * Dm[7] - Dm[1] * Dm[8]) / det;
        I[2] = (Dm[1] * Dm[5] - Dm[2] * Dm[4]) / det; I[3] = (Dm[5] * Dm[6] - Dm[3] * Dm[8]) / det;
        I[4] = (Dm[0] * Dm[8] - Dm[2] * Dm[6]) / det; I[5] = (Dm[2] * Dm[3] - Dm[0] * Dm[5]) / det;
        I[6] = (Dm[3] * Dm[7] - Dm[4] * Dm[6]) / det; I[7] = (Dm[1] * Dm[6] - Dm[0] * Dm[7]) / det;
        I[8] = (Dm[0] * Dm[4] - Dm[1] * Dm[3]) / det;
    }
    // free numbering
    s->free_ids.clear();
    s->free_index.assign(nV, -1);
    for (int v = 0; v < nV; ++v)
        if (!pinned[v]) { s->free_index[v] = (int)s->free_ids.size(); s->free_ids.push_back(v); }
    s->nVf = (int)s->free_ids.size();
    // incidence (ascending tet id) and valence
    std::vector<int> cnt(nV, 0);
    for (int64_t i = 0; i < 4LL * nT; ++i) cnt[tets[i]]++;
    s->valence = cnt;
    std::vector<int64_t> off(nV + 1, 0);
    for (int v = 0; v < nV; ++v) off[v + 1] = off[v] + cnt[v];
    std::vector<int> incall(off[nV]);
    std::vector<int64_t> pos(off.begin(), off.end() - 1);
    for (int t = 0; t < nT; ++t)
        for (int c = 0; c < 4; ++c) incall[pos[tets[4 * t + c]]++] = (t << 2) | c;
    // free one-ring, ascending
    std::vector<std::vector<int>> ringv(s->nVf);
    s->maxi = 0; s->K = 0;
    for (int f = 0; f < s->nVf; ++f) {
        const int v = s->free_ids[f];
        if (off[v + 1] == off[v]) return s->fail(JGS2_E_INVALID, "a free vertex belongs to no tet (it has no mass)");
        auto& r = ringv[f];
        for (int64_t k = off[v]; k < off[v + 1]; ++k) {
            const int t = incall[k] >> 2;
            for (int c = 0; c < 4; ++c) {
                const int a = tets[4 * t + c];
                if (a != v && !pinned[a]) r.push_back(a);
            }
        }
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
        s->maxi = std::max<int>(s->maxi, (int)(off[v + 1] - off[v]));
        s->K = std::max<int>(s->K, (int)r.size());
    }
    if (s->K > KMAX) return s->fail(JGS2_E_INVALID, "one-ring larger than 32 free vertices");
    if (s->maxi == 0) s->maxi = 1;
    if (s->K == 0) s->K = 1;
    const size_t nf = s->nVf;
    s->inc.assign(nf * s->maxi, -1);
    s->inc4.assign(nf * s->maxi, make_int4(-1, 0, 0, 0));
    s->incslot.assign(nf * s->maxi, 0xFFFFFFFFu);
    s->inc_n.assign(nf, 0);
    s->ring.assign(nf * s->K, -1);
    s->ring_n.assign(nf, 0);
    for (int f = 0; f < s->nVf; ++f) {
        const int v = s->free_ids[f];
        const auto& r = ringv[f];
        s->ring_n[f] = (int)r.size();
        for (size_t k = 0; k < r.size(); ++k) s->ring[(size_t)f * s->K + k] = r[k];
        int j = 0;
        for (int64_t k = off[v]; k < off[v + 1]; ++k, ++j) {
            const int pk = incall[k];
            const int t = pk >> 2;
            s->inc[(size_t)f * s->maxi + j] = pk;
            {
                const int c0 = pk & 3;
                s->inc4[(size_t)f * s->maxi + j] = make_int4(pk, tets[4 * t + ((c0 + 1) & 3)],
                                                             tets[4 * t + ((c0 + 2) & 3)], tets[4 * t + ((c0 + 3) & 3)]);
            }
            uint32_t sl = 0;
            for (int c = 0; c < 4; ++c) {
                const int a = tets[4 * t + c];
                uint32_t b;
                if (a == v) b = SLOT_SELF;
                else if (pinned[a]) b = SLOT_NONE;
                else b = (uint32_t)(std::lower_bound(r.begin(), r.end(), a) - r.begin());
                sl |= b << (8 * c);
            }
            s->incslot[(size_t)f * s->maxi + j] = sl;
        }
        s->inc_n[f] = j;
    }
    // greedy colouring of free vertices in id order
    s->color.assign(nV, -1);
    s->n_colors = 0;
    for (int f = 0; f < s->nVf; ++f) {
        std::vector<char> used(64, 0);
        for (int a : ringv[f]) {
            const int c = s->color[a];
            if (c >= 0) { if (c >= (int)used.size()) used.resize(c + 1, 0); used[c] = 1; }
        }
        int c = 0;
        while (c < (int)used.size() && used[c]) ++c;
        s->color[s->free_ids[f]] = c;
        s->n_colors = std::max(s->n_colors, c + 1);
    }
    s->col_off.assign(s->n_colors + 1, 0);
    for (int f = 0; f < s->nVf; ++f) s->col_off[s->color[s->free_ids[f]] + 1]++;
    for (int c = 0; c < s->n_colors; ++c) s->col_off[c + 1] += s->col_off[c];
    s->col_perm.assign(nf, 0);
    {
        std::vector<int> p(s->col_off.begin(), s->col_off.end() - 1);
        for (int f = 0; f < s->nVf; ++f) s->col_perm[p[s->color[s->free_ids[f]]]++] = f;
    }
    // device layout
    int r;
    const size_t V4 = (size_t)nV;
    if ((r = dalloc(s, s->d_X, V4)) || (r = dalloc(s, s->d_u, V4)) || (r = dalloc(s, s->d_unext, V4)) ||
        (r = dalloc(s, s->d_uhat, V4)) || (r = dalloc(s, s->d_vhat, V4)) || (r = dalloc(s, s->d_zu, V4)) ||
        (r = dalloc(s, s->d_g, V4)) || (r = dalloc(s, s->d_R, V4)) || (r = dalloc(s, s->d_mh2, (size_t)nV)) ||
        (r = dalloc(s, s->d_free, nf)) || (r = dalloc(s, s->d_inc, nf * s->maxi)) ||
        (r = dalloc(s, s->d_incslot, nf * s->maxi)) || (r = dalloc(s, s->d_inc_n, nf)) ||
        (r = dalloc(s, s->d_ring, nf * s->K)) || (r = dalloc(s, s->d_ring_n, nf)) ||
        (r = dalloc(s, s->d_colperm, nf)) || (r = dalloc(s, s->d_tet, (size_t)nT * TET_F4)) ||
        (r = dalloc(s, s->d_inc4, nf * s->maxi)) || (r = dalloc(s, s->d_uprev, V4)) ||
        (r = dalloc(s, s->d_coloff, (size_t)s->n_colors + 1)))
        return r;
    s->n_partial = std::max<int>((s->nVf + 1) / 2, (std::max(nT, s->nVf) + 255) / 256) + 1;
    if ((r = dalloc(s, s->d_partial, (size_t)s->n_partial)) || (r = dalloc(s, s->d_red, 4))) return r;
    std::vector<float4> Xs(V4), Rid(V4, make_float4(0.f, 0.f, 0.f, 1.f));
    for (int v = 0; v < nV; ++v)
        Xs[v] = make_float4((float)X[3 * (size_t)v], (float)X[3 * (size_t)v + 1], (float)X[3 * (size_t)v + 2], 0.f);
    if ((r = upload(s, s->d_X, Xs.data(), V4)) || (r = upload(s, s->d_R, Rid.data(), V4)) ||
        (r = upload(s, s->d_free, s->free_ids.data(), nf)) || (r = upload(s, s->d_inc, s->inc.data(), nf * s->maxi)) ||
        (r = upload(s, s->d_incslot, s->incslot.data(), nf * s->maxi)) || (r = upload(s, s->d_inc_n, s->inc_n.data(), nf)) ||
        (r = upload(s, s->d_ring, s->ring.data(), nf * s->K)) || (r = upload(s, s->d_ring_n, s->ring_n.data(), nf)) ||
        (r = upload(s, s->d_colperm, s->col_perm.data(), nf)) || (r = upload(s, s->d_inc4, s->inc4.data(), nf * s->maxi)) ||
        (r = upload(s, s->d_coloff, s->col_off.data(), (size_t)s->n_colors + 1)))
        return r;
    {
        std::vector<int> incnc(nf), vidc(nf);
        for (size_t q = 0; q < nf; ++q) {
            const int f = s->col_perm[q];
            incnc[q] = s->inc_n[f];
            vidc[q] = s->free_ids[f];
        }
        if ((r = dalloc(s, s->d_irec_c, nf * IREC_F4 * s->maxi)) || (r = dalloc(s, s->d_incn_c, nf)) ||
            (r = dalloc(s, s->d_vid_c, nf)) || (r = dalloc(s, s->d_fbody_c, nf)) ||
            (r = upload(s, s->d_incn_c, incnc.data(), nf)) || (r = upload(s, s->d_vid_c, vidc.data(), nf)))
            return r;
    }
    for (d4* d : {s->d_u, s->d_unext, s->d_uhat, s->d_zu}) HIPCHK(hipMemsetAsync(d, 0, V4 * sizeof(d4), s->stream));
    for (float4* d : {s->d_vhat, s->d_g}) HIPCHK(hipMemsetAsync(d, 0, V4 * sizeof(float4), s->stream));
    HIPCHK(hipMemsetAsync(s->d_mh2, 0, (size_t)nV * sizeof(float), s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    {
        std::vector<int32_t> zero((size_t)nV, 0);
        if ((r = jgs2_set_bodies(s, 1, zero.data())) != JGS2_OK) return r;
    }
    s->have_mesh = true;
    return JGS2_OK;
}

int32_t jgs2_set_material(jgs2_solver* s, const double* E, const double* nu, const double* rho) {
    if (!s) return JGS2_E_INVALID;
    if (!s->have_mesh) return s->fail(JGS2_E_NOT_READY, "no mesh");
    if (!E || !nu || !rho) return s->fail(JGS2_E_INVALID, "NULL material array");
    for (int t = 0; t < s->nT; ++t)
        if (!(E[t] >= 0) || !(nu[t] > -1 && nu[t] < 0.5) || !(rho[t] > 0) || !std::isfinite(E[t]))
            return s->fail(JGS2_E_INVALID, "material out of range");
    s->E.assign(E, E + s->nT);
    s->nu.assign(nu, nu + s->nT);
    s->rho.assign(rho, rho + s->nT);
    s->mass.assign(s->nV, 0.0);
    for (int t = 0; t < s->nT; ++t)
        for (int c = 0; c < 4; ++c) s->mass[s->tets[4 * t + c]] += rho[t] * s->vol[t] / 4.0;
    int r = upload_material_records(s);
    if (r != JGS2_OK) return r;
    if ((r = upload_incidence_records(s)) != JGS2_OK) return r;
    s->have_material = true;
    s->have_corr = s->have_full = false;
    s->ro_valid = false;
    return JGS2_OK;
}

int32_t jgs2_set_material_log_e(jgs2_solver* s, const double* log_E, const double* nu, const double* rho) {
    if (!s) return JGS2_E_INVALID;
    if (!s->have_mesh) return s->fail(JGS2_E_NOT_READY, "no mesh");
    if (!log_E) return s->fail(JGS2_E_INVALID, "NULL material array");
    std::vector<double> E((size_t)s->nT);
    for (int t = 0; t < s->nT; ++t) {
        if (!std::isfinite(log_E[t])) return s->fail(JGS2_E_INVALID, "non-finite log E");
        E[t] = std::exp(log_E[t]);
    }
    return jgs2_set_material(s, E.data(), nu, rho);
}

int32_t jgs2_get_ring_sizes(jgs2_solver* s, int32_t* nVf, int32_t* sizes) {
    if (!s) return JGS2_E_INVALID;
    if (!s->have_mesh) return s->fail(JGS2_E_NOT_READY, "no mesh");
    if (nVf) *nVf = s->nVf;
    if (sizes) std::copy(s->ring_n.begin(), s->ring_n.end(), sizes);
    return JGS2_OK;
}

// ---- precompute cache file ----
// Layout: a header (format tag, a 64-bit FNV-1a key over everything the
// precompute depends on, sizes), then the pose eigenvalues, the NNLS fits,
// the one-ring U-bar rows, the sample ids and records, and for the exact
// variant B^-1, the position tables, the tile maxima and every stored tile.
// The key includes this library build's date and time, so a rebuilt library
// never reads an older build's file.
namespace {
struct CacheHeader {
    char tag[8];
    uint64_t key;
    int32_t nV, nT, nVf, K, S, exact, n_poses, n_eigs;
    int64_t n_tiles;
};

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

uint64_t cache_key(const jgs2_solver* s, int S, int n_cand, uint64_t seed) {
    static const char build[] = __DATE__ " " __TIME__;
    uint64_t h = 1469598103934665603ull;
    h = fnv1a(h, build, sizeof(build));
    h = fnv1a(h, s->X.data(), s->X.size() * sizeof(double));
    h = fnv1a(h, s->tets.data(), s->tets.size() * sizeof(int));
    h = fnv1a(h, s->pinned.data(), s->pinned.size());
    h = fnv1a(h, s->E.data(), s->E.size() * sizeof(double));
    h = fnv1a(h, s->nu.data(), s->nu.size() * sizeof(double));
    h = fnv1a(h, s->rho.data(), s->rho.size() * sizeof(double));
    const int exact = s->p.variant == JGS2_EXACT;
    h = fnv1a(h, &s->p.dt, sizeof(double));
    h = fnv1a(h, &S, sizeof(S));
    h = fnv1a(h, &n_cand, sizeof(n_cand));
    h = fnv1a(h, &seed, sizeof(seed));
    return fnv1a(h, &exact, sizeof(exact));
}

constexpr size_t CACHE_CHUNK = (size_t)64 << 20;  // staging bytes per copy

bool put(FILE* f, const void* p, size_t n) { return n == 0 || std::fwrite(p, 1, n, f) == n; }
bool get(FILE* f, void* p, size_t n) { return n == 0 || std::fread(p, 1, n, f) == n; }

// Device buffer <-> file through one host staging buffer, chunk by chunk.
bool put_dev(FILE* f, const void* d, size_t n, std::vector<char>& stage) {
    for (size_t o = 0; o < n; o += CACHE_CHUNK) {
        const size_t m = std::min(CACHE_CHUNK, n - o);
        if (hipMemcpy(stage.data(), static_cast<const char*>(d) + o, m, hipMemcpyDeviceToHost) != hipSuccess ||
            !put(f, stage.data(), m))
            return false;
    }
    return true;
}

bool get_dev(FILE* f, void* d, size_t n, std::vector<char>& stage) {
    for (size_t o = 0; o < n; o += CACHE_CHUNK) {
        const size_t m = std::min(CACHE_CHUNK, n - o);
        if (!get(f, stage.data(), m) ||
            hipMemcpy(static_cast<char*>(d) + o, stage.data(), m, hipMemcpyHostToDevice) != hipSuccess)
            return false;
    }
    return true;
}

size_t tile_floats(const jgs2_solver* s) { return jgs2::mt_tiles(s->nVf) * jgs2::MT_Q * 9 * jgs2::MT_Q; }

int write_cache(jgs2_solver* s, const char* path, int n_cand, uint64_t seed) {
    if (s->tiles_fp16) return s->fail(JGS2_E_INVALID, "the cache holds FP32 tiles: write it before converting");
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return s->fail(JGS2_E_INVALID, "cannot write the precompute cache");
    (void)hipStreamSynchronize(s->stream);
    const size_t nf = s->nVf, S = s->S, K = s->K;
    CacheHeader hd;
    std::memset(&hd, 0, sizeof(hd));
    std::memcpy(hd.tag, "JGS2PC01", 8);
    hd.key = cache_key(s, s->S, n_cand, seed);
    hd.nV = s->nV; hd.nT = s->nT; hd.nVf = s->nVf; hd.K = s->K; hd.S = s->S;
    hd.exact = s->have_full; hd.n_poses = s->n_poses; hd.n_eigs = (int32_t)s->pose_eigs.size();
    hd.n_tiles = s->have_full ? (int64_t)s->tile_max.size() : 0;
    std::vector<char> stage(CACHE_CHUNK);
    bool ok = put(f, &hd, sizeof(hd)) && put(f, s->pose_eigs.data(), s->pose_eigs.size() * sizeof(double)) &&
              put(f, s->fit.data(), nf * sizeof(double)) &&
              put_dev(f, s->d_Uring, nf * 9 * K * sizeof(float), stage) &&
              put_dev(f, s->d_samp_e, nf * S * sizeof(int), stage) &&
              put_dev(f, s->d_samp, nf * jgs2::SREC * S * sizeof(float), stage);
    if (ok && s->have_full)
        ok = put_dev(f, s->d_Binv, nf * 9 * sizeof(float), stage) &&
             put_dev(f, s->d_qpos, (size_t)s->nV * sizeof(int), stage) &&
             put_dev(f, s->d_qvert, nf * sizeof(int), stage) && put_dev(f, s->d_qfree, nf * sizeof(int), stage) &&
             put(f, s->tile_max.data(), s->tile_max.size() * sizeof(float)) &&
             put_dev(f, s->d_Mt, tile_floats(s) * sizeof(float), stage);
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        (void)std::remove(tmp.c_str());
        return s->fail(JGS2_E_INVALID, "cannot write the precompute cache");
    }
    return JGS2_OK;
}

// 1: loaded; 0: no file, not this precompute's, or cut short (the tables
// are then recomputed); < 0: an allocation failure.
int read_cache(jgs2_solver* s, const char* path, int S, int n_cand, uint64_t seed) {
    FILE* f = std::fopen(path, "rb");
    if (!f) return 0;
    CacheHeader hd;
    const bool exact = s->p.variant == JGS2_EXACT;
    if (!get(f, &hd, sizeof(hd)) || std::memcmp(hd.tag, "JGS2PC01", 8) != 0 ||
        hd.key != cache_key(s, S, n_cand, seed) || hd.nV != s->nV || hd.nT != s->nT || hd.nVf != s->nVf ||
        hd.K != s->K || hd.S != S || hd.exact != (exact ? 1 : 0) || hd.n_eigs < 0 ||
        (exact && hd.n_tiles != (int64_t)jgs2::mt_tiles(s->nVf))) {
        std::fclose(f);
        return 0;
    }
    s->have_corr = s->have_full = false;
    const size_t nf = s->nVf, K = s->K;
    int r;
    if ((r = jgs2::alloc_tables(s, S)) != JGS2_OK || (exact && (r = jgs2::alloc_full_tables(s)) != JGS2_OK)) {
        std::fclose(f);
        return r;
    }
    (void)hipStreamSynchronize(s->stream);
    std::vector<char> stage(CACHE_CHUNK);
    s->pose_eigs.assign(hd.n_eigs, 0.0);
    s->fit.assign(nf, 0.0);
    bool ok = get(f, s->pose_eigs.data(), s->pose_eigs.size() * sizeof(double)) &&
              get(f, s->fit.data(), nf * sizeof(double)) &&
              get_dev(f, s->d_Uring, nf * 9 * K * sizeof(float), stage) &&
              get_dev(f, s->d_samp_e, nf * S * sizeof(int), stage) &&
              get_dev(f, s->d_samp, nf * jgs2::SREC * S * sizeof(float), stage);
    if (ok && exact) {
        s->tile_max.assign(hd.n_tiles, 0.0f);
        ok = get_dev(f, s->d_Binv, nf * 9 * sizeof(float), stage) &&
             get_dev(f, s->d_qpos, (size_t)s->nV * sizeof(int), stage) &&
             get_dev(f, s->d_qvert, nf * sizeof(int), stage) && get_dev(f, s->d_qfree, nf * sizeof(int), stage) &&
             get(f, s->tile_max.data(), s->tile_max.size() * sizeof(float)) &&
             get_dev(f, s->d_Mt, tile_floats(s) * sizeof(float), stage);
    }
    std::fclose(f);
    if (!ok) return 0;  // a matching header over a short or unreadable body: recompute and rewrite
    s->S = S;
    s->n_poses = hd.n_poses;
    s->have_corr = true;
    if (exact) {
        s->have_full = true;
        if ((r = jgs2::update_tile_mask(s)) != JGS2_OK) {
            s->have_full = false;
            return r;
        }
    }
    return 1;
}
}  // namespace

int32_t jgs2_precompute_cached(jgs2_solver* s, int32_t samples, int32_t n_cand, uint64_t seed, const char* path,
                               int32_t* loaded) {
    if (!s) return JGS2_E_INVALID;
    if (loaded) *loaded = 0;
    if (!path) return jgs2_precompute(s, samples, n_cand, seed);
    if (!s->have_mesh || !s->have_material) return s->fail(JGS2_E_NOT_READY, "no mesh or material");
    if (samples < 1 || samples > SMAX || n_cand < 1 || n_cand > 64)
        return s->fail(JGS2_E_INVALID, "samples in [1,8] and candidates in [1,64] required");
    TraceRange trace_range("jgs2_precompute_cached");
    int r = read_cache(s, path, samples, n_cand, seed);
    if (r < 0) return r;
    if (r == 1) {
        if (loaded) *loaded = 1;
        return JGS2_OK;
    }
    if ((r = jgs2_precompute(s, samples, n_cand, seed)) != JGS2_OK) return r;
    return write_cache(s, path, n_cand, seed);
}

int32_t jgs2_get_poses(jgs2_solver* s, int32_t* n_poses, double* eigenvalues) {
    if (!s) return JGS2_E_INVALID;
    if (n_poses) *n_poses = s->n_poses;
    if (eigenvalues) std::copy(s->pose_eigs.begin(), s->pose_eigs.end(), eigenvalues);
    return JGS2_OK;
}

int32_t jgs2_import_correction(jgs2_solver* s, int32_t S, const double* U_ring, const int32_t* samples,
                               const double* weights, const double* U_samp) {
    if (!s) return JGS2_E_INVALID;
    if (!s->have_mesh || !s->have_material) return s->fail(JGS2_E_NOT_READY, "no mesh or material");
    if (S < 0 || S > SMAX) return s->fail(JGS2_E_INVALID, "samples per vertex must be in [0, 8]");
    if (!U_ring || (S > 0 && (!samples || !weights || !U_samp))) return s->fail(JGS2_E_INVALID, "NULL table");
    const size_t nf = s->nVf, K = s->K;
    std::vector<float> Ur(nf * 9 * K, 0.0f);
    size_t row = 0;
    for (size_t f = 0; f < nf; ++f)
        for (int k = 0; k < s->ring_n[f]; ++k, ++row)
            for (int q = 0; q < 9; ++q) {
                const double val = U_ring[row * 9 + q];
                if (!std::isfinite(val)) return s->fail(JGS2_E_INVALID, "non-finite U-bar row");
                Ur[(f * 9 + q) * K + k] = (float)val;
            }
    const int Sd = S > 0 ? S : 1;
    std::vector<int> se(nf * Sd, -1);
    std::vector<float> sr(nf * SREC * Sd, 0.0f);
    for (size_t f = 0; f < nf && S > 0; ++f) {
        const int v = s->free_ids[f];
        const int* rb = &s->ring[f * K];
        const int rn = s->ring_n[f];
        for (int j = 0; j < S; ++j) {
            const int e = samples[f * S + j];
            if (e < -1 || e >= s->nT) return s->fail(JGS2_E_INVALID, "sample element out of range");
            if (e < 0) continue;
            const double w = weights[f * S + j];
            if (!(w >= 0) || !std::isfinite(w)) return s->fail(JGS2_E_INVALID, "bad cubature weight");
            se[f * S + j] = e;
            float* rec = &sr[f * SREC * S];
            rec[j] = (float)w;
            for (int c = 0; c < 4; ++c) {
                const int a = s->tets[4 * e + c];
                if (a == v) return s->fail(JGS2_E_INVALID, "sample element contains its own vertex");
                const bool in_ring = std::binary_search(rb, rb + rn, a);
                const double gc = (!s->pinned[a] && !in_ring) ? w / s->valence[a] : 0.0;
                rec[(1 + c) * S + j] = (float)gc;
                for (int q = 0; q < 9; ++q)
                    rec[(5 + 9 * c + q) * S + j] = (float)U_samp[((f * S + j) * 4 + c) * 9 + q];
            }
        }
    }
    int r;
    if ((r = alloc_tables(s, S))) return r;
    if ((r = upload(s, s->d_Uring, Ur.data(), Ur.size())) || (r = upload(s, s->d_samp_e, se.data(), se.size())) ||
        (r = upload(s, s->d_samp, sr.data(), sr.size())))
        return r;
    HIPCHK(hipStreamSynchronize(s->stream));
    s->S = S;
    s->have_corr = true;
    return JGS2_OK;
}

int32_t jgs2_export_correction(jgs2_solver* s, int32_t S, double* U_ring, int32_t* samples, double* weights,
                               double* U_samp, double* fit) {
    if (!s) return JGS2_E_INVALID;
    if (!s->have_corr) return s->fail(JGS2_E_NOT_READY, "no correction");
    if (S != s->S) return s->fail(JGS2_E_INVALID, "sample count differs from the stored correction");
    const size_t nf = s->nVf, K = s->K;
    const int Sd = S > 0 ? S : 1;
    std::vector<float> Ur(nf * 9 * K), sr(nf * SREC * Sd);
    std::vector<int> se(nf * Sd);
    HIPCHK(hipMemcpyAsync(Ur.data(), s->d_Uring, Ur.size() * 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(se.data(), s->d_samp_e, se.size() * 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(sr.data(), s->d_samp, sr.size() * 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    size_t row = 0;
    for (size_t f = 0; f < nf; ++f)
        for (int k = 0; k < s->ring_n[f]; ++k, ++row)
            for (int q = 0; q < 9; ++q)
                if (U_ring) U_ring[row * 9 + q] = Ur[(f * 9 + q) * K + k];
    for (size_t f = 0; f < nf && S > 0; ++f)
        for (int j = 0; j < S; ++j) {
            if (samples) samples[f * S + j] = se[f * S + j];
            const float* rec = &sr[f * SREC * S];
            if (weights) weights[f * S + j] = rec[j];
            if (U_samp)
                for (int c = 0; c < 4; ++c)
                    for (int q = 0; q < 9; ++q) U_samp[((f * S + j) * 4 + c) * 9 + q] = rec[(5 + 9 * c + q) * S + j];
        }
    if (fit) {
        for (size_t f = 0; f < nf; ++f) fit[f] = f < s->fit.size() ? s->fit[f] : 0.0;
    }
    return JGS2_OK;
}

int32_t jgs2_precompute(jgs2_solver* s, int32_t samples, int32_t n_cand, uint64_t seed) {
    TraceRange trace_range("jgs2_precompute");
    if (!s) return JGS2_E_INVALID;
    if (!s->have_mesh || !s->have_material) return s->fail(JGS2_E_NOT_READY, "no mesh or material");
    if (samples < 1 || samples > SMAX || n_cand < 1 || n_cand > 64)
        return s->fail(JGS2_E_INVALID, "samples in [1,8] and candidates in [1,64] required");
    return precompute_device(s, samples, n_cand, seed);
}

int32_t jgs2_set_state(jgs2_solver* s, const double* x, const double* v) {
    if (!s) return JGS2_E_INVALID;
    if (!s->have_mesh) return s->fail(JGS2_E_NOT_READY, "no mesh");
    if (!x || !v) return s->fail(JGS2_E_INVALID, "NULL state");
    const size_t nV = s->nV;
    std::vector<d4> u(nV);
    std::vector<float4> vv(nV);
    for (size_t a = 0; a < nV; ++a) {
        double uu[3];
        float vl[3];
        for (int i = 0; i < 3; ++i) {
            const double xi = x[3 * a + i], vi = v[3 * a + i];
            if (!std::isfinite(xi) || !std::isfinite(vi)) return s->fail(JGS2_E_INVALID, "non-finite state");
            uu[i] = xi - s->X[3 * a + i];
            vl[i] = s->pinned[a] ? 0.0f : (float)vi;
        }
        u[a] = make_d4(uu[0], uu[1], uu[2], 0.0);
        vv[a] = make_float4(vl[0], vl[1], vl[2], 0.f);
    }
    int r;
    if ((r = upload(s, s->d_uhat, u.data(), nV)) || (r = upload(s, s->d_u, u.data(), nV)) ||
        (r = upload(s, s->d_unext, u.data(), nV)) || (r = upload(s, s->d_vhat, vv.data(), nV)))
        return r;
    HIPCHK(hipStreamSynchronize(s->stream));
    s->have_state = true;
    s->in_step = false;
    s->phase1_valid = false;
    s->ro_valid = false;
    return JGS2_OK;
}

// Device-resident state: x, v are nV x 3 doubles in device memory.
__global__ void k_state_in(int nV, const double* __restrict__ X64, const uint8_t* __restrict__ pinned,
                           const double* __restrict__ x, const double* __restrict__ v, d4* __restrict__ uhat,
                           d4* __restrict__ u, d4* __restrict__ unext, float4* __restrict__ vhat,
                           int* __restrict__ bad) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nV) return;
    double uu[3];
    float vl[3];
    bool ok = true;
    for (int i = 0; i < 3; ++i) {
        const double xi = x[3 * a + i], vi = v[3 * a + i];
        ok = ok && isfinite(xi) && isfinite(vi);
        uu[i] = xi - X64[3 * a + i];
        vl[i] = pinned[a] ? 0.0f : (float)vi;
    }
    if (!ok) *bad = 1;
    const d4 ud = make_d4(uu[0], uu[1], uu[2], 0.0);
    uhat[a] = ud;
    u[a] = ud;
    unext[a] = ud;
    vhat[a] = make_float4(vl[0], vl[1], vl[2], 0.0f);
}

__global__ void k_state_out(int nV, const double* __restrict__ X64, const d4* __restrict__ u,
                            const float4* __restrict__ vhat, double* __restrict__ x, double* __restrict__ v) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= nV) return;
    const d4 ud = u[a];
    const float4 vv = vhat[a];
    if (x) {
        x[3 * a] = X64[3 * a] + ud.x;
        x[3 * a + 1] = X64[3 * a + 1] + ud.y;
        x[3 * a + 2] = X64[3 * a + 2] + ud.z;
    }
    if (v) {
        v[3 * a] = vv.x;
        v[3 * a + 1] = vv.y;
        v[3 * a + 2] = vv.z;
    }
}

// FP64 rest positions and pinned flags on the device, made on first use.
static int ensure_state_io(jgs2_solver* s) {
    if (s->d_X64) return JGS2_OK;
    const size_t nV = s->nV;
    int r;
    if ((r = dalloc(s, s->d_X64, 3 * nV)) || (r = dalloc(s, s->d_pin8, nV)) || (r = dalloc(s, s->d_flag, 1)))
        return r;
    std::vector<uint8_t> pin(nV);
    for (size_t a = 0; a < nV; ++a) pin[a] = s->pinned[a] ? 1 : 0;
    if ((r = upload(s, s->d_X64, s->X.data(), 3 * nV)) || (r = upload(s, s->d_pin8, pin.data(), nV))) return r;
    return JGS2_OK;
}

int32_t jgs2_set_state_device(jgs2_solver* s, const double* x, const double* v) {
    if (!s) return JGS2_E_INVALID;
    if (!s->have_mesh) return s->fail(JGS2_E_NOT_READY, "no mesh");
    if (!x || !v) return s->fail(JGS2_E_INVALID, "NULL state");
    int r = ensure_state_io(s);
    if (r != JGS2_OK) return r;
    HIPCHK(hipMemsetAsync(s->d_flag, 0, sizeof(int), s->stream));
    hipLaunchKernelGGL(k_state_in, dim3((s->nV + 255) / 256), dim3(256), 0, s->stream, s->nV,
                       (const double*)s->d_X64, (const uint8_t*)s->d_pin8, x, v, s->d_uhat, s->d_u, s->d_unext,
                       s->d_vhat, s->d_flag);
    HIPCHK(hipGetLastError());
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, s->d_flag, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (bad) {
        s->have_state = false;
        return s->fail(JGS2_E_INVALID, "non-finite state");
    }
    s->have_state = true;
    s->in_step = false;
    s->phase1_valid = false;
    s->ro_valid = false;
    return JGS2_OK;
}

int32_t jgs2_get_state_device(jgs2_solver* s, double* x, double* v) {
    if (!s) return JGS2_E_INVALID;
    if (!s->have_state) return s->fail(JGS2_E_NOT_READY, "no state");
    int r = ensure_state_io(s);
    if (r != JGS2_OK) return r;
    hipLaunchKernelGGL(k_state_out, dim3((s->nV + 255) / 256), dim3(256), 0, s->stream, s->nV,
                       (const double*)s->d_X64, (const d4*)s->d_u, (const float4*)s->d_vhat, x, v);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->stream));
    return JGS2_OK;
}

int32_t jgs2_get_state(jgs2_solver* s, double* x, double* v) {
    if (!s) return JGS2_E_INVALID;
    if (!s->have_state) return s->fail(JGS2_E_NOT_READY, "no state");
    const size_t nV = s->nV;
    std::vector<d4> u(nV);
    std::vector<float4> vv(nV);
    // inside a step the current iterate is u; otherwise uhat == u
    HIPCHK(hipMemcpyAsync(u.data(), s->d_u, nV * sizeof(d4), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(vv.data(), s->d_vhat, nV * sizeof(float4), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (size_t a = 0; a < nV; ++a) {
        const double uu[3] = {u[a].x, u[a].y, u[a].z};
        const float vl[3] = {vv[a].x, vv[a].y, vv[a].z};
        for (int i = 0; i < 3; ++i) {
            if (x) x[3 * a + i] = s->X[3 * a + i] + uu[i];
            if (v) v[3 * a + i] = vl[i];
        }
    }
    return JGS2_OK;
}

static int read_reduced(jgs2_solver* s, int n_partials, double* out) {
    launch_reduce(s, n_partials);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(out, s->d_red, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    prof_collect(s);
    return JGS2_OK;
}

__global__ void k_copy_d4(int n, const d4* __restrict__ src, d4* __restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

static void keep_iterate(jgs2_solver* s) {
    hipLaunchKernelGGL(k_copy_d4, dim3((s->nV + 255) / 256), dim3(256), 0, s->stream, s->nV, (const d4*)s->d_u,
                       s->d_uprev);
}

// Residual check, device part: gradient (and rotations) at the iterate, the
// per-body |g_b|^2, and (mask_k > 0) the per-body stop decision after mask_k
// sweeps and |x_k - x_{k-1}|^2 of the last sweep (the paper's convergence
// measure), in fixed chunk order.  Graph-capturable: kernels only.
static void residual_launches(jgs2_solver* s, int mask_k) {
    SweepArgs a;
    build_sweep_args(s, a);
    launch_phase1(s, a, s->p.variant != JGS2_PLAIN, mask_k > 0);
    if (mask_k > 0)
        launch_check(s, mask_k);  // per-body residuals, stop flags, update norm
    else
        launch_seg_norm2(s);
}

// Host part: read the per-body residuals and the count of bodies still on;
// |g|^2 over all bodies (summed in body order) into *g2.
static int residual_readback(jgs2_solver* s, double* g2) {
    const size_t nb = s->n_bodies;
    std::vector<double> rb(nb + 2);
    HIPCHK(hipMemcpyAsync(rb.data(), s->d_rb, (nb + 2) * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    std::copy(rb.begin() + 2, rb.end(), s->r2_host.begin());
    std::memcpy(&s->n_active, &rb[1], sizeof(int));
    s->dx_norm = std::sqrt(rb[0]);
    prof_collect(s);
    s->phase1_valid = true;
    double t = 0.0;
    for (size_t b = 0; b < nb; ++b) t += s->r2_host[b];
    *g2 = t;
    return JGS2_OK;
}

// Largest per-body relative residual at the last readback.
static double max_rel(jgs2_solver* s) {
    double m = 0.0;
    for (int b = 0; b < s->n_bodies; ++b)
        if (s->r0sq_host[b] > 0) m = std::max(m, std::sqrt(s->r2_host[b] / s->r0sq_host[b]));
    return m;
}

static int gradient_norm2(jgs2_solver* s, double* out) {
    residual_launches(s, 0);
    return residual_readback(s, out);
}

static bool ready_to_step(jgs2_solver* s) {
    if (!s->have_mesh || !s->have_material) { s->err = "no mesh or material"; return false; }
    if (!s->have_state) { s->err = "no state"; return false; }
    // the sweep kernels read the bodies' stop flags (a failed set_bodies leaves none)
    if (!s->have_bodies) { s->err = "no body tables (set_bodies failed)"; return false; }
    if (s->p.variant != JGS2_PLAIN && !s->have_corr) { s->err = "no correction (precompute or import)"; return false; }
    if (s->p.variant == JGS2_EXACT && !s->have_full) {
        s->err = "no H-bar^-1 tiles (precompute with the JGS2_EXACT variant)";
        return false;
    }
    return true;
}

// Sets *bad when a free vertex is on or behind a plane (FP64 distances).
__global__ void k_infeasible(SweepArgs a, int* __restrict__ bad) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= a.nVf) return;
    const int v = a.free_ids[f];
    const d4 u = a.u[v];
    const float4 X = a.X[v];
    for (int p = 0; p < a.n_planes; ++p) {
        const double d = (double)a.planes_d[p][0] * ((double)X.x + u.x) + (double)a.planes_d[p][1] * ((double)X.y + u.y) +
                         (double)a.planes_d[p][2] * ((double)X.z + u.z) - a.planes_d[p][3];
        if (!(d > 0.0)) atomicOr(bad, 1);
    }
}

int32_t jgs2_begin_step(jgs2_solver* s) {
    if (!s) return JGS2_E_INVALID;
    if (!ready_to_step(s)) return JGS2_E_NOT_READY;
    const float grav[3] = {(float)s->p.gravity[0], (float)s->p.gravity[1], (float)s->p.gravity[2]};
    // contact feasibility of the start state (on the device: one flag)
    if (s->p.n_planes > 0) {
        SweepArgs a;
        build_sweep_args(s, a);
        a.u = s->d_uhat;
        HIPCHK(hipMemsetAsync(s->d_nactive, 0, sizeof(int), s->stream));
        hipLaunchKernelGGL(k_infeasible, dim3((s->nVf + 255) / 256), dim3(256), 0, s->stream, a, s->d_nactive);
        HIPCHK(hipGetLastError());
        int bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, s->d_nactive, sizeof(int), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        if (bad) return s->fail(JGS2_E_INFEASIBLE, "a vertex is on or behind a contact plane");
    }
    launch_predict(s, (float)s->p.dt, grav);
    residual_launches(s, 0);
    launch_mask_init(s);
    double g2 = 0;
    int r = residual_readback(s, &g2);
    if (r != JGS2_OK) return r;
    if (!std::isfinite(g2)) return s->fail(JGS2_E_NONFINITE, "non-finite residual at the start of the step");
    s->r0sq_host = s->r2_host;
    s->r0 = std::sqrt(g2);
    s->dx_norm = 0.0;
    s->in_step = true;
    s->sweeps_in_step = 0;
    s->ls_halvings = 0;
    return JGS2_OK;
}

static void swap_u(jgs2_solver* s) {
    std::swap(s->d_u, s->d_unext);
    s->phase1_valid = false;
}

static int energy_of(jgs2_solver* s, d4* state, double* e) {
    SweepArgs a;
    build_sweep_args(s, a);
    a.u = state;
    launch_energy(s, a, s->nT);
    return read_reduced(s, (std::max(s->nT, s->nVf) + 255) / 256, e);
}

// Global backtracking on the incremental potential (FP64 sum of FP32
// terms): halve the Jacobi move while E(x + t dx) > E(x), at most 8 times.
static int line_search(jgs2_solver* s) {
    TraceRange trace_range("jgs2_line_search");
    double e0 = 0, e1 = 0;
    int r;
    if ((r = energy_of(s, s->d_u, &e0)) || (r = energy_of(s, s->d_unext, &e1))) return r;
    for (int k = 0; k < 8 && !(e1 <= e0); ++k) {
        SweepArgs a;
        build_sweep_args(s, a);
        launch_blend(s, a, 0.5f);
        s->ls_halvings++;
        if ((r = energy_of(s, s->d_unext, &e1))) return r;
    }
    return JGS2_OK;
}

// One sweep in the configured order and variant.
static int sweep_once(jgs2_solver* s) {
    SweepArgs a;
    build_sweep_args(s, a);
    const bool cub = s->p.variant == JGS2_CUBATURE;  // the two-phase R3 sweeps
    if (s->p.variant == JGS2_EXACT) {
        // gradients and rotations at the iterate, their rest-frame form in the
        // rows' order, then every row's exact local solve (Jacobi), or the
        // same for one colour at a time (GS, gradients refreshed per colour)
        if (s->p.order == JGS2_JACOBI) {
            if (!s->phase1_valid) launch_phase1(s, a, true, true);
            launch_reduced_gradient(s, a);
            launch_exact(s, a);
            if (s->p.line_search) {
                int r = line_search(s);
                if (r != JGS2_OK) return r;
            }
            swap_u(s);
        } else {
            for (int c = 0; c < s->n_colors; ++c) {
                SweepArgs all = a;
                launch_phase1(s, all, true, true);
                launch_reduced_gradient(s, all);
                SweepArgs ac = a;
                ac.list = s->d_colperm + s->col_off[c];
                ac.n_list = s->col_off[c + 1] - s->col_off[c];
                ac.in_place = 1;
                launch_exact(s, ac);
            }
            s->phase1_valid = false;
        }
        s->sweeps_in_step++;
        return jgs2::hip_check(s, hipGetLastError(), "sweep launch");
    }
    if (s->p.variant == JGS2_DAMPER) {
        // rotations of the sweep's starting iterate x^k (Sec. 4.3), held for
        // every colour; each row's gradient and diagonal block are gathered
        // fresh inside the fused kernel
        if (!s->phase1_valid) launch_rotations(s, a);
        if (s->p.order == JGS2_JACOBI) {
            launch_damper(s, a);
            if (s->p.line_search) {
                int r = line_search(s);
                if (r != JGS2_OK) return r;
            }
            swap_u(s);
        } else {
            for (int c = 0; c < s->n_colors; ++c) {
                SweepArgs ac = a;
                ac.list = s->d_colperm + s->col_off[c];
                ac.n_list = s->col_off[c + 1] - s->col_off[c];
                ac.in_place = 1;
                ac.cbase = s->col_off[c];
                launch_damper(s, ac);
            }
            s->phase1_valid = false;
        }
        s->sweeps_in_step++;
        return jgs2::hip_check(s, hipGetLastError(), "sweep launch");
    }
    if (s->p.order == JGS2_JACOBI) {
        if (cub) {
            if (!s->phase1_valid) launch_phase1(s, a, true, true);
            launch_phase2_cubature(s, a);
        } else {
            launch_plain(s, a);
        }
        if (s->p.line_search) {
            int r = line_search(s);
            if (r != JGS2_OK) return r;
        }
        swap_u(s);
    } else {
        for (int c = 0; c < s->n_colors; ++c) {
            SweepArgs ac = a;
            ac.list = s->d_colperm + s->col_off[c];
            ac.n_list = s->col_off[c + 1] - s->col_off[c];
            if (cub) {
                SweepArgs all = a;
                launch_phase1(s, all, true, true);
                launch_phase2_cubature(s, ac);
                launch_commit(s, ac);
            } else {
                ac.in_place = 1;
                ac.cbase = s->col_off[c];
                launch_plain(s, ac);
            }
        }
        s->phase1_valid = false;
    }
    s->sweeps_in_step++;
    return jgs2::hip_check(s, hipGetLastError(), "sweep launch");
}

// k sweeps followed by the residual launches (with the per-body stop
// decision); replayed from a captured graph when use_graph is set.
static int sweep_group(jgs2_solver* s, int k) {
    TraceRange trace_range("jgs2_sweep_group");
    if (s->persistent && s->p.variant == JGS2_PLAIN && s->p.order == JGS2_GS && !s->p.line_search && !s->prof) {
        // the whole group as one cooperative launch, then the residual check
        SweepArgs a;
        build_sweep_args(s, a);
        a.in_place = 1;
        int r = launch_plain_persistent(s, a, k);
        if (r != JGS2_OK) return r;
        residual_launches(s, k);
        s->sweeps_in_step += k;
        s->phase1_valid = false;
        return jgs2::hip_check(s, hipGetLastError(), "sweep launch");
    }
    const bool graphable = s->p.use_graph && !s->prof && !s->p.line_search;
    if (!graphable) {
        for (int i = 0; i < k; ++i) {
            if (i == k - 1) keep_iterate(s);
            int r = sweep_once(s);
            if (r != JGS2_OK) return r;
        }
        residual_launches(s, k);
        // the check's phase 1 left g (and, for the corrected variants, R) at
        // the iterate the next sweep starts from
        s->phase1_valid = s->p.variant != JGS2_PLAIN;
        return jgs2::hip_check(s, hipGetLastError(), "sweep launch");
    }
    // a Jacobi group of odd length leaves u and unext swapped: graphs are
    // keyed by the group length and the buffer holding the iterate
    if (s->stream == nullptr) {
        if (!s->own_stream) HIPCHK(hipStreamCreate(&s->own_stream));
        s->stream = s->own_stream;
    }
    int par = -1;
    for (int i = 0; i < 2; ++i)
        if (s->graph_exec[i] && s->graph_k[i] == k && s->graph_u[i] == s->d_u) par = i;
    if (par < 0) {
        par = !s->graph_exec[0] ? 0 : (!s->graph_exec[1] ? 1 : s->graph_next);
        s->graph_next = par ^ 1;
        if (s->graph_exec[par]) (void)hipGraphExecDestroy(s->graph_exec[par]);
        s->graph_exec[par] = nullptr;
        d4* u0 = s->d_u;
        const int sw0 = s->sweeps_in_step;
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
        int r = JGS2_OK;
        for (int i = 0; i < k && r == JGS2_OK; ++i) {
            if (i == k - 1) keep_iterate(s);
            r = sweep_once(s);
        }
        if (r == JGS2_OK) residual_launches(s, k);
        hipError_t e = hipStreamEndCapture(s->stream, &g);
        // capture only recorded the launches: put the bookkeeping back
        if (s->d_u != u0) std::swap(s->d_u, s->d_unext);
        s->sweeps_in_step = sw0;
        if (r != JGS2_OK) { if (g) (void)hipGraphDestroy(g); return r; }
        HIPCHK(e);
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPCHK(e);
        s->graph_exec[par] = ex;
        s->graph_k[par] = k;
        s->graph_u[par] = u0;
    }
    HIPCHK(hipGraphLaunch(s->graph_exec[par], s->stream));
    if (s->p.order == JGS2_JACOBI && (k & 1)) std::swap(s->d_u, s->d_unext);
    s->sweeps_in_step += k;
    s->phase1_valid = false;
    return JGS2_OK;
}

int32_t jgs2_iterate(jgs2_solver* s, int32_t n_sweeps, double* rel_res) {
    if (!s) return JGS2_E_INVALID;
    if (!s->in_step) return s->fail(JGS2_E_NOT_READY, "iterate outside begin_step/end_step");
    if (n_sweeps < 0) return s->fail(JGS2_E_INVALID, "negative sweep count");
    if (n_sweeps == 0) {
        double g2 = 0;
        int r = gradient_norm2(s, &g2);
        if (r != JGS2_OK) return r;
        if (rel_res) *rel_res = max_rel(s);
        return std::isfinite(g2) ? JGS2_OK : s->fail(JGS2_E_NONFINITE, "non-finite residual");
    }
    int r = sweep_group(s, n_sweeps);
    if (r != JGS2_OK) return r;
    double g2 = 0;
    if ((r = residual_readback(s, &g2)) != JGS2_OK) return r;
    const double rel = max_rel(s);
    if (rel_res) *rel_res = rel;
    if (!std::isfinite(g2)) return s->fail(JGS2_E_NONFINITE, "non-finite residual");
    if (rel > 1e8) return s->fail(JGS2_E_DIVERGED, "residual exceeded 1e8 x its start value");
    return JGS2_OK;
}

int32_t jgs2_end_step(jgs2_solver* s) {
    if (!s) return JGS2_E_INVALID;
    if (!s->in_step) return s->fail(JGS2_E_NOT_READY, "end_step without begin_step");
    launch_velocity(s, (float)s->p.dt);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(s->d_unext, s->d_u, (size_t)s->nV * sizeof(d4), hipMemcpyDeviceToDevice, s->stream));
    s->in_step = false;
    s->phase1_valid = false;
    return JGS2_OK;
}

static int abandon_step(jgs2_solver* s) {
    // restore the iterate to the start of the step
    (void)hipMemcpyAsync(s->d_u, s->d_uhat, (size_t)s->nV * sizeof(d4), hipMemcpyDeviceToDevice, s->stream);
    (void)hipMemcpyAsync(s->d_unext, s->d_uhat, (size_t)s->nV * sizeof(d4), hipMemcpyDeviceToDevice, s->stream);
    (void)hipStreamSynchronize(s->stream);
    s->in_step = false;
    s->phase1_valid = false;
    return JGS2_OK;
}

// Residual readback of a sweep group into pinned slot `slot`, without waiting.
static int enqueue_readback(jgs2_solver* s, int slot) {
    const size_t nb = s->n_bodies;
    HIPCHK(hipMemcpyAsync(s->h_rb[slot], s->d_rb, (nb + 2) * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipEventRecord(s->rb_ev[slot], s->stream));
    return JGS2_OK;
}

// Waits for a readback and takes it as the current per-body residuals.
static int finish_readback(jgs2_solver* s, int slot, double* rel) {
    HIPCHK(hipEventSynchronize(s->rb_ev[slot]));
    prof_collect(s);
    double g2 = 0.0;
    for (int b = 0; b < s->n_bodies; ++b) {
        s->r2_host[b] = s->h_r2[slot][b];
        g2 += s->r2_host[b];
    }
    s->n_active = *s->h_nact[slot];
    s->dx_norm = std::sqrt(*s->h_dx2[slot]);
    *rel = max_rel(s);
    if (!std::isfinite(g2)) return s->fail(JGS2_E_NONFINITE, "non-finite residual");
    if (*rel > 1e8) return s->fail(JGS2_E_DIVERGED, "residual exceeded 1e8 x its start value");
    return JGS2_OK;
}

int32_t jgs2_step(jgs2_solver* s, jgs2_step_stats* st) {
    TraceRange trace_range("jgs2_step");
    if (!s) return JGS2_E_INVALID;
    jgs2_step_stats loc;
    std::memset(&loc, 0, sizeof(loc));
    HIPCHK(hipEventRecord(s->ev0, s->stream));
    int r = jgs2_begin_step(s);
    if (r != JGS2_OK) { loc.status = r; if (st) *st = loc; return r; }
    double rel = s->r0 == 0.0 ? 0.0 : 1.0;
    auto failed = [&](int code) {
        loc.status = code; loc.sweeps = s->sweeps_in_step; loc.r0 = s->r0; loc.r_final = rel;
        abandon_step(s);
        if (st) *st = loc;
        return code;
    };
    if (s->p.line_search) {
        // the energy search reads back inside every sweep: plain synchronous loop
        while (s->n_active > 0 && s->sweeps_in_step < s->p.max_sweeps) {
            const int k = std::min(s->p.check_every, s->p.max_sweeps - s->sweeps_in_step);
            r = jgs2_iterate(s, k, &rel);
            if (r != JGS2_OK) return failed(r);
        }
    } else {
        // one sweep group stays in flight while the previous group's residuals
        // come back; the stop decision itself is taken on the device (per-body
        // masks), so a group issued after convergence changes nothing
        int pending = -1, slot = 0;
        double rel_prev = -1.0, rel_last = -1.0;  // residuals of the last two groups read back
        for (;;) {
            int issued = -1;
            // issue the next group before the in-flight one's residual is known
            // unless the rate so far says the in-flight group reaches rel_tol
            bool speculate = true;
            if (pending >= 0 && rel_prev > 0.0 && rel_last > 0.0) {
                const double predicted = rel_last * std::min(1.0, rel_last / rel_prev);
                speculate = predicted > s->p.rel_tol;
            }
            if (pending >= 0 && !speculate) {
                if ((r = finish_readback(s, pending, &rel)) != JGS2_OK) {
                    (void)hipStreamSynchronize(s->stream);
                    return failed(r);
                }
                rel_prev = rel_last;
                rel_last = rel;
                pending = -1;
            }
            if (s->n_active > 0 && s->sweeps_in_step < s->p.max_sweeps) {
                const int k = std::min(s->p.check_every, s->p.max_sweeps - s->sweeps_in_step);
                if ((r = sweep_group(s, k)) != JGS2_OK || (r = enqueue_readback(s, slot)) != JGS2_OK) {
                    (void)hipStreamSynchronize(s->stream);
                    return failed(r);
                }
                issued = slot;
                slot ^= 1;
            }
            if (pending >= 0) {
                if ((r = finish_readback(s, pending, &rel)) != JGS2_OK) {
                    (void)hipStreamSynchronize(s->stream);
                    return failed(r);
                }
                rel_prev = rel_last;
                rel_last = rel;
            }
            if (issued < 0) break;
            pending = issued;
        }
    }
    std::vector<int> bsw((size_t)s->n_bodies);
    HIPCHK(hipMemcpyAsync(bsw.data(), s->d_body_sweeps, bsw.size() * sizeof(int), hipMemcpyDeviceToHost, s->stream));
    r = jgs2_end_step(s);
    if (r != JGS2_OK) return r;
    HIPCHK(hipEventRecord(s->ev1, s->stream));
    HIPCHK(hipEventSynchronize(s->ev1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, s->ev0, s->ev1));
    int most = 0;
    for (int b : bsw) most = std::max(most, b);
    // a body still iterating at the last check reached max_sweeps above rel_tol
    const int status = s->n_active > 0 ? JGS2_NOT_CONVERGED : JGS2_OK;
    loc.sweeps = most; loc.status = status; loc.r0 = s->r0; loc.r_final = rel; loc.seconds = ms * 1e-3;
    loc.ls_halvings = s->ls_halvings;
    loc.dx_norm = s->dx_norm;
    if (s->d_bounds) {  // bounds-checked build: a failed index check fails the step
        int32_t line = 0;
        int64_t idx = 0, ext = 0;
        if ((r = jgs2_bounds_report(s, &line, &idx, &ext, 0)) != JGS2_OK) return r;
        if (line != 0) {
            loc.status = JGS2_E_BOUNDS;
            if (st) *st = loc;
            return s->fail(JGS2_E_BOUNDS, "index check failed in sweep.hip line " + std::to_string(line) +
                                              ": index " + std::to_string(idx) + " of extent " +
                                              std::to_string(ext));
        }
    }
    if (st) *st = loc;
    if (status != JGS2_OK) s->err = "max_sweeps reached above rel_tol";
    return status;
}

int32_t jgs2_residual(jgs2_solver* s, double* abs_res, double* rel_res) {
    if (!s) return JGS2_E_INVALID;
    if (!ready_to_step(s)) return JGS2_E_NOT_READY;
    double g2 = 0;
    int r = gradient_norm2(s, &g2);
    if (r != JGS2_OK) return r;
    if (abs_res) *abs_res = std::sqrt(g2);
    if (rel_res) *rel_res = s->r0 > 0 ? std::sqrt(g2) / s->r0 : 0.0;
    return JGS2_OK;
}

int32_t jgs2_energy(jgs2_solver* s, double* e) {
    if (!s) return JGS2_E_INVALID;
    if (!ready_to_step(s)) return JGS2_E_NOT_READY;
    SweepArgs a;
    build_sweep_args(s, a);
    launch_energy(s, a, s->nT);
    return read_reduced(s, (std::max(s->nT, s->nVf) + 255) / 256, e);
}

int32_t jgs2_energy_noalloc(jgs2_solver* s, double* e) {
    if (!s) return JGS2_E_INVALID;
    if (!e) return s->fail(JGS2_E_INVALID, "NULL output");
    if (!ready_to_step(s)) return JGS2_E_NOT_READY;
    const int n_partials = (std::max(s->nT, s->nVf) + 255) / 256;
    if (n_partials > JGS2_NOALLOC_MAX_PARTIALS)
        return s->fail(JGS2_E_INVALID, "jgs2_energy_noalloc: more than 256 x JGS2_NOALLOC_MAX_PARTIALS tets or "
                                       "free vertices (use jgs2_energy)");
    double* sp = (s->device >= 0 && s->device < kMaxDevices) ? g_scratch_ptr[s->device] : nullptr;
    if (!sp) return s->fail(JGS2_E_NOT_READY, "no scratch address for this device");
    // the same kernels as jgs2_energy, with the partials and the total in the
    // scratch array; launched without profiling events (no event creation)
    const bool prof = s->prof;
    s->prof = false;
    SweepArgs a;
    build_sweep_args(s, a);
    a.partial = sp;
    launch_energy(s, a, s->nT);
    launch_reduce_into(s, sp, n_partials, sp + JGS2_NOALLOC_MAX_PARTIALS);
    s->prof = prof;
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(e, sp + JGS2_NOALLOC_MAX_PARTIALS, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return JGS2_OK;
}

int32_t jgs2_get_phase1(jgs2_solver* s, double* g, double* R) {
    if (!s) return JGS2_E_INVALID;
    if (!s->have_mesh || !s->have_material || !s->have_state) return s->fail(JGS2_E_NOT_READY, "no state");
    if (!s->have_bodies) return s->fail(JGS2_E_NOT_READY, "no body tables (set_bodies failed)");
    SweepArgs a;
    build_sweep_args(s, a);
    launch_phase1(s, a, true);
    s->phase1_valid = s->in_step;
    HIPCHK(hipGetLastError());
    const size_t nV = s->nV;
    std::vector<float4> gg(nV), qq(nV);
    HIPCHK(hipMemcpyAsync(gg.data(), s->d_g, nV * sizeof(float4), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(qq.data(), s->d_R, nV * sizeof(float4), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (size_t v = 0; v < nV; ++v) {
        const double gv[3] = {gg[v].x, gg[v].y, gg[v].z};
        for (int i = 0; i < 3; ++i)
            if (g) g[3 * v + i] = s->pinned[v] ? 0.0 : gv[i];
        if (R) {
            double Rm[9];
            jgs2::rot_from_quat<double>(qq[v].x, qq[v].y, qq[v].z, qq[v].w, Rm);
            for (int i = 0; i < 9; ++i) R[9 * v + i] = s->pinned[v] ? ((i % 4 == 0) ? 1.0 : 0.0) : Rm[i];
        }
    }
    return JGS2_OK;
}

int32_t jgs2_set_profiling(jgs2_solver* s, int32_t on) {
    if (!s) return JGS2_E_INVALID;
    HIPCHK(hipStreamSynchronize(s->stream));
    prof_collect(s);
    s->prof = on != 0;
    for (int k = 0; k < JGS2_NKERNELS; ++k) { s->kt_ms[k] = 0.0; s->kt_n[k] = 0; }
    return JGS2_OK;
}

int32_t jgs2_kernel_times(jgs2_solver* s, double* ms, int64_t* launches) {
    if (!s) return JGS2_E_INVALID;
    HIPCHK(hipStreamSynchronize(s->stream));
    prof_collect(s);
    for (int k = 0; k < JGS2_NKERNELS; ++k) {
        if (ms) ms[k] = s->kt_ms[k];
        if (launches) launches[k] = s->kt_n[k];
    }
    return JGS2_OK;
}

int32_t jgs2_get_coloring(jgs2_solver* s, int32_t* color, int32_t* n_colors) {
    if (!s) return JGS2_E_INVALID;
    if (!s->have_mesh) return s->fail(JGS2_E_NOT_READY, "no mesh");
    if (color) std::copy(s->color.begin(), s->color.end(), color);
    if (n_colors) *n_colors = s->n_colors;
    return JGS2_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Differentiable rollout (adjoint of the step map through its optimality
// condition) with checkpointed recomputation.
// ---------------------------------------------------------------------------
template <typename T>
static int copy_v4(jgs2_solver* s, T* dst, const T* src) {
    return jgs2::hip_check(s, hipMemcpyAsync(dst, src, (size_t)s->nV * sizeof(T), hipMemcpyDeviceToDevice, s->stream),
                           "state copy");
}

static int save_checkpoint(jgs2_solver* s, int slot) {
    const size_t off = (size_t)slot * s->nV;
    int r;
    if ((r = copy_v4(s, s->d_ck_u + off, s->d_uhat)) || (r = copy_v4(s, s->d_ck_v + off, s->d_vhat))) return r;
    return JGS2_OK;
}

static int load_checkpoint(jgs2_solver* s, int slot) {
    const size_t off = (size_t)slot * s->nV;
    int r;
    if ((r = copy_v4(s, s->d_uhat, s->d_ck_u + off)) || (r = copy_v4(s, s->d_u, s->d_ck_u + off)) ||
        (r = copy_v4(s, s->d_unext, s->d_ck_u + off)) || (r = copy_v4(s, s->d_vhat, s->d_ck_v + off)))
        return r;
    s->in_step = false;
    s->phase1_valid = false;
    return JGS2_OK;
}

// |H y - rhs|^2 over free DOFs at the displacement a.u (no update).
static int linear_residual2(jgs2_solver* s, SweepArgs a, double* r2) {
    a.list = nullptr;
    a.n_list = 0;
    a.no_write = 1;
    a.ly = s->d_y;
    launch_linear(s, a);
    const int nv_blk = s->tune_block / s->tune_lpv;
    return read_reduced(s, (s->nVf + nv_blk - 1) / nv_blk, r2);
}

// Solves H(xstar) y = rhs (device d_rhs) by linear sweeps, warm-started from
// the y already in d_y.
static int adjoint_solve(jgs2_solver* s, const d4* xstar, int64_t* sweeps, double* rel) {
    SweepArgs a;
    build_sweep_args(s, a);
    a.u = xstar;
    a.lrhs = s->d_rhs;
    a.nactive = nullptr;  // the forward step's stop flags do not apply to the adjoint solve
    a.mh2 = s->d_mh2;
    double b2 = 0.0, r2 = 0.0;
    launch_norm2(s, s->d_rhs);
    int r = read_reduced(s, (s->nVf + 255) / 256, &b2);
    if (r != JGS2_OK) return r;
    if (!std::isfinite(b2)) return s->fail(JGS2_E_NONFINITE, "non-finite adjoint right-hand side");
    *rel = 0.0;
    if (b2 == 0.0) {
        HIPCHK(hipMemsetAsync(s->d_y, 0, (size_t)s->nV * sizeof(float4), s->stream));
        return JGS2_OK;
    }
    if ((r = linear_residual2(s, a, &r2)) != JGS2_OK) return r;
    *rel = std::sqrt(r2 / b2);
    const bool exact = s->p.variant == JGS2_EXACT;
    if (exact) launch_rotations(s, a);  // the co-rotated rows at x*
    int k = 0;
    while (*rel > s->p.adj_rel_tol && k < s->p.adj_max_sweeps) {
        const int n = std::min(s->p.check_every, s->p.adj_max_sweeps - k);
        for (int i = 0; i < n; ++i) {
            if (exact) {
                // the exact subspace's local systems of H(x*) y = rhs: residual
                // r = H y - rhs at every vertex, its rest-frame form, then the
                // rows (all of them, or one colour at a time with r refreshed)
                const int nc = s->p.order == JGS2_JACOBI ? 1 : s->n_colors;
                for (int c = 0; c < nc; ++c) {
                    SweepArgs ar = a;
                    ar.list = nullptr;
                    ar.n_list = 0;
                    ar.no_write = 1;
                    ar.ly = s->d_y;
                    ar.lres = s->d_g;
                    launch_linear(s, ar);
                    SweepArgs ah = a;
                    ah.g = s->d_g;
                    launch_reduced_gradient(s, ah);
                    SweepArgs ae = a;
                    ae.ly = s->d_y;
                    if (s->p.order == JGS2_JACOBI) {
                        ae.lynext = s->d_ynext;
                    } else {
                        ae.in_place = 1;
                        ae.list = s->d_colperm + s->col_off[c];
                        ae.n_list = s->col_off[c + 1] - s->col_off[c];
                    }
                    launch_exact_linear(s, ae);
                }
                if (s->p.order == JGS2_JACOBI) std::swap(s->d_y, s->d_ynext);
            } else if (s->p.order == JGS2_JACOBI) {
                SweepArgs aj = a;
                aj.ly = s->d_y;
                aj.lynext = s->d_ynext;
                launch_linear(s, aj);
                std::swap(s->d_y, s->d_ynext);
            } else {
                for (int c = 0; c < s->n_colors; ++c) {
                    SweepArgs ac = a;
                    ac.ly = s->d_y;
                    ac.in_place = 1;
                    ac.list = s->d_colperm + s->col_off[c];
                    ac.n_list = s->col_off[c + 1] - s->col_off[c];
                    ac.cbase = s->col_off[c];
                    launch_linear(s, ac);
                }
            }
        }
        HIPCHK(hipGetLastError());
        k += n;
        if ((r = linear_residual2(s, a, &r2)) != JGS2_OK) return r;
        *rel = std::sqrt(r2 / b2);
        if (!std::isfinite(*rel)) return s->fail(JGS2_E_NONFINITE, "non-finite adjoint residual");
        if (*rel > 1e8) return s->fail(JGS2_E_DIVERGED, "adjoint residual exceeded 1e8 x |b|");
    }
    *sweeps += k;
    return JGS2_OK;
}

extern "C" {

int32_t jgs2_rollout(jgs2_solver* s, int32_t n_steps, int32_t ckpt_every, jgs2_step_stats* last) {
    TraceRange trace_range("jgs2_rollout");
    if (!s) return JGS2_E_INVALID;
    if (n_steps < 1 || ckpt_every < 1) return s->fail(JGS2_E_INVALID, "n_steps and ckpt_every must be >= 1");
    if (!ready_to_step(s)) return JGS2_E_NOT_READY;
    if (s->in_step) return s->fail(JGS2_E_NOT_READY, "rollout inside begin_step/end_step");
    s->ro_valid = false;
    const int n_ck = (n_steps + ckpt_every - 1) / ckpt_every;
    const size_t nV = s->nV;
    int r;
    if ((r = dalloc(s, s->d_ck_u, (n_ck + 1) * nV)) || (r = dalloc(s, s->d_ck_v, (n_ck + 1) * nV)) ||
        (r = dalloc(s, s->d_seg, (size_t)std::min(ckpt_every, n_steps) * nV)))
        return r;
    jgs2_step_stats st;
    std::memset(&st, 0, sizeof(st));
    bool capped = false;
    for (int n = 0; n < n_steps; ++n) {
        if (n % ckpt_every == 0 && (r = save_checkpoint(s, n / ckpt_every)) != JGS2_OK) return r;
        r = jgs2_step(s, &st);
        if (r == JGS2_NOT_CONVERGED) {
            capped = true;
        } else if (r != JGS2_OK) {
            if (last) *last = st;
            return r;
        }
    }
    if ((r = save_checkpoint(s, n_ck)) != JGS2_OK) return r;
    HIPCHK(hipStreamSynchronize(s->stream));
    s->ro_steps = n_steps;
    s->ro_every = ckpt_every;
    s->ro_nck = n_ck;
    s->ro_valid = true;
    if (last) *last = st;
    if (capped) {
        s->err = "a step reached max_sweeps above rel_tol";
        return JGS2_NOT_CONVERGED;
    }
    return JGS2_OK;
}

int32_t jgs2_rollout_backward(jgs2_solver* s, const double* xbar, const double* vbar, double* thetabar,
                              double* xbar0, double* vbar0, double* ubar, jgs2_adjoint_stats* stats) {
    TraceRange trace_range("jgs2_rollout_backward");
    if (!s) return JGS2_E_INVALID;
    if (!s->ro_valid) return s->fail(JGS2_E_NOT_READY, "no rollout to differentiate");
    if (!xbar) return s->fail(JGS2_E_INVALID, "NULL xbar");
    jgs2_adjoint_stats loc;
    std::memset(&loc, 0, sizeof(loc));
    const size_t nV = s->nV;
    const double h = s->p.dt;
    std::vector<float4> xb(nV), vb(nV), rhs(nV);
    for (size_t a = 0; a < nV; ++a) {
        double x3[3] = {0, 0, 0}, v3[3] = {0, 0, 0};
        if (!s->pinned[a])
            for (int i = 0; i < 3; ++i) {
                x3[i] = xbar[3 * a + i];
                v3[i] = vbar ? vbar[3 * a + i] : 0.0;
                if (!std::isfinite(x3[i]) || !std::isfinite(v3[i])) return s->fail(JGS2_E_INVALID, "non-finite cotangent");
            }
        xb[a] = make_float4((float)x3[0], (float)x3[1], (float)x3[2], 0.f);
        vb[a] = make_float4((float)v3[0], (float)v3[1], (float)v3[2], 0.f);
        rhs[a] = make_float4((float)(x3[0] + v3[0] / h), (float)(x3[1] + v3[1] / h), (float)(x3[2] + v3[2] / h), 0.f);
    }
    int r;
    if ((r = dalloc(s, s->d_y, nV)) || (r = dalloc(s, s->d_ynext, nV)) || (r = dalloc(s, s->d_xbar, nV)) ||
        (r = dalloc(s, s->d_vbar, nV)) || (r = dalloc(s, s->d_rhs, nV)) || (r = dalloc(s, s->d_thbar, (size_t)s->nT)))
        return r;
    hipEvent_t e0 = pool_event(s), e1 = pool_event(s);
    struct EventReturn {  // the pair goes back to the pool on every return path
        jgs2_solver* s;
        hipEvent_t a, b;
        ~EventReturn() { s->ev_pool.push_back(a); s->ev_pool.push_back(b); }
    } event_return{s, e0, e1};
    HIPCHK(hipEventRecord(e0, s->stream));
    if ((r = upload(s, s->d_xbar, xb.data(), nV)) || (r = upload(s, s->d_vbar, vb.data(), nV)) ||
        (r = upload(s, s->d_rhs, rhs.data(), nV)))
        return r;
    HIPCHK(hipMemsetAsync(s->d_y, 0, nV * sizeof(float4), s->stream));
    HIPCHK(hipMemsetAsync(s->d_ynext, 0, nV * sizeof(float4), s->stream));
    HIPCHK(hipMemsetAsync(s->d_thbar, 0, (size_t)s->nT * sizeof(double), s->stream));
    int status = JGS2_OK;
    bool capped = false;  // a recomputed step or an adjoint solve ended at its sweep cap
    for (int k = s->ro_nck - 1; k >= 0 && status == JGS2_OK; --k) {
        const int n0 = k * s->ro_every, n1 = std::min(n0 + s->ro_every, s->ro_steps);
        if ((r = load_checkpoint(s, k)) != JGS2_OK) return r;
        for (int n = n0; n < n1 && status == JGS2_OK; ++n) {
            jgs2_step_stats st;
            status = jgs2_step(s, &st);
            if (status == JGS2_NOT_CONVERGED) {
                capped = true;
                status = JGS2_OK;
            }
            loc.forward_sweeps += st.sweeps;
            if (status == JGS2_OK && (r = copy_v4(s, s->d_seg + (size_t)(n - n0) * nV, s->d_uhat)) != JGS2_OK)
                return r;
        }
        for (int n = n1 - 1; n >= n0 && status == JGS2_OK; --n) {
            const d4* xstar = s->d_seg + (size_t)(n - n0) * nV;
            double rel = 0.0;
            status = adjoint_solve(s, xstar, &loc.adjoint_sweeps, &rel);
            if (status != JGS2_OK) break;
            if (rel > s->p.adj_rel_tol) capped = true;
            loc.max_rel_res = std::max(loc.max_rel_res, rel);
            launch_param_grad(s, xstar, s->d_y, s->d_thbar);
            launch_adj_vec(s, s->d_y, s->d_xbar, s->d_vbar, s->d_rhs);
            HIPCHK(hipGetLastError());
            loc.steps++;
        }
    }
    // leave the state at the end of the rollout
    if ((r = load_checkpoint(s, s->ro_nck)) != JGS2_OK) return r;
    HIPCHK(hipEventRecord(e1, s->stream));
    if (status == JGS2_OK) {
        std::vector<double> th((size_t)s->nT);
        HIPCHK(hipMemcpyAsync(th.data(), s->d_thbar, th.size() * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipMemcpyAsync(xb.data(), s->d_xbar, nV * sizeof(float4), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipMemcpyAsync(vb.data(), s->d_vbar, nV * sizeof(float4), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        if (thetabar) std::memcpy(thetabar, th.data(), th.size() * sizeof(double));
        // cotangent of one initial velocity shared by every free vertex:
        // the sum of vbar_0 over free vertices, in ascending vertex order
        double u3[3] = {0.0, 0.0, 0.0};
        for (size_t a = 0; a < nV; ++a) {
            const float x3[3] = {xb[a].x, xb[a].y, xb[a].z}, v3[3] = {vb[a].x, vb[a].y, vb[a].z};
            for (int i = 0; i < 3; ++i) {
                if (xbar0) xbar0[3 * a + i] = x3[i];
                if (vbar0) vbar0[3 * a + i] = v3[i];
                if (!s->pinned[a]) u3[i] += (double)v3[i];
            }
        }
        if (ubar)
            for (int i = 0; i < 3; ++i) ubar[i] = u3[i];
    }
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    loc.seconds = ms * 1e-3;
    if (status == JGS2_OK && capped) {
        status = JGS2_NOT_CONVERGED;
        s->err = "a recomputed step or an adjoint solve reached its sweep cap";
    }
    loc.status = status;
    if (stats) *stats = loc;
    // a recompute that differs from the rollout would leave ro_valid wrong;
    // the forward is deterministic, so the rollout stays usable
    return status;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Bodies, launch shape, autotuning
// ---------------------------------------------------------------------------
extern "C" {

int32_t jgs2_set_bodies(jgs2_solver* s, int32_t n_bodies, const int32_t* body_of_vertex) {
    if (!s) return JGS2_E_INVALID;
    // the tables below are replaced one by one: until the last upload has
    // succeeded nothing may read them, and a failure leaves none
    s->have_bodies = false;
    s->in_step = false;
    s->ro_valid = false;
    drop_graphs(s);
    if (!s->have_mesh && s->nV == 0) return s->fail(JGS2_E_NOT_READY, "no mesh");
    if (n_bodies < 1 || !body_of_vertex) return s->fail(JGS2_E_INVALID, "n_bodies must be >= 1");
    if (n_bodies > 1 && s->p.line_search) return s->fail(JGS2_E_INVALID, "the energy line search needs a single body");
    for (int v = 0; v < s->nV; ++v)
        if (body_of_vertex[v] < 0 || body_of_vertex[v] >= n_bodies) return s->fail(JGS2_E_INVALID, "body id out of range");
    for (int t = 0; t < s->nT; ++t) {
        const int b0 = body_of_vertex[s->tets[4 * (size_t)t]];
        for (int c = 1; c < 4; ++c)
            if (body_of_vertex[s->tets[4 * (size_t)t + c]] != b0) return s->fail(JGS2_E_INVALID, "a tet spans two bodies");
    }
    const int nf = s->nVf;
    std::vector<int> fbody(nf), off(n_bodies + 1, 0), idx(nf);
    for (int f = 0; f < nf; ++f) {
        fbody[f] = body_of_vertex[s->free_ids[f]];
        off[fbody[f] + 1]++;
    }
    for (int b = 0; b < n_bodies; ++b) off[b + 1] += off[b];
    std::vector<int> pos(off.begin(), off.end() - 1);
    for (int f = 0; f < nf; ++f) idx[pos[fbody[f]]++] = f;  // stable: ascending free index within a body
    // fixed chunks of each body's free vertices for the residual sums
    const int CH = seg_chunk_size();
    std::vector<int> clo, chi, boff(n_bodies + 1, 0);
    for (int b = 0; b < n_bodies; ++b) {
        for (int i = off[b]; i < off[b + 1]; i += CH) {
            clo.push_back(i);
            chi.push_back(std::min(i + CH, off[b + 1]));
        }
        boff[b + 1] = (int)clo.size();
    }
    const size_t nch = clo.size();
    int r;
    const size_t nb = n_bodies;
    if ((r = dalloc(s, s->d_chunk_lo, nch)) || (r = dalloc(s, s->d_chunk_hi, nch)) ||
        (r = dalloc(s, s->d_body_chunk_off, nb + 1)) || (r = dalloc(s, s->d_r2c, nch)) ||
        (r = dalloc(s, s->d_dx2c, nch)))
        return r;
    if (nch > 0 && ((r = upload(s, s->d_chunk_lo, clo.data(), nch)) || (r = upload(s, s->d_chunk_hi, chi.data(), nch))))
        return r;
    if ((r = upload(s, s->d_body_chunk_off, boff.data(), nb + 1))) return r;
    s->n_chunks = (int)nch;
    if ((r = dalloc(s, s->d_fbody, (size_t)nf)) ||
        (r = dalloc(s, s->d_seg_idx, (size_t)nf)) || (r = dalloc(s, s->d_body_on, nb)) ||
        (r = dalloc(s, s->d_body_sweeps, nb)) || (r = dalloc(s, s->d_rb, nb + 2)) || (r = dalloc(s, s->d_r0sq, nb)))
        return r;
    s->d_dx2 = s->d_rb;
    s->d_nactive = reinterpret_cast<int*>(s->d_rb + 1);
    s->d_r2 = s->d_rb + 2;
    HIPCHK(hipMemsetAsync(s->d_rb, 0, (nb + 2) * sizeof(double), s->stream));
    free_readback(s);
    for (int i = 0; i < 2; ++i) {
        HIPCHK(hipHostMalloc((void**)&s->h_rb[i], (nb + 2) * sizeof(double), hipHostMallocDefault));
        s->h_dx2[i] = s->h_rb[i];
        s->h_nact[i] = reinterpret_cast<int*>(s->h_rb[i] + 1);
        s->h_r2[i] = s->h_rb[i] + 2;
        std::memset(s->h_rb[i], 0, (nb + 2) * sizeof(double));
        if (!s->rb_ev[i]) HIPCHK(hipEventCreateWithFlags(&s->rb_ev[i], hipEventDisableTiming));
    }
    std::vector<int> ones(nb, 1), zeros(nb, 0);
    std::vector<int> fbodyc(nf);
    for (int q = 0; q < nf; ++q) fbodyc[q] = fbody[s->col_perm[q]];
    if ((r = upload(s, s->d_fbody_c, fbodyc.data(), (size_t)nf))) return r;
    if ((r = upload(s, s->d_fbody, fbody.data(), (size_t)nf)) ||
        (r = upload(s, s->d_seg_idx, idx.data(), (size_t)nf)) || (r = upload(s, s->d_body_on, ones.data(), nb)) ||
        (r = upload(s, s->d_body_sweeps, zeros.data(), nb)))
        return r;
    HIPCHK(hipStreamSynchronize(s->stream));
    s->n_bodies = n_bodies;
    s->body_of_vertex.assign(body_of_vertex, body_of_vertex + s->nV);
    s->seg_off = off;
    s->seg_idx = idx;
    s->r2_host.assign(nb, 0.0);
    s->r0sq_host.assign(nb, 0.0);
    s->n_active = n_bodies;
    s->have_bodies = true;
    return JGS2_OK;
}

int32_t jgs2_get_body_stats(jgs2_solver* s, int32_t* n_bodies, int32_t* sweeps, double* rel) {
    if (!s) return JGS2_E_INVALID;
    if (!s->have_mesh) return s->fail(JGS2_E_NOT_READY, "no mesh");
    if (!s->have_bodies) return s->fail(JGS2_E_NOT_READY, "no body tables (set_bodies failed)");
    if (n_bodies) *n_bodies = s->n_bodies;
    if (sweeps) {
        HIPCHK(hipMemcpyAsync(sweeps, s->d_body_sweeps, (size_t)s->n_bodies * sizeof(int), hipMemcpyDeviceToHost,
                              s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    if (rel)
        for (int b = 0; b < s->n_bodies; ++b)
            rel[b] = s->r0sq_host[b] > 0 ? std::sqrt(s->r2_host[b] / s->r0sq_host[b]) : 0.0;
    return JGS2_OK;
}

static bool valid_shape(int lpv, int block) {
    return (lpv == 4 || lpv == 8 || lpv == 16 || lpv == 32) &&
           (block == 64 || block == 128 || block == 256 || block == 512);
}

int32_t jgs2_set_tuning(jgs2_solver* s, int32_t lanes_per_vertex, int32_t block) {
    if (!s) return JGS2_E_INVALID;
    if (!valid_shape(lanes_per_vertex, block)) return s->fail(JGS2_E_INVALID, "unsupported launch shape");
    s->tune_lpv = lanes_per_vertex;
    s->tune_block = block;
    drop_graphs(s);
    return JGS2_OK;
}

int32_t jgs2_set_persistent(jgs2_solver* s, int32_t on) {
    if (!s) return JGS2_E_INVALID;
    if (on != 0 && on != 1) return s->fail(JGS2_E_INVALID, "persistent must be 0 or 1");
    if (on && s->n_cus == 0) {
        int r = hip_check(s, hipDeviceGetAttribute(&s->n_cus, hipDeviceAttributeMultiprocessorCount, s->device),
                          "compute unit count");
        if (r != JGS2_OK) return r;
    }
    s->persistent = on != 0;
    drop_graphs(s);
    return JGS2_OK;
}

int32_t jgs2_set_streaming(jgs2_solver* s, int32_t mode) {
    if (!s) return JGS2_E_INVALID;
    if (mode < -1 || mode > 1) return s->fail(JGS2_E_INVALID, "streaming mode must be -1, 0 or 1");
    s->stream_mode = mode;
    drop_graphs(s);  // captured launches hold the kernel variant
    return JGS2_OK;
}

int32_t jgs2_get_tuning(jgs2_solver* s, int32_t* lanes_per_vertex, int32_t* block) {
    if (!s) return JGS2_E_INVALID;
    if (lanes_per_vertex) *lanes_per_vertex = s->tune_lpv;
    if (block) *block = s->tune_block;
    return JGS2_OK;
}

int32_t jgs2_autotune(jgs2_solver* s, int32_t sweeps, int32_t* lanes_per_vertex, int32_t* block, double* ms) {
    if (!s) return JGS2_E_INVALID;
    if (sweeps < 1) return s->fail(JGS2_E_INVALID, "sweeps must be >= 1");
    if (s->in_step) return s->fail(JGS2_E_NOT_READY, "autotune inside begin_step/end_step");
    int r = jgs2_begin_step(s);
    if (r != JGS2_OK) return r;
    const int lanes[4] = {4, 8, 16, 32}, blocks[4] = {64, 128, 256, 512};
    const int keep_l = s->tune_lpv, keep_b = s->tune_block;
    double best = 1e300;
    int bl = keep_l, bb = keep_b;
    hipEvent_t e0 = pool_event(s), e1 = pool_event(s);
    for (int i = 0; i < 4 && r == JGS2_OK; ++i)
        for (int j = 0; j < 4 && r == JGS2_OK; ++j) {
            s->tune_lpv = lanes[i];
            s->tune_block = blocks[j];
            // every shape starts from the same iterate
            if ((r = copy_v4(s, s->d_u, s->d_uhat)) || (r = copy_v4(s, s->d_unext, s->d_uhat))) break;
            r = sweep_once(s);  // warm-up
            if (r != JGS2_OK) break;
            if ((r = copy_v4(s, s->d_u, s->d_uhat)) || (r = copy_v4(s, s->d_unext, s->d_uhat))) break;
            if ((r = jgs2::hip_check(s, hipEventRecord(e0, s->stream), "event"))) break;
            for (int k = 0; k < sweeps && r == JGS2_OK; ++k) r = sweep_once(s);
            if (r != JGS2_OK) break;
            if ((r = jgs2::hip_check(s, hipEventRecord(e1, s->stream), "event"))) break;
            if ((r = jgs2::hip_check(s, hipEventSynchronize(e1), "event"))) break;
            float t = 0.0f;
            if ((r = jgs2::hip_check(s, hipEventElapsedTime(&t, e0, e1), "event"))) break;
            if (ms) ms[4 * i + j] = t;
            if (t < best) { best = t; bl = lanes[i]; bb = blocks[j]; }
        }
    s->ev_pool.push_back(e0);
    s->ev_pool.push_back(e1);
    abandon_step(s);
    if (r != JGS2_OK) {
        s->tune_lpv = keep_l;
        s->tune_block = keep_b;
        return r;
    }
    s->tune_lpv = bl;
    s->tune_block = bb;
    drop_graphs(s);
    if (lanes_per_vertex) *lanes_per_vertex = bl;
    if (block) *block = bb;
    return JGS2_OK;
}

}  // extern "C"
