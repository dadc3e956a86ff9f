// The C ABI of libldrop (declared in include/ldrop.h): argument checking,
// device buffers, host/device pointer handling and the per-step launch
// sequence.  No C++ exception crosses this boundary.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "ld_host.h"

namespace ld {
namespace host {

thread_local std::string g_err;

ld_status fail(ld_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

bool is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Copy bytes into device memory from a host or device source.
hipError_t copy_in(void* dst, const void* src, size_t bytes, hipStream_t s) {
    return hipMemcpyAsync(dst, src, bytes,
                          is_device_ptr(src) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                          s);
}

// Copy bytes from device memory to a host or device destination; waits.
hipError_t copy_out(void* dst, const void* src, size_t bytes, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(
        dst, src, bytes, is_device_ptr(dst) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

ld_status check_params(const ld_params* p) {
    if (!p) return fail(LD_EINVAL, "params is NULL");
    if (p->n_types < 1 || p->n_types > LD_MAX_TYPES)
        return fail(LD_EINVAL, "n_types=%d outside [1,%d]", p->n_types, LD_MAX_TYPES);
    for (int t = 0; t < p->n_types; ++t) {
        if (!(p->sigma[t] > 0.0) || !std::isfinite(p->sigma[t]))
            return fail(LD_EINVAL, "sigma[%d]=%g must be positive", t, p->sigma[t]);
        if (!(p->eps[t] >= 0.0)) return fail(LD_EINVAL, "eps[%d]=%g must be >= 0", t, p->eps[t]);
        if (!(p->gamma[t] > 0.0))
            return fail(LD_EINVAL, "gamma[%d]=%g must be positive", t, p->gamma[t]);
        if (!(p->k_wall[t] >= 0.0))
            return fail(LD_EINVAL, "k_wall[%d]=%g must be >= 0", t, p->k_wall[t]);
        if (!std::isfinite(p->mass[t]) || !std::isfinite(p->wall_offset[t]))
            return fail(LD_EINVAL, "mass / wall_offset of type %d not finite", t);
        if (p->use_eps_matrix) {
            for (int u = 0; u < p->n_types; ++u) {
                const double a = p->eps_matrix[t * LD_MAX_TYPES + u];
                const double b = p->eps_matrix[u * LD_MAX_TYPES + t];
                if (!(a >= 0.0) || a != b)
                    return fail(LD_EINVAL, "eps_matrix must be symmetric and >= 0 (%d,%d)", t, u);
            }
        }
    }
    if (!(p->lj_cut > 0.0)) return fail(LD_EINVAL, "lj_cut=%g must be positive", p->lj_cut);
    if (p->coul_cut > 0.0)
        return fail(LD_EUNSUPPORTED, "coul_cut > 0 (truncated Coulomb) is not built");
    if (!(p->bjerrum >= 0.0) || !(p->kT >= 0.0))
        return fail(LD_EINVAL, "bjerrum and kT must be >= 0");
    if (p->rotation != 0 && p->rotation != 1) return fail(LD_EINVAL, "rotation must be 0 or 1");
    if (p->wall_band != 0 && p->wall_band != 1) return fail(LD_EINVAL, "wall_band must be 0/1");
    if (p->noise < 0 || p->noise > 2) return fail(LD_EINVAL, "noise must be 0, 1 or 2");
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(p->gravity[c])) return fail(LD_EINVAL, "gravity not finite");
    if (!std::isfinite(p->omega)) return fail(LD_EINVAL, "omega not finite");
    return LD_OK;
}

ld_status check_radius(const ld_radius* R) {
    if (!R) return fail(LD_EINVAL, "radius schedule is NULL");
    if (R->kind < LD_R_CONST || R->kind > LD_R_TABLE)
        return fail(LD_EINVAL, "radius kind %d unknown", R->kind);
    if (R->kind == LD_R_TABLE) {
        if (R->n_knots < 2 || R->n_knots > LD_R_TABLE_MAX)
            return fail(LD_EINVAL, "a radius table needs 2..%d knots", LD_R_TABLE_MAX);
        for (int k = 0; k < R->n_knots; ++k) {
            if (!std::isfinite(R->tab_t[k]) || !std::isfinite(R->tab_R[k]) || R->tab_R[k] < 0.0)
                return fail(LD_EINVAL, "radius table knot %d: finite time and radius >= 0", k);
            if (k > 0 && !(R->tab_t[k] > R->tab_t[k - 1]))
                return fail(LD_EINVAL, "radius table times must increase strictly");
        }
        return LD_OK;
    }
    if (!std::isfinite(R->R0) || R->R0 < 0.0) return fail(LD_EINVAL, "R0 must be >= 0");
    if (R->kind == LD_R_LINEAR && (!std::isfinite(R->R1) || R->R1 < 0.0 || !(R->T >= 0.0)))
        return fail(LD_EINVAL, "linear schedule needs R1 >= 0 and T >= 0");
    if (R->kind == LD_R_SQUARE_LAW && (!std::isfinite(R->a) || !(R->R_min >= 0.0)))
        return fail(LD_EINVAL, "square-law schedule needs finite a and R_min >= 0");
    return LD_OK;
}

void make_tables(const ld_params& p, const ld_radius& R, PairTable& tb, ExtParams& P) {
    std::memset(&tb, 0, sizeof tb);
    tb.T = p.n_types;
    double rc2max = 0.0;
    for (int a = 0; a < p.n_types; ++a)
        for (int b = 0; b < p.n_types; ++b) {
            const double s = 0.5 * (p.sigma[a] + p.sigma[b]);
            const double e = p.use_eps_matrix ? p.eps_matrix[a * LD_MAX_TYPES + b]
                                              : std::sqrt(p.eps[a] * p.eps[b]);
            const double rc = p.lj_cut * s;
            const int k = a * p.n_types + b;
            tb.sig2[k] = (float)(s * s);
            tb.rc2[k] = (float)(rc * rc);
            tb.e24[k] = (float)(24.0 * e);
            tb.e4[k] = (float)(4.0 * e);
            tb.sig2d[k] = s * s;
            tb.e24d[k] = 24.0 * e;
            tb.e4d[k] = 4.0 * e;
            tb.rc2d[k] = rc * rc;
            if (rc * rc > rc2max) rc2max = rc * rc;
        }
    tb.rc2max = (float)rc2max;

    std::memset(&P, 0, sizeof P);
    P.n_types = p.n_types;
    P.rotation = p.rotation;
    P.wall_band = p.wall_band;
    P.noise = p.noise;
    for (int k = 0; k < 3; ++k) P.gravity[k] = p.gravity[k];
    P.omega2 = p.omega * p.omega;
    P.kT = p.kT;
    P.jump_max = p.jump_max;
    for (int t = 0; t < p.n_types; ++t) {
        P.mu[t] = 1.0 / p.gamma[t];
        P.mass[t] = p.mass[t];
        P.k_wall[t] = p.k_wall[t];
        P.wall_offset[t] = p.wall_offset[t];
        P.half_sigma[t] = 0.5 * p.sigma[t];
    }
    P.R = R;
}

}  // namespace host

bool timing_events(ld_ctx* c, unsigned char kind, hipEvent_t* e0, hipEvent_t* e1) {
    for (int k = 0; k < 2; ++k)
        if (c->ev_used + k == c->ev_pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return false;
            c->ev_pool.push_back(e);
        }
    *e0 = c->ev_pool[c->ev_used];
    *e1 = c->ev_pool[c->ev_used + 1];
    c->ev_used += 2;
    c->ev_kind.push_back(kind);
    return true;
}
}  // namespace ld

namespace {

using namespace ld::host;

void build_tables(ld_ctx* c) { make_tables(c->p, c->R, c->tab, c->ext); }

void default_tuning(ld_ctx* c) {
    ld_tuning& t = c->tune;
    std::memset(&t, 0, sizeof t);
    const int64_t n = c->n;
    // Enough workgroups to fill 256 CUs (7 resident per CU) many times over
    // (a short tail), but at least 256 j per split so each workgroup streams
    // whole LDS tiles.
    // (block 64 with culling keeps a whole j tile in registers: one
    // wavefront per SIMD; 128 keeps eight)
    t.block = n >= 16384 ? 256 : 128;
    const int64_t tiles = (n + t.block - 1) / t.block;
    int64_t split = (32768 + tiles - 1) / tiles;
    int64_t cap = n / 256;
    if (cap < 1) cap = 1;
    if (split > cap) split = cap;
    if (split > 32) split = 32;
    if (split < 1) split = 1;
    t.j_split = (int)split;
    t.comp = 1;            // blocked Kahan over the FP32 blocks (costs ~1 %)
    t.sort_every = 50;
    t.cull = 1;
}

// A captured graph bakes in buffer pointers and parameter tables: drop it
// whenever either changes.
void invalidate_graph(ld_ctx* c) {
    if (c->graph) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
    }
}

ld_status ensure_split_capacity(ld_ctx* c, int split) {
    if (split <= c->j_split_cap) return LD_OK;
    invalidate_graph(c);
    if (c->Fpart) (void)hipFree(c->Fpart);
    c->Fpart = nullptr;
    c->j_split_cap = 0;
    if (hipMalloc(&c->Fpart, sizeof(double) * 3 * (size_t)c->n * split) != hipSuccess)
        return fail(LD_ENOMEM, "cannot allocate %d force partials", split);
    c->j_split_cap = split;
    return LD_OK;
}


ld_status run_pair(ld_ctx* c, bool diag, hipStream_t s, bool timed) {
    ld::PairLaunch L{};
    L.pos = c->pos;
    L.lo = c->lo;
    L.typ = c->typ;
    L.box = c->box;
    L.n = (int)c->n;
    L.block = c->tune.block;
    L.j_split = diag ? 1 : c->tune.j_split;
    L.comp = c->tune.comp;
    L.cull = (c->tune.cull && !diag) ? 1 : 0;
    L.Fpart = c->Fpart;
    L.S = diag ? c->S_slot : nullptr;
    L.U = diag ? c->U_slot : nullptr;
    L.nearbits = c->nearbits;
    L.nb_words = c->nb_words;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timed) {
        if (!ld::timing_events(c, ld::kTimedCoulomb, &e0, &e1))
            return fail(LD_EHIP, "cannot create timing events");
        HIP_TRY(hipEventRecord(e0, s));
    }
    // timed: the Coulomb kernel alone (the Lennard-Jones kernel follows it)
    HIP_TRY(ld::launch_pair(L, c->tab, s, timed ? e1 : nullptr));
    return LD_OK;
}

ld_status run_pair(ld_ctx* c, bool diag) { return run_pair(c, diag, c->stream, c->timing); }

ld_status run_sort(ld_ctx* c, hipStream_t s) {
    // the curve covers twice the largest droplet radius: particles thrown far
    // out by a blown-up step do not coarsen the order of the others
    const double rmax = ld::schedule_max_radius(c->R);
    const float clip = std::isfinite(rmax) && rmax > 0.0 ? (float)(2.0 * rmax) : INFINITY;
    HIP_TRY(ld::launch_sort(c->pos, c->lo, c->typ, c->oid, (int)c->n, c->sb, s, clip));
    HIP_TRY(ld::launch_boxes(c->pos, (int)c->n, c->box, s));
    c->steps_since_sort = 0;
    return LD_OK;
}

ld_status run_sort(ld_ctx* c) { return run_sort(c, c->stream); }

ld::StepLaunch step_launch(ld_ctx* c, double dt) {
    ld::StepLaunch L{};
    L.pos = c->pos;
    L.lo = c->lo;
    L.typ = c->typ;
    L.oid = c->oid;
    L.Fpart = c->Fpart;
    L.j_split = c->tune.j_split;
    L.n = (int)c->n;
    L.dt = dt;
    L.seed = c->seed;
    L.st = c->st;
    L.box = c->box;
    return L;
}

// One step (re-sorting first when due) on stream s.
ld_status enqueue_step(ld_ctx* c, double dt, hipStream_t s, bool timed) {
    if (c->pm) return ld::pm_step(c, dt, s);   // the paper's scheme sorts by cell itself
    if (c->tune.sort_every > 0 && c->steps_since_sort >= c->tune.sort_every) {
        ld_status st = run_sort(c, s);
        if (st != LD_OK) return st;
    }
    if (ld::ff_active(c)) {
        int js = 1;
        ld_status st = ld::ff_step_forces(c, s, &js);
        if (st != LD_OK) return st;
        ld::StepLaunch L = step_launch(c, dt);
        L.j_split = js;
        HIP_TRY(ld::launch_update(L, c->ext, s));
        ++c->steps_since_sort;
        return LD_OK;
    }
    ld_status st = run_pair(c, false, s, timed);
    if (st != LD_OK) return st;
    HIP_TRY(ld::launch_update(step_launch(c, dt), c->ext, s));
    ++c->steps_since_sort;
    return LD_OK;
}

// Capture `len` steps (a re-sort first when sorting is on) into a graph.
ld_status capture_chunk(ld_ctx* c, double dt, int len) {
    if (c->graph) {
        (void)hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
    }
    if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    const int64_t saved = c->steps_since_sort;
    HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    ld_status st = LD_OK;
    if (c->tune.sort_every > 0) c->steps_since_sort = c->tune.sort_every;
    for (int k = 0; k < len && st == LD_OK; ++k) st = enqueue_step(c, dt, c->cap_stream, false);
    hipGraph_t g = nullptr;
    hipError_t err = hipStreamEndCapture(c->cap_stream, &g);
    c->steps_since_sort = saved;
    if (st != LD_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (err != hipSuccess) return fail(LD_EHIP, "stream capture: %s", hipGetErrorString(err));
    err = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (err != hipSuccess) return fail(LD_EHIP, "graph instantiate: %s", hipGetErrorString(err));
    c->graph_dt = dt;
    c->graph_len = len;
    c->graph_key = c->tune;
    return LD_OK;
}

bool same_tuning(const ld_tuning& a, const ld_tuning& b) {
    return a.block == b.block && a.j_split == b.j_split && a.comp == b.comp &&
           a.sort_every == b.sort_every && a.cull == b.cull && a.graph_steps == b.graph_steps;
}

ld_status step_loop(ld_ctx* c, double dt, int64_t n_steps);
ld_status fill_diag(ld_ctx* c, ld_diag* d);

ld_status wait_stream(ld_ctx* c) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LD_OK;
}

// Report (once) and clear the device-side blow-up flag.
ld_status take_pending_error(ld_ctx* c) {
    ld::DevState st;
    HIP_TRY(hipMemcpyAsync(&st, c->st, sizeof st, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (st.bad_step != ~0ull) {
        const unsigned long long none = ~0ull;
        HIP_TRY(hipMemcpy(&c->st->bad_step, &none, sizeof none, hipMemcpyHostToDevice));
        return fail(LD_ENONFINITE, "step %llu produced a non-finite or too large move",
                    (unsigned long long)st.bad_step);
    }
    return LD_OK;
}

void free_all(ld_ctx* c) {
    ld::rec_free(c);
    ld::pm_free(c);
    ld::ag_free(c);
    void* bufs[] = {c->pos,     c->lo,     c->typ,         c->oid,       c->box,  c->aux,
                    c->Fpart,   c->S_slot, c->U_slot,      c->work,      c->st,  c->ref,
                    c->sb.keys, c->sb.tmp4, c->sb.tmp_i,   c->sb.bounds, c->sb.bounds_part,
                    c->sb.hist, c->pos2,  c->lo2,   c->typ2,       c->oid2, c->nearbits};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    ld::ff_free(c);
}

}  // namespace

// ---- initial placement (ld_init with pos = NULL) -------------------------

namespace {

constexpr int64_t kSampleTries = 100000;

// Philox4x32-10 on the host (Salmon, Moraes, Dror, Shaw, SC'11).
void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Uniform in the ball of radius R0, no pair closer than sigma_ij (section
// 2.1: NPs placed at random in the droplet without overlap).  Particle i in
// index order draws candidate k = 0, 1, ... from the Philox counter
// (i, k, 0, 1) with the noise key: v_c = 2 ((u_c >> 9) + 1/2) 2^-23 - 1 from
// the first three words, dropped if |v|^2 > 1, else x = FP32(R0 v), kept if
// |x - x_j|^2 >= sigma_ij^2 (FP64 on the FP32 values) for every kept j < i.
// Earlier particles are found through a hash of cells of side max sigma.
// Returns -1, or the first particle that found no place.
int64_t sample_ball(int64_t n, const int32_t* type, const double* sigma, double R0,
                    uint64_t seed, int64_t max_tries, float* x) {
#pragma clang fp contract(off)
    double smax = 0.0;
    for (int64_t i = 0; i < n; ++i) smax = std::max(smax, sigma[type[i]]);
    const double h = smax;                       // cell side >= any sigma_ij
    size_t cap = 1;
    while (cap < 2 * (size_t)n) cap <<= 1;
    std::vector<int64_t> head(cap, -1), next((size_t)n, -1);
    auto cell = [&](double v) { return (int64_t)std::floor(v / h); };
    auto slot = [&](int64_t a, int64_t b, int64_t c) {
        uint64_t k = (uint64_t)a * 0x9E3779B97F4A7C15ull ^ (uint64_t)b * 0xC2B2AE3D27D4EB4Full ^
                     (uint64_t)c * 0x165667B19E3779F9ull;
        return (size_t)((k ^ (k >> 29)) & (cap - 1));
    };
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int64_t i = 0; i < n; ++i) {
        bool placed = false;
        for (int64_t k = 0; k < max_tries && !placed; ++k) {
            uint32_t c[4] = {(uint32_t)i, (uint32_t)k, 0u, 1u};
            philox_host(c, k0, k1);
            double v[3];
            for (int d = 0; d < 3; ++d)
                v[d] = 2.0 * (((double)(c[d] >> 9) + 0.5) * (1.0 / 8388608.0)) - 1.0;
            if (v[0] * v[0] + v[1] * v[1] + v[2] * v[2] > 1.0) continue;
            double y[3];
            for (int d = 0; d < 3; ++d) y[d] = (double)(float)(R0 * v[d]);
            const int64_t cx = cell(y[0]), cy = cell(y[1]), cz = cell(y[2]);
            bool clash = false;
            for (int64_t a = cx - 1; a <= cx + 1 && !clash; ++a)
                for (int64_t b = cy - 1; b <= cy + 1 && !clash; ++b)
                    for (int64_t e = cz - 1; e <= cz + 1 && !clash; ++e)
                        for (int64_t j = head[slot(a, b, e)]; j >= 0 && !clash; j = next[j]) {
                            const double sij = 0.5 * (sigma[type[i]] + sigma[type[j]]);
                            const double dx = y[0] - (double)x[3 * j];
                            const double dy = y[1] - (double)x[3 * j + 1];
                            const double dz = y[2] - (double)x[3 * j + 2];
                            if (dx * dx + dy * dy + dz * dz < sij * sij) clash = true;
                        }
            if (clash) continue;
            for (int d = 0; d < 3; ++d) x[3 * i + d] = (float)y[d];
            const size_t sl = slot(cx, cy, cz);
            next[i] = head[sl];
            head[sl] = i;
            placed = true;
        }
        if (!placed) return i;
    }
    return -1;
}

}  // namespace

extern "C" {

const char* ld_last_error(void) { return g_err.c_str(); }

ld_status ld_init(ld_ctx** out, int64_t n, const int32_t* type, const double* charge,
                  const float* pos, const ld_params* p, const ld_radius* R, uint64_t seed,
                  void* stream) {
    g_err.clear();
    if (!out) return fail(LD_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 2 || n > (1 << 27)) return fail(LD_EINVAL, "n=%lld outside [2, 2^27]", (long long)n);
    if (!type || !charge) return fail(LD_EINVAL, "type and charge are required");
    ld_status st = check_params(p);
    if (st != LD_OK) return st;
    st = check_radius(R);
    if (st != LD_OK) return st;
    hipStream_t s = (hipStream_t)stream;

    std::vector<int32_t> ty;
    std::vector<double> q;
    std::vector<float> x;
    if ((st = read_host(ty, type, (size_t)n, s)) != LD_OK) return st;
    if ((st = read_host(q, charge, (size_t)n, s)) != LD_OK) return st;
    for (int64_t i = 0; i < n; ++i) {
        if (ty[i] < 0 || ty[i] >= p->n_types)
            return fail(LD_EINVAL, "type[%lld]=%d outside [0,%d)", (long long)i, ty[i], p->n_types);
        if (!std::isfinite(q[i])) return fail(LD_EINVAL, "charge[%lld] not finite", (long long)i);
    }
    if (pos) {
        if ((st = read_host(x, pos, (size_t)n * 3, s)) != LD_OK) return st;
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < 3; ++k)
                if (!std::isfinite(x[3 * i + k]))
                    return fail(LD_EINVAL, "pos[%lld] not finite", (long long)i);
    } else {
        const double R0 = ld::radius_at(*R, 0.0);
        if (!(R0 > 0.0)) return fail(LD_EINVAL, "sampling needs R(0) > 0");
        x.resize((size_t)n * 3);
        const int64_t bad = sample_ball(n, ty.data(), p->sigma, R0, seed, kSampleTries, x.data());
        if (bad >= 0)
            return fail(LD_EINVAL, "no place for particle %lld in the ball of radius %g after %lld "
                        "candidates (too dense)", (long long)bad, R0, (long long)kSampleTries);
    }

    ld_ctx* c = new (std::nothrow) ld_ctx();
    if (!c) return fail(LD_ENOMEM, "host allocation failed");
    c->n = n;
    c->stream = s;
    c->p = *p;
    c->R = *R;
    c->seed = seed;
    (void)hipGetDevice(&c->device);
    build_tables(c);
    default_tuning(c);

    const size_t N = (size_t)n;
    const int ngroups = (int)((n + ld::kGroup - 1) / ld::kGroup);
    int n_pow2 = 2048;
    while (n_pow2 < n) n_pow2 <<= 1;
    c->sb.n_pow2 = n_pow2;
    c->sb.bounds_parts = 64;
    bool ok = hipMalloc(&c->pos, sizeof(float4) * N) == hipSuccess &&
              hipMalloc(&c->lo, sizeof(float4) * N) == hipSuccess &&
              hipMalloc(&c->typ, sizeof(int) * N) == hipSuccess &&
              hipMalloc(&c->oid, sizeof(int) * N) == hipSuccess &&
              hipMalloc(&c->box, sizeof(ld::Box) * ngroups) == hipSuccess &&
              hipMalloc(&c->S_slot, sizeof(double) * N) == hipSuccess &&
              hipMalloc(&c->U_slot, sizeof(double) * 2 * N) == hipSuccess &&
              hipMalloc(&c->work, sizeof(double) * (16 * N + 64)) == hipSuccess &&
              hipMalloc(&c->aux, sizeof(double) * ld::kAuxWords) == hipSuccess &&
              hipMalloc(&c->ref, sizeof(double) * 3 * N) == hipSuccess &&
              hipMalloc(&c->st, sizeof(ld::DevState)) == hipSuccess &&
              hipMalloc(&c->sb.keys, sizeof(unsigned long long) * n_pow2) == hipSuccess &&
              hipMalloc(&c->sb.tmp4, sizeof(float4) * N) == hipSuccess &&
              hipMalloc(&c->sb.tmp_i, sizeof(int) * N) == hipSuccess &&
              hipMalloc(&c->sb.bounds, sizeof(float) * 8) == hipSuccess &&
              hipMalloc(&c->sb.bounds_part, sizeof(float) * 6 * 64) == hipSuccess &&
              hipMalloc(&c->sb.hist, sizeof(unsigned) * 256 * (ld::radix_tiles((int)n) + 1)) ==
                  hipSuccess;
    if (ok && n <= ld::kNearBitsMaxN) {
        c->nb_words = (ngroups + 31) / 32;
        const size_t bytes = sizeof(unsigned) * (size_t)ngroups * c->nb_words;
        ok = hipMalloc(&c->nearbits, bytes) == hipSuccess &&
             hipMemsetAsync(c->nearbits, 0, bytes, s) == hipSuccess;
    }
    if (!ok || ensure_split_capacity(c, c->tune.j_split) != LD_OK) {
        free_all(c);
        delete c;
        return fail(LD_ENOMEM, "device allocation failed for n=%lld", (long long)n);
    }

    const double qs = std::sqrt(p->kT * p->bjerrum);
    std::vector<float4> h4(N), l4(N);
    std::vector<int> ids(N);
    for (size_t i = 0; i < N; ++i) {
        h4[i] = make_float4(x[3 * i], x[3 * i + 1], x[3 * i + 2], (float)(q[i] * qs));
        l4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
        ids[i] = (int)i;
    }
    ld::DevState ds{};
    ds.step = 0;
    ds.t = 0.0;
    ds.bad_step = ~0ull;
    ds.pad0 = 0;
    hipError_t e = hipMemcpyAsync(c->pos, h4.data(), sizeof(float4) * N, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->lo, l4.data(), sizeof(float4) * N, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->typ, ty.data(), sizeof(int) * N, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->oid, ids.data(), sizeof(int) * N, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->st, &ds, sizeof ds, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = ld::launch_msd_ref(c->pos, c->lo, c->oid, (int)N, c->ref, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        free_all(c);
        delete c;
        return fail(LD_EHIP, "upload failed: %s", hipGetErrorString(e));
    }
    st = (c->tune.sort_every >= 0) ? run_sort(c) : LD_OK;
    if (st == LD_OK && c->tune.sort_every < 0) {
        e = ld::launch_boxes(c->pos, (int)n, c->box, s);
        if (e != hipSuccess) st = fail(LD_EHIP, "box kernel: %s", hipGetErrorString(e));
    }
    if (st == LD_OK) {
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = fail(LD_EHIP, "init: %s", hipGetErrorString(e));
    }
    if (st != LD_OK) {
        free_all(c);
        delete c;
        return st;
    }
    *out = c;
    return LD_OK;
}

void ld_destroy(ld_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

ld_status ld_forces(ld_ctx* c, double* F_pair, double* F_ext, double* S, double* U) {
    g_err.clear();
    if (!c) return fail(LD_EINVAL, "ctx is NULL");
    const bool diag = S || U;
    ld_status st = run_pair(c, diag);
    if (st != LD_OK) return st;
    const size_t N = (size_t)c->n;
    double* dF = c->work;                    // [3N]
    double* dE = c->work + 3 * N;            // [3N]
    double* dS = c->work + 6 * N;            // [N]
    double* dU = c->work + 7 * N;            // [2]
    HIP_TRY(ld::launch_gather(c->pos, c->lo, c->typ, c->oid, c->Fpart,
                              diag ? 1 : c->tune.j_split, c->S_slot, (int)N, c->st, c->ext,
                              F_pair ? dF : nullptr, F_ext ? dE : nullptr, S ? dS : nullptr,
                              c->stream));
    if (U) HIP_TRY(ld::launch_rowsum(c->U_slot, 2, (int)N, dU, c->stream));
    if (F_pair) HIP_TRY(copy_out(F_pair, dF, sizeof(double) * 3 * N, c->stream));
    if (F_ext) HIP_TRY(copy_out(F_ext, dE, sizeof(double) * 3 * N, c->stream));
    if (S) HIP_TRY(copy_out(S, dS, sizeof(double) * N, c->stream));
    if (U) HIP_TRY(copy_out(U, dU, sizeof(double) * 2, c->stream));
    return wait_stream(c);
}

ld_status ld_step(ld_ctx* c, double dt, int64_t n_steps, const ld_radius* R,
                  const uint64_t* seed, ld_diag* diag) {
    g_err.clear();
    if (!c) return fail(LD_EINVAL, "ctx is NULL");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(LD_EINVAL, "dt=%g must be positive", dt);
    if (n_steps < 0) return fail(LD_EINVAL, "n_steps must be >= 0");
    if (R) {
        ld_status st = check_radius(R);
        if (st != LD_OK) return st;
        // kernels already enqueued hold the old schedule in their arguments
        c->R = *R;
        invalidate_graph(c);
        build_tables(c);
    }
    if (seed && *seed != c->seed) {
        c->seed = *seed;
        invalidate_graph(c);
    }
    ld_status st = step_loop(c, dt, n_steps);
    if (st != LD_OK || !diag) return st;
    return fill_diag(c, diag);
}

ld_status ld_msd(ld_ctx* c, double* msd) {
    g_err.clear();
    if (!c || !msd) return fail(LD_EINVAL, "ctx and msd are required");
    double* res = c->aux;
    HIP_TRY(ld::launch_msd(c->pos, c->lo, c->oid, (int)c->n, c->ref, c->work, res, c->stream));
    HIP_TRY(copy_out(msd, res, sizeof(double), c->stream));
    return wait_stream(c);
}

ld_status ld_msd_reset(ld_ctx* c) {
    g_err.clear();
    if (!c) return fail(LD_EINVAL, "ctx is NULL");
    HIP_TRY(ld::launch_msd_ref(c->pos, c->lo, c->oid, (int)c->n, c->ref, c->stream));
    return wait_stream(c);
}

}  // extern "C"

namespace {

ld_status step_loop(ld_ctx* c, double dt, int64_t n_steps) {
    int64_t left = n_steps;
    const bool use_graph = c->tune.graph_steps > 0 && !c->timing && !ld::ff_active(c) && !c->pm &&
                           !c->rec;
    const int len = c->tune.sort_every > 0 ? c->tune.sort_every : c->tune.graph_steps;
    while (left > 0) {
        // A captured chunk starts with a re-sort when sorting is on, so it is
        // used once the current sort interval is used up.
        const bool at_chunk = c->tune.sort_every <= 0 || c->steps_since_sort >= c->tune.sort_every;
        if (use_graph && at_chunk && left >= len) {
            if (!c->graph || c->graph_dt != dt || c->graph_len != len ||
                !same_tuning(c->graph_key, c->tune)) {
                ld_status st = capture_chunk(c, dt, len);
                if (st != LD_OK) return st;
            }
            HIP_TRY(hipGraphLaunch(c->graph, c->stream));
            c->steps_since_sort = c->tune.sort_every > 0 ? len : 0;
            left -= len;
            continue;
        }
        ld_status st = enqueue_step(c, dt, c->stream, c->timing);
        if (st != LD_OK) return st;
        if (c->rec && (st = ld::rec_after_step(c, dt, c->stream)) != LD_OK) return st;
        --left;
    }
    return LD_OK;
}

// Wait for the steps, then the state and FP64 diagnostics at R(t) into *d;
// a pending blow-up is reported (once) as LD_ENONFINITE with d->bad_step.
ld_status fill_diag(ld_ctx* c, ld_diag* d) {
    double out[10];
    ld_status st = ld_diagnostics(c, out);
    if (st != LD_OK) return st;
    double* res = c->aux + 16;
    HIP_TRY(ld::launch_msd(c->pos, c->lo, c->oid, (int)c->n, c->ref, c->work, res, c->stream));
    double msd = 0.0;
    ld::DevState ds;
    HIP_TRY(hipMemcpyAsync(&msd, res, sizeof msd, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(&ds, c->st, sizeof ds, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    d->step = ds.step;
    d->t = ds.t;
    d->R = ld::radius_at(c->R, ds.t);
    for (int k = 0; k < 5; ++k) d->U[k] = out[k];
    for (int k = 0; k < 3; ++k) d->net_force[k] = out[5 + k];
    d->max_force = out[8];
    d->max_radius = out[9];
    d->msd = msd;
    d->bad_step = ds.bad_step == ~0ull ? -1 : (int64_t)ds.bad_step;
    return d->bad_step >= 0 ? take_pending_error(c) : LD_OK;
}

}  // namespace

extern "C" {

ld_status ld_sync(ld_ctx* c) {
    g_err.clear();
    if (!c) return fail(LD_EINVAL, "ctx is NULL");
    return take_pending_error(c);
}

ld_status ld_set_positions(ld_ctx* c, const float* pos, const float* pos_lo) {
    g_err.clear();
    if (!c || !pos) return fail(LD_EINVAL, "ctx and pos are required");
    const size_t N = (size_t)c->n;
    std::vector<float> x, xl;
    ld_status st = read_host(x, pos, 3 * N, c->stream);
    if (st != LD_OK) return st;
    if (pos_lo && (st = read_host(xl, pos_lo, 3 * N, c->stream)) != LD_OK) return st;
    for (size_t k = 0; k < 3 * N; ++k)
        if (!std::isfinite(x[k]) || (pos_lo && !std::isfinite(xl[k])))
            return fail(LD_EINVAL, "coordinate %zu of particle %zu is not finite", k % 3, k / 3);
    std::vector<float4> h(N), l(N);
    std::vector<int> ids(N);
    HIP_TRY(hipMemcpyAsync(h.data(), c->pos, sizeof(float4) * N, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(ids.data(), c->oid, sizeof(int) * N, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (size_t s = 0; s < N; ++s) {
        const size_t o = (size_t)ids[s];
        h[s] = make_float4(x[3 * o], x[3 * o + 1], x[3 * o + 2], h[s].w);   // q_hat stays
        l[s] = pos_lo ? make_float4(xl[3 * o], xl[3 * o + 1], xl[3 * o + 2], 0.f)
                      : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    HIP_TRY(hipMemcpyAsync(c->pos, h.data(), sizeof(float4) * N, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->lo, l.data(), sizeof(float4) * N, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(ld::launch_boxes(c->pos, (int)N, c->box, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->tune.sort_every > 0) c->steps_since_sort = c->tune.sort_every;
    return LD_OK;
}

ld_status ld_get_positions(ld_ctx* c, float* pos, float* pos_lo) {
    g_err.clear();
    if (!c) return fail(LD_EINVAL, "ctx is NULL");
    const size_t N = (size_t)c->n;
    std::vector<float4> h(N), l(N);
    std::vector<int> ids(N);
    HIP_TRY(hipMemcpyAsync(h.data(), c->pos, sizeof(float4) * N, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(l.data(), c->lo, sizeof(float4) * N, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(ids.data(), c->oid, sizeof(int) * N, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::vector<float> a(pos ? 3 * N : 0), b(pos_lo ? 3 * N : 0);
    for (size_t s = 0; s < N; ++s) {
        const size_t o = (size_t)ids[s];
        if (pos) { a[3 * o] = h[s].x; a[3 * o + 1] = h[s].y; a[3 * o + 2] = h[s].z; }
        if (pos_lo) { b[3 * o] = l[s].x; b[3 * o + 1] = l[s].y; b[3 * o + 2] = l[s].z; }
    }
    if (pos) {
        if (is_device_ptr(pos)) {
            HIP_TRY(hipMemcpyAsync(pos, a.data(), sizeof(float) * 3 * N, hipMemcpyHostToDevice,
                                   c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
        } else {
            std::memcpy(pos, a.data(), sizeof(float) * 3 * N);
        }
    }
    if (pos_lo) {
        if (is_device_ptr(pos_lo)) {
            HIP_TRY(hipMemcpyAsync(pos_lo, b.data(), sizeof(float) * 3 * N,
                                   hipMemcpyHostToDevice, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
        } else {
            std::memcpy(pos_lo, b.data(), sizeof(float) * 3 * N);
        }
    }
    return wait_stream(c);
}

ld_status ld_get_state(ld_ctx* c, int64_t* step, double* t, double* R) {
    g_err.clear();
    if (!c) return fail(LD_EINVAL, "ctx is NULL");
    ld::DevState st;
    HIP_TRY(hipMemcpyAsync(&st, c->st, sizeof st, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (step) *step = st.step;
    if (t) *t = st.t;
    if (R) *R = ld::radius_at(c->R, st.t);
    return LD_OK;
}

ld_status ld_set_params(ld_ctx* c, const ld_params* p, const ld_radius* R) {
    g_err.clear();
    if (!c) return fail(LD_EINVAL, "ctx is NULL");
    if (p) {
        ld_status st = check_params(p);
        if (st != LD_OK) return st;
        if (p->n_types < c->p.n_types)
            return fail(LD_EINVAL, "n_types cannot shrink below the types in use");
    }
    if (R) {
        ld_status st = check_radius(R);
        if (st != LD_OK) return st;
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (p) {
        const double old_s = std::sqrt(c->p.kT * c->p.bjerrum);
        const double new_s = std::sqrt(p->kT * p->bjerrum);
        if (old_s != new_s) {
            // rescale the stored charges q * sqrt(kT l_B)
            const size_t N = (size_t)c->n;
            std::vector<float4> h(N);
            std::vector<int> ids(N);
            HIP_TRY(hipMemcpy(h.data(), c->pos, sizeof(float4) * N, hipMemcpyDeviceToHost));
            HIP_TRY(hipMemcpy(ids.data(), c->oid, sizeof(int) * N, hipMemcpyDeviceToHost));
            if (old_s == 0.0)
                return fail(LD_ESTATE, "charges were stored with kT * l_B = 0 and are lost");
            std::vector<float> qh(N);
            for (size_t s = 0; s < N; ++s) qh[ids[s]] = (float)((double)h[s].w / old_s * new_s);
            float* dq = reinterpret_cast<float*>(c->work);
            HIP_TRY(hipMemcpy(dq, qh.data(), sizeof(float) * N, hipMemcpyHostToDevice));
            HIP_TRY(ld::launch_set_charge(c->pos, c->oid, dq, (int)N, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
        }
        c->p = *p;
    }
    if (R) c->R = *R;
    invalidate_graph(c);
    build_tables(c);
    return LD_OK;
}

ld_status ld_diagnostics(ld_ctx* c, double out[10]) {
    g_err.clear();
    if (!c || !out) return fail(LD_EINVAL, "ctx and out are required");
    ld_status st = run_pair(c, true);
    if (st != LD_OK) return st;
    const size_t N = (size_t)c->n;
    double* res = c->aux;
    HIP_TRY(ld::launch_diag(c->pos, c->lo, c->typ, c->Fpart, 1, c->U_slot, (int)N, c->st, c->ext,
                            c->work, res, c->stream));
    HIP_TRY(copy_out(out, res, sizeof(double) * 10, c->stream));
    return wait_stream(c);
}

ld_status ld_rdf(ld_ctx* c, double r_max, int32_t n_bins, double V, int32_t centre,
                 uint64_t* counts, double* g, uint64_t* ccounts, double* cbar) {
    g_err.clear();
    if (!c) return fail(LD_EINVAL, "ctx is NULL");
    if (!(r_max > 0.0) || !std::isfinite(r_max)) return fail(LD_EINVAL, "r_max must be > 0");
    if (n_bins < 1 || n_bins > 4096) return fail(LD_EINVAL, "n_bins must be in [1, 4096]");
    if (centre != 0 && centre != 1) return fail(LD_EINVAL, "centre must be 0 or 1");
    const size_t N = (size_t)c->n;
    unsigned long long* dcnt = reinterpret_cast<unsigned long long*>(c->aux);
    unsigned long long* dcc = dcnt + 4096;
    double* dctr = reinterpret_cast<double*>(dcc + 4096);
    double* mom = dctr + 4;
    if (centre == 1) {
        HIP_TRY(ld::launch_moments(c->pos, c->lo, (int)N, c->work, mom, c->stream));
        HIP_TRY(hipMemcpyAsync(dctr, mom, sizeof(double) * 3, hipMemcpyDeviceToDevice, c->stream));
    } else {
        const double z[4] = {0.0, 0.0, 0.0, 0.0};
        HIP_TRY(hipStreamSynchronize(c->stream));
        HIP_TRY(hipMemcpy(dctr, z, sizeof z, hipMemcpyHostToDevice));
    }
    // pair counts through the cell sort when r_max is short against the
    // droplet, else by the all-pairs histogram (same bins either way)
    bool cells = false;
    ld_status cst = ld::ag_rdf_pairs(c, r_max, n_bins, dcnt, &cells);
    if (cst != LD_OK) return cst;
    if (cells)
        HIP_TRY(ld::launch_centre_hist(c->pos, c->lo, nullptr, 0, (int)N, r_max, n_bins, dctr, dcc,
                                       c->stream));
    else
        HIP_TRY(ld::launch_rdf(c->pos, c->lo, (int)N, r_max, n_bins, dctr, dcnt, dcc, c->stream));
    std::vector<unsigned long long> hc(n_bins), hcc(n_bins);
    HIP_TRY(hipMemcpyAsync(hc.data(), dcnt, sizeof(unsigned long long) * n_bins,
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(hcc.data(), dcc, sizeof(unsigned long long) * n_bins,
                           hipMemcpyDeviceToHost, c->stream));
    ld::DevState ds;
    HIP_TRY(hipMemcpyAsync(&ds, c->st, sizeof ds, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (!(V > 0.0)) {
        const double Rn = ld::radius_at(c->R, ds.t);
        V = 4.0 / 3.0 * M_PI * Rn * Rn * Rn;
    }
    const double dr = r_max / n_bins;
    std::vector<double> hg(n_bins), hb(n_bins);
    const double n = (double)N;
    for (int b = 0; b < n_bins; ++b) {
        const double r0 = b * dr, r1 = (b + 1) * dr;
        const double dV = 4.0 / 3.0 * M_PI * (r1 * r1 * r1 - r0 * r0 * r0);
        // Eq. (6): sum_i psi_i / N over (N - 1) dV / V, sum_i psi_i = 2 C_b
        hg[b] = (2.0 * (double)hc[b] / n) / ((n - 1.0) * dV / V);
        // Eq. (8): (psi / N) / (dV / V)
        hb[b] = ((double)hcc[b] / n) / (dV / V);
    }
    auto put = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        if (!dst) return hipSuccess;
        if (is_device_ptr(dst)) {
            hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream);
            return e == hipSuccess ? hipStreamSynchronize(c->stream) : e;
        }
        std::memcpy(dst, src, bytes);
        return hipSuccess;
    };
    HIP_TRY(put(counts, hc.data(), sizeof(uint64_t) * n_bins));
    HIP_TRY(put(ccounts, hcc.data(), sizeof(uint64_t) * n_bins));
    HIP_TRY(put(g, hg.data(), sizeof(double) * n_bins));
    HIP_TRY(put(cbar, hb.data(), sizeof(double) * n_bins));
    return wait_stream(c);
}

ld_status ld_cbar_type(ld_ctx* c, int32_t type, double r_max, int32_t n_bins, double V,
                       int32_t centre, uint64_t* ccounts, double* cbar) {
    g_err.clear();
    if (!c) return fail(LD_EINVAL, "ctx is NULL");
    if (type < 0 || type >= c->p.n_types) return fail(LD_EINVAL, "type %d out of range", type);
    if (!(r_max > 0.0) || !std::isfinite(r_max)) return fail(LD_EINVAL, "r_max must be > 0");
    if (n_bins < 1 || n_bins > 4096) return fail(LD_EINVAL, "n_bins must be in [1, 4096]");
    if (centre != 0 && centre != 1) return fail(LD_EINVAL, "centre must be 0 or 1");
    const size_t N = (size_t)c->n;
    unsigned long long* dcc = reinterpret_cast<unsigned long long*>(c->aux) + 4096;
    double* dctr = reinterpret_cast<double*>(dcc + 4096);
    double* mom = dctr + 4;
    if (centre == 1) {
        HIP_TRY(ld::launch_moments(c->pos, c->lo, (int)N, c->work, mom, c->stream));
        HIP_TRY(hipMemcpyAsync(dctr, mom, sizeof(double) * 3, hipMemcpyDeviceToDevice, c->stream));
    } else {
        const double z[4] = {0.0, 0.0, 0.0, 0.0};
        HIP_TRY(hipStreamSynchronize(c->stream));
        HIP_TRY(hipMemcpy(dctr, z, sizeof z, hipMemcpyHostToDevice));
    }
    HIP_TRY(ld::launch_centre_hist(c->pos, c->lo, c->typ, type, (int)N, r_max, n_bins, dctr, dcc,
                                   c->stream));
    std::vector<unsigned long long> hcc(n_bins);
    std::vector<int32_t> ht(N);
    HIP_TRY(hipMemcpyAsync(hcc.data(), dcc, sizeof(unsigned long long) * n_bins,
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(ht.data(), c->typ, sizeof(int32_t) * N, hipMemcpyDeviceToHost,
                           c->stream));
    ld::DevState ds;
    HIP_TRY(hipMemcpyAsync(&ds, c->st, sizeof ds, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (!(V > 0.0)) {
        const double Rn = ld::radius_at(c->R, ds.t);
        V = 4.0 / 3.0 * M_PI * Rn * Rn * Rn;
    }
    double nt = 0.0;
    for (int32_t t : ht) nt += t == type ? 1.0 : 0.0;
    const double dr = r_max / n_bins;
    std::vector<double> hb(n_bins);
    for (int b = 0; b < n_bins; ++b) {
        const double r0 = b * dr, r1 = (b + 1) * dr;
        const double dV = 4.0 / 3.0 * M_PI * (r1 * r1 * r1 - r0 * r0 * r0);
        // Eq. (8) over the NPs of this type: (psi / N_t) / (dV / V)
        hb[b] = nt > 0.0 ? ((double)hcc[b] / nt) / (dV / V) : 0.0;
    }
    if (ccounts) HIP_TRY(put_out(ccounts, hcc.data(), sizeof(uint64_t) * n_bins, c->stream));
    if (cbar) HIP_TRY(put_out(cbar, hb.data(), sizeof(double) * n_bins, c->stream));
    return wait_stream(c);
}

ld_status ld_fractal(ld_ctx* c, double k_f, double d, double eps0, int32_t max_scales,
                     double out[4], int64_t* box_counts) {
    g_err.clear();
    if (!c || !out) return fail(LD_EINVAL, "ctx and out are required");
    if (!(k_f > 0.0)) return fail(LD_EINVAL, "k_f must be positive");
    if (max_scales < 0 || max_scales > 40) return fail(LD_EINVAL, "max_scales in [0, 40]");
    const size_t N = (size_t)c->n;
    // number-mean diameter and smallest diameter from the type histogram
    if (!(d > 0.0) || !(eps0 > 0.0)) {
        std::vector<int> ty(N);
        HIP_TRY(hipMemcpyAsync(ty.data(), c->typ, sizeof(int) * N, hipMemcpyDeviceToHost,
                               c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        double sum = 0.0, smin = INFINITY;
        for (size_t s = 0; s < N; ++s) {
            sum += c->p.sigma[ty[s]];
            smin = std::fmin(smin, c->p.sigma[ty[s]]);
        }
        if (!(d > 0.0)) d = sum / (double)N;
        if (!(eps0 > 0.0)) eps0 = smin;
    }
    double* mom = c->aux;
    double* lo3 = mom + 8;
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(lo3 + 4);
    HIP_TRY(ld::launch_moments(c->pos, c->lo, (int)N, c->work, mom, c->stream));
    double hm[4];
    HIP_TRY(copy_out(hm, mom, sizeof hm, c->stream));
    const double Rg = hm[3];
    out[0] = Rg;
    out[1] = std::log((double)N / k_f) / std::log(2.0 * Rg / d);
    HIP_TRY(ld::launch_pos_rows(c->pos, c->lo, (int)N, c->work, c->stream));
    HIP_TRY(ld::launch_rowmin(c->work, 3, (int)N, lo3, c->stream));
    // the extents decide, per scale, whether the box indices fit 32 bits
    double* hi3 = reinterpret_cast<double*>(cnt + 1);
    HIP_TRY(ld::launch_rowmax(c->work, 3, (int)N, hi3, c->stream));
    double hlo[3], hhi[3];
    HIP_TRY(copy_out(hlo, lo3, sizeof hlo, c->stream));
    HIP_TRY(copy_out(hhi, hi3, sizeof hhi, c->stream));
    std::vector<double> lx, ly;
    int K = 0;
    for (int k = 0; k < max_scales; ++k) {
        const double e = eps0 * std::ldexp(1.0, k);
        if (e > Rg) break;
        // boxes per axis: the largest index floor((hi - lo) / e) plus one, and one more
        double nb[3], prod = 1.0;
        for (int a = 0; a < 3; ++a) {
            nb[a] = std::floor((hhi[a] - hlo[a]) / e) + 2.0;
            prod *= nb[a];
        }
        if (prod <= 4294967296.0) {
            int bits = 1;
            while (bits < 32 && std::ldexp(1.0, bits) < prod) ++bits;
            HIP_TRY(ld::launch_boxcount_radix(c->pos, c->lo, (int)N, lo3, e,
                                              (unsigned long long)nb[1],
                                              (unsigned long long)nb[2], bits, c->sb.keys,
                                              reinterpret_cast<unsigned long long*>(c->sb.tmp4),
                                              c->sb.hist, cnt, c->stream));
        } else {
            HIP_TRY(ld::launch_boxcount(c->pos, c->lo, (int)N, lo3, e, c->sb.keys,
                                        c->sb.n_pow2, cnt, c->stream));
        }
        unsigned long long hc = 0;
        HIP_TRY(copy_out(&hc, cnt, sizeof hc, c->stream));
        if (box_counts) box_counts[k] = (int64_t)hc;
        lx.push_back(std::log(e));
        ly.push_back(std::log((double)hc));
        K = k + 1;
    }
    out[3] = (double)K;
    if (K >= 3) {
        double sx = 0, sy = 0, sxx = 0, sxy = 0;
        const int m = K - 1;
        for (int k = 1; k < K; ++k) { sx += lx[k]; sy += ly[k]; }
        const double mx = sx / m, my = sy / m;
        for (int k = 1; k < K; ++k) {
            sxx += (lx[k] - mx) * (lx[k] - mx);
            sxy += (lx[k] - mx) * (ly[k] - my);
        }
        out[2] = -sxy / sxx;
    } else {
        out[2] = NAN;
    }
    return wait_stream(c);
}

ld_status ld_get_tuning(ld_ctx* c, ld_tuning* t) {
    g_err.clear();
    if (!c || !t) return fail(LD_EINVAL, "ctx and t are required");
    *t = c->tune;
    return LD_OK;
}

ld_status ld_set_tuning(ld_ctx* c, const ld_tuning* t) {
    g_err.clear();
    if (!c || !t) return fail(LD_EINVAL, "ctx and t are required");
    ld_tuning u = *t;
    if (u.block == 0) u.block = c->tune.block;
    if (u.j_split == 0) u.j_split = c->tune.j_split;
    if (u.block != 64 && u.block != 128 && u.block != 256 && u.block != 512)
        return fail(LD_EINVAL, "block must be 64, 128, 256 or 512");
    if (u.j_split < 1 || u.j_split > 64) return fail(LD_EINVAL, "j_split must be in [1, 64]");
    if (u.comp != 0 && u.comp != 1) return fail(LD_EINVAL, "comp must be 0 or 1");
    if (u.cull != 0 && u.cull != 1) return fail(LD_EINVAL, "cull must be 0 or 1");
    if (u.graph_steps < 0 || u.graph_steps > 4096)
        return fail(LD_EINVAL, "graph_steps must be in [0, 4096]");
    if (u.sort_every > 4096) return fail(LD_EINVAL, "sort_every must be <= 4096");
    HIP_TRY(hipStreamSynchronize(c->stream));
    ld_status st = ensure_split_capacity(c, u.j_split);
    if (st != LD_OK) return st;
    c->tune = u;
    invalidate_graph(c);
    return LD_OK;
}

namespace {
constexpr char kMagic[8] = {'L', 'D', 'R', 'O', 'P', 'C', 'K', '2'};
}

ld_status ld_checkpoint_save(ld_ctx* c, const char* path) {
    g_err.clear();
    if (!c || !path) return fail(LD_EINVAL, "ctx and path are required");
    if (c->pm) return fail(LD_ESTATE, "checkpoints hold no velocities (ld_paper_disable first)");
    const size_t N = (size_t)c->n;
    std::vector<float4> h(N), l(N);
    std::vector<int> ty(N), ids(N);
    ld::DevState ds;
    HIP_TRY(hipMemcpyAsync(h.data(), c->pos, sizeof(float4) * N, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(l.data(), c->lo, sizeof(float4) * N, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(ty.data(), c->typ, sizeof(int) * N, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(ids.data(), c->oid, sizeof(int) * N, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(&ds, c->st, sizeof ds, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(LD_ESTATE, "cannot open %s for writing", path);
    const int64_t n64 = c->n, sss = c->steps_since_sort;
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&n64, 8, 1, f) == 1 &&
              std::fwrite(&c->p, sizeof c->p, 1, f) == 1 &&
              std::fwrite(&c->R, sizeof c->R, 1, f) == 1 &&
              std::fwrite(&c->seed, 8, 1, f) == 1 &&
              std::fwrite(&c->tune, sizeof c->tune, 1, f) == 1 &&
              std::fwrite(&ds.step, 8, 1, f) == 1 && std::fwrite(&ds.t, 8, 1, f) == 1 &&
              std::fwrite(&sss, 8, 1, f) == 1 &&
              std::fwrite(h.data(), sizeof(float4), N, f) == N &&
              std::fwrite(l.data(), sizeof(float4), N, f) == N &&
              std::fwrite(ty.data(), sizeof(int), N, f) == N &&
              std::fwrite(ids.data(), sizeof(int), N, f) == N;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(LD_ESTATE, "writing %s failed", path);
    return LD_OK;
}

ld_status ld_checkpoint_load(ld_ctx** out, const char* path, void* stream) {
    g_err.clear();
    if (!out || !path) return fail(LD_EINVAL, "out and path are required");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(LD_ESTATE, "cannot open %s", path);
    char magic[8];
    int64_t n64 = 0, step = 0, sss = 0;
    double t = 0.0;
    ld_params p;
    ld_radius R;
    uint64_t seed = 0;
    ld_tuning tune;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 &&
              std::fread(&n64, 8, 1, f) == 1 && n64 >= 2 && n64 <= (1 << 27) &&
              std::fread(&p, sizeof p, 1, f) == 1 && std::fread(&R, sizeof R, 1, f) == 1 &&
              std::fread(&seed, 8, 1, f) == 1 && std::fread(&tune, sizeof tune, 1, f) == 1 &&
              std::fread(&step, 8, 1, f) == 1 && std::fread(&t, 8, 1, f) == 1 &&
              std::fread(&sss, 8, 1, f) == 1;
    const size_t N = ok ? (size_t)n64 : 0;
    std::vector<float4> h(N), l(N);
    std::vector<int> ty(N), ids(N);
    ok = ok && std::fread(h.data(), sizeof(float4), N, f) == N &&
         std::fread(l.data(), sizeof(float4), N, f) == N &&
         std::fread(ty.data(), sizeof(int), N, f) == N &&
         std::fread(ids.data(), sizeof(int), N, f) == N;
    std::fclose(f);
    if (!ok) return fail(LD_EINVAL, "%s is not a complete checkpoint of this version", path);
    // a context in original order, then overwrite its slot arrays and clock
    std::vector<int32_t> ty_orig(N);
    std::vector<double> q_orig(N);
    std::vector<float> x_orig(3 * N);
    const double qs = std::sqrt(p.kT * p.bjerrum);
    std::vector<bool> seen(N, false);
    for (size_t s = 0; s < N; ++s) {
        const int o = ids[s];
        if (o < 0 || (size_t)o >= N || seen[o])
            return fail(LD_EINVAL, "%s: slot permutation is corrupt", path);
        seen[o] = true;
        ty_orig[o] = ty[s];
        q_orig[o] = qs > 0.0 ? (double)h[s].w / qs : 0.0;
        x_orig[3 * o] = h[s].x;
        x_orig[3 * o + 1] = h[s].y;
        x_orig[3 * o + 2] = h[s].z;
    }
    ld_ctx* c = nullptr;
    ld_status st = ld_init(&c, n64, ty_orig.data(), q_orig.data(), x_orig.data(), &p, &R, seed,
                           stream);
    if (st != LD_OK) return st;
    ld::DevState ds{};
    ds.step = step;
    ds.t = t;
    ds.bad_step = ~0ull;
    hipError_t e = hipMemcpyAsync(c->pos, h.data(), sizeof(float4) * N, hipMemcpyHostToDevice,
                                  c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->lo, l.data(), sizeof(float4) * N, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->typ, ty.data(), sizeof(int) * N, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->oid, ids.data(), sizeof(int) * N, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->st, &ds, sizeof ds, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = ld::launch_msd_ref(c->pos, c->lo, c->oid, (int)N, c->ref, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        ld_destroy(c);
        return fail(LD_EHIP, "restoring state: %s", hipGetErrorString(e));
    }
    st = ld_set_tuning(c, &tune);
    if (st == LD_OK) {
        e = ld::launch_boxes(c->pos, (int)N, c->box, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) st = fail(LD_EHIP, "boxes: %s", hipGetErrorString(e));
    }
    if (st != LD_OK) {
        ld_destroy(c);
        return st;
    }
    c->steps_since_sort = sss;
    *out = c;
    return LD_OK;
}

ld_status ld_autotune(ld_ctx* c, const char* cache_path, int32_t force, ld_tuning* out) {
    g_err.clear();
    if (!c) return fail(LD_EINVAL, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(c->stream));
    // cache key: architecture, size bucket (quarter octaves), types, mode
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, c->device));
    char arch[64];
    std::snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
    for (char* q = arch; *q; ++q)
        if (*q == ':' || *q == ' ') *q = '_';
    const int bucket = (int)std::floor(std::log2((double)c->n) * 4.0);
    char key[160];
    std::snprintf(key, sizeof key, "%s/nb%d/T%d/cull%d/comp%d", arch, bucket, c->p.n_types,
                  c->tune.cull, c->tune.comp);
    std::vector<std::string> lines;
    if (cache_path && !force) {
        if (FILE* f = std::fopen(cache_path, "r")) {
            char k[160];
            int b = 0, js = 0;
            double ms = 0.0;
            while (std::fscanf(f, "%159s %d %d %lf", k, &b, &js, &ms) == 4) {
                if (std::strcmp(k, key) == 0) {
                    std::fclose(f);
                    ld_tuning u = c->tune;
                    u.block = b;
                    u.j_split = js;
                    ld_status st = ld_set_tuning(c, &u);
                    if (st != LD_OK) return st;
                    if (out) *out = c->tune;
                    return LD_OK;
                }
            }
            std::fclose(f);
        }
    }
    const ld_tuning saved = c->tune;
    const bool saved_timing = c->timing;
    c->timing = false;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int blocks[] = {128, 256, 512};
    const int splits[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32};
    int64_t cap = c->n / 256;
    if (cap < 1) cap = 1;
    double best_ms = INFINITY;
    ld_tuning best = saved;
    ld_status st = LD_OK;
    for (int b : blocks) {
        for (int js : splits) {
            if (js > cap || (c->n + b - 1) / b * (int64_t)js > 65535 * 8) continue;
            if (ensure_split_capacity(c, js) != LD_OK) continue;
            c->tune.block = b;
            c->tune.j_split = js;
            double ms_min = INFINITY;
            for (int rep = 0; rep < 4 && st == LD_OK; ++rep) {
                if (hipEventRecord(e0, c->stream) != hipSuccess) st = LD_EHIP;
                if (st == LD_OK) st = run_pair(c, false, c->stream, false);
                if (st == LD_OK && hipEventRecord(e1, c->stream) != hipSuccess) st = LD_EHIP;
                if (st == LD_OK && hipEventSynchronize(e1) != hipSuccess) st = LD_EHIP;
                float ms = 0.f;
                if (st == LD_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = LD_EHIP;
                if (rep > 0 && ms < ms_min) ms_min = ms;   // first launch is a warm-up
            }
            if (st != LD_OK) break;
            if (ms_min < best_ms) {
                best_ms = ms_min;
                best = c->tune;
            }
        }
        if (st != LD_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->timing = saved_timing;
    if (st != LD_OK) {
        c->tune = saved;
        return fail(LD_EHIP, "autotune launch failed");
    }
    c->tune = best;
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "r")) {
            char buf[256];
            while (std::fgets(buf, sizeof buf, f)) {
                if (std::strncmp(buf, key, std::strlen(key)) != 0 || buf[std::strlen(key)] != ' ')
                    lines.emplace_back(buf);
            }
            std::fclose(f);
        }
        if (FILE* f = std::fopen(cache_path, "w")) {
            for (const std::string& l : lines) std::fputs(l.c_str(), f);
            std::fprintf(f, "%s %d %d %.6f\n", key, best.block, best.j_split, best_ms);
            std::fclose(f);
        }
    }
    if (out) *out = c->tune;
    return LD_OK;
}

ld_status ld_kernel_timing(ld_ctx* c, int32_t enable) {
    g_err.clear();
    if (!c) return fail(LD_EINVAL, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->timing = enable != 0;
    if (enable) {
        c->ev_used = 0;
        c->ev_kind.clear();
    }
    return LD_OK;
}

namespace {
ld_status timed_total(ld_ctx* c, unsigned char kind, int64_t* launches, double* total_ms) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    double tot = 0.0;
    int64_t cnt = 0;
    for (size_t p = 0; p < c->ev_kind.size() && 2 * p + 1 < c->ev_used; ++p) {
        if (c->ev_kind[p] != kind) continue;
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev_pool[2 * p], c->ev_pool[2 * p + 1]));
        tot += ms;
        ++cnt;
    }
    if (launches) *launches = cnt;
    if (total_ms) *total_ms = tot;
    return LD_OK;
}
}  // namespace

ld_status ld_kernel_time(ld_ctx* c, int64_t* launches, double* total_ms) {
    g_err.clear();
    if (!c) return fail(LD_EINVAL, "ctx is NULL");
    return timed_total(c, ld::kTimedCoulomb, launches, total_ms);
}

ld_status ld_near_kernel_time(ld_ctx* c, int64_t* launches, double* total_ms) {
    g_err.clear();
    if (!c) return fail(LD_EINVAL, "ctx is NULL");
    return timed_total(c, ld::kTimedNear, launches, total_ms);
}

}  // extern "C"
