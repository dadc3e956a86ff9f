// Internal declarations of libldrop: device data layout, kernel parameter
// blocks and the host-side launchers each .hip file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "ldrop.h"

namespace ld {

constexpr int kMaxTypes = LD_MAX_TYPES;
constexpr int kGroup = 64;            // one wavefront: the unit of tile culling
// Largest n with a near-group bitmap (ceil(n/64)^2 bits: 32 MiB at 2^20)
constexpr int64_t kNearBitsMaxN = 1 << 20;

// Far-away, uncharged filler for the padded tail of a j tile: its Coulomb
// weight is exactly zero and it never enters the LJ range.
constexpr float kFarAway = 1.0e18f;

// Words (8 bytes) of the small auxiliary buffer: two 4096-bin histograms plus
// a few scalars.
constexpr int kAuxWords = 2 * 4096 + 64;

// Per type-pair LJ constants in FP32 (LDS-resident inside the pair kernel).
struct PairTable {
    int T;
    float rc2max;                        // max_ij (lj_cut sigma_ij)^2
    float sig2[kMaxTypes * kMaxTypes];   // sigma_ij^2
    float rc2[kMaxTypes * kMaxTypes];    // (lj_cut sigma_ij)^2
    float e24[kMaxTypes * kMaxTypes];    // 24 eps_ij
    float e4[kMaxTypes * kMaxTypes];     // 4 eps_ij
    // FP64 copies for the Lennard-Jones arithmetic (near the minimum the
    // force is a small difference of two large terms)
    double sig2d[kMaxTypes * kMaxTypes];
    double e24d[kMaxTypes * kMaxTypes];
    double e4d[kMaxTypes * kMaxTypes];
    double rc2d[kMaxTypes * kMaxTypes];
};

// Per-type constants and globals for the O(N) kernels, all FP64.
struct ExtParams {
    int n_types, rotation, wall_band, noise;
    double gravity[3];
    double omega2;                       // omega^2
    double kT, jump_max;
    double mu[kMaxTypes];                // 1 / gamma
    double mass[kMaxTypes];
    double k_wall[kMaxTypes];
    double wall_offset[kMaxTypes];
    double half_sigma[kMaxTypes];
    ld_radius R;
};

// Device-resident step state.  Kernels of a step read it; a one-thread
// kernel after the update advances it, so captured graphs replay correctly.
struct DevState {
    long long step;                      // global step counter n
    double t;                            // time t_n
    unsigned long long bad_step;         // first step with a blow-up (~0: none)
    unsigned int pad0;                   // unused
    unsigned int pad;
};

struct Box {
    float4 lo, hi;                       // .w unused
};

// Radius schedule, FP64.
__host__ __device__ inline double radius_at(const ld_radius& R, double t) {
    if (R.kind == LD_R_LINEAR) {
        double f = R.T > 0.0 ? t / R.T : 1.0;
        f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
        return R.R0 + (R.R1 - R.R0) * f;
    }
    if (R.kind == LD_R_SQUARE_LAW) {
        double r2 = R.R0 * R.R0 - 2.0 * R.a * t;
        double m2 = R.R_min * R.R_min;
        return sqrt(r2 < m2 ? m2 : r2);
    }
    if (R.kind == LD_R_TABLE) {
        const int m = R.n_knots;
        if (t <= R.tab_t[0]) return R.tab_R[0];
        for (int k = 1; k < m; ++k)
            if (t < R.tab_t[k]) {
                const double f = (t - R.tab_t[k - 1]) / (R.tab_t[k] - R.tab_t[k - 1]);
                return R.tab_R[k - 1] + (R.tab_R[k] - R.tab_R[k - 1]) * f;
            }
        return R.tab_R[m - 1];
    }
    return R.R0;
}

// ---- launchers (each returns hipSuccess or the first HIP error) --------

struct PairLaunch {
    const float4* pos;
    const float4* lo;                    // low words of the positions
    const int* typ;
    const Box* box;                      // per 64-slot group, or nullptr
    int n;
    int block;
    int j_split;
    int comp;
    int cull;
    double* Fpart;                       // [j_split][3][n]
    double* S;                           // [n] or nullptr (diagnostic mode)
    double* U;                           // [2][n] or nullptr (diagnostic mode)
    // Near-group bitmap [ceil(n/64)][nb_words] (or nullptr): the Coulomb
    // kernel sets bit (gi, gj) for every group pair it takes as near, the
    // Lennard-Jones kernel reads and clears row gi (all zero between launches).
    unsigned* nearbits;
    int nb_words;
};
// The Coulomb kernel (k_pair) and then the FP64 Lennard-Jones kernel (k_lj);
// after_coulomb, if given, is recorded between the two.
hipError_t launch_pair(const PairLaunch& L, const PairTable& tab, hipStream_t s,
                       hipEvent_t after_coulomb = nullptr);
// Mean square displacement against FP64 reference positions [3][n] in
// original order: store the reference, or reduce the mean into out[0].
hipError_t launch_msd_ref(const float4* pos, const float4* lo, const int* oid, int n,
                          double* ref, hipStream_t s);
hipError_t launch_msd(const float4* pos, const float4* lo, const int* oid, int n,
                      const double* ref, double* work, double* out, hipStream_t s);

struct StepLaunch {
    float4* pos;
    float4* lo;
    const int* typ;
    const int* oid;
    const double* Fpart;
    int j_split;
    int n;
    double dt;
    unsigned long long seed;
    DevState* st;
    Box* box;                            // refreshed for the new positions
};
hipError_t launch_update(const StepLaunch& L, const ExtParams& P, hipStream_t s);
// Step counter + 1 and t + dt (enqueued after an update).
hipError_t launch_advance(DevState* st, double dt, hipStream_t s);

hipError_t launch_boxes(const float4* pos, int n, Box* box, hipStream_t s);

// Gather into original order: pair force totals, external forces at R(t),
// and optional S.  Any output may be null.
hipError_t launch_gather(const float4* pos, const float4* lo, const int* typ, const int* oid,
                         const double* Fpart, int j_split, const double* S_slot, int n,
                         const DevState* st, const ExtParams& P, double* F_pair,
                         double* F_ext, double* S, hipStream_t s);

// Deterministic FP64 sum of m rows of length n: out[r] = sum_s in[r*n + s].
hipError_t launch_rowsum(const double* in, int rows, int n, double* out, hipStream_t s);
hipError_t launch_rowmin(const double* in, int rows, int n, double* out, hipStream_t s);
hipError_t launch_rowmax(const double* in, int rows, int n, double* out, hipStream_t s);

// Positions hi + lo as FP64 rows work[0..2][n].
hipError_t launch_pos_rows(const float4* pos, const float4* lo, int n, double* work,
                           hipStream_t s);

// Replace the charge word of every slot: pos[s].w = qhat[oid[s]].
hipError_t launch_set_charge(float4* pos, const int* oid, const float* qhat, int n,
                             hipStream_t s);

// Per-slot diagnostic terms -> out[10] (see ld_diagnostics).
hipError_t launch_diag(const float4* pos, const float4* lo, const int* typ,
                       const double* Fpart, int j_split, const double* U_slot, int n,
                       const DevState* st, const ExtParams& P, double* work, double* out,
                       hipStream_t s);

// Hilbert index of a point with BITS-bit coordinates (J. Skilling,
// "Programming the Hilbert curve", AIP Conf. Proc. 707 (2004): the transpose
// form -- undo the excess work, Gray-encode, then interleave the bits).
// Consecutive indices are face neighbours, so runs of 64 particles along the
// curve are more compact than Morton runs (about half as many pairs of
// 64-particle groups come within LJ range of each other at the large
// workload).
template <int BITS>
__device__ __forceinline__ unsigned hilbert_index(unsigned x0, unsigned x1, unsigned x2) {
    unsigned X[3] = {x0, x1, x2};
    const unsigned M = 1u << (BITS - 1);
    for (unsigned Q = M; Q > 1; Q >>= 1) {
        const unsigned P = Q - 1;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                const unsigned t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    unsigned t = 0;
    for (unsigned Q = M; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    X[0] ^= t; X[1] ^= t; X[2] ^= t;
    unsigned key = 0;
    for (int b = BITS - 1; b >= 0; --b)
        key = (key << 3) | (((X[0] >> b) & 1u) << 2) | (((X[1] >> b) & 1u) << 1) |
              ((X[2] >> b) & 1u);
    return key;
}

// Spatial ordering: Hilbert keys over the current bounding cube, sort, and
// permutation of every per-slot array.
struct SortBuffers {
    unsigned long long* keys;            // [n_pow2]
    int n_pow2;
    float4* tmp4;                        // [n]
    int* tmp_i;                          // [n]
    float* bounds;                       // [8] device scratch
    float* bounds_part;                  // per-block partial min/max
    int bounds_parts;
    unsigned* hist;                      // [256 * (radix_tiles(n) + 1)] radix digit counts
                                         // and the 256 digit totals (or null)
};
// Hilbert-curve order of the slots over the particles' bounding box clipped
// to [-clip, clip] per axis (INFINITY: no clip).
hipError_t launch_sort(float4* pos, float4* lo, int* typ, int* oid, int n,
                       const SortBuffers& B, hipStream_t s, float clip);

// Largest radius a schedule reaches (INFINITY if it grows without bound).
inline double schedule_max_radius(const ld_radius& R) {
    if (R.kind == LD_R_LINEAR) return R.R0 > R.R1 ? R.R0 : R.R1;
    if (R.kind == LD_R_SQUARE_LAW) return R.a >= 0.0 ? R.R0 : INFINITY;
    if (R.kind == LD_R_TABLE) {
        double m = 0.0;
        for (int k = 0; k < R.n_knots; ++k) m = R.tab_R[k] > m ? R.tab_R[k] : m;
        return m;
    }
    return R.R0;
}

// Sort B.keys (filled by the caller: high word = sort key, low word = slot;
// padding keys ~0) and permute the slot arrays accordingly.
hipError_t launch_sort_by_keys(float4* pos, float4* lo, int* typ, int* oid, int n,
                               const SortBuffers& B, hipStream_t s);

// 64-bit bitonic sort of n_pow2 keys (ascending).
hipError_t launch_bitonic(unsigned long long* keys, int n_pow2, hipStream_t s);

// Slot arrays permuted by B.keys (low word of keys[s] = source slot of s).
hipError_t permute_slots(float4* pos, float4* lo, int* typ, int* oid, int n,
                         const SortBuffers& B, hipStream_t s);

// Radix sort geometry: a workgroup of 256 handles a tile of 8 rounds x 256
// keys; B.hist holds 256 digit counts per tile (digit-major).
constexpr int kRadixThreads = 256;
constexpr int kRadixRounds = 8;
constexpr int kRadixTile = kRadixThreads * kRadixRounds;
int radix_tiles(int n);

// Stable sort of keys[0, n) by the high word, which is below 2^bits (LSD
// radix, 8-bit digits; tmp holds n keys, hist 256 * (radix_tiles(n) + 1)).
// first_counted: hist already holds the first pass's digit counts.
// sorted: if given, receives the buffer holding the result (keys or tmp);
// otherwise the result is copied into keys.
hipError_t launch_radix_by_high(unsigned long long* keys, unsigned long long* tmp, int n, int bits,
                                unsigned* hist, hipStream_t s, bool first_counted = false,
                                unsigned long long** sorted = nullptr);

// First slots of the cells of keys sorted by cell (cell << 32 | slot):
// cfirst[c] = the first slot whose cell is >= c, for c <= M (n past the last
// key), so the slots of cells a..b are [cfirst[a], cfirst[b + 1]).  Called
// by every work-item s of a one-dimensional launch over the keys; the slot
// that starts cell c (previous slot in cell p < c) fills cells p+1 .. c, the
// last slot cells c+1 .. M.  Gaps of up to 8 cells are filled by their own
// lane; a wavefront fills each longer gap together, 64 cells per pass, so
// long runs of empty cells cost little.
__device__ __forceinline__ void fill_cell_first(const unsigned long long* __restrict__ keys, int n,
                                                int M, int s, int* cfirst) {
    const int lane = threadIdx.x % 64;
    int p = 0, c = 0;
    bool gap = false, tail = false;
    if (s < n) {
        c = (int)(keys[s] >> 32);
        p = s == 0 ? -1 : (int)(keys[s - 1] >> 32);
        gap = c != p;
        tail = s == n - 1;
    }
    const bool own = gap && c - p <= 8;
    if (own)
        for (int q = p + 1; q <= c; ++q) cfirst[q] = s;
    unsigned long long todo = __ballot(gap && !own);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int gp = __shfl(p, leader), gc = __shfl(c, leader), gs = __shfl(s, leader);
        for (int q = gp + 1 + lane; q <= gc; q += 64) cfirst[q] = gs;
        todo &= todo - 1ull;
    }
    const unsigned long long last = __ballot(tail);
    if (last) {
        const int leader = __ffsll((long long)last) - 1;
        const int gc = __shfl(c, leader);
        for (int q = gc + 1 + lane; q <= M; q += 64) cfirst[q] = n;
    }
}

// dst arrays[s] = src arrays[low word of keys[s]] for s < n, one launch.
hipError_t permute_slots_into(const unsigned long long* keys, int n, const float4* pos,
                              const float4* lo, const int* typ, const int* oid, float4* pos2,
                              float4* lo2, int* typ2, int* oid2, hipStream_t s);

// Post-processing.
hipError_t launch_rdf(const float4* pos, const float4* lo, int n, double r_max, int n_bins,
                      const double* centre, unsigned long long* counts,
                      unsigned long long* ccounts, hipStream_t s);
// Eq. (8) counts of the NPs of type `want` only (typ in slot order).
hipError_t launch_centre_hist(const float4* pos, const float4* lo, const int* typ, int want, int n,
                              double r_max, int n_bins, const double* centre,
                              unsigned long long* ccounts, hipStream_t s);
hipError_t launch_moments(const float4* pos, const float4* lo, int n, double* work,
                          double* out4, hipStream_t s);
hipError_t launch_boxcount(const float4* pos, const float4* lo, int n, const double* lo3,
                           double eps, unsigned long long* keys, int n_pow2,
                           unsigned long long* count, hipStream_t s);
// Box counting by compact box indices below 2^bits <= 2^32 (ny, nz boxes
// along y and z) and the radix sort; keys and tmp hold n keys each, hist as
// for the radix sort.
hipError_t launch_boxcount_radix(const float4* pos, const float4* lo, int n, const double* lo3,
                                 double eps, unsigned long long ny, unsigned long long nz,
                                 int bits, unsigned long long* keys, unsigned long long* tmp,
                                 unsigned* hist, unsigned long long* count, hipStream_t s);

struct FarField;
struct PaperMode;
struct Recorder;

}  // namespace ld

// The opaque context behind the C ABI.
struct ld_ctx {
    int64_t n = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    ld_params p{};
    ld_radius R{};
    uint64_t seed = 0;
    ld_tuning tune{};
    ld::PairTable tab{};
    ld::ExtParams ext{};

    float4* pos = nullptr;               // [n] {x_hi, y_hi, z_hi, q_hat}, slot order
    float4* lo = nullptr;                // [n] {x_lo, y_lo, z_lo, 0}
    int* typ = nullptr;                  // [n] type per slot
    int* oid = nullptr;                  // [n] original index per slot
    // second slot arrays (allocated by the learned path: its cell sort
    // permutes into them and swaps them with the four above)
    float4* pos2 = nullptr;
    float4* lo2 = nullptr;
    int* typ2 = nullptr;
    int* oid2 = nullptr;
    ld::Box* box = nullptr;              // [ceil(n/64)] group boxes
    unsigned* nearbits = nullptr;        // near-group bitmap (n <= kNearBitsMaxN), zero at rest
    int nb_words = 0;
    double* Fpart = nullptr;             // [j_split_cap][3][n]
    int j_split_cap = 0;
    double* S_slot = nullptr;            // [n]
    double* U_slot = nullptr;            // [2][n]
    double* work = nullptr;              // [16][n] FP64 scratch (outputs, reductions)
    double* aux = nullptr;               // [kAuxWords] histograms and small results
    double* ref = nullptr;               // [3][n] MSD reference positions, original order
    ld::DevState* st = nullptr;
    ld::SortBuffers sb{};
    int64_t steps_since_sort = 0;

    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    // what each timed (start, end) event pair brackets: kTimedCoulomb or
    // kTimedNear
    std::vector<unsigned char> ev_kind;

    // captured step chunk (HIP graph)
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph = nullptr;
    double graph_dt = 0.0;
    int graph_len = 0;
    ld_tuning graph_key{};

    // learned far field (null until ld_ff_enable)
    ld::FarField* ff = nullptr;
    // the paper's own scheme (null until ld_paper_enable)
    ld::PaperMode* pm = nullptr;
    // scratch of the aggregate statistics (null until first used)
    void* agg = nullptr;
    // open trajectory recording (null when none)
    ld::Recorder* rec = nullptr;
};

namespace ld {
constexpr unsigned char kTimedCoulomb = 0;   // the all-pairs Coulomb kernel
constexpr unsigned char kTimedNear = 1;      // the learned path's near-field kernels
// A (start, end) pair of timing events from the context's pool, recorded as
// bracketing `kind`; false when no event could be created.
bool timing_events(ld_ctx* c, unsigned char kind, hipEvent_t* e0, hipEvent_t* e1);
// Learned far field hooks used by the step loop (defined in ld_ff.hip).
void ff_free(ld_ctx* c);
bool ff_active(const ld_ctx* c);
// Pair forces of one step into Fpart: the learned path (one partial) or the
// direct path; *j_split_used says how many partials the update must sum.
ld_status ff_step_forces(ld_ctx* c, hipStream_t s, int* j_split_used);
// The paper's own scheme (defined in ld_paper.hip): one step, and release.
ld_status pm_step(ld_ctx* c, double dt, hipStream_t s);
void pm_free(ld_ctx* c);
// Aggregate statistics scratch (ld_agg.hip).
void ag_free(ld_ctx* c);
// Eq. (6) pair counts through the cell sort (ld_agg.hip); *used = false when
// the cells would be too coarse and the all-pairs histogram should count.
ld_status ag_rdf_pairs(ld_ctx* c, double r_max, int n_bins, unsigned long long* counts,
                       bool* used);
// Trajectory recording (ld_record.hip): after each enqueued step.
ld_status rec_after_step(ld_ctx* c, double dt, hipStream_t s);
void rec_free(ld_ctx* c);
}  // namespace ld
