// Internal declarations shared by the host runtime and the device code of the
// MPdist / snippet library.  Not part of the public ABI (include/pst.h is).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pst {

// Profile kernel geometry (workgroup size and tile width depend on w: see
// profile_tile_windows and profile_slots).
constexpr int kMaxW = 1025;            // largest supported w = m - l + 1
constexpr int kScanBlock = 4096;       // elements per block of the prefix-sum scan
constexpr int kSumBlock = 8192;        // windows per block of the greedy area sums
constexpr int kStatsPad = 16;          // zeroed elements after each per-window statistic and the series

// Statistics of the length-l subsequences of one series.  The paper evaluates
// the distance matrix from dot products, means and standard deviations
// (section 4.1, eq. 9, after its ref. [7]); means here are of the series
// centred by its global mean.
struct Stats {
    const double *xc;  // series minus its global mean, [len] (+ kStatsPad zeros)
    const double *mu;  // centred mean of each window, [Nl] (each per-window array + kStatsPad zeros)
    const float *inv;  // 1 / (sigma * sqrt(l)); 0 for a constant window, [Nl]
    const float *h;    // 0.5 for a constant window, else 0, [Nl]
    const float *df;   // (x[j+l] - x[j]) / 2, [Nl]; 0 at the last window
    const float *dg;   // (x[j+l] - mu[j+1]) + (x[j] - mu[j]), [Nl]; 0 at the last
};

// Device layout of the statistics of one series of length len.
struct StatsLayout {
    int64_t len, Nl;
    int32_t l, nblk;
    size_t xc, mu, inv, h, df, dg, pre, blk, part, misc, total;
};
StatsLayout stats_layout(int64_t len, int32_t l);
Stats stats_view(char *base, const StatsLayout &L);
// misc[0] global mean, misc[1] max |x|, misc[2] 1.0 if any value is not finite.
inline double *stats_misc(char *base, const StatsLayout &L) { return (double *)(base + L.misc); }
hipError_t launch_series_stats(const double *x, char *base, const StatsLayout &L, hipStream_t st);

// One profile-kernel problem: `nq` queries (segments of T, or one external
// query) against all windows of T.
struct ProfileJob {
    Stats col;             // statistics of T
    Stats row;             // statistics of the rows' series (T itself, or the query)
    int64_t row_stride;    // rows of query s start at s * row_stride of the row series
    int64_t n, Nl, Nm;
    int32_t m, l, w, k, nq;
    float *D;              // out: D[s * ld + j]
    int64_t ld;
    float *rw;             // scratch: profile_scratch_floats(grid, w) floats
    unsigned *dmax_bits;   // optional: atomic max of D's bit patterns
    int32_t grid;          // persistent workgroups
    int32_t anchor_every;  // > 0: also re-anchor every diagonal at rows i % anchor_every == 0
};
// Up to kMaxJobs problems (for example every candidate m of a length sweep)
// run in one persistent launch; tiles are striped over the workgroups, or
// handed out by a device counter when `counter` is set (zeroed beforehand).
constexpr int kMaxJobs = 16;
struct ProfileBatch {
    ProfileJob J[kMaxJobs];
    int64_t tile_end[kMaxJobs];   // job j owns tiles [tile_end[j-1], tile_end[j])
    int32_t njobs;
    size_t slot_floats;           // scratch floats per workgroup
    uint32_t *counter;
};
int64_t profile_tiles(const ProfileJob &j);
hipError_t profile_prepare(int32_t wmax);  // kernel attributes; call outside graph capture
hipError_t launch_profile_batch(const ProfileJob *jobs, int n, int32_t grid, uint32_t *counter,
                                hipStream_t st);
int32_t profile_tile_windows(int32_t w);  // windows per tile
int32_t profile_slots(int32_t w);                 // profile workgroups resident at once
int32_t profile_shape(int32_t w);                 // equal for w that get the same workgroup shape
int32_t profile_grid(int64_t tiles, int32_t w);   // persistent grid for that many tiles
size_t profile_scratch_floats(int32_t grid, int32_t w);
hipError_t launch_profile(const ProfileJob &job, hipStream_t st);
size_t profile_lds_bytes(int32_t w);   // dynamic LDS of one profile workgroup
// Tile geometry of the profile kernel for w (workgroup size, diagonals per
// thread, rows per chunk, selection threads, sub-tile width) as one code: the
// one in use, the candidates the kernels can run, and an override for w
// (code 0 restores the built-in choice; false if the code is not a
// candidate).  Results of different geometries agree within the profile
// tolerance, not bit for bit (sub-tiles anchor their diagonals afresh).
int32_t profile_geometry(int32_t w);
int32_t profile_geometry_candidates(int32_t w, int32_t *codes, int32_t max);
bool profile_set_geometry(int32_t w, int32_t code);
// Profile scratch floats that any candidate geometry needs for nq queries.
size_t profile_scratch_bound(int64_t Nm, int64_t nq, int32_t w);

// Greedy snippet search and its by-products, all on device (eqs. 6-8, 16-18).
struct GreedyJob {
    const float *D;
    int64_t ld, Nm;
    int32_t nseg, K;
    float *M;             // [Nm] representativeness curve
    double *part;         // [nseg * nblk] partial areas
    int32_t nblk;
    int32_t *pick;        // [K]
    double *area;         // [K]
    uint8_t *chosen;      // [nseg]
    int32_t *count;       // [K] neighbours per snippet
    int32_t *owner;       // [Nm] or null
    float *profiles;      // [K * Nm] or null
    double *crit;         // [nblk2 + 1] criterion partial sums; crit[nblk2] = total
    int32_t nblk2;
};
hipError_t launch_greedy(const GreedyJob &g, hipStream_t st);
// Up to kMaxJobs greedy searches (and their neighbours) in the same launches,
// one job per slice of each grid; every job's arithmetic is the same as alone.
hipError_t launch_greedy_batch(const GreedyJob *g, int n, hipStream_t st);
hipError_t launch_owner_batch(const GreedyJob *g, int n, hipStream_t st);
// The greedy search's steps one by one (M = +inf and nothing chosen; the
// area partials of g.nseg segments of g.D; the pick of round iter; M folded
// with row g.pick[iter] of g.D), for callers that produce D in pieces.
hipError_t launch_greedy_init(const GreedyJob &g, hipStream_t st);
hipError_t launch_area_parts(const GreedyJob &g, hipStream_t st);
hipError_t launch_pick(const GreedyJob &g, int iter, hipStream_t st);
hipError_t launch_update_M(const GreedyJob &g, int iter, hipStream_t st);
// Fill n 32-bit words with v by a kernel (no memset nodes, so it is safe to
// capture in a graph).
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st);
hipError_t launch_owner(const GreedyJob &g, hipStream_t st);
hipError_t launch_criterion(const GreedyJob &g, hipStream_t st);

// Per-candidate results of a length sweep gathered into one device buffer:
// for candidate i, out[i*(3+3K) ..] = crit total, max D (float bits), the
// non-finite flag, then K areas, K picks, K neighbour counts (as doubles).
struct SweepGather {
    int32_t nm, K;
    const double *crit[kMaxJobs];
    const uint32_t *dmax[kMaxJobs];
    const double *bad[kMaxJobs];
    const double *area[kMaxJobs];
    const int32_t *pick[kMaxJobs];
    const int32_t *count[kMaxJobs];
    double *out;
};
hipError_t launch_gather(const SweepGather &g, hipStream_t st);

// A served request's results packed for one copy to the host, at
// out[off[i]]: the 4 statistics words (misc), K picks (int32), K areas
// (double), K neighbour counts (int32) and max D (float bits), each part at
// the double offset 4, 4+K, 4+2K, 4+3K.
struct ResultPack {
    int32_t n;
    int32_t K[kMaxJobs];
    int64_t off[kMaxJobs];
    const double *misc[kMaxJobs];
    const int32_t *pick[kMaxJobs];
    const double *area[kMaxJobs];
    const int32_t *count[kMaxJobs];
    const uint32_t *dmax[kMaxJobs];
    double *out;
};
hipError_t launch_pack_results(const ResultPack &r, hipStream_t st);

// Labelling score: owner array of K snippets against true classes.
struct LabelJob {
    const int32_t *owner;  // [n-m+1] greedy rank of each window's nearest snippet
    const int32_t *truth;  // [n] true class of each element
    int64_t n;
    int32_t m, K, C;
    bool lds;              // confusion counts through LDS (set by the launcher)
    unsigned *conf;        // [K*C] out
    unsigned *bad;         // out: elements with a label outside range
    int32_t *map;          // [K] out: class of each snippet
    double *prec, *rec, *f1;  // [C] out
    double *macro;         // out
};
hipError_t launch_label_f1(const LabelJob &job, hipStream_t st);

// The fixed device scratch of the allocation-free entry point: its size, and
// its device address on `device` (which must be current), looked up once.
size_t static_scratch_bytes();
hipError_t static_scratch(int device, void **ptr);

}  // namespace pst
