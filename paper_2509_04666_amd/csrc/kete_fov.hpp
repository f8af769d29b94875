// Field-of-view stage: parameters shared by the host layer and kernels.
#pragma once

#include "kete_internal.hpp"

namespace kete {

constexpr int kBatchStride = 17;        // doubles per batch record
constexpr int kExactRec = 24;           // doubles per exact-test frame record
constexpr double kMaxLightDays = 1.0;   // light time covered by the staged window

// Sub-frame locator of a frame with several sub-frames: a tangent basis at
// the frame's cap centre and a kLocL x kLocL grid over the gnomonic
// bounding box of its sub-frames, each cell with a bit mask (two 64-bit
// words) of the sub-frames whose gnomonic box overlaps it.  Record:
//   [0..2] centre c, [3..5] e1, [6..8] e2, [9] X0, [10] Y0, [11] 1/dX,
//   [12] 1/dY, [13] 1 when usable (every vertex in the hemisphere around
//   c), [14] X1 = X0 + kLocL dX, [15] Y1, then kLocL^2 x 2 mask words.
constexpr int kLocL = 8;
constexpr int kLocHead = 16;
constexpr int kLocStride = kLocHead + 2 * kLocL * kLocL;     // doubles per frame

// Exact-test candidates and pairs share one 64-bit key: frame << 32 |
// sub-frame << 25 | object; a candidate with bit 63 set stands for every
// sub-frame of its frame.
constexpr unsigned long long kAllSubs = 1ull << 63;

struct FovParams {
    EphemArgs eph;
    const double* x_epoch;      // [B][N][6]
    const int32_t* status;      // [N] or null
    int32_t n_obj;
    int32_t n_batch;
    int64_t n_frames;
    const double* t_ref;        // [B]
    const int32_t* batch_off;   // [B+1]
    const int32_t* frame_order; // [F]
    const double* ft;           // [F]
    const double* fobs;         // [F][3]
    const double* normals;      // [F][S][4][3]
    int32_t n_sub;
    int32_t pad0;
    double* fcap;               // [F][8]: centre, cos R, sin R
    double* loc;                // [F][kLocStride] sub-frame locators in cell order, or null (one sub-frame)
    double* btab;               // [B][kBatchStride]
    int32_t* cell_start;        // [B G^3 + 1]
    int32_t* cell_frames;       // [F]
    double* cell_caps;          // [F][8]: frame caps in cell order, slot 5 = frame index
    // What the join reads of a frame, in cell order, so that the frames of
    // neighbouring cells sit together in memory: time and observer
    // position, and the sub-frame normals.
    double* cell_obs;           // [F][4]: t, observer x, y, z
    float* cell_normals;        // [F][S][4][3] single-precision copies (the join widens its margin by their rounding)
    // What the exact test reads of a frame, by frame index, in one record
    // (kExactRec doubles): its time, its batch's epoch, the observer, the
    // Sun's state at the epoch, the offset of the batch's states in
    // x_epoch (int64 bits) and the Sun's cubic about the frame time
    // (position, velocity, acceleration, jerk).
    double* exact_rec;          // [F][kExactRec]
    unsigned long long* pairs;  // [cap] packed (frame << 32 | sub << 25 | obj)
    unsigned long long* n_pairs;
    int64_t cap;
    unsigned long long* stats;  // [4] or null: candidates, exact tests, brute-force objects
    unsigned long long* cand;   // [cand_cap] keys (frame, sub-frame or kAllSubs, object) for the exact test
    unsigned long long* n_cand;
    int64_t cand_cap;
    int32_t* frame_batch;       // [F] batch of each frame
    // Batch -> object structure.  Batch b tests the local objects
    // 0 .. b_poff[b+1]-b_poff[b]-1 of its job; local object j is global
    // object b_obj0[b] + j with its state at x_epoch + b_xoff[b] + 6 j.
    // A single job of N objects has b_poff[b] = b N, b_obj0[b] = 0 and
    // b_xoff[b] = 6 b N.
    const int64_t* b_poff;      // [B+1]
    const int32_t* b_obj0;      // [B]
    const int64_t* b_xoff;      // [B]
    int64_t n_pairs_total;      // b_poff[B]
    int64_t max_batch_obj;      // the most objects of any batch
    // Sky grid of batch b: G_b cells per axis over [-1, 1]^3 (G_b = 1 puts
    // every frame in one cell); its keys start at b_koff[b] and number
    // G_b^3 + 1 (the last one collects objects with wide motion caps).
    int32_t* b_G;               // [B] sky-grid size per batch (lowered for large frames)
    const int64_t* b_koff;      // [B+1]
    int64_t n_keys;             // b_koff[B]
    const int32_t* obj_sorted;  // [n_pairs_total] local objects of each batch ordered by sky cell
    const int32_t* obj_start;   // [n_keys + 1] start of each key's objects in obj_sorted
    const int32_t* obj_count;   // [n_keys] objects per key
    unsigned long long* items;  // work items of the per-cell join: key << 32 | object chunk
    const int32_t* item_start;  // [n_keys + 1] exclusive scan of items per key (total at n_keys)
    unsigned int* item_next;    // work-queue cursors, kJoinCursorWords unsigned ints
    unsigned long long* wide;   // [n_pairs_total] (batch << 32 | local obj) of objects with wide motion caps
    unsigned long long* n_wide;
    // The wide join's work is split into parts: about 64 grid cells of an
    // object's cap box, or kWidePartFrames frames of its batch when it has
    // no usable cap, wide_max_parts at most.  wide_parts[w] counts the parts of wide object w and
    // wide_off is their exclusive scan (total at n_pairs_total).
    int32_t* wide_parts;        // [n_pairs_total]
    int32_t* wide_off;          // [n_pairs_total + 1]
    unsigned int* wide_next;    // work-queue cursors, kJoinCursorWords unsigned ints
    int32_t wide_max_parts;     // parts per object at most (their total must stay below 2^31)
    int32_t pad2;
    double mu, smu, c_light, lt_tol;
    int32_t lt_iter;
    int32_t max_cells;
    double sin_overflow;
    int32_t kepler_iter;
    int32_t pad1;
    // hops that ended on the Kepler iteration cap: fail[j] = 1 for global
    // object j (zeroed by the caller), and KETE_ST_KEPLER_NOCONV in
    // status_out[j] when status_out is not null; *n_fail counts them
    int32_t* fail;
    int32_t* status_out;
    unsigned long long* n_fail;
};

hipError_t fov_prepare(const FovParams& p, int32_t* qkey, int32_t* cnt, int32_t* cursor, void* scan_scratch,
                       hipStream_t s);
// Objects of every batch into sky-cell order (sorted, with start/cnt per
// key), each cell's objects ordered by their sub-cell key (osub, scratch of
// n_pairs_total entries) so that the join's 64-object items are compact.
hipError_t fov_sort_objects(const FovParams& p, int32_t* okey, int32_t* orank, int32_t* cnt, int32_t* start,
                            int32_t* sorted, int32_t* osub, void* scan_scratch, hipStream_t s);
// Workgroups are dealt to the chip's XCDs round-robin (workgroup i to XCD
// i mod kXcds), each XCD with its own L2.  The per-cell join splits its
// work list into kXcds slices, one cursor each, kCursorStride unsigned ints
// (128 bytes) apart.
constexpr int kXcds = 8;
constexpr int kCursorStride = 32;
constexpr int kJoinCursorWords = kXcds * kCursorStride;
constexpr int kWidePartFrames = 1024;

// Candidate generation.  icnt and istart are [n_keys + 1] int32 scratch
// (istart becomes p.item_start), items holds n_keys + n_pairs_total / 64 + 1
// entries, scan_scratch >= scan_scratch_bytes(n_keys), wide_scan_scratch >=
// scan_scratch_bytes(n_pairs_total); p.wide_parts, p.wide_off and
// p.wide_next must be set.
hipError_t fov_candidates(FovParams& p, int32_t* icnt, int32_t* istart, unsigned long long* items,
                          unsigned int* item_next, void* scan_scratch, void* wide_scan_scratch, hipStream_t s);
inline int64_t fov_item_capacity(int64_t n_keys, int64_t n_pairs_total) { return n_keys + n_pairs_total / 64 + 1; }
// Doubles of the frame copies (cell_obs, cell_normals as floats, exact_rec).
inline int64_t fov_cell_frame_doubles(int64_t n_frames, int n_sub) {
    return n_frames * (4 + 6 * (int64_t)n_sub + kExactRec);
}
hipError_t fov_exact(const FovParams& p, hipStream_t s);
hipError_t fov_drop_failed(const unsigned long long* keys, int64_t n, const int32_t* fail, unsigned long long* out,
                           unsigned long long* n_out, hipStream_t s);
// Pair keys of objects 0 .. n_obj - 1 and n_sub sub-frames to the output
// arrays, sorted by (frame, sub-frame, object).
hipError_t fov_sort(unsigned long long* keys, int64_t n, int64_t n_frames, int64_t n_obj, int n_sub, int32_t* fcnt,
                    int32_t* fstart, unsigned long long* sorted, void* scan_scratch, int32_t* pf, int32_t* ps,
                    int32_t* po, hipStream_t s);
hipError_t launch_directions(const FovParams& p, const double* x_ref, double t_ref, const double* t_obs,
                             const double* obs, int64_t n_q, double* d, double* tau, hipStream_t s);
hipError_t launch_ephem_eval(const EphemArgs& E, const double* t, int64_t n_q, double* out, hipStream_t s);
hipError_t fov_single_job_layout(int64_t* b_poff, int32_t* b_obj0, int64_t* b_xoff, int32_t* b_G, int64_t* b_koff,
                                 int64_t n_batch, int64_t n_obj, int G, hipStream_t s);
hipError_t fill_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace kete
