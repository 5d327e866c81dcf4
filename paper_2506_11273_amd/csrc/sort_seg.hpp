// Device-side descriptors and workspace layout of the segmented radix sort.
#pragma once

#include "common.hpp"

namespace rr {

// One segment: keys [off, off + n) of the key array, its tiles starting at
// global tile index tile_off.  Segments are listed in increasing off and
// tile_off order.
struct SortSeg {
  uint32_t off, n, tile_off, ntiles;
};

struct SortHdr {
  uint32_t nseg, total_tiles, total_keys, pad;
};

// Digits chosen on the device for the most-significant-digit sort: dh the
// highest 8-bit digit in which the keys differ, dl the next one below it
// (any other digit when no lower one differs).
struct MsdPlan {
  uint32_t dh, dl, n;
  uint32_t big;  // nonzero when some (dh, dl) bucket holds more than kWaveCap keys
};

// hist holds hist_copies copies of every segment's digit histograms
// (passes x radix words each); a single-segment sort spreads its histogram
// flush over several copies, summed again by the scatter passes.
// The most-significant-digit sort (msd) adds: the plan, a header and 256
// segments (one per value of digit dh), their digit-dl histograms (hist2,
// 256 x 256 words, also the bucket sizes), the start of every (dh, dl)
// bucket (bstart), and look-back words for its two passes (status2, two
// passes of status2_stride words; gstatus2 likewise).
struct SegLayout {
  size_t keys_alt, idx_alt, hdr, segs, hist, counters, status, gstatus, total;
  size_t plan, hdr2, segs2, hist2, bstart, status2, gstatus2;
  uint32_t passes, tile, max_seg, max_tiles, status_stride, gstatus_stride, hist_copies;
  uint32_t status2_stride, gstatus2_stride;
  bool msd;
};

SegLayout seg_layout(int64_t n_max, uint32_t max_seg, uint32_t key_bits, uint32_t db, uint32_t kpt);
// Layout of the single-segment most-significant-digit sort (8-bit digits,
// kpt keys per thread in its two scatter passes).
SegLayout msd_layout(int64_t n_max, uint32_t key_bits, uint32_t kpt);
// The most-significant-digit sort exists for 64-bit keys below 2^27
// (msd_supported); rr_sort and the fused call run it only when asked to
// (force_msd), else the LSD sort.
bool msd_supported(int64_t n_max, uint32_t key_bits);

// Sorts every segment described by the device header and segment table
// hdr / segs.  With hdr == nullptr one segment of min(*count_dev, n_max)
// keys (n_max without count_dev) is set up on the device, in the workspace.
// counted: the scatter passes take tiles from a counter (for sorts that may
// share the device with other kernels) instead of in a fixed order.
// gather_out: the last pass also moves the rays into sorted order,
// gather_out[i] = gather_in[idx[i]] (gather_n rays in), and leaves the keys
// of that pass unwritten.
rr_status launch_seg_sort(void* keys, uint32_t* idx, const SegLayout& L, void* ws, SortHdr* hdr, SortSeg* segs,
                          const uint32_t* count_dev, uint32_t n_max, uint32_t key_bits, uint32_t db, uint32_t kpt,
                          bool counted, hipStream_t st, const rr_ray* gather_in = nullptr,
                          rr_ray* gather_out = nullptr, uint32_t gather_n = 0);

// The keys of rays[0, n) (as the keys kernel computes them for plan, with
// the identity index) sorted by the single-segment sort with 8-bit digits
// and kpt keys per thread, the histogram counted while the keys are
// computed, and the rays gathered into key order by the last pass
// (rays_out[i] = rays[idx[i]]).  keys / idx receive n entries; ws holds the
// sort workspace of seg_layout(n, 1, key bits, 8, kpt).  force_msd takes the
// most-significant-digit sort at any supported size.
rr_status launch_keys_sort_gather(const rr_ray* rays, int64_t n, const KeyPlan& plan, void* keys, uint32_t* idx,
                                  uint32_t kpt, void* ws, size_t ws_bytes, rr_ray* rays_out, hipStream_t st,
                                  bool force_msd = false);

// Runs the one-time occupancy queries of a sort configuration, so that a
// later stream capture records kernel launches only.
void sort_warm(uint32_t key_bits, uint32_t db, uint32_t kpt);

}  // namespace rr
