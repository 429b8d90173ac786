// Static description of the network and the per-call memory plan of the Radar-STDA library.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/stda.h"

namespace stda {

// Mobile encoder / decoder blocks: input / output widths, decoder flag, input / output level
// (level l = map downsampled by 2^l).
struct BlockCfg {
  int cin, cout;
  bool dec;
  int lin, lout;
};
constexpr BlockCfg kBlocks[4] = {
    {16, 32, false, 0, 1},  // encoder block 0
    {32, 64, false, 1, 2},  // encoder block 1
    {64, 32, true, 2, 1},   // decoder block 0
    {32, 16, true, 1, 0},   // decoder block 1
};

constexpr int kMaxSegs = 8;
constexpr int kMaxGrid = 2048;       // blocks of per-pixel kernels (bounds partial buffers)
constexpr int kTileGrid = 1024;      // blocks of the persistent LDS-tile kernels (4 per CU)
constexpr int kMaxTiles = 16;        // blocks per clip of per-clip kernels
constexpr int kMaxWgradGrid = 512;   // blocks of weight-gradient kernels
constexpr int kNumGradBufs = 13;

struct ParamEntry {
  char name[40];
  int64_t offset, count;
  int ndim;
  int shape[4];
  int fan_in;
};

struct BlockOffsets {
  int64_t pw_w, pw_g, pw_b, dw_w, dw_g, dw_b, id_g, id_b, main_w, main_g, main_b, res_w, eca_w;
  int64_t bn_pw, bn_dw, bn_id, bn_main;  // offsets into the running / statistics buffers
};

struct NetOffsets {
  int64_t stem_w, stem_g, stem_b, head_w, head_b;
  BlockOffsets blk[4];
  int64_t running_count, param_count;
};

// Architecture readings (STDA_ARCH_* bits) set by stda_set_arch; a call reads them once into its
// plan and passes that value on.
int current_arch();
const std::vector<ParamEntry>& param_table(int arch);
const NetOffsets& net_offsets(int arch);

// Byte offsets of one segment's activations (in `saved` for TRAIN, in `ws` for EVAL).
struct BlockActs {
  size_t X1, T, Y, Xn, a, g, mask;  // mask: stage-2 ReLU decisions, 4 bits per byte
  size_t m1;                        // stage-1 ReLU decisions (X1 > 0), 1 bit per element
  bool inner_in_ws;                 // X1, T, m1 live in ws (recomputed in the backward)
};
struct SegPlan {
  int n, H, W;
  int64_t x_off, z_off;
  size_t stats;  // [mean C][invstd C] per BN layer, running-buffer layout
  size_t s0;
  size_t zs;     // TRAIN with the sigmoid output: FP32 copy of z (in saved), else 0
  BlockActs blk[4];
  size_t scr;     // byte offset of the segment's region in the full-resolution scratch (ws_R, ws_g)
  int64_t clip0;  // clips of the segments before this one (per-clip scratch rows)
};

struct Plan {
  int n_segs, dtype, mode, arch;
  SegPlan seg[kMaxSegs];
  // ws regions (byte offsets)
  size_t ws_wk, ws_dense, ws_R, ws_part, ws_sums, ws_gap, ws_eval_stats, ws_loss;
  size_t ws_g[kNumGradBufs];
  size_t ws_coef_e, ws_coef, ws_ecaw, ws_wpart, ws_frag;
  int64_t dense_f[4][2], dense_d[4][2];  // element offsets inside ws_dense (main, residual)
  size_t ws_pwx;                         // depthwise 1x1 reading: diagonal C x C weights
  int64_t pwx_off[4];                    // element offsets inside ws_pwx per block
  size_t part_cap, wpart_cap;            // floats of ws_part and ws_wpart
  size_t saved_bytes, ws_bytes;
};

void build_plan(const stda_segment* segs, int n_segs, int dtype, int mode, int recompute, Plan& P);

}  // namespace stda
