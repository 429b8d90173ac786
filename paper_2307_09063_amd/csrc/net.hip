// Host orchestration of the Radar-STDA forward / backward / loss / SGD behind the C ABI.
//
// Network (Radar-STDA, arXiv 2307.09063, Sec. IV): input module (Conv3x3 3->16, BN, ReLU on
// the channel concatenation of frames t, t-1, t-2), two mobile encoder blocks (16->32->64),
// two mobile decoder blocks (64->32->16), each block followed by ECA, skip additions of the
// same-size encoder features after the decoder blocks, output module Conv3x3 16->1 + bias.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/stda.h"
#include "dense_mfma.h"
#include "net_bwd_kernels.h"
#include "net_kernels.h"
#include "plan.h"
#include "s2_tile.h"
#include "stage1_tile.h"
#include "stem_tile.h"
#include "head_tile.h"
#include "eval_folded.h"

using namespace stda;

namespace {

thread_local int g_last_hip = 0;

#define HIP_TRY(expr)                         \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) {                   \
      g_last_hip = (int)e_;                   \
      return STDA_E_HIP;                      \
    }                                         \
  } while (0)
#define LAUNCH_CHECK() HIP_TRY(hipGetLastError())

// ------------------------------------------------------------------ per-kernel timing hook
// When a tag is selected, every launch carrying that tag is bracketed by two HIP events
// recorded on the launch stream; stda_profile_read sums their elapsed times.
struct Prof {
  std::mutex mu;
  std::string tag;  // "*" records every tagged launch
  bool on = false;
  std::vector<hipEvent_t> ev;
  std::vector<std::string> evtag;  // tag of each recorded pair
  size_t used = 0;
};
Prof& prof() {
  static Prof p;
  return p;
}
struct ProfScope {
  hipStream_t st;
  long idx = -1;
  ProfScope(const std::string& tag, hipStream_t s) : st(s) {
    Prof& p = prof();
    if (!p.on) return;
    std::lock_guard<std::mutex> lk(p.mu);
    if (p.tag != "*" && tag != p.tag) return;
    if (p.used + 2 > p.ev.size()) {
      for (int k = 0; k < 2; ++k) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        p.ev.push_back(e);
      }
    }
    idx = (long)p.used;
    p.used += 2;
    if (p.evtag.size() < p.used / 2) p.evtag.resize(p.used / 2);
    p.evtag[idx / 2] = tag;
    // a failed record only leaves this measurement out (stda_profile_read reports the error)
    (void)hipEventRecord(p.ev[idx], st);
  }
  ~ProfScope() {
    if (idx >= 0) (void)hipEventRecord(prof().ev[idx + 1], st);
  }
};
const char* const kBlockName[4] = {"enc0", "enc1", "dec0", "dec1"};
std::string tagk(const char* kind, int k) { return std::string(kind) + "." + kBlockName[k]; }

#define KLAUNCH(tag, ...)               \
  do {                                  \
    ProfScope ps_((tag), c.st);         \
    __VA_ARGS__;                        \
  } while (0);                          \
  LAUNCH_CHECK()

int grid_for(int64_t items, int cap = 2048) {
  int64_t g = (items + STDA_BLOCK - 1) / STDA_BLOCK;
  if (g < 1) g = 1;
  return (int)std::min<int64_t>(g, cap);
}

// Upper bound on the workgroups of the tiled network kernels (stda_set_grid_cap; 0 = none).  The
// kernels walk their tiles with a grid-stride (or XCD-chunked) schedule and keep accumulators
// across tiles, so a small cap makes every workgroup of a small batch take several tiles.
std::atomic<int> g_grid_cap{0};
int64_t capped(int64_t g) {
  const int c = g_grid_cap.load(std::memory_order_relaxed);
  return c > 0 ? std::min<int64_t>(g, c) : g;
}

// Workspace of stda_forward_noalloc: one array per GPU, resident until the process ends.  In host
// code its name is only a stand-in; kernels get the device address that hipGetSymbolAddress
// reports for the current device, looked up once per device and kept here.
static __device__ __align__(256) unsigned char scratch[STDA_NOALLOC_WS_MAX];

int noalloc_scratch(hipStream_t stream, char** out) {
  static std::mutex mu;
  static std::vector<char*> addr;  // per device ordinal
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (stream) {
    hipDevice_t sdev = 0;
    HIP_TRY(hipStreamGetDevice(stream, &sdev));
    if ((int)sdev != dev) return STDA_E_INVALID;  // the stream must belong to the current device
  }
  std::lock_guard<std::mutex> lk(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return STDA_E_HIP;
    addr[dev] = static_cast<char*>(p);
  }
  *out = addr[dev];
  return STDA_OK;
}

}  // namespace

namespace stda {

// ------------------------------------------------------------------- parameter table
std::atomic<int> g_arch{0};  // STDA_ARCH_* bits, see stda_set_arch
int current_arch() { return g_arch.load(std::memory_order_relaxed); }

static std::vector<ParamEntry> build_param_table(int arch) {
  std::vector<ParamEntry> t;
  int64_t off = 0;
  auto add = [&](const std::string& name, std::vector<int> shape, int fan_in) {
    ParamEntry e{};
    std::snprintf(e.name, sizeof(e.name), "%s", name.c_str());
    e.offset = off;
    e.ndim = (int)shape.size();
    int64_t n = 1;
    for (int i = 0; i < e.ndim; ++i) {
      e.shape[i] = shape[i];
      n *= shape[i];
    }
    e.fan_in = fan_in;
    e.count = n;
    off += n;
    t.push_back(e);
  };
  const int rk = (arch & STDA_ARCH_RES3) ? 3 : 4;  // decoder long-residual kernel
  const bool pw_dw = (arch & STDA_ARCH_PW_DW) != 0;  // stage-1 1x1 branch depthwise
  add("stem.conv.w", {16, 3, 3, 3}, 27);
  add("stem.bn.gamma", {16}, 0);
  add("stem.bn.beta", {16}, 0);
  const char* names[4] = {"enc0", "enc1", "dec0", "dec1"};
  for (int k = 0; k < 4; ++k) {
    const BlockCfg& b = kBlocks[k];
    const int c = b.cin, co = b.cout;
    const std::string n = names[k];
    if (pw_dw)
      add(n + ".s1.pw.w", {c, 1, 1, 1}, 1);
    else
      add(n + ".s1.pw.w", {c, c, 1, 1}, c);
    add(n + ".s1.pw_bn.gamma", {c}, 0);
    add(n + ".s1.pw_bn.beta", {c}, 0);
    add(n + ".s1.dw.w", {c, 1, 3, 3}, 9);
    add(n + ".s1.dw_bn.gamma", {c}, 0);
    add(n + ".s1.dw_bn.beta", {c}, 0);
    add(n + ".s1.id_bn.gamma", {c}, 0);
    add(n + ".s1.id_bn.beta", {c}, 0);
    if (b.dec)
      add(n + ".s2.main.w", {c, co, 4, 4}, c * 16);
    else
      add(n + ".s2.main.w", {co, c, 3, 3}, c * 9);
    add(n + ".s2.main_bn.gamma", {co}, 0);
    add(n + ".s2.main_bn.beta", {co}, 0);
    if (b.dec)
      add(n + ".s2.res.w", {c, co, rk, rk}, c * rk * rk);
    else
      add(n + ".s2.res.w", {co, c, 3, 3}, c * 9);
    add(n + ".eca.w", {3}, 3);
  }
  add("head.conv.w", {1, 16, 3, 3}, 144);
  add("head.conv.b", {1}, 0);
  return t;
}

// One table per combination of readings (the output nonlinearity leaves it unchanged).
constexpr int kArchCombos = 8;
const std::vector<ParamEntry>& param_table(int arch) {
  static const std::vector<ParamEntry> tab[kArchCombos] = {build_param_table(0), build_param_table(1),
                                                          build_param_table(2), build_param_table(3),
                                                          build_param_table(4), build_param_table(5),
                                                          build_param_table(6), build_param_table(7)};
  return tab[arch & (kArchCombos - 1)];
}

static int64_t param_offset(const std::vector<ParamEntry>& t, const std::string& name) {
  for (const auto& e : t)
    if (name == e.name) return e.offset;
  return -1;
}

static NetOffsets build_net_offsets(int arch) {
  const std::vector<ParamEntry>& t = param_table(arch);
  NetOffsets n{};
  n.stem_w = param_offset(t, "stem.conv.w");
  n.stem_g = param_offset(t, "stem.bn.gamma");
  n.stem_b = param_offset(t, "stem.bn.beta");
  const char* names[4] = {"enc0", "enc1", "dec0", "dec1"};
  int64_t run = 32;  // stem BN occupies running[0..32)
  for (int k = 0; k < 4; ++k) {
    const std::string p = names[k];
    BlockOffsets& b = n.blk[k];
    b.pw_w = param_offset(t, p + ".s1.pw.w");
    b.pw_g = param_offset(t, p + ".s1.pw_bn.gamma");
    b.pw_b = param_offset(t, p + ".s1.pw_bn.beta");
    b.dw_w = param_offset(t, p + ".s1.dw.w");
    b.dw_g = param_offset(t, p + ".s1.dw_bn.gamma");
    b.dw_b = param_offset(t, p + ".s1.dw_bn.beta");
    b.id_g = param_offset(t, p + ".s1.id_bn.gamma");
    b.id_b = param_offset(t, p + ".s1.id_bn.beta");
    b.main_w = param_offset(t, p + ".s2.main.w");
    b.main_g = param_offset(t, p + ".s2.main_bn.gamma");
    b.main_b = param_offset(t, p + ".s2.main_bn.beta");
    b.res_w = param_offset(t, p + ".s2.res.w");
    b.eca_w = param_offset(t, p + ".eca.w");
    const int c = kBlocks[k].cin, co = kBlocks[k].cout;
    b.bn_pw = run;
    run += 2 * c;
    b.bn_dw = run;
    run += 2 * c;
    b.bn_id = run;
    run += 2 * c;
    b.bn_main = run;
    run += 2 * co;
  }
  n.head_w = param_offset(t, "head.conv.w");
  n.head_b = param_offset(t, "head.conv.b");
  n.running_count = run;
  n.param_count = t.back().offset + t.back().count;
  return n;
}

const NetOffsets& net_offsets(int arch) {
  static const NetOffsets o[kArchCombos] = {build_net_offsets(0), build_net_offsets(1), build_net_offsets(2),
                                            build_net_offsets(3), build_net_offsets(4), build_net_offsets(5),
                                            build_net_offsets(6), build_net_offsets(7)};
  return o[arch & (kArchCombos - 1)];
}

}  // namespace stda

// ===================================================================== weight preparation
namespace {

// Dense stride-2 weights re-laid out for the implicit-GEMM kernels:
//   fwd   [tap][K = layer input channels][N = layer output channels]
//   dgrad [tap][K = layer output channels][N = layer input channels]
// Conv weights are [Cout][Cin][3][3], deconv weights [Cin][Cout][4][4].
struct PrepJob {
  int dec, cin, cout;
  int64_t src, dst_f, dst_d;
};
struct PrepJobs {
  int n;
  int bf16;
  PrepJob j[8];
};

__global__ void k_prep_dense(const float* __restrict__ w, float* __restrict__ out, PrepJobs jobs) {
  const PrepJob J = jobs.j[blockIdx.y];
  const int ks = J.dec ? 4 : 3, taps = ks * ks;
  const int64_t total = (int64_t)taps * J.cin * J.cout;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    // i enumerates the PyTorch layout
    int64_t r = i;
    const int t = (int)(r % taps);
    r /= taps;
    int ci, co;
    if (J.dec) {
      co = (int)(r % J.cout);
      ci = (int)(r / J.cout);
    } else {
      ci = (int)(r % J.cin);
      co = (int)(r / J.cin);
    }
    float v = w[J.src + i];
    if (jobs.bf16) v = round_bf16(v);
    out[J.dst_f + ((int64_t)t * J.cin + ci) * J.cout + co] = v;
    out[J.dst_d + ((int64_t)t * J.cout + co) * J.cin + ci] = v;
  }
}

// Working copy of all parameters; in BF16 mode the listed ranges are rounded to BF16.
struct RoundRanges {
  int n;
  int64_t off[24];
  int64_t cnt[24];
};
__global__ void k_working_weights(const float* __restrict__ w, float* __restrict__ wk, int64_t n, RoundRanges rr) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float v = w[i];
    for (int r = 0; r < rr.n; ++r)
      if (i >= rr.off[r] && i < rr.off[r] + rr.cnt[r]) v = round_bf16(v);
    wk[i] = v;
  }
}

// Depthwise 1x1 reading: the per-channel weights of each block's 1x1 branch written as the
// diagonal of a dense C x C matrix, so that the dense pointwise kernels compute exactly the
// depthwise branch (the off-diagonal products are exact zeros).
struct PwDiag {
  int64_t src[4], dst[4];
  int C[4];
};
__global__ void k_pw_diag(const float* __restrict__ w, float* __restrict__ out, PwDiag d) {
  const int k = blockIdx.y, C = d.C[k];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < C * C; i += gridDim.x * blockDim.x) {
    const int r = i / C, q = i % C;
    out[d.dst[k] + i] = r == q ? w[d.src[k] + r] : 0.f;
  }
}

}  // namespace

// ===================================================================== plan
namespace stda {

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

struct Bump {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  }
};

void build_plan(const stda_segment* segs, int n_segs, int dtype, int mode, int recompute, Plan& P) {
  P = Plan{};
  P.n_segs = n_segs;
  P.dtype = dtype;
  P.mode = mode;
  P.arch = current_arch();
  const bool sigmoid_save = (P.arch & STDA_ARCH_SIGMOID) && mode == STDA_TRAIN;
  const size_t es = dtype == STDA_BF16 ? 2 : 4;
  Bump sv, ws;
  const bool train = mode == STDA_TRAIN;
  Bump& acts = train ? sv : ws;
  // per-call scratch shared by all segments
  P.ws_wk = ws.take(sizeof(float) * net_offsets(P.arch).param_count);
  int64_t dense_elems = 0;
  for (int k = 0; k < 4; ++k) {
    const BlockCfg& b = kBlocks[k];
    const int64_t per = (int64_t)(b.dec ? 16 : 9) * b.cin * b.cout;
    for (int m = 0; m < 2; ++m) {
      P.dense_f[k][m] = dense_elems;
      dense_elems += per;
      P.dense_d[k][m] = dense_elems;
      dense_elems += per;
    }
  }
  P.ws_dense = ws.take(sizeof(float) * dense_elems);
  int64_t pwx = 0;
  for (int k = 0; k < 4; ++k) {
    P.pwx_off[k] = pwx;
    pwx += (int64_t)kBlocks[k].cin * kBlocks[k].cin;
  }
  P.ws_pwx = ws.take(sizeof(float) * pwx);
  P.ws_frag = ws.take(sizeof(float) * dense_elems);  // same element offsets as ws_dense
  // per-segment regions: full-resolution scratch by pixels, per-clip scratch by clips
  int64_t tot_pix = 0, tot_clips = 0;
  size_t part_cap = 0;
  for (int s = 0; s < n_segs; ++s) {
    P.seg[s].scr = es * 16 * (size_t)tot_pix;
    P.seg[s].clip0 = tot_clips;
    tot_pix += (int64_t)segs[s].n * segs[s].H * segs[s].W;
    tot_clips += segs[s].n;
    // per-block partials: up to 9 x 64 floats (+ a count) per block of a per-pixel kernel, or
    // 2 x 64 per (clip, tile) block of the per-clip stage-2 adjoint; regions with counts are
    // aligned to 64 floats
    part_cap += std::max<size_t>((size_t)kMaxGrid * (9 * 64 + 1), (size_t)segs[s].n * kMaxTiles * (2 * 64 + 1)) + 64;
  }
  const size_t full16 = es * 16 * (size_t)tot_pix;  // largest per-level activation of all segments
  P.ws_R = ws.take(full16);
  P.part_cap = part_cap;
  P.ws_part = ws.take(sizeof(float) * part_cap);
  P.ws_sums = ws.take(sizeof(double) * 6 * 64);
  P.ws_gap = ws.take(sizeof(float) * (size_t)tot_clips * kMaxTiles * 64);
  P.ws_eval_stats = ws.take(sizeof(float) * stda_running_count());
  P.ws_loss = ws.take(sizeof(double) * kMaxGrid);
  P.wpart_cap = 0;
  if (train) {
    for (int i = 0; i < kNumGradBufs; ++i) P.ws_g[i] = ws.take(full16);
    P.ws_coef_e = ws.take(sizeof(float) * (size_t)tot_clips * 64);
    P.ws_coef = ws.take(sizeof(float) * (size_t)n_segs * 4 * 64);
    P.ws_ecaw = ws.take(sizeof(float) * (size_t)tot_clips * 3);
    // weight-gradient partial rows of one launch: at most kMaxWgradGrid x 32768 floats a segment
    P.wpart_cap = (size_t)n_segs * kMaxWgradGrid * 32768;
    P.ws_wpart = ws.take(sizeof(float) * P.wpart_cap);
  }
  const bool rec = train && recompute;
  for (int s = 0; s < n_segs; ++s) {
    SegPlan& S = P.seg[s];
    const int64_t n = segs[s].n, H = segs[s].H, W = segs[s].W;
    S.n = (int)n;
    S.H = (int)H;
    S.W = (int)W;
    S.x_off = segs[s].x_off;
    S.z_off = segs[s].z_off;
    const int64_t HW = H * W;
    S.stats = (train ? sv : ws).take(sizeof(float) * stda_running_count());
    S.s0 = acts.take(es * 16 * n * HW);
    S.zs = sigmoid_save ? sv.take(sizeof(float) * n * HW) : 0;
    // recompute: one scratch set of block internals in ws per segment, shared by its blocks
    size_t rx1 = 0, rt = 0, rm1 = 0;
    if (rec) {
      size_t mx1 = 0, mty = 0;
      for (int k = 0; k < 4; ++k) {
        const BlockCfg& b = kBlocks[k];
        mx1 = std::max(mx1, (size_t)b.cin * n * (H >> b.lin) * (W >> b.lin));
        mty = std::max(mty, (size_t)b.cout * n * (H >> b.lout) * (W >> b.lout));
      }
      rx1 = ws.take(es * mx1);
      rm1 = ws.take(mx1 / 8);
      rt = ws.take(es * mty);
    }
    for (int k = 0; k < 4; ++k) {
      const BlockCfg& b = kBlocks[k];
      const int64_t hin = H >> b.lin, win = W >> b.lin, hout = H >> b.lout, wout = W >> b.lout;
      BlockActs& A = S.blk[k];
      A.inner_in_ws = rec;
      if (rec) {
        A.X1 = rx1;
        A.T = rt;
        A.m1 = rm1;
      } else {
        A.X1 = acts.take(es * b.cin * n * hin * win);
        A.T = acts.take(es * b.cout * n * hout * wout);
        A.m1 = train ? acts.take((size_t)b.cin * n * hin * win / 8) : 0;
      }
      // the block output before ECA and the stage-2 ReLU decisions are kept in both modes: the
      // recompute rebuilds the rest of the block (x1, its decisions, t) from the block input
      A.Y = acts.take(es * b.cout * n * hout * wout);
      A.mask = train ? acts.take((size_t)b.cout * n * hout * wout / 4) : 0;
      A.Xn = acts.take(es * b.cout * n * hout * wout);
      A.a = acts.take(sizeof(float) * b.cout * n);
      A.g = acts.take(sizeof(float) * b.cout * n);
    }
  }
  P.saved_bytes = train ? sv.off : 0;
  P.ws_bytes = ws.off;
}

}  // namespace stda

// ===================================================================== forward
namespace {

// Consecutive per-segment regions of a partial-sums buffer (one region per segment of a launch).
// Regions without per-row counts follow each other with no gap, so a column sum over all rows
// of all segments is one reduction; regions with counts start on 256-byte boundaries.
struct Parts {
  float* base;
  size_t cap, used = 0;  // floats
  int n = 0;
  bool over = false;     // a region did not fit: nothing may be launched with these regions
  float* p[kMaxSegs] = {};
  int rows[kMaxSegs] = {};
  Parts(float* b, size_t c) : base(b), cap(c) {}
  // the next segment's region: r rows of `row` floats, followed (counts) by one count per row
  float* take(int r, int64_t row, bool counts) {
    if (counts) used = (used + 63) & ~(size_t)63;
    const size_t need = (size_t)r * (size_t)row + (counts ? (size_t)r : 0);
    if (n >= kMaxSegs || used + need > cap) {
      over = true;
      return base;
    }
    p[n] = base + used;
    rows[n] = r;
    used += need;
    return p[n++];
  }
  int total_rows() const {
    int t = 0;
    for (int i = 0; i < n; ++i) t += rows[i];
    return t;
  }
};

// The arguments of one launch over all segments (see SegL): segment s's workgroups start at the
// first multiple of 8 after the previous segment's.
template <class A>
struct Batch {
  SegL<A> L{};
  int end = 0;
  void add(int grid, const A& a) {
    const int s = L.n++;
    L.base[s] = (end + 7) & ~7;
    L.grid[s] = grid;
    L.a[s] = a;
    end = L.base[s] + grid;
  }
  unsigned blocks() const { return (unsigned)end; }
};

template <class T>
struct Ctx {
  const Plan* P;
  char* sv;  // activations base (saved in TRAIN, ws in EVAL)
  char* ws;
  const float* w;   // working weights (rounded in BF16 mode)
  const float* dl;  // dense layouts
  hipStream_t st;
  bool train;
  bool rec_pass = false;  // re-running a block's forward inside the backward (recompute mode)
  int ns() const { return P->n_segs; }
  const SegPlan& S(int s) const { return P->seg[s]; }
  template <class U> U* act(size_t off) const { return reinterpret_cast<U*>(sv + off); }
  template <class U> U* inner(const BlockActs& A, size_t off) const {
    return reinterpret_cast<U*>((A.inner_in_ws ? ws : sv) + off);
  }
  template <class U> U* scr(size_t off) const { return reinterpret_cast<U*>(ws + off); }
  float* stats(int s, int64_t bn_off) const {
    return reinterpret_cast<float*>((train ? sv : ws) + P->seg[s].stats) + bn_off;
  }
  // segment s's regions of the per-call scratch
  T* R(int s) const { return scr<T>(P->ws_R + P->seg[s].scr); }
  T* grad(int s, int i) const { return scr<T>(P->ws_g[i] + P->seg[s].scr); }
  float* gap(int s) const { return scr<float>(P->ws_gap) + P->seg[s].clip0 * kMaxTiles * 64; }
  float* coef(int s) const { return scr<float>(P->ws_coef) + (size_t)s * 4 * 64; }
  float* coef_e(int s) const { return scr<float>(P->ws_coef_e) + P->seg[s].clip0 * 64; }
  float* ecaw(int s) const { return scr<float>(P->ws_ecaw) + P->seg[s].clip0 * 3; }
  Parts part() const { return Parts(scr<float>(P->ws_part), P->part_cap); }
  Parts wpart() const { return Parts(scr<float>(P->ws_wpart), P->wpart_cap); }
  int clips() const {
    int t = 0;
    for (int s = 0; s < P->n_segs; ++s) t += P->seg[s].n;
    return t;
  }
};

// One segment's operands of a dense stage-2 launch.
template <class T>
struct DenseOps {
  int n = 0;
  const T* src[kMaxSegs];
  T* dst[kMaxSegs];
  int clips[kMaxSegs], hd[kMaxSegs], wd[kMaxSegs];
  void add(const T* s, T* d, int b, int h, int w) {
    src[n] = s;
    dst[n] = d;
    clips[n] = b;
    hd[n] = h;
    wd[n] = w;
    ++n;
  }
};

int tiles_for(int64_t hw, int G) {
  const int64_t item_blocks = (hw * G + STDA_BLOCK - 1) / STDA_BLOCK;
  return (int)std::max<int64_t>(1, capped(std::min<int64_t>(kMaxTiles, (item_blocks + 3) / 4)));
}

// Tiling variant of each tunable launch, [dtype][kind][block]: kinds 0 forward, 1 input gradient
// of the dense stage-2 layers (0..2 the LDS-tiled kernel with the tilings listed in
// launch_s2_variant, 3 the register-gather kernel), 2 their weight gradient (tilings listed in
// launch_wgrad), 3 the fused stage-1 adjoint (tilings listed in launch_s1b).  Set by
// stda_tune_set (the autotuner); 0 by default.  Atomic entries: a call that plans while another
// thread tunes reads each entry whole (which tiling a launch gets is then up to the ordering).
constexpr int kS2Variants = 4;
constexpr int kTuneKinds = 4;
constexpr double kTuneMargin = 0.03;
std::atomic<int> g_s2_variant[2][kTuneKinds][4] = {};
int tuned(int dtype_idx, int kind, int blk) {
  return g_s2_variant[dtype_idx][kind][blk].load(std::memory_order_relaxed);
}
void set_tuned(int dtype_idx, int kind, int blk, int v) {
  g_s2_variant[dtype_idx][kind][blk].store(v, std::memory_order_relaxed);
}

// Dense stride-2 layer on LDS tiles over every segment; with STATS, each segment's BN partials
// go to a region of *pm.
template <class T, int OP, int K, int N, int NB, int TH, int TW, bool STATS, int WV = 4>
int launch_s2_cfg(const Ctx<T>& c, const std::string& tag, const DenseOps<T>& D, const T* frag, Parts* pm) {
  typedef S2Cfg<T, OP, K, N, NB, TH, TW, WV> C;
  const int64_t per_cu = std::max<int64_t>(1, (160 * 1024) / C::LDS_BYTES);
  Batch<k_s2_tile_args<T, OP, K, N, NB, TH, TW, STATS, WV>> b;
  for (int s = 0; s < D.n; ++s) {
    const int64_t ntiles = (int64_t)D.clips[s] * ((D.hd[s] + TH - 1) / TH) * ((D.wd[s] + TW - 1) / TW);
    int64_t gx = capped(std::min<int64_t>(ntiles, std::min<int64_t>(256 * per_cu * 2, kMaxGrid)));
    if (gx >= 64) gx &= ~(int64_t)7;  // whole XCD groups: tiles are handed out XCD by XCD
    gx = std::max<int64_t>(gx, 1);
    float* part = nullptr;
    if constexpr (STATS) part = pm->take((int)gx, 2 * N, true);
    b.add((int)gx, {D.src[s], frag, D.dst[s], part, D.clips[s], D.hd[s], D.wd[s]});
  }
  if (STATS && pm->over) return STDA_E_WORKSPACE;
  KLAUNCH(tag, k_s2_tile<T, OP, K, N, NB, TH, TW, STATS, WV><<<dim3(b.blocks(), N / NB), C::BLK, 0, c.st>>>(b.L));
  return STDA_OK;
}

template <class T, int OP, int K, int N, bool STATS>
int launch_gather(const Ctx<T>& c, const std::string& tag, const DenseOps<T>& D, const T* frag, Parts* pm) {
  constexpr int R = 4;
  constexpr bool down = OpGeo<OP>::DOWN;
  const int phases = down ? 1 : 4;
  Batch<k_dense_mfma_args<T, OP, K, N, R, STATS>> b;
  for (int s = 0; s < D.n; ++s) {
    const int64_t hd = D.hd[s], wd = D.wd[s];
    const int64_t P = (int64_t)D.clips[s] * (down ? hd * wd : (hd / 2) * (wd / 2));
    const int64_t tiles = (P + 64 * R - 1) / (64 * R);
    const int gx = (int)std::max<int64_t>(1, capped(std::min<int64_t>(tiles, kMaxGrid / phases)));
    float* part = nullptr;
    if constexpr (STATS) part = pm->take(gx * phases, 2 * N, true);
    b.add(gx, {D.src[s], frag, D.dst[s], part, D.clips[s], D.hd[s], D.wd[s]});
  }
  if (STATS && pm->over) return STDA_E_WORKSPACE;
  KLAUNCH(tag, k_dense_mfma<T, OP, K, N, R, STATS><<<dim3(b.blocks(), phases), 256, 0, c.st>>>(b.L));
  return STDA_OK;
}

// The candidate tilings (NB output channels per workgroup, TH x TW output pixels) of each
// operator; all fit the 160 KB of LDS of a gfx950 workgroup (checked at compile time).
template <class T, int OP, int K, int N, bool STATS>
int launch_s2_variant(int v, const Ctx<T>& c, const std::string& tag, const DenseOps<T>& D, const T* frag,
                      Parts* pm) {
  constexpr bool BF = sizeof(T) == 2;
#define S2V(NB_, TH_, TW_) launch_s2_cfg<T, OP, K, N, NB_, TH_, TW_, STATS>(c, tag, D, frag, pm)
  // 8 waves per workgroup: tilings whose LDS leaves room for one workgroup per CU
#define S2W(NB_, TH_, TW_) \
  launch_s2_cfg<T, OP, K, N, NB_, TH_, TW_, STATS, 8>(c, tag, D, frag, pm)
  if (v == 3) return launch_gather<T, OP, K, N, STATS>(c, tag, D, frag, pm);
  if constexpr (OP == OP_ENC_FWD && K == 16) {
    if constexpr (BF) return v == 1 ? S2V(32, 8, 16) : v == 2 ? S2W(32, 16, 16) : S2V(32, 8, 32);
    else return v == 1 ? S2V(32, 8, 8) : v == 2 ? S2W(32, 8, 16) : S2V(32, 8, 16);
  } else if constexpr (OP == OP_ENC_FWD) {
    if constexpr (BF) return v == 1 ? S2V(64, 8, 8) : v == 2 ? S2W(32, 8, 16) : S2V(64, 8, 16);
    else return v == 1 ? S2V(64, 8, 8) : v == 2 ? S2W(16, 8, 16) : S2V(32, 8, 8);
  } else if constexpr (OP == OP_DEC_FWD && K == 64) {
    if constexpr (BF) return v == 1 ? S2V(16, 16, 16) : v == 2 ? S2W(32, 16, 32) : S2V(32, 16, 16);
    else return v == 1 ? S2V(16, 32, 16) : v == 2 ? S2W(16, 16, 32) : S2V(16, 16, 16);
  } else if constexpr (OP == OP_DEC_FWD) {
    if constexpr (BF) return v == 1 ? S2V(16, 16, 16) : v == 2 ? S2W(16, 32, 32) : S2V(16, 16, 32);
    else return v == 1 ? S2V(16, 16, 32) : v == 2 ? S2W(16, 32, 32) : S2V(16, 16, 16);
  } else if constexpr (OP == OP_ENC_DGRAD && K == 32) {
    if constexpr (BF) return v == 1 ? S2V(16, 16, 16) : v == 2 ? S2W(16, 32, 32) : S2V(16, 16, 32);
    else return v == 1 ? S2V(16, 16, 32) : v == 2 ? S2W(16, 32, 32) : S2V(16, 16, 16);
  } else if constexpr (OP == OP_ENC_DGRAD) {
    if constexpr (BF) return v == 1 ? S2V(16, 16, 16) : v == 2 ? S2V(32, 16, 32) : S2V(32, 16, 16);
    else return v == 1 ? S2V(32, 16, 16) : v == 2 ? S2W(16, 16, 32) : S2V(16, 16, 16);
  } else if constexpr (OP == OP_DEC_DGRAD && K == 32) {
    if constexpr (BF) return v == 1 ? S2V(32, 8, 8) : v == 2 ? S2V(32, 8, 16) : S2V(64, 8, 8);
    else return v == 1 ? S2V(32, 8, 8) : v == 2 ? S2W(16, 8, 16) : S2V(16, 8, 8);
  } else {
    if constexpr (BF) return v == 1 ? S2V(32, 8, 8) : v == 2 ? S2W(32, 16, 16) : S2V(32, 8, 16);
    else return v == 1 ? S2W(32, 8, 16) : v == 2 ? S2V(16, 8, 16) : S2V(32, 8, 8);
  }
#undef S2V
#undef S2W
}

// Dense stride-2 layer of block `blk` on the matrix cores over every segment, with the tiling the
// tuner chose for it; with STATS the BN partials go to *pm.
template <class T, int OP, int K, int N, bool STATS>
int launch_dense(const Ctx<T>& c, int blk, const std::string& tag, const DenseOps<T>& D, int64_t frag_off, Parts* pm) {
  const T* frag = c.template scr<T>(c.P->ws_frag) + frag_off;
  const bool dgrad = OP == OP_ENC_DGRAD || OP == OP_DEC_DGRAD;
  const int v = tuned(sizeof(T) == 2 ? 1 : 0, dgrad ? 1 : 0, blk);
  return launch_s2_variant<T, OP, K, N, STATS>(v, c, tag, D, frag, pm);
}

// Blocks of the tiled stage-1 kernels: one per tile, at most kMaxGrid (they loop over tiles).
template <int C>
int s1_grid(int n, int h, int w) {
  const int64_t tiles = (int64_t)n * ((h + S1Tile<C>::TH - 1) / S1Tile<C>::TH) * ((w + S1Tile<C>::TW - 1) / S1Tile<C>::TW);
  return (int)std::max<int64_t>(1, capped(std::min<int64_t>(tiles, kTileGrid)));
}

// Blocks of the tiled input-module kernels (8 x 32 pixel tiles), at most kTileGrid.
int stem_grid(int n, int H, int W) {
  const int64_t tiles = (int64_t)n * ((H + 7) / 8) * ((W + 31) / 32);
  return (int)std::max<int64_t>(1, capped(std::min<int64_t>(tiles, kTileGrid)));
}

// Blocks of the tiled output-module kernels, at most kTileGrid.
int head_grid(int n, int H, int W) {
  const int64_t tiles = (int64_t)n * ((H + kHeadTH - 1) / kHeadTH) * ((W + kHeadTW - 1) / kHeadTW);
  return (int)std::max<int64_t>(1, capped(std::min<int64_t>(tiles, kTileGrid)));
}

// FP64 merge of the per-block BN statistics (count, mean, m2) followed by the finalize, for every
// segment of the launch whose partials are in pm; NB layers of C channels at the given offsets
// of the statistics layout.  `running` (null: no update) gets one update per segment.
template <class T>
int bn_finalize(const Ctx<T>& c, const Parts& pm, int NB, int C, const int64_t* bn_off, float* running) {
  BnSegs sg{};
  sg.n = pm.n;
  for (int s = 0; s < pm.n; ++s) {
    sg.part[s] = pm.p[s];
    sg.rows[s] = pm.rows[s];
    sg.stats[s] = c.stats(s, 0);
  }
  BnLayers L{};
  for (int i = 0; i < NB; ++i) L.off[i] = bn_off[i];
  KLAUNCH("bn_finalize", k_bn_stats_reduce<<<NB * C, 256, 0, c.st>>>(sg, NB, C, L, running));
  return STDA_OK;
}

// One segment's operands of mobile block k.
template <class T>
struct BlockView {
  int n, hin, win, hout, wout;
  const T* X;  // block input
  T *X1, *Tm, *Y, *Xn;
  uint8_t *m1, *mask;  // ReLU decisions (TRAIN), else null
  float *a, *g;        // ECA scale and average (saved)
  const T* skip;       // decoder blocks: the encoder output added to the block output
};
template <class T>
BlockView<T> block_view(const Ctx<T>& c, int s, int k) {
  const BlockCfg& bc = kBlocks[k];
  const SegPlan& S = c.S(s);
  const BlockActs& A = S.blk[k];
  BlockView<T> v;
  v.n = S.n;
  v.hin = S.H >> bc.lin;
  v.win = S.W >> bc.lin;
  v.hout = S.H >> bc.lout;
  v.wout = S.W >> bc.lout;
  v.X = k == 0 ? c.template act<T>(S.s0) : c.template act<T>(S.blk[k - 1].Xn);
  v.X1 = c.template inner<T>(A, A.X1);
  v.Tm = c.template inner<T>(A, A.T);
  v.Y = c.template act<T>(A.Y);
  v.Xn = c.template act<T>(A.Xn);
  v.m1 = c.train ? c.template inner<uint8_t>(A, A.m1) : nullptr;
  v.mask = c.train ? c.template act<uint8_t>(A.mask) : nullptr;
  v.a = c.template act<float>(A.a);
  v.g = c.template act<float>(A.g);
  v.skip = k == 2 ? c.template act<T>(S.blk[0].Xn) : (k == 3 ? c.template act<T>(S.s0) : nullptr);
  return v;
}

// Stage-1 parameters of block k with segment s's statistics.
template <class T>
S1Params s1_params(const Ctx<T>& c, int s, int k) {
  const BlockOffsets& bo = net_offsets(c.P->arch).blk[k];
  S1Params sp{};
  sp.wpw = (c.P->arch & STDA_ARCH_PW_DW) ? c.template scr<float>(c.P->ws_pwx) + c.P->pwx_off[k] : c.w + bo.pw_w;
  sp.wdw = c.w + bo.dw_w;
  sp.stats[0] = c.stats(s, bo.bn_pw);
  sp.stats[1] = c.stats(s, bo.bn_dw);
  sp.stats[2] = c.stats(s, bo.bn_id);
  sp.gamma[0] = c.w + bo.pw_g;
  sp.gamma[1] = c.w + bo.dw_g;
  sp.gamma[2] = c.w + bo.id_g;
  sp.beta[0] = c.w + bo.pw_b;
  sp.beta[1] = c.w + bo.dw_b;
  sp.beta[2] = c.w + bo.id_b;
  return sp;
}

// ECA scale of each clip and the next block input Xn = a * Y (+ skip) over every segment; the
// GAP partials of segment s are gap(s, clip) = gaps[s] + clip * gap_tiles[s] * COUT.
template <class T, int COUT, bool SKIP>
int launch_eca_next(const Ctx<T>& c, int k, const BlockView<T>* v, float* const* gaps, const int* gap_tiles,
                    const float* weca) {
  Batch<k_eca_next_args<T, COUT, SKIP>> b;
  for (int s = 0; s < c.ns(); ++s) {
    const int hw = v[s].hout * v[s].wout, tiles = tiles_for(hw, COUT / 4);
    b.add(tiles * v[s].n, {v[s].Y, v[s].skip, v[s].Xn, gaps[s], weca, v[s].g, v[s].a, hw, gap_tiles[s], tiles});
  }
  KLAUNCH(tagk("eca_next", k), k_eca_next<T, COUT, SKIP><<<b.blocks(), 256, 0, c.st>>>(b.L));
  return STDA_OK;
}

template <class T, int CIN, int COUT, bool DEC>
int fwd_block(const Ctx<T>& c, int k, float* running) {
  const BlockOffsets& bo = net_offsets(c.P->arch).blk[k];
  const int ns = c.ns();
  BlockView<T> v[kMaxSegs];
  S1Params sp[kMaxSegs];
  for (int s = 0; s < ns; ++s) {
    v[s] = block_view(c, s, k);
    sp[s] = s1_params(c, s, k);
  }
  // stage 1
  const bool stats_pass = c.train && !c.rec_pass;
  if (stats_pass) {
    Parts pm = c.part();
    Batch<k_s1_tile_args<T, CIN, DEC, 0>> b;
    for (int s = 0; s < ns; ++s) {
      const int g = s1_grid<CIN>(v[s].n, v[s].hin, v[s].win);
      b.add(g, {v[s].X, nullptr, nullptr, pm.take(g, 6 * CIN, true), sp[s], v[s].n, v[s].hin, v[s].win});
    }
    if (pm.over) return STDA_E_WORKSPACE;
    KLAUNCH(tagk("s1_stats", k), k_s1_tile<T, CIN, DEC, 0><<<b.blocks(), 256, 0, c.st>>>(b.L));
    const int64_t offs[3] = {bo.bn_pw, bo.bn_dw, bo.bn_id};
    if (int r = bn_finalize(c, pm, 3, CIN, offs, running)) return r;
  }
  {
    Batch<k_s1_tile_args<T, CIN, DEC, 1>> b;
    for (int s = 0; s < ns; ++s)
      b.add(s1_grid<CIN>(v[s].n, v[s].hin, v[s].win),
            {v[s].X, v[s].X1, v[s].m1, nullptr, sp[s], v[s].n, v[s].hin, v[s].win});
    KLAUNCH(tagk("s1_apply", k), k_s1_tile<T, CIN, DEC, 1><<<b.blocks(), 256, 0, c.st>>>(b.L));
  }
  // stage 2: main (with statistics) and residual
  constexpr int OPF = DEC ? OP_DEC_FWD : OP_ENC_FWD;
  DenseOps<T> dm, dr;
  for (int s = 0; s < ns; ++s) {
    dm.add(v[s].X1, v[s].Tm, v[s].n, v[s].hout, v[s].wout);
    dr.add(v[s].X, c.R(s), v[s].n, v[s].hout, v[s].wout);
  }
  if (stats_pass) {
    Parts pm = c.part();
    if (int r = launch_dense<T, OPF, CIN, COUT, true>(c, k, tagk("dense_fwd_main", k), dm, c.P->dense_f[k][0], &pm))
      return r;
    const int64_t offs[1] = {bo.bn_main};
    if (int r = bn_finalize(c, pm, 1, COUT, offs, running)) return r;
  } else {
    if (int r = launch_dense<T, OPF, CIN, COUT, false>(c, k, tagk("dense_fwd_main", k), dm, c.P->dense_f[k][0], nullptr))
      return r;
  }
  // recompute: x1, its decisions and t are rebuilt; the block output y, its ReLU decisions and
  // everything after them were kept from the forward
  if (c.rec_pass) return STDA_OK;
  bool res_done = false;
  if constexpr (DEC) {
    if (c.P->arch & STDA_ARCH_RES3) {
      // DeConv3x3-s2-p1 (output padding 1): the input-gradient operator of a Conv3x3-s2-p1
      if (int r = launch_dense<T, OP_ENC_DGRAD, CIN, COUT, false>(c, k, tagk("dense_fwd_res", k), dr, c.P->dense_f[k][1], nullptr))
        return r;
      res_done = true;
    }
  }
  if (!res_done)
    if (int r = launch_dense<T, OPF, CIN, COUT, false>(c, k, tagk("dense_fwd_res", k), dr, c.P->dense_f[k][1], nullptr))
      return r;
  // Y = ReLU(BN(T)) + R, GAP partials; then ECA and the skip
  float* gaps[kMaxSegs];
  int gtiles[kMaxSegs];
  {
    Batch<k_s2_apply_args<T, COUT>> b;
    for (int s = 0; s < ns; ++s) {
      const int hw = v[s].hout * v[s].wout, tiles = tiles_for(hw, COUT / 4);
      gaps[s] = c.gap(s);
      gtiles[s] = tiles;
      b.add(tiles * v[s].n, {v[s].Tm, c.R(s), v[s].Y, v[s].mask, gaps[s], c.stats(s, bo.bn_main), c.w + bo.main_g,
                             c.w + bo.main_b, hw, tiles});
    }
    KLAUNCH(tagk("s2_apply", k), k_s2_apply<T, COUT><<<b.blocks(), 256, 0, c.st>>>(b.L));
  }
  if (k >= 2) return launch_eca_next<T, COUT, true>(c, k, v, gaps, gtiles, c.w + bo.eca_w);
  return launch_eca_next<T, COUT, false>(c, k, v, gaps, gtiles, c.w + bo.eca_w);
}

template <class T, bool SIG>
int launch_head_fwd(const Ctx<T>& c, const float* wh, const float* bh, float* z) {
  Batch<k_head_fwd_tile_args<T, SIG>> b;
  for (int s = 0; s < c.ns(); ++s) {
    const SegPlan& S = c.S(s);
    float* zs = SIG && S.zs ? c.template act<float>(S.zs) : nullptr;
    b.add(head_grid(S.n, S.H, S.W), {c.template act<T>(S.blk[3].Xn), wh, bh, z + S.z_off, zs, S.n, S.H, S.W});
  }
  KLAUNCH("head_fwd", k_head_fwd_tile<T, SIG><<<b.blocks(), 256, 0, c.st>>>(b.L));
  return STDA_OK;
}

// The network forward over every segment: one launch per kernel kind and layer.
template <class T>
int forward_net(const Ctx<T>& c, const float* x, float* running, float* z) {
  const NetOffsets& no = net_offsets(c.P->arch);
  const int ns = c.ns();
  auto stem_args = [&](int s, float* part) {
    const SegPlan& S = c.S(s);
    return StemArgs{x + S.x_off, c.w + no.stem_w, c.stats(s, 0), c.w + no.stem_g, c.w + no.stem_b, nullptr, part};
  };
  if (c.train) {
    Parts pm = c.part();
    Batch<k_stem_tile_args<T, 0>> b;
    for (int s = 0; s < ns; ++s) {
      const SegPlan& S = c.S(s);
      const int g = stem_grid(S.n, S.H, S.W);
      b.add(g, {stem_args(s, pm.take(g, 32, true)), nullptr, nullptr, nullptr, S.n, S.H, S.W});
    }
    if (pm.over) return STDA_E_WORKSPACE;
    KLAUNCH("stem_stats", k_stem_tile<T, 0><<<b.blocks(), 256, 0, c.st>>>(b.L));
    const int64_t offs[1] = {0};
    if (int r = bn_finalize(c, pm, 1, 16, offs, running)) return r;
  }
  {
    Batch<k_stem_tile_args<T, 1>> b;
    for (int s = 0; s < ns; ++s) {
      const SegPlan& S = c.S(s);
      b.add(stem_grid(S.n, S.H, S.W), {stem_args(s, nullptr), nullptr, nullptr, c.template act<T>(S.s0), S.n, S.H, S.W});
    }
    KLAUNCH("stem_apply", k_stem_tile<T, 1><<<b.blocks(), 256, 0, c.st>>>(b.L));
  }
  if (int r = fwd_block<T, 16, 32, false>(c, 0, running)) return r;
  if (int r = fwd_block<T, 32, 64, false>(c, 1, running)) return r;
  if (int r = fwd_block<T, 64, 32, true>(c, 2, running)) return r;
  if (int r = fwd_block<T, 32, 16, true>(c, 3, running)) return r;
  if (c.P->arch & STDA_ARCH_SIGMOID) return launch_head_fwd<T, true>(c, c.w + no.head_w, c.w + no.head_b, z);
  return launch_head_fwd<T, false>(c, c.w + no.head_w, c.w + no.head_b, z);
}

int validate_segs(const stda_segment* segs, int n_segs) {
  if (!segs || n_segs < 1 || n_segs > kMaxSegs) return STDA_E_INVALID;
  for (int s = 0; s < n_segs; ++s) {
    const stda_segment& g = segs[s];
    if (g.n < 1 || g.x_off < 0 || g.z_off < 0) return STDA_E_INVALID;
    if (g.H < 8 || g.W < 8 || g.H > 4096 || g.W > 4096 || (g.H % 4) || (g.W % 4)) return STDA_E_SHAPE;
  }
  return STDA_OK;
}

// Per-call preparation: working weights and dense layouts.
int prepare_weights(const Plan& P, const float* w, char* ws, hipStream_t st, const float** wk_out) {
  float* wk = reinterpret_cast<float*>(ws + P.ws_wk);
  const NetOffsets& no = net_offsets(P.arch);
  const int64_t np = no.param_count;
  const bool res3 = (P.arch & STDA_ARCH_RES3) != 0;
  const float* src = w;
  if (P.dtype == STDA_BF16) {
    RoundRanges rr{};
    for (const auto& e : param_table(P.arch)) {
      // only the weights the matrix cores consume (the stride-2 layers) are rounded; the
      // SIMT layers (input / output modules, pointwise, depthwise) keep FP32 weights
      const bool mfma_w = std::strstr(e.name, ".s2.main.w") != nullptr || std::strstr(e.name, ".s2.res.w") != nullptr;
      if (mfma_w) {
        rr.off[rr.n] = e.offset;
        rr.cnt[rr.n] = e.count;
        ++rr.n;
      }
    }
    {
      ProfScope ps_("prep_weights", st);
      k_working_weights<<<grid_for(np, 256), 256, 0, st>>>(w, wk, np, rr);
    }
    LAUNCH_CHECK();
    src = wk;
  }
  PrepJobs jobs{};
  jobs.bf16 = P.dtype == STDA_BF16;
  for (int k = 0; k < 4; ++k)
    for (int m = 0; m < 2; ++m) {
      PrepJob& j = jobs.j[jobs.n++];
      j.src = m == 0 ? no.blk[k].main_w : no.blk[k].res_w;
      if (res3 && m == 1 && kBlocks[k].dec) {
        // DeConv3x3-s2-p1 with output padding 1 is the adjoint of a Conv3x3-s2-p1 whose input
        // is the residual's output (Cout channels) and whose output is its input (Cin): the
        // same [Cin][Cout][3][3] array read as that conv's [out][in][3][3] weight.  Its
        // forward layout is that conv's input-gradient layout and vice versa.
        j.dec = 0;
        j.cin = kBlocks[k].cout;
        j.cout = kBlocks[k].cin;
        j.dst_f = P.dense_d[k][m];
        j.dst_d = P.dense_f[k][m];
      } else {
        j.dec = kBlocks[k].dec;
        j.cin = kBlocks[k].cin;
        j.cout = kBlocks[k].cout;
        j.dst_f = P.dense_f[k][m];
        j.dst_d = P.dense_d[k][m];
      }
    }
  {
    ProfScope ps_("prep_weights", st);
    k_prep_dense<<<dim3(32, jobs.n), 256, 0, st>>>(w, reinterpret_cast<float*>(ws + P.ws_dense), jobs);
  }
  LAUNCH_CHECK();
  if (P.arch & STDA_ARCH_PW_DW) {
    PwDiag d{};
    for (int k = 0; k < 4; ++k) {
      d.src[k] = no.blk[k].pw_w;
      d.dst[k] = P.pwx_off[k];
      d.C[k] = kBlocks[k].cin;
    }
    k_pw_diag<<<dim3(16, 4), 256, 0, st>>>(w, reinterpret_cast<float*>(ws + P.ws_pwx), d);
    LAUNCH_CHECK();
  }
  FragJobs fj{};
  for (int k = 0; k < 4; ++k)
    for (int m = 0; m < 2; ++m) {
      const int taps = kBlocks[k].dec && !(res3 && m == 1) ? 16 : 9;
      fj.j[fj.n++] = FragJob{P.dense_f[k][m], P.dense_f[k][m], taps, kBlocks[k].cin, kBlocks[k].cout};
      fj.j[fj.n++] = FragJob{P.dense_d[k][m], P.dense_d[k][m], taps, kBlocks[k].cout, kBlocks[k].cin};
    }
  const float* dl = reinterpret_cast<const float*>(ws + P.ws_dense);
  {
    ProfScope ps_("prep_weights", st);
    if (P.dtype == STDA_BF16)
      k_prep_frag<bf16><<<dim3(16, fj.n), 256, 0, st>>>(dl, reinterpret_cast<bf16*>(ws + P.ws_frag), fj);
    else
      k_prep_frag<float><<<dim3(16, fj.n), 256, 0, st>>>(dl, reinterpret_cast<float*>(ws + P.ws_frag), fj);
  }
  LAUNCH_CHECK();
  *wk_out = src;
  return STDA_OK;
}

template <class T>
int forward_all(const Plan& P, const float* x, const float* w, float* running, float* z, char* saved, char* ws,
                hipStream_t st) {
  const float* wk = nullptr;
  if (int r = prepare_weights(P, w, ws, st, &wk)) return r;
  const bool train = P.mode == STDA_TRAIN;
  Ctx<T> c{&P, train ? saved : ws, ws, wk, reinterpret_cast<float*>(ws + P.ws_dense), st, train};
  if (!train) {
    BnTable tab{};
    int off = 0;
    tab.off[tab.n] = off;
    tab.C[tab.n++] = 16;
    off += 32;
    for (int k = 0; k < 4; ++k) {
      const int cs[4] = {kBlocks[k].cin, kBlocks[k].cin, kBlocks[k].cin, kBlocks[k].cout};
      for (int q = 0; q < 4; ++q) {
        tab.off[tab.n] = off;
        tab.C[tab.n++] = cs[q];
        off += 2 * cs[q];
      }
    }
    tab.nseg = P.n_segs;
    for (int s = 0; s < P.n_segs; ++s) tab.stats[s] = c.stats(s, 0);
    {
      ProfScope ps_("eval_stats", st);
      k_eval_stats<<<1, 256, 0, st>>>(running, tab);
    }
    LAUNCH_CHECK();
  }
  return forward_net<T>(c, x, running, z);
}

// ------------------------------------------------------------------ folded EVAL inference
// Layout of the folded-parameter buffer: the weight regions of the per-call workspace (working
// weights, dense and fragment-order layouts; their offsets do not depend on the batch), then the
// folded parameter vector, then the identity statistics.
struct FoldLayout {
  Plan P;
  size_t wf_off, bytes;
};
bool fold_arch_ok(int arch) { return (arch & (STDA_ARCH_RES3 | STDA_ARCH_PW_DW)) == 0; }
FoldLayout fold_layout(int dtype) {
  FoldLayout L;
  const stda_segment one{1, 8, 8, 0, 0};
  build_plan(&one, 1, dtype, STDA_EVAL, 0, L.P);
  L.wf_off = L.P.ws_R;  // ws_wk, ws_dense, ws_pwx and ws_frag come first
  L.bytes = align_up(L.wf_off + sizeof(float) * (net_offsets(L.P.arch).param_count + kFoldIds));
  return L;
}

#define FLAUNCH(tag, ...)             \
  do {                                \
    ProfScope ps_((tag), st);         \
    __VA_ARGS__;                      \
  } while (0);                        \
  LAUNCH_CHECK()

// ECA partial sums of block k in the folded path: per (clip, phase, row tile) and channel.
int64_t folded_gap_floats(const SegPlan& S, int k) {
  const BlockCfg& b = kBlocks[k];
  const int64_t ho = S.H >> b.lout, wo = S.W >> b.lout;
  const int64_t rows = b.dec ? (ho / 2) * (wo / 2) : ho * wo;  // one clip's phase grid
  return (int64_t)S.n * (b.dec ? 4 : 1) * ((rows + 63) / 64) * b.cout;
}

template <class T, int CIN, int COUT, bool DEC>
int folded_block(const Plan& P, int k, const char* fold, const float* wk, const float* ids, char* ws, hipStream_t st) {
  const BlockOffsets& bo = net_offsets(P.arch).blk[k];
  // the whole buffer is ws (EVAL), so the context's views serve here
  const Ctx<T> c{&P, ws, ws, wk, nullptr, st, false};
  const int ns = c.ns();
  BlockView<T> v[kMaxSegs];
  for (int s = 0; s < ns; ++s) v[s] = block_view(c, s, k);
  S1Params sp{};
  sp.wpw = wk + bo.pw_w;
  sp.wdw = wk + bo.dw_w;
  for (int q = 0; q < 3; ++q) sp.stats[q] = ids + fold_ids_off(CIN);
  sp.gamma[0] = wk + bo.pw_g;
  sp.gamma[1] = wk + bo.dw_g;
  sp.gamma[2] = wk + bo.id_g;
  sp.beta[0] = wk + bo.pw_b;
  sp.beta[1] = wk + bo.dw_b;
  sp.beta[2] = wk + bo.id_b;
  {
    Batch<k_s1_tile_args<T, CIN, DEC, 1>> b;
    for (int s = 0; s < ns; ++s)
      b.add(s1_grid<CIN>(v[s].n, v[s].hin, v[s].win), {v[s].X, v[s].X1, nullptr, nullptr, sp, v[s].n, v[s].hin, v[s].win});
    FLAUNCH(tagk("s1_apply", k), k_s1_tile<T, CIN, DEC, 1><<<b.blocks(), 256, 0, st>>>(b.L));
  }
  constexpr int OPF = DEC ? OP_DEC_FWD : OP_ENC_FWD, PH = DEC ? 4 : 1, R = 1;
  const T* frag = reinterpret_cast<const T*>(fold + P.ws_frag);
  // the residual buffer is not needed here: it holds the ECA partial sums, segment after segment
  float* gap = reinterpret_cast<float*>(ws + P.ws_R);
  float* gaps[kMaxSegs];
  int gtiles[kMaxSegs];
  {
    Batch<k_s2_eval_args<T, OPF, CIN, COUT, R>> b;
    for (int s = 0; s < ns; ++s) {
      const int64_t rows = DEC ? (int64_t)(v[s].hout / 2) * (v[s].wout / 2) : (int64_t)v[s].hout * v[s].wout;
      const int tx = (int)((rows + 64 * R - 1) / (64 * R));
      gaps[s] = gap;
      gtiles[s] = tx * PH;
      b.add(tx * v[s].n, {v[s].X1, v[s].X, frag + P.dense_f[k][0], frag + P.dense_f[k][1], wk + bo.main_b, v[s].Y,
                          gap, v[s].hout, v[s].wout, tx});
      gap += folded_gap_floats(P.seg[s], k);
    }
    FLAUNCH(tagk("s2_eval", k), k_s2_eval<T, OPF, CIN, COUT, R><<<dim3(b.blocks(), PH), 256, 0, st>>>(b.L));
  }
  if (k >= 2) return launch_eca_next<T, COUT, true>(c, k, v, gaps, gtiles, wk + bo.eca_w);
  return launch_eca_next<T, COUT, false>(c, k, v, gaps, gtiles, wk + bo.eca_w);
}

template <class T>
int forward_folded_all(const Plan& P, const FoldLayout& L, const float* x, const char* fold, float* z, char* ws,
                       hipStream_t st) {
  const NetOffsets& no = net_offsets(P.arch);
  const float* wf = reinterpret_cast<const float*>(fold + L.wf_off);
  const float* ids = wf + no.param_count;
  // working weights: the folded vector (BF16: its copy with the stage-2 weights rounded)
  const float* wk = P.dtype == STDA_BF16 ? reinterpret_cast<const float*>(fold + L.P.ws_wk) : wf;
  // the ECA partial sums of every block fit the residual buffer
  for (int k = 0; k < 4; ++k) {
    int64_t need = 0;
    for (int s = 0; s < P.n_segs; ++s) need += folded_gap_floats(P.seg[s], k) * (int64_t)sizeof(float);
    if (need > (int64_t)(P.ws_part - P.ws_R)) return STDA_E_WORKSPACE;
  }
  const Ctx<T> c{&P, ws, ws, wk, nullptr, st, false};
  {
    Batch<k_stem_tile_args<T, 1>> b;
    for (int s = 0; s < P.n_segs; ++s) {
      const SegPlan& S = P.seg[s];
      const StemArgs sa{x + S.x_off, wk + no.stem_w, ids + fold_ids_off(16), wk + no.stem_g, wk + no.stem_b, nullptr, nullptr};
      b.add(stem_grid(S.n, S.H, S.W), {sa, nullptr, nullptr, reinterpret_cast<T*>(ws + S.s0), S.n, S.H, S.W});
    }
    FLAUNCH("stem_apply", k_stem_tile<T, 1><<<b.blocks(), 256, 0, st>>>(b.L));
  }
  if (int r = folded_block<T, 16, 32, false>(P, 0, fold, wk, ids, ws, st)) return r;
  if (int r = folded_block<T, 32, 64, false>(P, 1, fold, wk, ids, ws, st)) return r;
  if (int r = folded_block<T, 64, 32, true>(P, 2, fold, wk, ids, ws, st)) return r;
  if (int r = folded_block<T, 32, 16, true>(P, 3, fold, wk, ids, ws, st)) return r;
  if (P.arch & STDA_ARCH_SIGMOID) return launch_head_fwd<T, true>(c, wk + no.head_w, wk + no.head_b, z);
  return launch_head_fwd<T, false>(c, wk + no.head_w, wk + no.head_b, z);
}
#undef FLAUNCH

}  // namespace

// ===================================================================== backward
namespace {

template <class T>
int colsum_to(const Ctx<T>& c, const float* part, int nrows, int ncols, float* dst, ColMap map, int acc,
              const std::string& tag = "colsum") {
  if (ncols >= 16384) {
    KLAUNCH(tag, k_colsum<64><<<(ncols + 63) / 64, 256, 0, c.st>>>(part, nrows, ncols, nullptr, dst, map, acc));
  } else if (ncols >= 4096) {  // too few 64-column blocks to fill the chip: more row groups each
    KLAUNCH(tag, k_colsum<64, 1024><<<(ncols + 63) / 64, 1024, 0, c.st>>>(part, nrows, ncols, nullptr, dst, map, acc));
  } else {
    KLAUNCH(tag, k_colsum<16><<<(ncols + 15) / 16, 256, 0, c.st>>>(part, nrows, ncols, nullptr, dst, map, acc));
  }
  return STDA_OK;
}

// Stage-2 weight gradient of block `blk` on LDS tiles; encoder: Lo = output gradient on the
// hout x wout grid, Hi = layer input; decoder: Lo = layer input on the hin x win grid, Hi = output
// gradient.
// Workgroups of a tiled weight-gradient launch: enough to keep 4 per CU where the partial rows
// (one per workgroup, `cols` floats each) fit the partial buffer, at least 256.
int64_t wgrad_rows(int64_t cols) {
  const int64_t fit = (int64_t)kMaxWgradGrid * 32768 / cols;
  return std::max<int64_t>(256, std::min<int64_t>(1024, fit));
}

// One segment's operands of a stage-2 weight gradient: x the layer input (hin x win), d the
// gradient of its output.
template <class T>
struct WgOps {
  int n = 0;
  const T* x[kMaxSegs];
  const T* d[kMaxSegs];
  int clips[kMaxSegs], hin[kMaxSegs], win[kMaxSegs];
  void add(const T* xs, const T* ds, int b, int h, int w) {
    x[n] = xs;
    d[n] = ds;
    clips[n] = b;
    hin[n] = h;
    win[n] = w;
    ++n;
  }
};

// Weight-gradient launch with tiling (TH, TW) over every segment: Lo / Hi operands and the grid
// of Lo per segment; one partial row per workgroup, all segments' rows summed by one reduction.
template <class T, bool DEC, int CL, int CH, int TH, int TW, bool VEC>
int launch_wgrad_cfg(const Ctx<T>& c, const std::string& tag, const WgOps<T>& O, float* dst, ColMap map) {
  constexpr int TAPS = VEC ? WgVCfg<T, DEC, CL, CH, TH, TW>::TAPS : WgCfg<T, DEC, CL, CH, TH, TW>::TAPS;
  const int64_t cols = (int64_t)TAPS * CH * CL;
  typedef std::conditional_t<VEC, k_s2_wgrad_v_args<T, DEC, CL, CH, TH, TW>, k_s2_wgrad_args<T, DEC, CL, CH, TH, TW>> A;
  Batch<A> b;
  Parts pm = c.wpart();
  for (int s = 0; s < O.n; ++s) {
    const T* lo = DEC ? O.x[s] : O.d[s];
    const T* hi = DEC ? O.d[s] : O.x[s];
    const int h = DEC ? O.hin[s] : O.hin[s] / 2, w = DEC ? O.win[s] : O.win[s] / 2;
    const int64_t ntiles = (int64_t)O.clips[s] * ((h + TH - 1) / TH) * ((w + TW - 1) / TW);
    int64_t gx = capped(std::min<int64_t>(ntiles, wgrad_rows(cols)));
    if (gx >= 64) gx &= ~(int64_t)7;
    gx = std::max<int64_t>(gx, 1);
    b.add((int)gx, {lo, hi, pm.take((int)gx, cols, false), O.clips[s], h, w});
  }
  if (pm.over) return STDA_E_WORKSPACE;
  if constexpr (VEC) {
    KLAUNCH(tag, k_s2_wgrad_v<T, DEC, CL, CH, TH, TW><<<b.blocks(), 256, 0, c.st>>>(b.L));
  } else {
    KLAUNCH(tag, k_s2_wgrad<T, DEC, CL, CH, TH, TW><<<b.blocks(), 256, 0, c.st>>>(b.L));
  }
  return colsum_to(c, pm.base, pm.total_rows(), (int)cols, dst, map, 0, "wgrad_sum" + tag.substr(5));
}

template <class T, bool DEC, int CIN, int COUT>
int launch_wgrad(const Ctx<T>& c, int blk, const std::string& tag, const WgOps<T>& O, float* dst) {
  const int v = tuned(sizeof(T) == 2 ? 1 : 0, 2, blk);
  constexpr int CL = DEC ? CIN : COUT, CH = DEC ? COUT : CIN;
  const ColMap map{DEC ? MAP_DEC_S2 : MAP_ENC_S2, CIN, COUT};
  constexpr bool SMALL = CL * CH <= 512;  // 16 x 32 channel pairs: larger tiles fit
#define WGV(TH_, TW_) launch_wgrad_cfg<T, DEC, CL, CH, TH_, TW_, false>(c, tag, O, dst, map)
#define WGVV(TH_, TW_) launch_wgrad_cfg<T, DEC, CL, CH, TH_, TW_, true>(c, tag, O, dst, map)
  // 0, 1, 3: vector-operand kernel; 2: scalar-operand kernel (BF16) or the vector-operand kernel on
  // smaller tiles (FP32)
  constexpr bool BF = sizeof(T) == 2;
  if (v == 3) {
    if constexpr (BF) return WGVV(4, 8);
    else return WGVV(2, 8);
  }
  if (v == 2) {
    if constexpr (BF && SMALL) return WGV(8, 16);
    else if constexpr (BF) return WGV(8, 8);
    else if constexpr (SMALL) return WGVV(4, 8);
    else return WGVV(4, 4);
  }
  if constexpr (SMALL) return v == 1 ? WGVV(8, 8) : WGVV(8, 16);
  else return v == 1 ? WGVV(4, 8) : WGVV(8, 8);
#undef WGV
#undef WGVV
}

// One segment's operands of the fused stage-1 adjoint.
template <class T>
struct S1bOps {
  const T* X;
  const uint8_t* M1;
  const T *dX1, *dXr, *skipg;
  S1Params sp;
  T* dXout;
  const float* coef;
  int n, h, w;
};

// Fused stage-1 adjoint of block `blk` with the tiling chosen for it (tuning kind 3): TH x TW
// pixel tiles, MINW waves per SIMD; weight-gradient partial rows (one per workgroup) go to
// *pw (pointwise) and *dw (depthwise), segment after segment.
template <class T, int C, bool DEC, int TH, int TW, int MINW, bool LC = false>
int launch_s1b_cfg(const Ctx<T>& c, int blk, const S1bOps<T>* O, Parts& pw, Parts& dw) {
  Batch<k_s1_bwd_fused_args<T, C, DEC, !DEC, TH, TW, MINW, LC>> b;
  for (int s = 0; s < c.ns(); ++s) {
    const S1bOps<T>& o = O[s];
    const int64_t tiles = (int64_t)o.n * ((o.h + TH - 1) / TH) * ((o.w + TW - 1) / TW);
    const int g = (int)std::max<int64_t>(1, capped(std::min<int64_t>(tiles, kTileGrid)));
    b.add(g, {o.X, o.M1, o.dX1, o.dXr, o.skipg, o.coef, o.sp, o.dXout, pw.take(g, C * C, false), dw.take(g, 9 * C, false),
              o.n, o.h, o.w});
  }
  if (pw.over || dw.over) return STDA_E_WORKSPACE;
  KLAUNCH(tagk("s1_bwd_fused", blk),
          (k_s1_bwd_fused<T, C, DEC, !DEC, TH, TW, MINW, LC><<<b.blocks(), 256, 0, c.st>>>(b.L)));
  return STDA_OK;
}

template <class T, int C, bool DEC>
int launch_s1b(const Ctx<T>& c, int blk, const S1bOps<T>* O, Parts& pw, Parts& dw) {
  const int v = tuned(sizeof(T) == 2 ? 1 : 0, 3, blk);
#define S1B(TH_, TW_, W_) launch_s1b_cfg<T, C, DEC, TH_, TW_, W_>(c, blk, O, pw, dw)
  // LC: depthwise taps and BN-adjoint coefficients read from LDS, three waves per SIMD at 16
  // channels (above, the LDS of three workgroups does not fit and two are asked for)
#define S1L(TH_, TW_) launch_s1b_cfg<T, C, DEC, TH_, TW_, C == 16 ? 3 : 2, true>(c, blk, O, pw, dw)
  if constexpr (C == 16) return v == 1 ? S1B(16, 8, 2) : v == 2 ? S1B(4, 32, 2) : v == 3 ? S1L(8, 16) : S1B(8, 16, 2);
  else if constexpr (C == 32) return v == 1 ? S1B(4, 16, 2) : v == 2 ? S1B(16, 4, 2) : v == 3 ? S1L(8, 8) : S1B(8, 8, 2);
  else return v == 1 ? S1B(2, 8, 2) : v == 2 ? S1L(4, 4) : v == 3 ? S1B(4, 4, 1) : S1B(4, 4, 2);
#undef S1B
#undef S1L
}

// BN adjoint reduction over every segment of the launch whose partials are in pm: NS sums per
// channel, count[s] elements per channel in segment s; gamma / beta gradients summed over the
// segments, coefficients per segment.
template <class T>
int bn_bwd(const Ctx<T>& c, const Parts& pm, int NS, int C, const double* count, float* const* dg, float* const* db) {
  if (NS > 4) return STDA_E_INVALID;
  BnBwdSegs sg{};
  sg.n = pm.n;
  for (int s = 0; s < pm.n; ++s) {
    sg.part[s] = pm.p[s];
    sg.rows[s] = pm.rows[s];
    sg.count[s] = count[s];
    sg.coef[s] = c.coef(s);
  }
  BnBwdOut o{};
  for (int k = 0; k < NS - 1; ++k) {
    o.dgamma[k] = dg[k];
    o.dbeta[k] = db[k];
  }
  KLAUNCH("bn_bwd_finalize", k_bn_bwd_reduce<<<NS * C, 256, 0, c.st>>>(sg, NS, C, o, 0));
  return STDA_OK;
}

// Gradient buffers (ws, one region per segment): 0 dd1 (grad of d1), 1 dd0 (grad of d0), 2 de1,
// 3 de0, 4 ds0, 5 dT, 6 dY, 7 dX1, 8 dXr, 9 dP, 10 dD, 11 dX0, 12 dTp (input module).
// Block k's adjoint reads the output gradient from buffer gin and writes the input gradient to
// gout; the encoder blocks add the skip gradient from buffer gskip (decoder blocks: -1).
template <class T, int CIN, int COUT, bool DEC>
int bwd_block(const Ctx<T>& c, int k, int gin, int gout, int gskip, float* dw) {
  const BlockOffsets& bo = net_offsets(c.P->arch).blk[k];
  const int ns = c.ns();
  // the encoder blocks receive a skip gradient (from the decoder), the decoder blocks none
  if ((gskip >= 0) != !DEC) return STDA_E_INVALID;
  BlockView<T> v[kMaxSegs];
  S1Params sp[kMaxSegs];
  int tiles[kMaxSegs];
  double cin_n[kMaxSegs], cout_n[kMaxSegs];
  for (int s = 0; s < ns; ++s) {
    v[s] = block_view(c, s, k);
    sp[s] = s1_params(c, s, k);
    tiles[s] = tiles_for(v[s].hout * v[s].wout, COUT / 4);
    cin_n[s] = (double)v[s].n * v[s].hin * v[s].win;
    cout_n[s] = (double)v[s].n * v[s].hout * v[s].wout;
  }
  auto G = [&](int s, int i) { return c.grad(s, i); };
  // ECA adjoint partials and stage-2 BN statistics
  {
    Batch<k_eca_bwd_part_args<T, COUT>> b;
    for (int s = 0; s < ns; ++s)
      b.add(tiles[s] * v[s].n, {G(s, gin), v[s].Y, c.gap(s), v[s].hout * v[s].wout, tiles[s]});
    KLAUNCH(tagk("eca_bwd", k), k_eca_bwd_part<T, COUT><<<b.blocks(), 256, 0, c.st>>>(b.L));
  }
  {
    Parts pm = c.part();
    Batch<k_s2_bwd_stats_args<T, COUT>> b;
    for (int s = 0; s < ns; ++s)
      b.add(tiles[s] * v[s].n, {G(s, gin), v[s].Tm, v[s].mask, c.gap(s), v[s].a, v[s].g, c.w + bo.eca_w,
                                c.stats(s, bo.bn_main), c.w + bo.main_g, c.w + bo.main_b, c.coef_e(s), c.ecaw(s),
                                pm.take(tiles[s] * v[s].n, 2 * COUT, false), v[s].hout * v[s].wout, tiles[s],
                                tiles[s]});
    if (pm.over) return STDA_E_WORKSPACE;
    KLAUNCH(tagk("s2_bwd_stats", k), k_s2_bwd_stats<T, COUT><<<b.blocks(), 256, 0, c.st>>>(b.L));
    // ECA weight gradient: the per-clip rows of all segments are contiguous
    if (int r = colsum_to(c, c.ecaw(0), c.clips(), 3, dw + bo.eca_w, ColMap{MAP_IDENT, 0, 0}, 0)) return r;
    float* dg[1] = {dw + bo.main_g};
    float* db[1] = {dw + bo.main_b};
    if (int r = bn_bwd(c, pm, 2, COUT, cout_n, dg, db)) return r;
  }
  {
    Batch<k_s2_bwd_apply_args<T, COUT>> b;
    for (int s = 0; s < ns; ++s)
      b.add(tiles[s] * v[s].n, {G(s, gin), v[s].Tm, v[s].mask, v[s].a, c.coef_e(s), c.coef(s), c.stats(s, bo.bn_main),
                                c.w + bo.main_g, c.w + bo.main_b, G(s, 5), G(s, 6), v[s].hout * v[s].wout, tiles[s]});
    KLAUNCH(tagk("s2_bwd_apply", k), k_s2_bwd_apply<T, COUT><<<b.blocks(), 256, 0, c.st>>>(b.L));
  }
  // dense adjoints: dX1 from dT, dXr from dY
  constexpr int OPD = DEC ? OP_DEC_DGRAD : OP_ENC_DGRAD;
  DenseOps<T> dm, dr;
  for (int s = 0; s < ns; ++s) {
    dm.add(G(s, 5), G(s, 7), v[s].n, v[s].hin, v[s].win);
    dr.add(G(s, 6), G(s, 8), v[s].n, v[s].hin, v[s].win);
  }
  if (int r = launch_dense<T, OPD, COUT, CIN, false>(c, k, tagk("dense_dgrad_main", k), dm, c.P->dense_d[k][0], nullptr))
    return r;
  const bool res3 = DEC && (c.P->arch & STDA_ARCH_RES3);
  if constexpr (DEC) {
    if (res3)  // adjoint of the DeConv3x3-s2-p1 residual: a Conv3x3-s2-p1 of dY
      if (int r = launch_dense<T, OP_ENC_FWD, COUT, CIN, false>(c, k, tagk("dense_dgrad_res", k), dr, c.P->dense_d[k][1], nullptr))
        return r;
  }
  if (!res3)
    if (int r = launch_dense<T, OPD, COUT, CIN, false>(c, k, tagk("dense_dgrad_res", k), dr, c.P->dense_d[k][1], nullptr))
      return r;
  // dense weight gradients
  {
    WgOps<T> om, orr;
    for (int s = 0; s < ns; ++s) {
      om.add(v[s].X1, G(s, 5), v[s].n, v[s].hin, v[s].win);
      if (res3)  // the weight gradient of that Conv3x3-s2-p1 with input dY and output gradient X
        orr.add(G(s, 6), v[s].X, v[s].n, v[s].hout, v[s].wout);
      else
        orr.add(v[s].X, G(s, 6), v[s].n, v[s].hin, v[s].win);
    }
    if (int r = launch_wgrad<T, DEC, CIN, COUT>(c, k, tagk("wgrad_main", k), om, dw + bo.main_w)) return r;
    if constexpr (DEC) {
      if (res3)
        if (int r = launch_wgrad<T, false, COUT, CIN>(c, k, tagk("wgrad_res", k), orr, dw + bo.res_w)) return r;
    }
    if (!res3)
      if (int r = launch_wgrad<T, DEC, CIN, COUT>(c, k, tagk("wgrad_res", k), orr, dw + bo.res_w)) return r;
  }
  // stage 1
  {
    Parts pm = c.part();
    Batch<k_s1_bwd_stats_tile_args<T, CIN, DEC>> b;
    for (int s = 0; s < ns; ++s) {
      const int g = s1_grid<CIN>(v[s].n, v[s].hin, v[s].win);
      b.add(g, {v[s].X, v[s].m1, G(s, 7), pm.take(g, 4 * CIN, false), sp[s], v[s].n, v[s].hin, v[s].win});
    }
    if (pm.over) return STDA_E_WORKSPACE;
    KLAUNCH(tagk("s1_bwd_stats", k), k_s1_bwd_stats_tile<T, CIN, DEC><<<b.blocks(), 256, 0, c.st>>>(b.L));
    float* dg[3] = {dw + bo.pw_g, dw + bo.dw_g, dw + bo.id_g};
    float* db[3] = {dw + bo.pw_b, dw + bo.dw_b, dw + bo.id_b};
    if (int r = bn_bwd(c, pm, 4, CIN, cin_n, dg, db)) return r;
  }
  S1bOps<T> o[kMaxSegs];
  for (int s = 0; s < ns; ++s)
    o[s] = S1bOps<T>{v[s].X, v[s].m1, G(s, 7), G(s, 8), gskip >= 0 ? G(s, gskip) : nullptr, sp[s], G(s, gout),
                     c.coef(s), v[s].n, v[s].hin, v[s].win};
  Parts pw = c.wpart(), dwp = c.part();
  if (int r = launch_s1b<T, CIN, DEC>(c, k, o, pw, dwp)) return r;
  const ColMap pwmap = (c.P->arch & STDA_ARCH_PW_DW) ? ColMap{MAP_PW_DIAG, CIN, 0}
                                                      : ColMap{DEC ? MAP_IDENT : MAP_PW_CONV, CIN, 0};
  // both weight gradients of stage 1 (pointwise, depthwise) in one reduction launch
  const int rows = pw.total_rows();
  const ColJob ja{pw.base, dw + bo.pw_w, pwmap, rows, CIN * CIN, (CIN * CIN + 15) / 16};
  const ColJob jb{dwp.base, dw + bo.dw_w, ColMap{MAP_DW, CIN, 0}, rows, 9 * CIN, (9 * CIN + 15) / 16};
  KLAUNCH(tagk("s1_bwd_fused_sum", k), k_colsum2<<<ja.nblk + jb.nblk, 256, 0, c.st>>>(ja, jb, 0));
  return STDA_OK;
}

template <class T, bool SIG>
int launch_head_bwd(const Ctx<T>& c, const float* dz, const float* wh, Parts& pm) {
  Batch<k_head_bwd_tile_args<T, SIG>> b;
  for (int s = 0; s < c.ns(); ++s) {
    const SegPlan& S = c.S(s);
    const int g = head_grid(S.n, S.H, S.W);
    b.add(g, {dz + S.z_off, SIG ? c.template act<float>(S.zs) : nullptr, wh, c.template act<T>(S.blk[3].Xn),
              c.grad(s, 0), pm.take(g, 10 * 16, false), S.n, S.H, S.W});
  }
  if (pm.over) return STDA_E_WORKSPACE;
  KLAUNCH("head_bwd", k_head_bwd_tile<T, SIG><<<b.blocks(), 256, 0, c.st>>>(b.L));
  return STDA_OK;
}

// The network adjoint over every segment: one launch per kernel kind and layer; parameter
// gradients summed over all segments.
template <class T>
int backward_net(const Ctx<T>& c, const float* dz, const float* x, float* dw, float* dx) {
  const NetOffsets& no = net_offsets(c.P->arch);
  const int ns = c.ns();
  // output module
  {
    Parts pm = c.part();
    const int r = (c.P->arch & STDA_ARCH_SIGMOID) ? launch_head_bwd<T, true>(c, dz, c.w + no.head_w, pm)
                                                  : launch_head_bwd<T, false>(c, dz, c.w + no.head_w, pm);
    if (r) return r;
    if (int e = colsum_to(c, pm.base, pm.total_rows(), 10 * 16, dw + no.head_w, ColMap{MAP_HEAD, 0, 0}, 0)) return e;
  }
  // decoder 1 (input d0, output d1 = ECA + s0), decoder 0 (input e1, output d0 = ECA + e0)
  // recompute mode: rebuild a block's x1, its decisions and t (saved statistics) right before its
  // adjoint
  Ctx<T> rc = c;
  rc.rec_pass = true;
  const bool rec = c.S(0).blk[0].inner_in_ws;
  if (rec)
    if (int r = fwd_block<T, 32, 16, true>(rc, 3, nullptr)) return r;
  if (int r = bwd_block<T, 32, 16, true>(c, 3, 0, 1, -1, dw)) return r;
  if (rec)
    if (int r = fwd_block<T, 64, 32, true>(rc, 2, nullptr)) return r;
  if (int r = bwd_block<T, 64, 32, true>(c, 2, 1, 2, -1, dw)) return r;
  // encoder 1 (input e0: its gradient also receives dd0 through the skip), encoder 0
  if (rec)
    if (int r = fwd_block<T, 32, 64, false>(rc, 1, nullptr)) return r;
  if (int r = bwd_block<T, 32, 64, false>(c, 1, 2, 3, 1, dw)) return r;
  if (rec)
    if (int r = fwd_block<T, 16, 32, false>(rc, 0, nullptr)) return r;
  if (int r = bwd_block<T, 16, 32, false>(c, 0, 3, 4, 0, dw)) return r;
  // input module
  auto stem_args = [&](int s, float* part) {
    const SegPlan& S = c.S(s);
    return StemArgs{x + S.x_off, c.w + no.stem_w, c.stats(s, 0), c.w + no.stem_g, c.w + no.stem_b, c.coef(s), part};
  };
  {
    Parts pm = c.part();
    Batch<k_stem_tile_args<T, 2>> b;
    double cnt[kMaxSegs];
    for (int s = 0; s < ns; ++s) {
      const SegPlan& S = c.S(s);
      const int g = stem_grid(S.n, S.H, S.W);
      cnt[s] = (double)S.n * S.H * S.W;
      b.add(g, {stem_args(s, pm.take(g, 2 * 16, false)), c.grad(s, 4), c.template act<T>(S.s0), nullptr, S.n, S.H, S.W});
    }
    if (pm.over) return STDA_E_WORKSPACE;
    KLAUNCH("stem_bwd_stats", k_stem_tile<T, 2><<<b.blocks(), 256, 0, c.st>>>(b.L));
    float* dg[1] = {dw + no.stem_g};
    float* db[1] = {dw + no.stem_b};
    if (int r = bn_bwd(c, pm, 2, 16, cnt, dg, db)) return r;
  }
  {
    Parts pm = c.part();
    Batch<k_stem_tile_args<T, 3>> b;
    for (int s = 0; s < ns; ++s) {
      const SegPlan& S = c.S(s);
      const int g = stem_grid(S.n, S.H, S.W);
      b.add(g, {stem_args(s, pm.take(g, 27 * 16, false)), c.grad(s, 4), c.template act<T>(S.s0),
                dx ? c.grad(s, 12) : nullptr, S.n, S.H, S.W});
    }
    if (pm.over) return STDA_E_WORKSPACE;
    KLAUNCH("stem_bwd_apply", k_stem_tile<T, 3><<<b.blocks(), 256, 0, c.st>>>(b.L));
    if (int r = colsum_to(c, pm.base, pm.total_rows(), 27 * 16, dw + no.stem_w, ColMap{MAP_STEM, 0, 0}, 0)) return r;
  }
  if (dx) {
    Batch<k_stem_dx_args<T>> b;
    for (int s = 0; s < ns; ++s) {
      const SegPlan& S = c.S(s);
      b.add(grid_for((int64_t)S.n * S.H * S.W), {c.grad(s, 12), c.w + no.stem_w, dx + S.x_off, S.n, S.H, S.W});
    }
    KLAUNCH("stem_dx", k_stem_dx<T><<<b.blocks(), 256, 0, c.st>>>(b.L));
  }
  return STDA_OK;
}

template <class T>
int backward_all(const Plan& P, const float* dz, const float* x, const float* w, const char* saved, float* dw,
                 float* dx, char* ws, hipStream_t st) {
  const float* wk = nullptr;
  if (int r = prepare_weights(P, w, ws, st, &wk)) return r;
  Ctx<T> c{&P, const_cast<char*>(saved), ws, wk, reinterpret_cast<float*>(ws + P.ws_dense), st, true};
  return backward_net<T>(c, dz, x, dw, dx);
}

}  // namespace

// ===================================================================== saved-buffer records
namespace {

// The layout of `saved` follows from (segments, dtype, recompute, architecture reading).  Every
// TRAIN forward records that key for its `saved` pointer on the host, and stda_backward accepts a
// `saved` only under the key it was filled with, so that a backward with another dtype, recompute
// flag, reading or segment list is refused instead of reading the buffer at the wrong offsets.
// Host-side, so that neither call waits on the device (both stay capturable into graphs).
uint64_t saved_key(const stda_segment* segs, int n_segs, int dtype, int recompute, int arch) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the fields
  auto mix = [&h](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xffu;
      h *= 1099511628211ull;
    }
  };
  mix((uint64_t)dtype);
  mix((uint64_t)(recompute != 0));
  mix((uint64_t)arch);
  mix((uint64_t)n_segs);
  for (int s = 0; s < n_segs; ++s) {
    mix((uint64_t)segs[s].n);
    mix((uint64_t)segs[s].H);
    mix((uint64_t)segs[s].W);
    mix((uint64_t)segs[s].x_off);
    mix((uint64_t)segs[s].z_off);
  }
  return h;
}

struct SavedRec {
  const void* ptr;
  uint64_t key;
};
constexpr size_t kSavedRecs = 256;  // most recent TRAIN forwards remembered
std::mutex g_saved_mu;
std::vector<SavedRec> g_saved_recs;

void saved_record(const void* p, uint64_t key) {
  std::lock_guard<std::mutex> lk(g_saved_mu);
  for (auto it = g_saved_recs.begin(); it != g_saved_recs.end(); ++it)
    if (it->ptr == p) {
      g_saved_recs.erase(it);
      break;
    }
  if (g_saved_recs.size() >= kSavedRecs) g_saved_recs.erase(g_saved_recs.begin());
  g_saved_recs.push_back(SavedRec{p, key});
}

bool saved_matches(const void* p, uint64_t key) {
  std::lock_guard<std::mutex> lk(g_saved_mu);
  for (const auto& r : g_saved_recs)
    if (r.ptr == p) return r.key == key;
  return false;
}

}  // namespace

// ===================================================================== C ABI
extern "C" {

const char* stda_status_string(int s) {
  switch (s) {
    case STDA_OK: return "ok";
    case STDA_E_INVALID: return "invalid argument";
    case STDA_E_SHAPE: return "unsupported shape (H, W must be multiples of 4 in [8, 4096])";
    case STDA_E_WORKSPACE: return "workspace or saved buffer too small";
    case STDA_E_HIP: return "HIP runtime error";
    case STDA_E_NONFINITE: return "non-finite value";
    default: return "unknown status";
  }
}

int stda_last_hip_error(void) { return g_last_hip; }

size_t stda_param_count(void) { return (size_t)net_offsets(current_arch()).param_count; }

int stda_param_table(stda_param_desc* out, int cap) {
  const auto& t = param_table(current_arch());
  if (out) {
    for (int i = 0; i < (int)t.size() && i < cap; ++i) {
      std::memset(&out[i], 0, sizeof(out[i]));
      std::snprintf(out[i].name, sizeof(out[i].name), "%s", t[i].name);
      out[i].offset = t[i].offset;
      out[i].ndim = t[i].ndim;
      for (int d = 0; d < 4; ++d) out[i].shape[d] = d < t[i].ndim ? t[i].shape[d] : 0;
      out[i].fan_in = t[i].fan_in;
    }
  }
  return (int)t.size();
}

struct stda_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // extern "C"

namespace {
// Captures the work `enqueue` puts on `stream` into an instantiated graph.
template <class F>
int capture_graph(hipStream_t stream, F enqueue, stda_graph* out) {
  {
    Prof& p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    if (p.on) return STDA_E_INVALID;  // the timing hook records events; keep it out of graphs
  }
  HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
  const int r = enqueue();
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(stream, &g);
  if (r) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    return STDA_E_HIP;
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e2 != hipSuccess) {
    (void)hipGraphDestroy(g);
    g_last_hip = (int)e2;
    return STDA_E_HIP;
  }
  stda_graph h = new (std::nothrow) stda_graph_s;
  if (!h) {
    (void)hipGraphExecDestroy(ex);
    (void)hipGraphDestroy(g);
    return STDA_E_INVALID;
  }
  h->graph = g;
  h->exec = ex;
  *out = h;
  return STDA_OK;
}
}  // namespace

extern "C" {

int stda_forward_graph_create(const stda_segment* segs, int n_segs, const float* x, const float* w, float* running,
                              float* z, void* saved, size_t saved_bytes, void* ws, size_t ws_bytes, int dtype,
                              int mode, hipStream_t stream, stda_graph* out) {
  if (!out || !stream) return STDA_E_INVALID;
  *out = nullptr;
  size_t sv = 0, wb = 0;
  if (int r = stda_workspace_size(segs, n_segs, dtype, mode, 0, &sv, &wb)) return r;
  if (!x || !w || !running || !z || !ws || (mode == STDA_TRAIN && !saved)) return STDA_E_INVALID;
  if (ws_bytes < wb || (mode == STDA_TRAIN && saved_bytes < sv)) return STDA_E_WORKSPACE;
  return capture_graph(
      stream,
      [&]() {
        return stda_forward(segs, n_segs, x, w, running, z, saved, saved_bytes, ws, ws_bytes, dtype, mode, 0,
                            stream);
      },
      out);
}

int stda_forward_folded_graph_create(const stda_segment* segs, int n_segs, const float* x, const void* folded,
                                     size_t folded_bytes, float* z, void* ws, size_t ws_bytes, int dtype,
                                     hipStream_t stream, stda_graph* out) {
  if (!out || !stream) return STDA_E_INVALID;
  *out = nullptr;
  if (int r = validate_segs(segs, n_segs)) return r;
  if ((dtype != STDA_FP32 && dtype != STDA_BF16) || !x || !folded || !z || !ws) return STDA_E_INVALID;
  if (!fold_arch_ok(current_arch())) return STDA_E_INVALID;
  size_t sv = 0, wb = 0;
  if (int r = stda_workspace_size(segs, n_segs, dtype, STDA_EVAL, 0, &sv, &wb)) return r;
  if (ws_bytes < wb || folded_bytes < fold_layout(dtype).bytes) return STDA_E_WORKSPACE;
  return capture_graph(
      stream, [&]() { return stda_forward_folded(segs, n_segs, x, folded, folded_bytes, z, ws, ws_bytes, dtype, stream); },
      out);
}

int stda_train_step_graph_create(const stda_segment* segs, int n_segs, const float* x, const float* y, float* w,
                                 float* running, float* z, double* loss, float* dz, float* dw, void* saved,
                                 size_t saved_bytes, void* ws, size_t ws_bytes, int dtype, int recompute, float lr,
                                 float weight_decay, uint16_t* w_bf16, hipStream_t stream, stda_graph* out) {
  if (!out || !stream) return STDA_E_INVALID;
  *out = nullptr;
  // validate everything before capture starts, so that a failing call leaves nothing captured
  size_t sv = 0, wb = 0;
  if (int r = stda_workspace_size(segs, n_segs, dtype, STDA_TRAIN, recompute, &sv, &wb)) return r;
  if (!x || !y || !w || !running || !z || !loss || !dz || !dw || !saved || !ws) return STDA_E_INVALID;
  if (saved_bytes < sv || ws_bytes < wb) return STDA_E_WORKSPACE;
  return capture_graph(
      stream,
      [&]() {
        int r = stda_forward(segs, n_segs, x, w, running, z, saved, saved_bytes, ws, ws_bytes, dtype, STDA_TRAIN,
                             recompute, stream);
        if (!r) r = stda_mse_loss(segs, n_segs, z, y, loss, dz, ws, ws_bytes, stream);
        if (!r)
          r = stda_backward(segs, n_segs, x, dz, w, saved, saved_bytes, dw, nullptr, ws, ws_bytes, dtype, recompute,
                            stream);
        if (!r) r = stda_sgd_step(w, dw, (int64_t)stda_param_count(), lr, weight_decay, w_bf16, stream);
        return r;
      },
      out);
}

int stda_graph_launch(stda_graph g, hipStream_t stream) {
  if (!g || !g->exec) return STDA_E_INVALID;
  HIP_TRY(hipGraphLaunch(g->exec, stream));
  return STDA_OK;
}

int stda_graph_destroy(stda_graph g) {
  if (!g) return STDA_OK;
  hipError_t e = hipSuccess;
  if (g->exec) e = hipGraphExecDestroy(g->exec);
  if (g->graph) {
    const hipError_t e2 = hipGraphDestroy(g->graph);
    if (e == hipSuccess) e = e2;
  }
  delete g;
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    return STDA_E_HIP;
  }
  return STDA_OK;
}

int stda_profile_select(const char* tag) {
  Prof& p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  p.tag = tag ? tag : "";
  p.on = !p.tag.empty();
  p.used = 0;
  return STDA_OK;
}

int stda_profile_read(double* total_ms, int* count) {
  if (!total_ms || !count) return STDA_E_INVALID;
  Prof& p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  double tot = 0.0;
  for (size_t i = 0; i + 1 < p.used; i += 2) {
    HIP_TRY(hipEventSynchronize(p.ev[i + 1]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, p.ev[i], p.ev[i + 1]));
    tot += ms;
  }
  *total_ms = tot;
  *count = (int)(p.used / 2);
  return STDA_OK;
}

int stda_tune_count(int kind) { return (kind >= 0 && kind < kTuneKinds) ? kS2Variants : STDA_E_INVALID; }

int stda_tune_set(int kind, int dtype, int block, int variant) {
  if (kind < 0 || kind >= kTuneKinds || (dtype != STDA_FP32 && dtype != STDA_BF16) || block < 0 || block > 3 ||
      variant < 0 || variant >= kS2Variants)
    return STDA_E_INVALID;
  set_tuned(dtype, kind, block, variant);
  return STDA_OK;
}

int stda_tune_get(int kind, int dtype, int block, int* variant) {
  if (kind < 0 || kind >= kTuneKinds || (dtype != STDA_FP32 && dtype != STDA_BF16) || block < 0 || block > 3 ||
      !variant)
    return STDA_E_INVALID;
  *variant = tuned(dtype, kind, block);
  return STDA_OK;
}

int stda_autotune(const stda_segment* segs, int n_segs, const float* x, const float* y, const float* w,
                  float* running, float* z, double* loss_dev, float* dz, float* dw, void* saved, size_t saved_bytes,
                  void* ws, size_t ws_bytes, int dtype, int recompute, int reps, hipStream_t stream, char* report,
                  size_t cap, size_t* needed) {
  if (dtype != STDA_FP32 && dtype != STDA_BF16) return STDA_E_INVALID;
  if (reps < 1) reps = 1;
  {
    Prof& p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    if (p.on) return STDA_E_INVALID;
  }
  auto step = [&]() -> int {
    int r = stda_forward(segs, n_segs, x, w, running, z, saved, saved_bytes, ws, ws_bytes, dtype, STDA_TRAIN,
                         recompute, stream);
    if (!r) r = stda_mse_loss(segs, n_segs, z, y, loss_dev, dz, ws, ws_bytes, stream);
    if (!r)
      r = stda_backward(segs, n_segs, x, dz, w, saved, saved_bytes, dw, nullptr, ws, ws_bytes, dtype, recompute,
                        stream);
    return r;
  };
  int saved_choice[kTuneKinds][4];
  for (int kind = 0; kind < kTuneKinds; ++kind)
    for (int b = 0; b < 4; ++b) saved_choice[kind][b] = tuned(dtype, kind, b);
  auto restore = [&]() {
    for (int kind = 0; kind < kTuneKinds; ++kind)
      for (int b = 0; b < 4; ++b) set_tuned(dtype, kind, b, saved_choice[kind][b]);
  };
  double cost[kTuneKinds][4][kS2Variants] = {};
  for (int v = 0; v < kS2Variants; ++v) {
    for (int kind = 0; kind < kTuneKinds; ++kind)
      for (int b = 0; b < 4; ++b) set_tuned(dtype, kind, b, v);
    int r = step();  // untimed
    if (!r) {
      stda_profile_select("*");
      for (int i = 0; i < reps && !r; ++i) r = step();
    }
    if (r) {
      stda_profile_select(nullptr);
      restore();
      return r;
    }
    Prof& p = prof();
    std::lock_guard<std::mutex> lk(p.mu);
    for (size_t i = 0; i + 1 < p.used; i += 2) {
      float ms = 0.f;
      hipError_t e = hipEventSynchronize(p.ev[i + 1]);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.ev[i], p.ev[i + 1]);
      if (e != hipSuccess) {
        g_last_hip = (int)e;
        p.on = false;
        p.tag.clear();
        p.used = 0;
        restore();
        return STDA_E_HIP;
      }
      const std::string& t = p.evtag[i / 2];
      const int kind = t.rfind("dense_fwd_", 0) == 0     ? 0
                       : t.rfind("dense_dgrad_", 0) == 0 ? 1
                       : t.rfind("wgrad_", 0) == 0       ? 2
                       : t.rfind("s1_bwd_fused", 0) == 0 ? 3
                                                         : -1;
      if (kind < 0) continue;
      for (int b = 0; b < 4; ++b)
        if (t.size() > 5 && t.compare(t.size() - 4, 4, kBlockName[b]) == 0) cost[kind][b][v] += ms;
    }
    p.on = false;
    p.tag.clear();
    p.used = 0;
    // the loss of the last timed step: times measured on NaN / Inf values are not kept
    double loss_h = 0.0;
    hipError_t e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = hipMemcpy(&loss_h, loss_dev, sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      restore();
      return STDA_E_HIP;
    }
    if (!std::isfinite(loss_h)) {
      restore();
      return STDA_E_NONFINITE;
    }
  }
  std::string out;
  char line[256];
  for (int kind = 0; kind < kTuneKinds; ++kind)
    for (int b = 0; b < 4; ++b) {
      // another tiling replaces the default only when it is faster by kTuneMargin, so that
      // near-ties do not flip with timing noise
      int best = 0;
      for (int v = 1; v < kS2Variants; ++v)
        if (cost[kind][b][v] < cost[kind][b][best] && cost[kind][b][v] < (1.0 - kTuneMargin) * cost[kind][b][0])
          best = v;
      set_tuned(dtype, kind, b, best);
      int n = std::snprintf(line, sizeof(line), "%d\t%d", kind, b);
      for (int v = 0; v < kS2Variants; ++v)
        n += std::snprintf(line + n, sizeof(line) - n, "\t%.6f", cost[kind][b][v] / reps);
      std::snprintf(line + n, sizeof(line) - n, "\t%d\n", best);
      out += line;
    }
  if (needed) *needed = out.size() + 1;
  if (report && cap > 0) {
    const size_t k = std::min(cap - 1, out.size());
    std::memcpy(report, out.data(), k);
    report[k] = '\0';
  }
  return STDA_OK;
}

int stda_profile_report(char* buf, size_t cap, size_t* needed) {
  Prof& p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  std::vector<std::string> order;
  std::vector<double> tot;
  std::vector<int> cnt;
  for (size_t i = 0; i + 1 < p.used; i += 2) {
    HIP_TRY(hipEventSynchronize(p.ev[i + 1]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, p.ev[i], p.ev[i + 1]));
    const std::string& t = p.evtag[i / 2];
    size_t k = 0;
    while (k < order.size() && order[k] != t) ++k;
    if (k == order.size()) {
      order.push_back(t);
      tot.push_back(0.0);
      cnt.push_back(0);
    }
    tot[k] += ms;
    cnt[k] += 1;
  }
  std::string out;
  char line[160];
  for (size_t k = 0; k < order.size(); ++k) {
    std::snprintf(line, sizeof(line), "%s\t%d\t%.6f\n", order[k].c_str(), cnt[k], tot[k]);
    out += line;
  }
  if (needed) *needed = out.size() + 1;
  if (buf && cap > 0) {
    const size_t n = std::min(cap - 1, out.size());
    std::memcpy(buf, out.data(), n);
    buf[n] = 0;
  }
  return STDA_OK;
}

int stda_set_grid_cap(int cap) {
  if (cap < 0) return STDA_E_INVALID;
  g_grid_cap.store(cap, std::memory_order_relaxed);
  return STDA_OK;
}

int stda_get_grid_cap(void) { return g_grid_cap.load(std::memory_order_relaxed); }

int stda_bn_layer_count(void) { return 17; }
size_t stda_running_count(void) { return (size_t)net_offsets(0).running_count; }

int stda_set_arch(int flags) {
  if (flags & ~(STDA_ARCH_RES3 | STDA_ARCH_SIGMOID | STDA_ARCH_PW_DW)) return STDA_E_INVALID;
  g_arch.store(flags, std::memory_order_relaxed);
  return STDA_OK;
}

int stda_get_arch(void) { return current_arch(); }

int stda_workspace_size(const stda_segment* segs, int n_segs, int dtype, int mode, int recompute,
                        size_t* saved_bytes, size_t* ws_bytes) {
  if (int r = validate_segs(segs, n_segs)) return r;
  if ((dtype != STDA_FP32 && dtype != STDA_BF16) || (mode != STDA_EVAL && mode != STDA_TRAIN)) return STDA_E_INVALID;
  Plan P;
  build_plan(segs, n_segs, dtype, mode, recompute, P);
  if (saved_bytes) *saved_bytes = P.saved_bytes;
  if (ws_bytes) *ws_bytes = P.ws_bytes;
  return STDA_OK;
}

int stda_forward(const stda_segment* segs, int n_segs, const float* x, const float* w, float* running, float* z,
                 void* saved, size_t saved_bytes, void* ws, size_t ws_bytes, int dtype, int mode, int recompute,
                 hipStream_t stream) {
  try {
    if (int r = validate_segs(segs, n_segs)) return r;
    if ((dtype != STDA_FP32 && dtype != STDA_BF16) || (mode != STDA_EVAL && mode != STDA_TRAIN)) return STDA_E_INVALID;
    if (!x || !w || !running || !z || !ws) return STDA_E_INVALID;
    Plan P;
    build_plan(segs, n_segs, dtype, mode, recompute, P);
    if (ws_bytes < P.ws_bytes) return STDA_E_WORKSPACE;
    if (mode == STDA_TRAIN && (!saved || saved_bytes < P.saved_bytes)) return STDA_E_WORKSPACE;
    const int r = dtype == STDA_BF16 ? forward_all<bf16>(P, x, w, running, z, (char*)saved, (char*)ws, stream)
                                     : forward_all<float>(P, x, w, running, z, (char*)saved, (char*)ws, stream);
    if (r == STDA_OK && mode == STDA_TRAIN) saved_record(saved, saved_key(segs, n_segs, dtype, recompute, P.arch));
    return r;
  } catch (...) {
    return STDA_E_INVALID;
  }
}

int stda_forward_noalloc(const stda_segment* segs, int n_segs, const float* x, const float* w, const float* running,
                         float* z, int dtype, hipStream_t stream) {
  try {
    if (int r = validate_segs(segs, n_segs)) return r;
    if (dtype != STDA_FP32 && dtype != STDA_BF16) return STDA_E_INVALID;
    if (!x || !w || !running || !z) return STDA_E_INVALID;
    Plan P;
    build_plan(segs, n_segs, dtype, STDA_EVAL, 0, P);
    if (P.ws_bytes > STDA_NOALLOC_WS_MAX) return STDA_E_WORKSPACE;
    char* ws = nullptr;
    if (int r = noalloc_scratch(stream, &ws)) return r;
    // EVAL reads the running statistics only
    float* rn = const_cast<float*>(running);
    return dtype == STDA_BF16 ? forward_all<bf16>(P, x, w, rn, z, nullptr, ws, stream)
                              : forward_all<float>(P, x, w, rn, z, nullptr, ws, stream);
  } catch (...) {
    return STDA_E_INVALID;
  }
}

int stda_eval_fold_size(int dtype, size_t* bytes) {
  if ((dtype != STDA_FP32 && dtype != STDA_BF16) || !bytes) return STDA_E_INVALID;
  if (!fold_arch_ok(current_arch())) return STDA_E_INVALID;
  *bytes = fold_layout(dtype).bytes;
  return STDA_OK;
}

int stda_eval_fold(const float* w, const float* running, void* folded, size_t folded_bytes, int dtype,
                   hipStream_t stream) {
  try {
    if ((dtype != STDA_FP32 && dtype != STDA_BF16) || !w || !running || !folded) return STDA_E_INVALID;
    if (!fold_arch_ok(current_arch())) return STDA_E_INVALID;
    const FoldLayout L = fold_layout(dtype);
    if (folded_bytes < L.bytes) return STDA_E_WORKSPACE;
    char* base = static_cast<char*>(folded);
    float* wf = reinterpret_cast<float*>(base + L.wf_off);
    const NetOffsets& no = net_offsets(L.P.arch);
    HIP_TRY(hipMemcpyAsync(wf, w, sizeof(float) * no.param_count, hipMemcpyDeviceToDevice, stream));
    FoldArgs fa{};
    fa.no = no;
    for (int k = 0; k < 4; ++k) {
      fa.cin[k] = kBlocks[k].cin;
      fa.cout[k] = kBlocks[k].cout;
      fa.dec[k] = kBlocks[k].dec;
    }
    fa.ids = no.param_count;
    k_fold_eval<<<10, 256, 0, stream>>>(w, running, wf, fa);
    HIP_TRY(hipGetLastError());
    const float* wk = nullptr;
    return prepare_weights(L.P, wf, base, stream, &wk);
  } catch (...) {
    return STDA_E_INVALID;
  }
}

int stda_forward_folded(const stda_segment* segs, int n_segs, const float* x, const void* folded, size_t folded_bytes,
                        float* z, void* ws, size_t ws_bytes, int dtype, hipStream_t stream) {
  try {
    if (int r = validate_segs(segs, n_segs)) return r;
    if ((dtype != STDA_FP32 && dtype != STDA_BF16) || !x || !folded || !z || !ws) return STDA_E_INVALID;
    if (!fold_arch_ok(current_arch())) return STDA_E_INVALID;
    const FoldLayout L = fold_layout(dtype);
    Plan P;
    build_plan(segs, n_segs, dtype, STDA_EVAL, 0, P);
    if (folded_bytes < L.bytes || ws_bytes < P.ws_bytes) return STDA_E_WORKSPACE;
    return dtype == STDA_BF16 ? forward_folded_all<bf16>(P, L, x, static_cast<const char*>(folded), z, (char*)ws, stream)
                              : forward_folded_all<float>(P, L, x, static_cast<const char*>(folded), z, (char*)ws, stream);
  } catch (...) {
    return STDA_E_INVALID;
  }
}

int stda_backward(const stda_segment* segs, int n_segs, const float* x, const float* dz, const float* w,
                  const void* saved, size_t saved_bytes, float* dw, float* dx, void* ws, size_t ws_bytes, int dtype,
                  int recompute, hipStream_t stream) {
  try {
    if (int r = validate_segs(segs, n_segs)) return r;
    if (dtype != STDA_FP32 && dtype != STDA_BF16) return STDA_E_INVALID;
    if (!x || !dz || !w || !saved || !dw || !ws) return STDA_E_INVALID;
    Plan P;
    build_plan(segs, n_segs, dtype, STDA_TRAIN, recompute, P);
    if (ws_bytes < P.ws_bytes || saved_bytes < P.saved_bytes) return STDA_E_WORKSPACE;
    if (!saved_matches(saved, saved_key(segs, n_segs, dtype, recompute, P.arch))) return STDA_E_INVALID;
    if (dtype == STDA_BF16)
      return backward_all<bf16>(P, dz, x, w, (const char*)saved, dw, dx, (char*)ws, stream);
    return backward_all<float>(P, dz, x, w, (const char*)saved, dw, dx, (char*)ws, stream);
  } catch (...) {
    return STDA_E_INVALID;
  }
}

int stda_mse_loss(const stda_segment* segs, int n_segs, const float* z, const float* y, double* loss_dev, float* dz,
                  void* ws, size_t ws_bytes, hipStream_t stream) {
  if (int r = validate_segs(segs, n_segs)) return r;
  if (!z || !y || !loss_dev || !dz || !ws) return STDA_E_INVALID;
  // the loss uses the first kMaxGrid doubles of ws (any workspace of these segments holds them)
  if (ws_bytes < sizeof(double) * kMaxGrid) return STDA_E_WORKSPACE;
  double* part = reinterpret_cast<double*>(ws);
  int used = 0;
  for (int s = 0; s < n_segs; ++s) {
    const int64_t n = (int64_t)segs[s].n * segs[s].H * segs[s].W;
    const int g = std::min(grid_for(n), kMaxGrid / n_segs);
    k_mse<<<g, 256, 0, stream>>>(z + segs[s].z_off, y + segs[s].z_off, dz + segs[s].z_off, part + used, n);
    LAUNCH_CHECK();
    used += g;
  }
  k_sum_f64<<<1, 256, 0, stream>>>(part, used, loss_dev);
  LAUNCH_CHECK();
  return STDA_OK;
}

int stda_sinr(const float* maps, const uint8_t* o_mask, const uint8_t* n_mask, int n_maps, int H, int W,
              double* out_dev, hipStream_t stream) {
  if (!maps || !o_mask || !n_mask || !out_dev || n_maps < 1 || H < 1 || W < 1) return STDA_E_INVALID;
  k_sinr<<<n_maps, 256, 0, stream>>>(maps, o_mask, n_mask, (int64_t)H * W, out_dev);
  LAUNCH_CHECK();
  return STDA_OK;
}

int stda_sgd_step(float* w, const float* dw, int64_t n, float lr, float weight_decay, uint16_t* w_bf16,
                  hipStream_t stream) {
  if (!w || !dw || n < 0) return STDA_E_INVALID;
  if (n == 0) return STDA_OK;
  k_sgd<<<grid_for(n, 1024), 256, 0, stream>>>(w, dw, n, lr, weight_decay, w_bf16);
  LAUNCH_CHECK();
  return STDA_OK;
}

}  // extern "C"
