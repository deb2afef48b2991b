// Host side of libmra.so: contexts, resident reference sets, validation,
// chunk planning and the launch sequence of one MRA pass (Algorithm 1).
// Every entry point is extern "C", catches everything, and reports through
// an int status plus a per-context message (see include/mra.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mra.h"
#include "mra_common.h"

using namespace mra;

namespace {

constexpr size_t kLdsMax = 160 * 1024;

// Device scratch of mra_align_noalloc (callers that cannot allocate): the
// per-chunk particle operand and row results live here instead of the
// context's workspace.  Each device holds its own copy for the life of the
// process; host code reaches it only through the address that
// hipGetSymbolAddress returns for the device (scratch_ptr), never through
// the symbol itself.
constexpr size_t kScratchBytes = 256ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Refset {
  mra_geom g{};
  int K = 0, R = 0, R4 = 0, NS = 0, n_kt = 0;
  float* B32 = nullptr;
  uint16_t* B16 = nullptr;
  float2* G1 = nullptr;    // K = 1: spectrum table of the fused single-reference kernel
  float* qhat = nullptr;
  double* norm = nullptr;
  Stencil* stencil = nullptr;
  float b_scale = 1.f;
  int dmin = 0, dmax = 0;  // range of stencil floor offsets
  int variant = 0;         // correlation kernel tile configuration
  int chunk = 0;           // particles per chunk (0: from the workspace cap)
  int prune = 1;           // exact pruning of the inverse FFT in the correlation kernel
  int run_tiles = 0;       // row tiles per correlation workgroup (0: from the launch size)
};

struct Fail {
  int code;
  std::string msg;
};

}  // namespace

struct mra_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  uint64_t cap = 0;
  bool failed = false;
  std::string err;
  std::map<int32_t, Refset> refs;
  double2* cs64 = nullptr;
  float2* cs32 = nullptr;
  std::map<std::string, DevBuf> ws;
  int n_cu = 256;
  void* scratch = nullptr; // this device's copy of the no-allocation scratch
  bool profiling = false;
  std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> prof;
};

namespace {

void hip_check(mra_ctx* c, hipError_t e, const char* what) {
  if (e != hipSuccess) {
    c->failed = true;
    throw Fail{MRA_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e)};
  }
}

// Address of the no-allocation scratch on c's device (current at the call):
// resolved once per device, kept for every later context on it.
void* scratch_ptr(mra_ctx* c) {
  if (c->device < 0 || c->device >= kMaxDevices) throw Fail{MRA_E_INVAL, "device ordinal out of range"};
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  void*& p = g_scratch_ptr[c->device];
  if (!p) {
    void* q = nullptr;
    hip_check(c, hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!q) throw Fail{MRA_E_DEVICE, "no device address for the scratch array"};
    p = q;
  }
  return p;
}

void* alloc(mra_ctx* c, size_t bytes, const char* what) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes < 16 ? 16 : bytes);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    throw Fail{MRA_E_NOMEM, std::string("out of device memory allocating ") + what};
  }
  hip_check(c, e, what);
  return p;
}

void* ws_get(mra_ctx* c, const std::string& name, size_t bytes) {
  DevBuf& b = c->ws[name];
  if (b.bytes < bytes) {
    uint64_t total = bytes;  // the workspace after this buffer grows
    for (const auto& kv : c->ws)
      if (&kv.second != &b) total += kv.second.bytes;
    if (total > c->cap)
      throw Fail{MRA_E_NOMEM, "workspace cap of " + std::to_string(c->cap) + " bytes is too small (" + name +
                                  " needs " + std::to_string(bytes) + " bytes)"};
    if (b.p) hip_check(c, hipFree(b.p), "hipFree");
    b.p = nullptr;
    b.bytes = 0;
    b.p = alloc(c, bytes, name.c_str());
    b.bytes = bytes;
  }
  return b.p;
}

// Runs `launch` between two events on the context stream when profiling.
template <class F>
void timed(mra_ctx* c, const char* group, F&& launch) {
  if (!c->profiling) {
    launch();
    return;
  }
  hipEvent_t a, b;
  hip_check(c, hipEventCreate(&a), "hipEventCreate");
  hip_check(c, hipEventCreate(&b), "hipEventCreate");
  hip_check(c, hipEventRecord(a, c->stream), "hipEventRecord");
  launch();
  hip_check(c, hipEventRecord(b, c->stream), "hipEventRecord");
  c->prof[group].emplace_back(a, b);
}

void clear_profile(mra_ctx* c) {
  for (auto& kv : c->prof)
    for (auto& e : kv.second) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  c->prof.clear();
}

void free_refset(Refset& r) {
  for (void* p : {(void*)r.B32, (void*)r.B16, (void*)r.G1, (void*)r.qhat, (void*)r.norm, (void*)r.stencil})
    if (p) (void)hipFree(p);
  r = Refset{};
}

// cos / sin of 2 pi j / n built from the first octant so that the table is
// exactly symmetric (cos even, sin odd, quarter turns exact).
void build_cs(int n, std::vector<double>& c, std::vector<double>& s) {
  c.assign(n, 0.0);
  s.assign(n, 0.0);
  const double two_pi = 6.283185307179586476925286766559;
  const int q = n / 4, e = n / 8;
  std::vector<double> c0(q + 1), s0(q + 1);
  for (int j = 0; j <= e; ++j) {
    c0[j] = std::cos(two_pi * j / n);
    s0[j] = std::sin(two_pi * j / n);
  }
  for (int j = e + 1; j <= q; ++j) {
    c0[j] = s0[q - j];
    s0[j] = c0[q - j];
  }
  for (int j = 0; j < n; ++j) {
    int jj = j, sc = 1, ss = 1;
    if (jj > n / 2) { jj = n - jj; ss = -1; }          // theta -> -theta
    if (jj > q) { jj = n / 2 - jj; sc = -1; }          // theta -> pi - theta
    c[j] = sc * c0[jj];
    s[j] = ss * s0[jj];
  }
}

void check_geom(const mra_geom* g) {
  auto bad = [](const char* m) { throw Fail{MRA_E_INVAL, m}; };
  if (!g) bad("geometry is NULL");
  if (g->L < 8 || g->L > 160) bad("L must be in [8, 160]");
  if (g->r_min < 1 || g->r_max < g->r_min || g->r_max > 64) bad("need 1 <= r_min <= r_max <= 64");
  if (g->n_phi != kNphi) bad("n_phi must be 256 (the only angular sampling the kernels implement)");
  if (g->shift_max < 0 || g->shift_max > 8) bad("shift_max must be in [0, 8]");
  if (g->mirror != 0 && g->mirror != 1) bad("mirror must be 0 or 1");
  if (g->precision < 0 || g->precision > 2) bad("precision must be MRA_FP32, MRA_BF16 or MRA_FP16");
  if (g->normalize != 0 && g->normalize != 1) bad("normalize must be 0 or 1");
  if (g->rescore_rows < 0 || g->rescore_rows > 8) bad("rescore_rows must be in [0, 8]");
}

// Range of the floor offsets of the polar stencil (r cos, r sin) over the
// rings of g: the pixels a zero shift touches lie in [c + dmin, c + dmax + 1].
void stencil_range(const mra_geom& g, int& dmin, int& dmax) {
  std::vector<double> cs, sn;
  build_cs(kNphi, cs, sn);
  dmin = 0;
  dmax = 0;
  for (int r = g.r_min; r <= g.r_max; ++r)
    for (int j = 0; j < kNphi; ++j) {
      const int fx = (int)std::floor(r * cs[j]), fy = (int)std::floor(r * sn[j]);
      dmin = std::min({dmin, fx, fy});
      dmax = std::max({dmax, fx, fy});
    }
}

// The flat candidate index iota = (((k M + m) S1 + sy) S1 + sx) n_phi + a is
// an int32 in every kernel and 0x7fffffff marks "no candidate", so
// K * M * S * n_phi must stay below 2^31.
void check_index_range(int64_t K, int M, int T) {
  const int64_t S1 = 2 * (int64_t)T + 1;
  if (K * M * S1 * S1 * kNphi > (int64_t)INT32_MAX)
    throw Fail{MRA_E_INVAL, "K * mirrors * (2 shift_max + 1)^2 * n_phi must be below 2^31 (int32 candidate index); "
                            "split the references into several refsets"};
}

Refset& get_refset(mra_ctx* c, int32_t id) {
  auto it = c->refs.find(id);
  if (it == c->refs.end()) throw Fail{MRA_E_NOREF, "refset " + std::to_string(id) + " is not loaded"};
  return it->second;
}

struct Plan {
  int T, S1, S, M, pad, Lp, cx;
  int pad_r, Lp_r;  // border and side for the kernels that sample with the FP64 stencil table
};

Plan plan_for(const Refset& rs, int T) {
  if (T < 0 || T > 8) throw Fail{MRA_E_INVAL, "shift_max must be in [0, 8]"};
  check_index_range(rs.K, rs.g.mirror ? 2 : 1, T);
  Plan p;
  p.T = T;
  p.S1 = 2 * T + 1;
  p.S = p.S1 * p.S1;
  p.M = rs.g.mirror ? 2 : 1;
  p.cx = rs.g.L / 2;
  // lowest and highest pixel index touched; the resamplers that take the
  // floor of single-precision positions reach one pixel further either side
  const int lo = p.cx - T + rs.dmin;
  const int hi = p.cx + T + rs.dmax + 1;
  p.pad_r = std::max(0, std::max(-lo, hi - (rs.g.L - 1)));
  p.Lp_r = rs.g.L + 2 * p.pad_r;
  p.pad = std::max(0, std::max(-(lo - 1), hi + 1 - (rs.g.L - 1)));
  p.Lp = rs.g.L + 2 * p.pad;
  if (polar_lds_bytes(p.Lp) > kLdsMax)
    throw Fail{MRA_E_INVAL, "box plus search range too large for the LDS-staged resampler"};
  return p;
}

void check_result(const mra_result* r) {
  if (!r || !r->ref || !r->shift_x || !r->shift_y || !r->psi || !r->mirror || !r->cc)
    throw Fail{MRA_E_INVAL, "result arrays must be non-NULL (cc2, flat_index may be NULL)"};
}

// bytes of the correlation operand A per particle row (one eighth of a tile)
// the operand's element size: 16-bit for the 16-bit contractions
size_t a_elem(const Refset& rs) { return a_elem_bytes(a_layout_for(rs.g.precision, rs.variant)); }
size_t a_bytes_per_row(const Refset& rs) { return (size_t)kSlots * rs.R4 * 64 * a_elem(rs) / kRowTile; }

int64_t chunk_particles(mra_ctx* c, const Refset& rs, const Plan& p) {
  if (rs.chunk > 0) return rs.chunk;
  const uint64_t budget = c->cap / 2;
  const uint64_t per = (uint64_t)p.S * a_bytes_per_row(rs);
  int64_t n = (int64_t)(budget / per);
  return std::max<int64_t>(n, 1);
}

// Device buffers of one alignment chunk of nc particles.
struct ChunkBufs {
  float* A = nullptr;       // particle operand, ceil(nc S / 8) row tiles
  float* rcc = nullptr;     // [nc S] best CC per row
  int* ridx = nullptr;      // [nc S] its flat index
  float* maxabs = nullptr;  // FP16: [nc] max |pixel|
  int32_t* win = nullptr;   // cc2: [nc] chunk-local winner copy
};

size_t tile_bytes_of(const Refset& rs) { return (size_t)kSlots * rs.R4 * 64 * a_elem(rs); }

// Lays the buffers of an nc-particle chunk out from `base` (256-byte
// aligned pieces); returns the bytes used.  base = nullptr only measures.
size_t carve_chunk(const Refset& rs, const Plan& p, int64_t nc, bool fp16, bool cc2, char* base, ChunkBufs* b) {
  const size_t rows = (size_t)nc * p.S;
  const size_t tiles = (rows + kRowTile - 1) / kRowTile;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return q;
  };
  char* A = take(tiles * tile_bytes_of(rs));
  char* rcc = take(rows * sizeof(float));
  char* ridx = take(rows * sizeof(int));
  char* mx = fp16 ? take((size_t)nc * sizeof(float)) : nullptr;
  char* win = cc2 ? take((size_t)nc * sizeof(int32_t)) : nullptr;
  if (b) {
    b->A = (float*)A;
    b->rcc = (float*)rcc;
    b->ridx = (int*)ridx;
    b->maxabs = (float*)mx;
    b->win = (int32_t*)win;
  }
  return off;
}

// Buffers of a chunk from the context's workspace (grown on demand).
ChunkBufs ws_chunk(mra_ctx* c, const Refset& rs, const Plan& p, int nc, const mra_result* out) {
  ChunkBufs b;
  const size_t rows = (size_t)nc * p.S;
  const size_t tiles = (rows + kRowTile - 1) / kRowTile;
  b.A = (float*)ws_get(c, "A", tiles * tile_bytes_of(rs));
  b.rcc = (float*)ws_get(c, "row_cc", rows * sizeof(float));
  b.ridx = (int*)ws_get(c, "row_idx", rows * sizeof(int));
  if (rs.g.precision == kFP16) b.maxabs = (float*)ws_get(c, "maxabs", (size_t)nc * sizeof(float));
  if (out && out->cc2) b.win = (int32_t*)ws_get(c, "win", (size_t)nc * sizeof(int32_t));
  return b;
}

// Largest chunk whose buffers fit `bytes` of scratch (0 if not one particle).
int64_t scratch_chunk(const Refset& rs, const Plan& p, bool cc2, size_t bytes) {
  const bool fp16 = rs.g.precision == kFP16;
  if (carve_chunk(rs, p, 1, fp16, cc2, nullptr, nullptr) > bytes) return 0;
  // the buffers grow with the chunk: bisect for the largest that fits
  int64_t lo = 1, hi = std::min<int64_t>(INT32_MAX / p.S / 2, (int64_t)(bytes / ((size_t)p.S * 8)) + 1);
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (carve_chunk(rs, p, mid, fp16, cc2, nullptr, nullptr) <= bytes) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Sub-step angles of particles n0 .. n0 + nc - 1 from their final parameters.
void refine_chunk(mra_ctx* c, const Refset& rs, const Plan& p, const float* parts, int64_t n0, int64_t nc,
                  const mra_result* out) {
  const int L = rs.g.L;
  const int64_t step = INT32_MAX / 2;
  for (int64_t o = 0; o < nc; o += step) {
    RescoreArgs ra{};
    ra.parts = parts + (size_t)(n0 + o) * L * L;
    ra.n_part = (int)std::min<int64_t>(step, nc - o);
    ra.out_off = n0 + o;
    ra.L = L; ra.R = rs.R; ra.r_min = rs.g.r_min; ra.Lp = p.Lp_r; ra.pad = p.pad_r; ra.cx = p.cx;
    ra.K = rs.K; ra.T = p.T;
    ra.stencil = rs.stencil;
    ra.qhat = rs.qhat;
    ra.ref = out->ref; ra.shift_x = out->shift_x; ra.shift_y = out->shift_y;
    ra.psi = out->psi; ra.mirror = out->mirror;
    ra.psi_frac = out->psi_frac;
    timed(c, "refine", [&] { hip_check(c, launch_refine(ra, c->stream), "refine"); });
  }
}

// One chunk of the alignment pass: resample + FFT -> correlation -> merge
// (-> FP32 re-score for 16-bit contractions).  mode 0 = production,
// mode 3 = debug CC table into `table`.
void run_chunk(mra_ctx* c, const Refset& rs, const Plan& p, const float* parts, int64_t n0, int nc,
               const mra_result* out, float* table, const ChunkBufs& bufs) {
  hipStream_t st = c->stream;
  const int L = rs.g.L;
  const int rows = nc * p.S;
  const int tiles = (rows + kRowTile - 1) / kRowTile;
  const size_t tile_bytes = tile_bytes_of(rs);
  float* A = bufs.A;
  float* rcc = bufs.rcc;
  int* ridx = bufs.ridx;
  // rows past the chunk in its last tile are read as zeros
  if (rows % kRowTile)
    hip_check(c, launch_fill_zero((char*)A + (size_t)(tiles - 1) * tile_bytes, tile_bytes, st), "fill");
  const float* src = parts + (size_t)n0 * L * L;

  float* maxabs = nullptr;
  if (rs.g.precision == kFP16) {
    maxabs = bufs.maxabs;
    timed(c, "maxabs", [&] { hip_check(c, launch_part_maxabs(src, nc, L, maxabs, st), "maxabs"); });
  }

  PolarArgs pa{};
  pa.parts = src;
  pa.n_part = nc;
  pa.L = L; pa.R = rs.R; pa.R4 = rs.R4; pa.T = p.T; pa.S1 = p.S1; pa.S = p.S;
  pa.Lp = p.Lp; pa.pad = p.pad; pa.cx = p.cx;
  pa.r_min = rs.g.r_min;
  // the CC table is written by the form launch_corr picks for it
  pa.a_layout = a_layout_for(rs.g.precision, table ? (rs.g.precision == kFP32 ? 2 : 0) : rs.variant);
  pa.prec = rs.g.precision;
  pa.maxabs = maxabs;
  pa.cs64 = c->cs64;
  pa.out = A;
  timed(c, "polar", [&] { hip_check(c, launch_polar(0, pa, st), "polar"); });

  CorrArgs ca{};
  ca.A = A;
  ca.a_layout = pa.a_layout;
  ca.n_row_tiles = tiles;
  ca.rows = rows;
  ca.B32 = rs.B32;
  ca.B16 = rs.B16;
  ca.R = rs.R; ca.R4 = rs.R4; ca.NS = rs.NS; ca.BT = b16_tail_width(rs.R4); ca.n_ref_tiles = rs.n_kt; ca.K = rs.K; ca.S = p.S; ca.M = p.M;
  ca.maxabs = maxabs;
  ca.b_scale = rs.b_scale;
  ca.cs32 = c->cs32;
  ca.row_cc = rcc;
  ca.row_idx = ridx;
  ca.table = table;
  ca.prune = rs.prune;
  ca.tiles_per_run = table ? 1 : (rs.run_tiles > 0 ? rs.run_tiles : corr_tiles_per_run(tiles, c->n_cu));
  ca.margin = rs.g.rescore_rows >= 2 ? rerank_margin(rs.g.precision) : 0.f;
  timed(c, "corr", [&] { hip_check(c, launch_corr(rs.g.precision, rs.variant, table != nullptr, ca, st), "corr"); });
  if (table) return;

  MergeArgs ma{};
  ma.row_cc = rcc; ma.row_idx = ridx;
  ma.n_part = nc; ma.S = p.S; ma.S1 = p.S1; ma.T = p.T; ma.M = p.M;
  ma.out_off = n0;
  ma.ref = out->ref; ma.shift_x = out->shift_x; ma.shift_y = out->shift_y;
  ma.psi = out->psi; ma.mirror = out->mirror; ma.flat = out->flat_index;
  ma.cc = out->cc; ma.cc2 = out->cc2;
  int32_t* win = out->cc2 ? bufs.win : nullptr;
  ma.win = win;
  timed(c, "merge", [&] { hip_check(c, launch_merge(ma, st), "merge"); });

  if (rs.g.precision != kFP32) {
    RescoreArgs ra{};
    ra.parts = src;
    ra.n_part = nc;
    ra.out_off = n0;
    ra.L = L; ra.R = rs.R; ra.r_min = rs.g.r_min; ra.Lp = p.Lp_r; ra.pad = p.pad_r; ra.cx = p.cx;
    ra.K = rs.K; ra.T = p.T;
    ra.stencil = rs.stencil;
    ra.qhat = rs.qhat;
    ra.ref = out->ref; ra.shift_x = out->shift_x; ra.shift_y = out->shift_y;
    ra.psi = out->psi; ra.mirror = out->mirror;
    ra.cc = out->cc;
    ra.rows = rs.g.rescore_rows;
    ra.margin = rerank_margin(rs.g.precision);
    ra.S1 = p.S1; ra.S = p.S; ra.M = p.M;
    ra.row_cc = rcc; ra.row_idx = ridx;
    ra.ref_w = out->ref; ra.shift_x_w = out->shift_x; ra.shift_y_w = out->shift_y;
    ra.psi_w = out->psi; ra.mirror_w = out->mirror; ra.flat_w = out->flat_index;
    ra.win = win;
    timed(c, "rescore", [&] { hip_check(c, launch_rescore(ra, st), "rescore"); });
  }

  if (out->cc2) {
    // runner-up: the same contraction with each particle's winner left out;
    // the best that remains is the best over every other candidate
    ca.excl = win;
    timed(c, "corr2", [&] { hip_check(c, launch_corr_runner_up(rs.g.precision, ca, st), "corr2"); });
    MergeArgs m2 = ma;
    m2.win = nullptr;
    m2.runner_up = 1;
    timed(c, "merge", [&] { hip_check(c, launch_merge(m2, st), "merge"); });
  }
  if (out->psi_frac) refine_chunk(c, rs, p, parts, n0, nc, out);
}

// One reference (K = 1): the fused single-reference kernel over the whole
// stack; it needs no workspace.
void run_single(mra_ctx* c, const Refset& rs, const Plan& p, const float* parts, int64_t N, const mra_result* out) {
  const int L = rs.g.L;
  const int64_t step = INT32_MAX / 2;
  for (int64_t n0 = 0; n0 < N; n0 += step) {
    RfaArgs ra{};
    ra.parts = parts + (size_t)n0 * L * L;
    ra.n_part = (int)std::min<int64_t>(step, N - n0);
    ra.out_off = n0;
    ra.L = L; ra.R = rs.R; ra.T = p.T; ra.S1 = p.S1; ra.S = p.S; ra.M = p.M;
    ra.Lp = p.Lp; ra.pad = p.pad; ra.cx = p.cx; ra.r_min = rs.g.r_min;
    ra.stencil = rs.stencil;
    ra.cs64 = c->cs64;
    ra.G = rs.G1;
    ra.ref = out->ref; ra.shift_x = out->shift_x; ra.shift_y = out->shift_y;
    ra.psi = out->psi; ra.mirror = out->mirror; ra.flat = out->flat_index;
    ra.cc = out->cc; ra.cc2 = out->cc2;
    timed(c, "rfa", [&] { hip_check(c, launch_rfa(ra, c->stream), "rfa"); });
  }
  if (out->psi_frac) refine_chunk(c, rs, p, parts, 0, N, out);
}

// noalloc: the chunk buffers come from the device scratch array instead of
// the workspace, so nothing is allocated (the path of mra_align_noalloc).
void align_impl(mra_ctx* c, int32_t id, const float* parts, int64_t N, int T, const mra_result* out,
                float* table, bool noalloc = false) {
  Refset& rs = get_refset(c, id);
  if (N < 0) throw Fail{MRA_E_INVAL, "N must be >= 0"};
  if (N == 0) return;
  if (!parts) throw Fail{MRA_E_INVAL, "parts is NULL"};
  if (!table) check_result(out);
  const Plan p = plan_for(rs, T < 0 ? rs.g.shift_max : T);
  if (rs.K == 1 && !table) {
    run_single(c, rs, p, parts, N, out);
    return;
  }
  int64_t step = std::min<int64_t>(chunk_particles(c, rs, p), (int64_t)(INT32_MAX / p.S / 2));
  if (noalloc) {
    step = scratch_chunk(rs, p, out && out->cc2, kScratchBytes);
    if (step < 1)
      throw Fail{MRA_E_INVAL, "one particle's operand exceeds the " + std::to_string(kScratchBytes >> 20) +
                                  " MiB no-allocation scratch"};
    if (!c->scratch) throw Fail{MRA_E_DEVICE, "no-allocation scratch not resolved on this device"};
  }
  for (int64_t n0 = 0; n0 < N; n0 += step) {
    const int nc = (int)std::min<int64_t>(step, N - n0);
    float* tab = table ? table + (size_t)n0 * rs.K * p.M * p.S * kNphi : nullptr;
    ChunkBufs b;
    if (noalloc) carve_chunk(rs, p, nc, rs.g.precision == kFP16, out && out->cc2, (char*)c->scratch, &b);
    else b = ws_chunk(c, rs, p, nc, out);
    run_chunk(c, rs, p, parts, n0, nc, out, tab, b);
  }
}

// One piece of a stack inside a batched wave.
struct Piece {
  int stack;
  const Refset* rs;
  Plan p;
  int64_t n0;
  int nc;
  size_t a_off;  // first byte of the piece in the wave's A buffer
  size_t row0;   // first row in the wave's row-result buffers
};

void launch_wave(mra_ctx* c, const mra_stack* stacks, std::vector<Piece>& w) {
  hipStream_t st = c->stream;
  if (w.size() == 1) {  // one piece fills the chip by itself: the plain per-chunk launches
    const Piece& pc = w[0];
    const mra_stack& sk = stacks[pc.stack];
    run_chunk(c, *pc.rs, pc.p, sk.parts, pc.n0, pc.nc, &sk.out, nullptr, ws_chunk(c, *pc.rs, pc.p, pc.nc, &sk.out));
    return;
  }
  const Refset& rs0 = *w[0].rs;
  const int prec = rs0.g.precision, variant = rs0.variant;
  size_t a_bytes = 0, rows = 0, part_total = 0;
  for (Piece& pc : w) {
    part_total += pc.nc;
    pc.a_off = a_bytes;
    pc.row0 = rows;
    const size_t r = (size_t)pc.nc * pc.p.S;
    a_bytes += (r + kRowTile - 1) / kRowTile * tile_bytes_of(*pc.rs);
    rows += r;
  }
  char* A = (char*)ws_get(c, "A", a_bytes);
  float* rcc = (float*)ws_get(c, "row_cc", rows * sizeof(float));
  int* ridx = (int*)ws_get(c, "row_idx", rows * sizeof(int));
  float* maxabs = prec == kFP16 ? (float*)ws_get(c, "maxabs", (size_t)part_total * sizeof(float)) : nullptr;

  PolarBatch pb{};
  CorrBatch cb{};
  MergeBatch mb{};
  RescoreBatch rb{};
  pb.n = cb.n = mb.n = rb.n = (int)w.size();
  int part = 0, run = 0;
  for (size_t i = 0; i < w.size(); ++i) {
    const Piece& pc = w[i];
    const Refset& rs = *pc.rs;
    const mra_stack& sk = stacks[pc.stack];
    const int L = rs.g.L;
    const int prow = pc.nc * pc.p.S;
    const int ptiles = (prow + kRowTile - 1) / kRowTile;
    const size_t tile_bytes = tile_bytes_of(rs);
    float* Ap = (float*)(A + pc.a_off);
    const float* src = sk.parts + (size_t)pc.n0 * L * L;
    if (prow % kRowTile)
      hip_check(c, launch_fill_zero((char*)Ap + (size_t)(ptiles - 1) * tile_bytes, tile_bytes, st), "fill");
    float* mx = nullptr;
    if (maxabs) {
      mx = maxabs + part;
      timed(c, "maxabs", [&] { hip_check(c, launch_part_maxabs(src, pc.nc, L, mx, st), "maxabs"); });
    }
    PolarArgs& pa = pb.piece[i];
    pa.parts = src; pa.n_part = pc.nc;
    pa.L = L; pa.R = rs.R; pa.R4 = rs.R4; pa.T = pc.p.T; pa.S1 = pc.p.S1; pa.S = pc.p.S;
    pa.Lp = pc.p.Lp; pa.pad = pc.p.pad; pa.cx = pc.p.cx; pa.r_min = rs.g.r_min; pa.cs64 = c->cs64; pa.out = Ap;
    pa.a_layout = a_layout_for(prec, variant);
    pa.prec = prec;
    pa.maxabs = mx;
    pb.start[i] = part;

    CorrArgs& ca = cb.piece[i];
    ca.A = Ap; ca.a_layout = pa.a_layout; ca.n_row_tiles = ptiles; ca.rows = prow;
    ca.B32 = rs.B32; ca.B16 = rs.B16;
    ca.R = rs.R; ca.R4 = rs.R4; ca.NS = rs.NS; ca.BT = b16_tail_width(rs.R4); ca.n_ref_tiles = rs.n_kt; ca.K = rs.K; ca.S = pc.p.S; ca.M = pc.p.M;
    ca.maxabs = mx; ca.b_scale = rs.b_scale; ca.cs32 = c->cs32;
    ca.row_cc = rcc + pc.row0; ca.row_idx = ridx + pc.row0; ca.table = nullptr; ca.prune = rs.prune;
    ca.tiles_per_run = rs.run_tiles > 0 ? rs.run_tiles : corr_tiles_per_run(ptiles, c->n_cu);
    ca.margin = rs.g.rescore_rows >= 2 ? rerank_margin(prec) : 0.f;
    cb.run_start[i] = run;

    MergeArgs& ma = mb.piece[i];
    ma.row_cc = rcc + pc.row0; ma.row_idx = ridx + pc.row0;
    ma.n_part = pc.nc; ma.S = pc.p.S; ma.S1 = pc.p.S1; ma.T = pc.p.T; ma.M = pc.p.M; ma.out_off = pc.n0;
    ma.ref = sk.out.ref; ma.shift_x = sk.out.shift_x; ma.shift_y = sk.out.shift_y; ma.psi = sk.out.psi;
    ma.mirror = sk.out.mirror; ma.flat = sk.out.flat_index; ma.cc = sk.out.cc; ma.cc2 = sk.out.cc2;
    mb.start[i] = part;

    RescoreArgs& ra = rb.piece[i];
    ra.parts = src; ra.n_part = pc.nc; ra.out_off = pc.n0;
    ra.L = L; ra.R = rs.R; ra.r_min = rs.g.r_min; ra.Lp = pc.p.Lp_r; ra.pad = pc.p.pad_r; ra.cx = pc.p.cx;
    ra.K = rs.K; ra.T = pc.p.T; ra.stencil = rs.stencil; ra.qhat = rs.qhat;
    ra.ref = sk.out.ref; ra.shift_x = sk.out.shift_x; ra.shift_y = sk.out.shift_y; ra.psi = sk.out.psi;
    ra.mirror = sk.out.mirror; ra.cc = sk.out.cc;
    ra.rows = rs.g.rescore_rows; ra.margin = rerank_margin(prec); ra.S1 = pc.p.S1; ra.S = pc.p.S; ra.M = pc.p.M;
    ra.row_cc = rcc + pc.row0; ra.row_idx = ridx + pc.row0;
    ra.ref_w = sk.out.ref; ra.shift_x_w = sk.out.shift_x; ra.shift_y_w = sk.out.shift_y;
    ra.psi_w = sk.out.psi; ra.mirror_w = sk.out.mirror; ra.flat_w = sk.out.flat_index;
    ra.win = nullptr;
    rb.start[i] = part;

    part += pc.nc;
    run += (ptiles + ca.tiles_per_run - 1) / ca.tiles_per_run;
  }
  pb.start[w.size()] = mb.start[w.size()] = rb.start[w.size()] = part;
  cb.run_start[w.size()] = run;
  timed(c, "polar", [&] { hip_check(c, launch_polar_batch(pb, st), "polar batch"); });
  const int grid = run;
  timed(c, "corr", [&] { hip_check(c, launch_corr_batch(prec, variant, cb, grid, st), "corr batch"); });
  timed(c, "merge", [&] { hip_check(c, launch_merge_batch(mb, st), "merge batch"); });
  if (prec != kFP32) timed(c, "rescore", [&] { hip_check(c, launch_rescore_batch(rb, st), "rescore batch"); });
}

void run_batch(mra_ctx* c, const mra_stack* stacks, int n, const std::vector<Plan>& plans) {
  const uint64_t budget = c->cap / 2;
  // stacks that share a correlation instantiation (precision, tile variant,
  // and the ring bucket: for the 16-bit forms R4 <= 8, 9..12 or 13..16, for
  // the FP32 resident 8-wave variant the exact R4; launches that mix them
  // take the kernel's slower run-time form) are packed into the same waves;
  // within a group the caller's order holds
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  auto group = [](const Refset& rs) {
    const int bucket = rs.g.precision == kFP32 ? (rs.variant == 0 ? rs.R4 : 0)
                                               : (rs.R4 <= 8 ? 0 : (rs.R4 <= 12 ? 1 : 2));
    return (rs.g.precision * 16 + rs.variant) * 32 + bucket;
  };
  auto key = [&](int i) {
    if (stacks[i].N <= 0) return 0;
    return group(get_refset(c, stacks[i].refset_id));
  };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return key(x) < key(y); });
  std::vector<Piece> wave;
  uint64_t used = 0;
  for (int i : order) {
    const mra_stack& s = stacks[i];
    if (s.N <= 0) continue;
    const Refset& rs = get_refset(c, s.refset_id);
    const Plan& p = plans[i];
    if (rs.K == 1) {  // one reference: the fused single-reference kernel
      run_single(c, rs, p, s.parts, s.N, &s.out);
      continue;
    }
    if (s.out.cc2 || s.out.psi_frac) {  // runner-up or refinement: the per-chunk path
      const int64_t step = std::min<int64_t>(chunk_particles(c, rs, p), (int64_t)(INT32_MAX / p.S / 2));
      for (int64_t n0 = 0; n0 < s.N; n0 += step) {
        const int nc = (int)std::min<int64_t>(step, s.N - n0);
        run_chunk(c, rs, p, s.parts, n0, nc, &s.out, nullptr, ws_chunk(c, rs, p, nc, &s.out));
      }
      continue;
    }
    const uint64_t per = (uint64_t)p.S * a_bytes_per_row(rs);
    const int64_t cap_n = rs.chunk > 0 ? rs.chunk : std::max<int64_t>(1, (int64_t)(budget / per));
    for (int64_t n0 = 0; n0 < s.N;) {
      const bool compatible = wave.empty() || group(*wave[0].rs) == group(rs);
      if (!compatible || (int)wave.size() == kMaxBatchPieces || used + per > budget) {
        if (!wave.empty()) launch_wave(c, stacks, wave);
        wave.clear();
        used = 0;
      }
      const int64_t room = std::max<int64_t>(1, (int64_t)((budget - used) / per));
      const int nc = (int)std::min<int64_t>({s.N - n0, room, cap_n, (int64_t)(INT32_MAX / p.S / 2)});
      wave.push_back(Piece{i, &rs, p, n0, nc, 0, 0});
      used += (uint64_t)nc * per + (uint64_t)kRowTile * a_bytes_per_row(rs);
      n0 += nc;
    }
  }
  if (!wave.empty()) launch_wave(c, stacks, wave);
}

void load_refs_impl(mra_ctx* c, int32_t id, const float* refs, int32_t K, const mra_geom* g) {
  check_geom(g);
  if (K < 1) throw Fail{MRA_E_INVAL, "K must be >= 1"};
  check_index_range(K, g->mirror ? 2 : 1, g->shift_max);
  if (!refs) throw Fail{MRA_E_INVAL, "refs is NULL"};
  Refset rs;
  rs.g = *g;
  rs.K = K;
  rs.R = g->r_max - g->r_min + 1;
  rs.R4 = (rs.R + 3) / 4;
  rs.NS = (rs.R4 + 7) / 8;
  rs.n_kt = (K + kRefTile - 1) / kRefTile;
  rs.variant = corr_default_variant(g->precision, rs.R4);
  hipStream_t st = c->stream;
  try {
    // particle sampling stencil, exactly symmetric in j <-> 256 - j
    std::vector<double> cs, sn;
    build_cs(kNphi, cs, sn);
    std::vector<Stencil> sten((size_t)rs.R * kNphi);
    rs.dmin = 0;
    rs.dmax = 0;
    for (int r = 0; r < rs.R; ++r)
      for (int j = 0; j < kNphi; ++j) {
        const double rr = g->r_min + r;
        const double x = rr * cs[j], y = rr * sn[j];
        const double fx = std::floor(x), fy = std::floor(y);
        Stencil s;
        s.bx = 4 * (int)fx;
        s.dy = (int)fy;
        s.fx = (float)(x - fx);
        s.fy = (float)(y - fy);
        sten[(size_t)r * kNphi + j] = s;
        rs.dmin = std::min({rs.dmin, (int)fx, (int)fy});
        rs.dmax = std::max({rs.dmax, (int)fx, (int)fy});
      }
    rs.stencil = (Stencil*)alloc(c, sten.size() * sizeof(Stencil), "stencil");
    hip_check(c, hipMemcpyAsync(rs.stencil, sten.data(), sten.size() * sizeof(Stencil), hipMemcpyHostToDevice, st), "memcpy");

    RefArgs ra{};
    ra.refs = refs;
    ra.K = K; ra.L = g->L; ra.r_min = g->r_min; ra.R = rs.R; ra.R4 = rs.R4; ra.NS = rs.NS;
    ra.n_ref_tiles = rs.n_kt; ra.normalize = g->normalize; ra.prec = g->precision;
    ra.cs64 = c->cs64;
    ra.q64 = (double*)ws_get(c, "ref_q64", (size_t)K * rs.R * kNphi * sizeof(double));
    ra.inv = (double*)ws_get(c, "ref_inv", (size_t)K * sizeof(double));
    ra.Qs = (double2*)ws_get(c, "ref_Qs", (size_t)K * 129 * rs.R * sizeof(double2));
    ra.bmax = (float*)ws_get(c, "ref_bmax", 256);
    rs.norm = (double*)alloc(c, (size_t)K * sizeof(double), "norm");
    rs.qhat = (float*)alloc(c, (size_t)K * rs.R * kNphi * sizeof(float), "qhat");
    ra.norm = rs.norm;
    ra.qhat32 = rs.qhat;
    hip_check(c, hipMemsetAsync(ra.bmax, 0, sizeof(float), st), "memset");
    hip_check(c, launch_ref_stage1(ra, st), "ref stage 1");
    std::vector<double> norms(K);
    float bmax = 0.f;
    hip_check(c, hipMemcpyAsync(norms.data(), rs.norm, K * sizeof(double), hipMemcpyDeviceToHost, st), "memcpy");
    hip_check(c, hipMemcpyAsync(&bmax, ra.bmax, sizeof(float), hipMemcpyDeviceToHost, st), "memcpy");
    hip_check(c, hipStreamSynchronize(st), "sync");
    if (g->normalize)
      for (int k = 0; k < K; ++k)
        if (!(norms[k] > 0.0))
          throw Fail{MRA_E_DEGENERATE, "reference " + std::to_string(k) + " has zero weighted ring norm"};
    rs.b_scale = 1.f;
    if (g->precision == kFP16 && bmax > 0.f) rs.b_scale = std::ldexp(1.f, 14 - (int)std::ceil(std::log2(bmax)));
    ra.b_scale = rs.b_scale;
    if (g->precision == kFP32)
      rs.B32 = (float*)alloc(c, (size_t)rs.n_kt * kSlots * rs.R4 * 64 * sizeof(float), "B32");
    else
      rs.B16 = (uint16_t*)alloc(c, (size_t)rs.n_kt * kSlots * b16_slot_elems(rs.R4) * sizeof(uint16_t), "B16");
    ra.B32 = rs.B32;
    ra.B16 = rs.B16;
    if (K == 1) rs.G1 = (float2*)alloc(c, (size_t)rs.R * kSlots * sizeof(float2), "G1");
    ra.G1 = rs.G1;
    hip_check(c, launch_ref_stage2(ra, st), "ref stage 2");
  } catch (...) {
    free_refset(rs);
    throw;
  }
  auto it = c->refs.find(id);
  if (it != c->refs.end()) {
    hip_check(c, hipStreamSynchronize(st), "sync");
    free_refset(it->second);
    c->refs.erase(it);
  }
  c->refs[id] = rs;
}

void averages_core(mra_ctx* c, int K, int L, const float* parts, int64_t N, const mra_result* params,
                   float* averages, int32_t* counts) {
  if (N < 0 || N > (int64_t)INT32_MAX / 2) throw Fail{MRA_E_INVAL, "N out of range"};
  if (!averages || !counts) throw Fail{MRA_E_INVAL, "averages and counts must be non-NULL"};
  if (!params || !params->ref || !params->shift_x || !params->shift_y || !params->psi || !params->mirror)
    throw Fail{MRA_E_INVAL, "params arrays must be non-NULL"};
  if (N > 0 && !parts) throw Fail{MRA_E_INVAL, "parts is NULL"};
  hipStream_t st = c->stream;
  if (N == 0) {
    hip_check(c, hipMemsetAsync(counts, 0, K * sizeof(int32_t), st), "memset");
    return;
  }
  AvgArgs a{};
  a.parts = parts;
  a.N = N;
  a.K = K; a.L = L; a.cx = L / 2;
  a.ref = params->ref; a.shift_x = params->shift_x; a.shift_y = params->shift_y;
  a.psi = params->psi; a.mirror = params->mirror;
  a.cs64 = c->cs64;
  a.n_blk = (int)((N + 1023) / 1024);
  a.max_chunks = (int)((N + kAvgChunk - 1) / kAvgChunk) + K;
  a.blk_cnt = (int*)ws_get(c, "avg_blk_cnt", (size_t)a.n_blk * K * sizeof(int));
  a.blk_off = (int*)ws_get(c, "avg_blk_off", (size_t)a.n_blk * K * sizeof(int));
  a.cls_start = (int*)ws_get(c, "avg_cls", (size_t)(K + 1) * sizeof(int));
  a.chunk_start = (int*)ws_get(c, "avg_chunk", (size_t)(K + 1) * sizeof(int));
  a.order = (int*)ws_get(c, "avg_order", (size_t)N * sizeof(int));
  a.partial = (float*)ws_get(c, "avg_partial", (size_t)a.max_chunks * L * L * sizeof(float));
  a.averages = averages;
  a.counts = counts;
  timed(c, "averages", [&] { hip_check(c, launch_averages(a, st), "averages"); });
}

void update_averages_impl(mra_ctx* c, int32_t id, const float* parts, int64_t N, const mra_result* params,
                          float* averages, int32_t* counts) {
  const Refset& rs = get_refset(c, id);
  averages_core(c, rs.K, rs.g.L, parts, N, params, averages, counts);
}

// The outer repeat: load the averages as references, align, count the
// particles whose key (class, or with by_flat the whole parameter set)
// changed since the previous pass, update the averages.
void iterate_impl(mra_ctx* c, int32_t id, const mra_geom* g, const float* parts, int64_t N, float* averages,
                  int32_t K, int32_t max_iter, double max_changed_frac, const mra_result* out, int32_t* counts,
                  int32_t* n_iter, int64_t* changed, bool by_flat) {
  // a tuning set on this refset id carries over when the geometry matches
  int variant = -1, chunk = 0, prune = 1, run_tiles = 0;
  auto old = c->refs.find(id);
  if (old != c->refs.end() && old->second.K == K && std::memcmp(&old->second.g, g, sizeof(mra_geom)) == 0) {
    variant = old->second.variant;
    chunk = old->second.chunk;
    prune = old->second.prune;
    run_tiles = old->second.run_tiles;
  }
  hipStream_t st = c->stream;
  mra_result o = *out;
  if (by_flat && !o.flat_index) o.flat_index = (int32_t*)ws_get(c, "iter_flat", (size_t)N * sizeof(int32_t));
  const int32_t* key = by_flat ? o.flat_index : o.ref;
  int32_t* prev = (int32_t*)ws_get(c, "iter_prev", (size_t)N * sizeof(int32_t));
  int* cnt = (int*)ws_get(c, "iter_count", 256);
  *n_iter = 0;
  for (int it = 1; it <= max_iter; ++it) {
    load_refs_impl(c, id, averages, K, g);
    if (variant >= 0) {
      Refset& rs = c->refs[id];
      rs.variant = variant;
      rs.chunk = chunk;
      rs.prune = prune;
      rs.run_tiles = run_tiles;
    }
    align_impl(c, id, parts, N, -1, &o, nullptr);
    int64_t n_changed = N;
    if (it == 1) {
      hip_check(c, hipMemcpyAsync(prev, key, (size_t)N * sizeof(int32_t), hipMemcpyDeviceToDevice, st), "memcpy");
    } else {
      int h = 0;
      hip_check(c, hipMemsetAsync(cnt, 0, sizeof(int), st), "memset");
      hip_check(c, launch_count_changed(key, prev, (int)N, cnt, st), "count changed");
      hip_check(c, hipMemcpyAsync(&h, cnt, sizeof(int), hipMemcpyDeviceToHost, st), "memcpy");
      hip_check(c, hipStreamSynchronize(st), "sync");
      n_changed = h;
    }
    update_averages_impl(c, id, parts, N, &o, averages, counts);
    if (changed) changed[it - 1] = n_changed;
    *n_iter = it;
    if (it > 1 && (double)n_changed <= max_changed_frac * (double)N) break;
  }
  hip_check(c, hipStreamSynchronize(st), "sync");
}

void check_loop_args(const mra_geom* g, const float* parts, int64_t N, const float* averages, int32_t max_iter,
                     double max_changed_frac, const mra_result* out, const int32_t* n_iter) {
  check_geom(g);
  if (N < 1 || N > (int64_t)INT32_MAX / 2) throw Fail{MRA_E_INVAL, "N out of range"};
  if (!parts || !averages || !n_iter) throw Fail{MRA_E_INVAL, "NULL argument"};
  if (max_iter < 1) throw Fail{MRA_E_INVAL, "max_iter must be >= 1"};
  if (!(max_changed_frac >= 0.0 && max_changed_frac <= 1.0))
    throw Fail{MRA_E_INVAL, "max_changed_frac must lie in [0, 1]"};
  check_result(out);
}

template <class F>
int guard(mra_ctx* c, F&& fn) {
  if (!c) return MRA_E_INVAL;
  if (c->failed) {
    c->err = "context failed after an earlier device error";
    return MRA_E_DEVICE;
  }
  try {
    hip_check(c, hipSetDevice(c->device), "hipSetDevice");
    fn();
    return MRA_OK;
  } catch (const Fail& f) {
    c->err = f.msg;
    return f.code;
  } catch (const std::bad_alloc&) {
    c->err = "host out of memory";
    return MRA_E_NOMEM;
  } catch (...) {
    c->err = "unexpected internal error";
    return MRA_E_INVAL;
  }
}

}  // namespace

extern "C" {

int mra_create(mra_ctx** out, int device, void* hip_stream, uint64_t workspace_cap_bytes) {
  if (!out) return MRA_E_INVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return MRA_E_INVAL;
  }
  mra_ctx* c = new (std::nothrow) mra_ctx;
  if (!c) return MRA_E_NOMEM;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->cap = workspace_cap_bytes ? workspace_cap_bytes : (32ull << 30);
  int rc = guard(c, [&] {
    std::vector<double> cs, sn;
    build_cs(kNphi, cs, sn);
    std::vector<double2> h64(kNphi);
    std::vector<float2> h32(kNphi);
    for (int j = 0; j < kNphi; ++j) {
      h64[j] = make_double2(cs[j], sn[j]);
      h32[j] = make_float2((float)cs[j], (float)sn[j]);
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
      c->n_cu = ncu;
    c->scratch = scratch_ptr(c);
    c->cs64 = (double2*)alloc(c, kNphi * sizeof(double2), "cs64");
    c->cs32 = (float2*)alloc(c, kNphi * sizeof(float2), "cs32");
    hip_check(c, hipMemcpy(c->cs64, h64.data(), kNphi * sizeof(double2), hipMemcpyHostToDevice), "memcpy");
    hip_check(c, hipMemcpy(c->cs32, h32.data(), kNphi * sizeof(float2), hipMemcpyHostToDevice), "memcpy");
  });
  if (rc != MRA_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return MRA_OK;
}

int mra_destroy(mra_ctx* c) {
  if (!c) return MRA_E_INVAL;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  clear_profile(c);
  for (auto& kv : c->refs) free_refset(kv.second);
  for (auto& kv : c->ws)
    if (kv.second.p) (void)hipFree(kv.second.p);
  if (c->cs64) (void)hipFree(c->cs64);
  if (c->cs32) (void)hipFree(c->cs32);
  delete c;
  return MRA_OK;
}

int mra_load_refs(mra_ctx* c, int32_t id, const float* refs, int32_t K, const mra_geom* g) {
  return guard(c, [&] { load_refs_impl(c, id, refs, K, g); });
}

int mra_check_geom(const mra_geom* g, int32_t K, int32_t shift_max) {
  try {
    check_geom(g);
    if (K < 1) return MRA_E_INVAL;
    const int T = shift_max < 0 ? g->shift_max : shift_max;
    if (T > 8) return MRA_E_INVAL;
    check_index_range(K, g->mirror ? 2 : 1, T);
    Refset rs;
    rs.g = *g;
    rs.K = K;
    stencil_range(*g, rs.dmin, rs.dmax);
    (void)plan_for(rs, T);
    return MRA_OK;
  } catch (const Fail& f) {
    return f.code;
  } catch (...) {
    return MRA_E_INVAL;
  }
}

int mra_unload_refs(mra_ctx* c, int32_t id) {
  return guard(c, [&] {
    Refset& rs = get_refset(c, id);
    hip_check(c, hipStreamSynchronize(c->stream), "sync");
    free_refset(rs);
    c->refs.erase(id);
  });
}

int mra_refset_info(mra_ctx* c, int32_t id, int32_t* K, mra_geom* g) {
  return guard(c, [&] {
    Refset& rs = get_refset(c, id);
    if (K) *K = rs.K;
    if (g) *g = rs.g;
  });
}

int mra_align(mra_ctx* c, int32_t id, const float* parts, int64_t N, mra_result* out) {
  return guard(c, [&] { align_impl(c, id, parts, N, -1, out, nullptr); });
}

int mra_align_noalloc(mra_ctx* c, int32_t id, const float* parts, int64_t N, mra_result* out) {
  return guard(c, [&] { align_impl(c, id, parts, N, -1, out, nullptr, true); });
}

int mra_align_batch(mra_ctx* c, const mra_stack* stacks, int32_t n) {
  return guard(c, [&] {
    if (n < 0 || (n > 0 && !stacks)) throw Fail{MRA_E_INVAL, "bad stack list"};
    std::vector<Plan> plans(n);
    for (int i = 0; i < n; ++i) {  // validate everything before enqueueing anything
      const mra_stack& s = stacks[i];
      Refset& rs = get_refset(c, s.refset_id);
      if (s.N < 0) throw Fail{MRA_E_INVAL, "stack N must be >= 0"};
      plans[i] = plan_for(rs, s.shift_max < 0 ? rs.g.shift_max : s.shift_max);
      if (s.N > 0) {
        if (!s.parts) throw Fail{MRA_E_INVAL, "stack parts is NULL"};
        check_result(&s.out);
        if (s.N * (int64_t)plans[i].S > INT32_MAX / 2) throw Fail{MRA_E_INVAL, "stack too large"};
      }
    }
    run_batch(c, stacks, n, plans);
  });
}

int mra_update_averages(mra_ctx* c, int32_t id, const float* parts, int64_t N, const mra_result* params,
                        float* averages, int32_t* counts) {
  return guard(c, [&] { update_averages_impl(c, id, parts, N, params, averages, counts); });
}

int mra_classify(mra_ctx* c, int32_t id, const mra_geom* g, const float* parts, int64_t N, float* averages,
                 int32_t K, int32_t max_iter, double max_changed_frac, mra_result* out, int32_t* counts,
                 int32_t* n_iter, int64_t* changed) {
  return guard(c, [&] {
    check_loop_args(g, parts, N, averages, max_iter, max_changed_frac, out, n_iter);
    if (K < 1) throw Fail{MRA_E_INVAL, "K must be >= 1"};
    if (!counts) throw Fail{MRA_E_INVAL, "counts is NULL"};
    iterate_impl(c, id, g, parts, N, averages, K, max_iter, max_changed_frac, out, counts, n_iter, changed, false);
  });
}

int mra_rfa(mra_ctx* c, int32_t id, const mra_geom* g, const float* parts, int64_t N, float* average,
            int32_t start_from_mean, int32_t max_iter, double max_changed_frac, mra_result* out, int32_t* n_iter,
            int64_t* changed) {
  return guard(c, [&] {
    check_loop_args(g, parts, N, average, max_iter, max_changed_frac, out, n_iter);
    int32_t* cnt = (int32_t*)ws_get(c, "rfa_count", 256);
    if (start_from_mean) {  // the plain mean: the average update with every parameter zero
      hipStream_t st = c->stream;
      for (int32_t* p : {out->ref, out->shift_x, out->shift_y, out->psi, out->mirror})
        hip_check(c, hipMemsetAsync(p, 0, (size_t)N * sizeof(int32_t), st), "memset");
      averages_core(c, 1, g->L, parts, N, out, average, cnt);
    }
    iterate_impl(c, id, g, parts, N, average, 1, max_iter, max_changed_frac, out, cnt, n_iter, changed, true);
  });
}

int mra_debug_polar(mra_ctx* c, int32_t id, const float* parts, int64_t N, float* out) {
  return guard(c, [&] {
    Refset& rs = get_refset(c, id);
    if (N < 0 || N > INT32_MAX || (N > 0 && (!parts || !out))) throw Fail{MRA_E_INVAL, "bad arguments"};
    const Plan p = plan_for(rs, rs.g.shift_max);
    PolarArgs pa{};
    pa.parts = parts; pa.n_part = (int)N;
    pa.L = rs.g.L; pa.R = rs.R; pa.R4 = rs.R4; pa.T = p.T; pa.S1 = p.S1; pa.S = p.S;
    pa.Lp = p.Lp; pa.pad = p.pad; pa.cx = p.cx; pa.r_min = rs.g.r_min; pa.cs64 = c->cs64; pa.out = out;
    hip_check(c, launch_polar(1, pa, c->stream), "polar");
  });
}

int mra_debug_spectra(mra_ctx* c, int32_t id, const float* parts, int64_t N, float* out) {
  return guard(c, [&] {
    Refset& rs = get_refset(c, id);
    if (N < 0 || N > INT32_MAX || (N > 0 && (!parts || !out))) throw Fail{MRA_E_INVAL, "bad arguments"};
    const Plan p = plan_for(rs, rs.g.shift_max);
    PolarArgs pa{};
    pa.parts = parts; pa.n_part = (int)N;
    pa.L = rs.g.L; pa.R = rs.R; pa.R4 = rs.R4; pa.T = p.T; pa.S1 = p.S1; pa.S = p.S;
    pa.Lp = p.Lp; pa.pad = p.pad; pa.cx = p.cx; pa.r_min = rs.g.r_min; pa.cs64 = c->cs64; pa.out = out;
    hip_check(c, launch_polar(2, pa, c->stream), "polar");
  });
}

int mra_debug_cctable(mra_ctx* c, int32_t id, const float* parts, int64_t N, float* out) {
  return guard(c, [&] {
    if (N > 0 && !out) throw Fail{MRA_E_INVAL, "out is NULL"};
    align_impl(c, id, parts, N, -1, nullptr, out);
  });
}

int mra_debug_refs(mra_ctx* c, int32_t id, float* qhat, double* norm) {
  return guard(c, [&] {
    Refset& rs = get_refset(c, id);
    if (qhat)
      hip_check(c, hipMemcpyAsync(qhat, rs.qhat, (size_t)rs.K * rs.R * kNphi * sizeof(float), hipMemcpyDeviceToDevice, c->stream), "memcpy");
    if (norm)
      hip_check(c, hipMemcpyAsync(norm, rs.norm, (size_t)rs.K * sizeof(double), hipMemcpyDeviceToDevice, c->stream), "memcpy");
  });
}

int mra_set_tuning(mra_ctx* c, int32_t id, const mra_tuning* t) {
  return guard(c, [&] {
    Refset& rs = get_refset(c, id);
    if (!t) throw Fail{MRA_E_INVAL, "tuning is NULL"};
    const int v = t->corr_variant < 0 ? corr_default_variant(rs.g.precision, rs.R4) : t->corr_variant;
    if (!corr_variant_ok(rs.g.precision, v, rs.R4)) throw Fail{MRA_E_INVAL, "variant cannot serve this geometry"};
    if (t->chunk_particles < 0) throw Fail{MRA_E_INVAL, "chunk_particles must be >= 0"};
    if (t->prune < -1 || t->prune > 1) throw Fail{MRA_E_INVAL, "prune must be -1, 0 or 1"};
    if (t->run_tiles < 0 || t->run_tiles > 64) throw Fail{MRA_E_INVAL, "run_tiles must be in [0, 64]"};
    rs.variant = v;
    rs.chunk = t->chunk_particles;
    rs.prune = t->prune != 0;
    rs.run_tiles = t->run_tiles;
  });
}

int mra_get_tuning(mra_ctx* c, int32_t id, mra_tuning* t) {
  return guard(c, [&] {
    Refset& rs = get_refset(c, id);
    if (!t) throw Fail{MRA_E_INVAL, "tuning is NULL"};
    t->corr_variant = rs.variant;
    t->chunk_particles = rs.chunk;
    t->prune = rs.prune;
    t->run_tiles = rs.run_tiles;
  });
}

int mra_profile(mra_ctx* c, int enable) {
  return guard(c, [&] {
    hip_check(c, hipStreamSynchronize(c->stream), "sync");
    if (enable) clear_profile(c);
    c->profiling = enable != 0;
  });
}

int mra_profile_read(mra_ctx* c, const char* kernel, double* total_ms, int64_t* launches) {
  return guard(c, [&] {
    if (!kernel) throw Fail{MRA_E_INVAL, "kernel name is NULL"};
    hip_check(c, hipStreamSynchronize(c->stream), "sync");
    double tot = 0.0;
    int64_t cnt = 0;
    auto it = c->prof.find(kernel);
    if (it != c->prof.end())
      for (auto& e : it->second) {
        float ms = 0.f;
        hip_check(c, hipEventElapsedTime(&ms, e.first, e.second), "hipEventElapsedTime");
        tot += ms;
        ++cnt;
      }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = cnt;
  });
}

const char* mra_last_error(mra_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

const char* mra_strerror(int code) {
  switch (code) {
    case MRA_OK: return "ok";
    case MRA_E_INVAL: return "invalid argument";
    case MRA_E_NOREF: return "refset not loaded";
    case MRA_E_NOMEM: return "out of device memory";
    case MRA_E_DEVICE: return "device error";
    case MRA_E_DEGENERATE: return "degenerate reference (zero norm)";
    default: return "unknown error";
  }
}

}  // extern "C"
