// C ABI of libtfmm: contexts, operator setup/import/export, translation,
// kernel timing and the continuous-batching scheduler (include/tfmm.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host_math.h"
#include "internal.h"
#include "launch.h"
#include "noalloc.h"
#include "setup_gpu.h"
#include "tfmm.h"

using tfmm::cd;

namespace {

thread_local std::string g_last_error;

tfmm_status fail(tfmm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define HIP_TRY(expr)                                                                               \
  do {                                                                                              \
    hipError_t _e = (expr);                                                                         \
    if (_e != hipSuccess)                                                                           \
      return fail(TFMM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));                 \
  } while (0)

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool supported_len(int n) {
  switch (n) {
    case 8: case 16: case 24: case 32: case 48: case 64: return true;
    default: return false;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Objects
// ---------------------------------------------------------------------------

struct ScratchSlot {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// A tile-configuration choice of the autotuner: -1 / 0 = keep the default.
struct TuneChoice {
  int fused = -1;  // 1: fused one-kernel path (when the grid allows), 0: three-pass
  int cb = 0;      // three-pass pencil tile: 64*cb pencils per block
  int tk2 = -1;    // Tucker family: 1 register-chained, 0 LDS-staged restoration
};

struct tfmm_op_s {
  tfmm_ctx ctx = nullptr;
  tfmm_format fmt = TFMM_FMT_FULL;
  tfmm_precision prec = TFMM_PREC_FP32;
  int K[3] = {0, 0, 0}, n[3] = {0, 0, 0};
  int ndir = 0, L = 0, nq = 0;
  tfmm::Factors host;                  // complex128 factors (export / import layout)
  float4* d_full = nullptr;            // FULL operator, [p][n3/2][nq]
  float2* d_data = nullptr;            // compressed factors, complex64, import layout
  int* d_desc = nullptr;               // [ndir][8] z-stage descriptors
  size_t dev_bytes = 0;                // bytes charged to the budget
  size_t stored_elems = 0;
  std::vector<int> desc;               // host copy of the descriptors
  // derived plan: three-pass pipeline (cb, KC, lds) and, for small cubic
  // grids, the fused single-kernel path (fused, fKC, flds)
  int zfmt = 0, cb = 1, KC = 8, lds = 0, rg = 1;
  bool fused = false;
  int fKC = 8, flds = 0;
  // Tucker family: register-chained restoration (3-pass tile / fused tile)
  bool tk2 = false, ftk2 = false;
  // 4-D formats on the three-pass path: the x-mode product W1[fx][b][c] of each
  // direction's core is formed by a batched GEMM per direction chunk, and the
  // z-stage restores from it (ZF_TUCKER_W1)
  bool use_w1 = false;
  double tol = 0.0;                    // compression tolerance of tfmm_setup_compressed (0: imported)
  // TT-3D on the three-pass path with register-chained restoration: the x-y
  // products W_p[q][b] = sum_a U1_p[fx][a] C_p[a][fy][b] of every direction are
  // formed by one batched GEMM per call (wtt_elems complex64 of scratch)
  size_t wtt_elems = 0;
  size_t a1_bytes = 0;                 // scratch for per-direction cores (4-D formats)
  int* d_perm = nullptr;               // direction order, costliest restoration first (NULL: identity)
  float2* d_roots_z = nullptr;         // exp(-2 pi i m / n3), m < n3 (context table)
  float2* d_roots_x = nullptr;         // exp(-2 pi i m / n1) when n1 > 64 (context table), else NULL
  // physics of the problem (set by tfmm_setup_compressed from a direction grid):
  // directions, quadrature weights, wavenumber and box size, for the far-field
  // patterns of tfmm_basis_setup
  bool physical = false;
  std::vector<double> khat, wts;
  double k_re = 0.0, k_im = 0.0, box = 0.0;
  // captured translations, keyed by (nrhs, A, B) and the scratch generation
  struct GraphEntry {
    int nrhs;
    const void* A;
    void* B;
    unsigned gen;
    hipGraph_t g;
    hipGraphExec_t x;
  };
  std::vector<GraphEntry> graphs;      // least recently used first
  TuneChoice choice;                   // plan overrides in effect
  bool tuned = false;                  // choice came from the autotuner or its cache
  tfmm_op_info info{};
  std::atomic<int> refs{0};
};

struct tfmm_near_s {
  tfmm_ctx ctx = nullptr;
  int n = 0;
  long long nnz = 0;
  int* d_rp = nullptr;                 // [n + 1]
  int* d_ci = nullptr;                 // [nnz]
  float2* d_val = nullptr;             // [nnz] complex64
};

struct tfmm_basis_s {
  tfmm_ctx ctx = nullptr;
  tfmm_op op = nullptr;                // operator whose directions and grid the patterns follow
  int N = 0, nbox = 0, ndir = 0;
  float4* d_pat = nullptr;             // [p][n] (theta.u, phi.u, Re e, Im e), sorted order
  int* d_start = nullptr;              // [nbox + 1] sorted range of each box
  int* d_orig = nullptr;               // [N] caller index of sorted basis n
  int* d_boxof = nullptr;              // [N] box of sorted basis n
  float* d_w = nullptr;                // [ndir] quadrature weights
  size_t bytes = 0;
};

struct Job {
  tfmm_ticket id = 0;
  tfmm_op op = nullptr;
  const float2* A = nullptr;
  float2* B = nullptr;
  int nrhs = 0;
  double t_submit = 0.0, t_done = 0.0;
  size_t charged = 0;                  // A and B bytes charged to the budget while admitted
  std::atomic<int> done{0};
  tfmm_status status = TFMM_OK;
};

struct InFlight {
  hipEvent_t ev = nullptr;
  std::vector<std::shared_ptr<Job>> jobs;
  int slot = 0;
};

struct KernelStat {
  double total_ms = 0.0;
  int n = 0;
};

struct tfmm_ctx_s {
  int device = 0;
  bool no_fused = false;               // TFMM_NO_FUSED=1: always use the three-pass pipeline
  bool no_tk2 = false;                 // TFMM_NO_TK2=1: Tucker restoration through LDS-staged products
  bool no_w1 = false;                  // TFMM_NO_W1=1: 4-D formats restore the x-mode product in the z-stage
  bool host_compress = false;          // TFMM_HOST_COMPRESS=1: compress the 4-D formats on the host
  size_t hcap = (size_t)256 << 20;     // three-pass half-spectrum chunk (budget / 8, TFMM_HCAP_MB)
  size_t budget = 0, used = 0;
  std::recursive_mutex mu;
  // translation scratch, one per stream slot (slot 0 = tfmm_translate; 1..S = scheduler streams)
  static constexpr int kSlots = 3;
  ScratchSlot scratch[kSlots];
  unsigned scratch_gen[kSlots] = {0, 0, 0};  // bumped when a slot's buffer moves
  // recorded after the last work enqueued on each slot's scratch: a slot's buffer
  // is freed only once its own work is done (no device-wide synchronisation)
  hipEvent_t slot_ev[kSlots] = {nullptr, nullptr, nullptr};
  bool slot_ev_set[kSlots] = {false, false, false};
  // per slot, a second stream for the per-call GEMMs (a1 and the formed
  // products), which depend on the operator only: forked from the slot's
  // stream at the start of a translation and joined before the first z-stage,
  // so they run beside the first x pass, which depends on A only
  hipStream_t side[kSlots] = {nullptr, nullptr, nullptr};
  hipEvent_t fork_ev[kSlots] = {nullptr, nullptr, nullptr};
  hipEvent_t join_ev[kSlots] = {nullptr, nullptr, nullptr};
  int* counters = nullptr;             // device work counters of the persistent launches, one per slot
  int ncu = 0;                         // compute units
  hipStream_t cap_stream = nullptr;    // stream used only for graph capture
  // graph policy (TFMM_GRAPH): 0 never capture, 1 always, 2 (default) only
  // multi-launch translations; TFMM_NO_GRAPH=1 is the same as 0
  int graph_mode = 2;
  // autotuner results: key -> choice, loaded from / appended to TFMM_TUNE_CACHE
  std::map<std::string, TuneChoice> tune;
  std::string tune_path;
  std::map<int, float2*> roots;        // n3 -> device table exp(-2 pi i m/n3)
  // profiling
  bool prof = false;
  struct Pending {
    std::string name;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  std::map<std::string, KernelStat> stats;
  hipEvent_t take_event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  // scheduler
  hipStream_t streams[2] = {nullptr, nullptr};
  std::thread worker, completer;
  std::mutex qmu;
  std::condition_variable qcv, fcv;
  std::deque<std::shared_ptr<Job>> queue;
  std::deque<InFlight> inflight;
  std::unordered_map<tfmm_ticket, std::shared_ptr<Job>> jobs;
  std::atomic<tfmm_ticket> next_ticket{1};
  bool stop = false;
  int slot_busy[2] = {0, 0};
  // scheduler statistics: launches started, times the head of the queue had to
  // wait for memory, jobs completed and jobs failed
  uint64_t n_launch = 0, n_parked = 0, n_done = 0, n_failed = 0;
  std::vector<tfmm_op> ops;
  std::vector<tfmm_basis> bases;
  std::vector<tfmm_near> nears;
  // far-field matvec intermediates (A and B of the translation), grown on demand
  void* mv_buf = nullptr;
  size_t mv_bytes = 0;
  std::string noalloc_error;           // why the fixed scratch is unavailable (empty: available)
};

namespace tfmm {
int near_rows(tfmm_near m) { return m ? m->n : 0; }
void set_last_error(const std::string& msg) { g_last_error = msg; }
}  // namespace tfmm

static void free_basis(tfmm_ctx c, tfmm_basis b);

// ---------------------------------------------------------------------------
// Budget and scratch
// ---------------------------------------------------------------------------
namespace {

tfmm_status charge(tfmm_ctx c, size_t bytes) {
  if (c->used + bytes > c->budget)
    return fail(TFMM_ERR_BUDGET, "device-memory budget exhausted: need " + std::to_string(bytes) + " B, " +
                                     std::to_string(c->budget - c->used) + " B left");
  c->used += bytes;
  return TFMM_OK;
}

void uncharge(tfmm_ctx c, size_t bytes) { c->used -= std::min(c->used, bytes); }

tfmm_status dev_alloc(tfmm_ctx c, void** p, size_t bytes) {
  tfmm_status s = charge(c, bytes);
  if (s != TFMM_OK) return s;
  if (hipMalloc(p, bytes) != hipSuccess) {
    uncharge(c, bytes);
    (void)hipGetLastError();
    return fail(TFMM_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " B failed");
  }
  return TFMM_OK;
}

void dev_free(tfmm_ctx c, void* p, size_t bytes) {
  if (p) {
    (void)hipFree(p);
    uncharge(c, bytes);
  }
}

void mark_slot(tfmm_ctx c, int slot, hipStream_t st) {
  if (hipEventRecord(c->slot_ev[slot], st) == hipSuccess) c->slot_ev_set[slot] = true;
}

// Free a slot's scratch once the work enqueued on it has finished.
void release_scratch(tfmm_ctx c, int slot) {
  ScratchSlot& s = c->scratch[slot];
  if (!s.ptr) return;
  if (c->slot_ev_set[slot]) (void)hipEventSynchronize(c->slot_ev[slot]);
  dev_free(c, s.ptr, s.bytes);
  s.ptr = nullptr;
  s.bytes = 0;
  ++c->scratch_gen[slot];
}

tfmm_status ensure_scratch(tfmm_ctx c, int slot, size_t bytes, void** out) {
  ScratchSlot& s = c->scratch[slot];
  if (s.bytes < bytes) {
    release_scratch(c, slot);
    size_t want = bytes + bytes / 8;
    tfmm_status st = dev_alloc(c, &s.ptr, want);
    if (st != TFMM_OK) {
      st = dev_alloc(c, &s.ptr, bytes);
      if (st != TFMM_OK) return st;
      want = bytes;
    }
    s.bytes = want;
    ++c->scratch_gen[slot];
  }
  *out = s.ptr;
  return TFMM_OK;
}

tfmm_status roots_table(tfmm_ctx c, int n3, float2** out) {
  auto it = c->roots.find(n3);
  if (it != c->roots.end()) {
    *out = it->second;
    return TFMM_OK;
  }
  std::vector<float2> h(n3);
  for (int m = 0; m < n3; ++m) {
    const double a = -2.0 * 3.14159265358979323846264338327950288 * m / n3;
    h[m] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  void* d = nullptr;
  tfmm_status s = dev_alloc(c, &d, n3 * sizeof(float2));
  if (s != TFMM_OK) return s;
  HIP_TRY(hipMemcpy(d, h.data(), n3 * sizeof(float2), hipMemcpyHostToDevice));
  c->roots[n3] = (float2*)d;
  *out = (float2*)d;
  return TFMM_OK;
}

// ---------------------------------------------------------------------------
// Operator build from host factors
// ---------------------------------------------------------------------------

tfmm_status validate_grid(const int K[3]) {
  for (int i = 0; i < 3; ++i)
    if (K[i] < 1) return fail(TFMM_ERR_INVALID_ARG, "box grid dimensions must be positive");
  for (int i = 0; i < 3; ++i) {
    const bool long_x = i == 0 && (K[i] == 64 || K[i] == 128);
    if (!supported_len(2 * K[i]) && !long_x)
      return fail(TFMM_ERR_UNSUPPORTED, "box grid dimension " + std::to_string(K[i]) +
                                            " unsupported (need 4, 8, 12, 16, 24 or 32; Kx may also be 64 or 128)");
  }
  // one z-plane of the xy spectrum must fit the 64 KB LDS slab of the xy passes
  if ((size_t)4 * K[0] * K[1] * sizeof(float2) > 65536)
    return fail(TFMM_ERR_UNSUPPORTED, "x-y plane too large (need Kx * Ky <= 2048)");
  return TFMM_OK;
}

int pick_cb(int n2, int nq, int max_cb) {
  // pencil tile 64*cb must be a multiple of n2 and divide nq; prefer 256 pencils
  for (int cb : {4, 3, 2, 1}) {
    const int qt = 64 * cb;
    if (cb <= max_cb && qt % n2 == 0 && nq % qt == 0) return cb;
  }
  return 0;
}

int max_cb_for(int n3) {
  // accumulator registers: (n3/8) * cb * 4 per lane; keep them <= 96
  return n3 >= 64 ? 2 : (n3 >= 48 ? 3 : 4);
}

bool cb_valid(int cb, int n2, int nq, int n3) {
  const int qt = 64 * cb;
  return cb >= 1 && cb <= max_cb_for(n3) && qt % n2 == 0 && nq % qt == 0;
}

tfmm_status plan_zstage(tfmm_op op) {
  const int n1 = op->n[0], n2 = op->n[1], n3 = op->n[2];
  op->nq = n1 * n2;
  const TuneChoice& ch = op->choice;
  op->cb = cb_valid(ch.cb, n2, op->nq, n3) ? ch.cb : pick_cb(n2, op->nq, max_cb_for(n3));
  if (op->cb == 0) return fail(TFMM_ERR_UNSUPPORTED, "no pencil tiling for this grid");
  switch (op->fmt) {
    case TFMM_FMT_FULL: op->zfmt = tfmm::ZF_FULL; break;
    case TFMM_FMT_TT3D: op->zfmt = tfmm::ZF_TT3D; break;
    case TFMM_FMT_TT4D: op->zfmt = tfmm::ZF_TT4D; break;
    default: op->zfmt = tfmm::ZF_TUCKER; break;
  }
  op->lds = 0;
  // largest ranks over directions bound the LDS need
  int r1 = 1, r2 = 1;
  if (op->zfmt != tfmm::ZF_FULL)
    for (int p = 0; p < op->ndir; ++p) {
      r1 = std::max(r1, op->desc[8 * p + 4]);
      r2 = std::max(r2, op->desc[8 * p + 5]);
    }
  const size_t lds_max = 160 * 1024 - 64;  // leaves room for the work-item slot
  const bool bf = op->prec == TFMM_PREC_BF16X3;
  op->tk2 = op->ftk2 = false;
  int kfmt = op->zfmt;  // the z-stage kernel family this plan launches
  if (op->zfmt != tfmm::ZF_FULL) {
    const size_t cap = 96 * 1024;
    int KC = 16;
    while (KC > 1 && tfmm::zstage_lds_bytes(op->zfmt, n1, n2, n3, 64 * op->cb, KC, r1, r2) > cap) KC /= 2;
    size_t need = tfmm::zstage_lds_bytes(op->zfmt, n1, n2, n3, 64 * op->cb, KC, r1, r2);
    if (op->zfmt == tfmm::ZF_TUCKER && !op->ctx->no_tk2 && ch.tk2 != 0) {
      // the 4-D formats restore from a formed x-mode product on this path
      // (no core chunk in LDS), unless TFMM_NO_W1=1
      const bool w1 = (op->fmt == TFMM_FMT_TUCKER4D || op->fmt == TFMM_FMT_HTUCKER4D) && !op->ctx->no_w1;
      const size_t need2 = tfmm::tucker2_lds_bytes(n2, n3, 64 * op->cb, r1, r2, bf, w1);
      if (need2 <= lds_max) {
        op->tk2 = true;
        need = need2;
        if (w1) kfmt = tfmm::ZF_TUCKER_W1;
      }
    } else if ((op->zfmt == tfmm::ZF_TT4D || op->zfmt == tfmm::ZF_TT3D) && !op->ctx->no_tk2 && ch.tk2 != 0) {
      const size_t need2 = tfmm::tt4d_chained_lds_bytes(n3, r2, bf);
      if (need2 <= lds_max) {
        op->tk2 = true;
        need = need2;
      }
    }
    if (need > lds_max) return fail(TFMM_ERR_UNSUPPORTED, "ranks too large for the LDS-resident restoration");
    op->KC = KC;
    op->lds = (int)need;
  }
  // the z-stage's y- and z-stages reuse the restoration's LDS; RHS go through in
  // groups of rg half spectra.  Where the kernel is built for two waves per
  // SIMD (n3 <= 32), the largest group that lets two blocks share a compute
  // unit's LDS comes first; otherwise as many as fit.
  op->rg = 0;
  if (tfmm::zplanes_waves_per_simd(kfmt, n3 / 8) == 2) {
    const size_t two = 80 * 1024 - 64 - TFMM_LDS_SLOT;
    for (int rg : {4, 2, 1})
      if (std::max<size_t>((size_t)op->lds, tfmm::zplanes_lds_bytes(n3, op->cb, rg)) <= two) {
        op->rg = rg;
        break;
      }
  }
  if (op->rg == 0) {
    op->rg = 1;
    for (int rg : {4, 2})
      if (tfmm::zplanes_lds_bytes(n3, op->cb, rg) <= lds_max) {
        op->rg = rg;
        break;
      }
  }
  op->lds = (int)std::max<size_t>((size_t)op->lds, tfmm::zplanes_lds_bytes(n3, op->cb, op->rg));
  // fused path: cubic grids whose half spectrum (n*n*zp complex64) fits in LDS
  op->fused = false;
  if (!op->ctx->no_fused && ch.fused != 0 && n1 == n2 && n2 == n3 &&
      (n1 == 8 || n1 == 16 || n1 == 24 || n1 == 32)) {
    const int K3 = n3 / 2, zp = (K3 & 1) ? K3 : K3 + 1;
    const size_t hbytes = (size_t)n1 * n2 * zp * sizeof(float2);
    int KC = 16;
    size_t rb = 0;
    bool ftk2 = false;
    if (op->zfmt != tfmm::ZF_FULL) {
      while (KC > 1 && tfmm::zstage_lds_bytes(op->zfmt, n1, n2, n3, n1 * n2, KC, r1, r2) > lds_max) KC /= 2;
      rb = tfmm::zstage_lds_bytes(op->zfmt, n1, n2, n3, n1 * n2, KC, r1, r2);
      if (op->zfmt == tfmm::ZF_TUCKER && !op->ctx->no_tk2 && ch.tk2 != 0) {
        const size_t rb2 = tfmm::tucker2_lds_bytes(n2, n3, n1 * n2, r1, r2, bf);
        if (rb2 <= lds_max) {
          ftk2 = true;
          rb = rb2;
        }
      } else if (op->zfmt == tfmm::ZF_TT4D && !op->ctx->no_tk2 && ch.tk2 != 0) {
        const size_t rb2 = tfmm::tt4d_chained_lds_bytes(n3, r2, bf);
        if (rb2 <= lds_max) {
          ftk2 = true;
          rb = rb2;
        }
      }
    }
    if (hbytes <= lds_max && rb <= lds_max) {
      op->fused = true;
      op->ftk2 = ftk2;
      op->fKC = KC;
      op->flds = (int)std::max(hbytes, rb);
    }
  }
  // the three-pass LDS above was planned for the formed product when tk2 holds
  op->use_w1 = (op->fmt == TFMM_FMT_TUCKER4D || op->fmt == TFMM_FMT_HTUCKER4D) && !op->fused && op->tk2 &&
               !op->ctx->no_w1;
  return TFMM_OK;
}

tfmm_status build_device_op(tfmm_ctx c, tfmm_op op) {
  const tfmm::Factors& F = op->host;
  const int n1 = op->n[0], n2 = op->n[1], n3 = op->n[2], nd = op->ndir;
  const long long N = (long long)n1 * n2 * n3;
  op->nq = n1 * n2;
  // twiddle tables of the z-stage and of long x lines, shared per context
  tfmm_status st0 = roots_table(c, n3, &op->d_roots_z);
  if (st0 == TFMM_OK && n1 > 64) st0 = roots_table(c, n1, &op->d_roots_x);
  if (st0 != TFMM_OK) return st0;
  if (op->fmt == TFMM_FMT_FULL) {
    std::vector<float4> h((size_t)nd * N / 2);
    for (int p = 0; p < nd; ++p)
      for (int q = 0; q < op->nq; ++q)
        for (int zp = 0; zp < n3 / 2; ++zp) {
          const cd a = F.data[(size_t)p * N + (size_t)q * n3 + 2 * zp];
          const cd b = F.data[(size_t)p * N + (size_t)q * n3 + 2 * zp + 1];
          h[((size_t)p * (n3 / 2) + zp) * op->nq + q] =
              make_float4((float)a.real(), (float)a.imag(), (float)b.real(), (float)b.imag());
        }
    op->dev_bytes = h.size() * sizeof(float4);
    tfmm_status s = dev_alloc(c, (void**)&op->d_full, op->dev_bytes);
    if (s != TFMM_OK) return s;
    HIP_TRY(hipMemcpy(op->d_full, h.data(), op->dev_bytes, hipMemcpyHostToDevice));
    op->stored_elems = (size_t)nd * N;
    return plan_zstage(op);
  }
  // compressed: factors as complex64 in the import layout
  std::vector<float2> h(F.data.size());
  for (size_t i = 0; i < h.size(); ++i) h[i] = make_float2((float)F.data[i].real(), (float)F.data[i].imag());
  if (op->fmt == TFMM_FMT_HTUCKER4D) {
    // the root transfer matrix B is absorbed into the (3,4) interior node, in
    // FP64: E[(a3 a4)][b] = sum_b' C34[(a3 a4)][b'] B[b][b'] (r3 r4 x r12) follows
    // C12 on the device in place of C34 and B (an equivalent tree with an
    // identity root)
    const std::vector<int32_t>& rk = F.ranks;
    const int r1 = rk[0], r2 = rk[1], r3 = rk[2], r4 = rk[3], r12 = rk[4], r34 = rk[5];
    const size_t oU4 = (size_t)n1 * r1 + (size_t)n2 * r2 + (size_t)n3 * r3, oC12 = oU4 + (size_t)nd * r4,
                 oC34 = oC12 + (size_t)r1 * r2 * r12, oB = oC34 + (size_t)r3 * r4 * r34;
    const size_t rows = (size_t)r3 * r4;
    h.resize(oC34 + rows * r12);
    std::vector<std::thread> pool;
    const int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    for (int t = 0; t < nt; ++t)
      pool.emplace_back([&, t] {
        for (size_t m = t; m < rows; m += nt)
          for (int b = 0; b < r12; ++b) {
            cd acc = 0.0;
            for (int k = 0; k < r34; ++k) acc += F.data[oC34 + m * r34 + k] * F.data[oB + (size_t)b * r34 + k];
            h[oC34 + m * r12 + b] = make_float2((float)acc.real(), (float)acc.imag());
          }
      });
    for (auto& th : pool) th.join();
  }
  op->stored_elems = h.size();
  op->desc.assign((size_t)8 * nd, 0);
  const std::vector<int32_t>& r = F.ranks;
  size_t a1 = 0;
  if (op->fmt == TFMM_FMT_TUCKER3D) {
    long long off = 0;
    for (int p = 0; p < nd; ++p) {
      const int r1 = r[3 * p], r2 = r[3 * p + 1], r3 = r[3 * p + 2];
      int* d = &op->desc[8 * p];
      d[0] = (int)off;
      d[1] = (int)(off + (long long)r1 * r2 * r3);
      d[2] = (int)(d[1] + (long long)n1 * r1);
      d[3] = (int)(d[2] + (long long)n2 * r2);
      d[4] = r1; d[5] = r2; d[6] = r3;
      off = d[3] + (long long)n3 * r3;
    }
  } else if (op->fmt == TFMM_FMT_TT3D) {
    long long off = 0, woff = 0;
    for (int p = 0; p < nd; ++p) {
      const int r1 = r[2 * p], r2 = r[2 * p + 1];
      int* d = &op->desc[8 * p];
      d[1] = (int)off;
      d[0] = (int)(off + (long long)n1 * r1);
      d[3] = (int)(d[0] + (long long)r1 * n2 * r2);
      d[4] = r1; d[5] = r2;
      off = d[3] + (long long)n3 * r2;
      d[7] = (int)woff;  // W_p = U1_p . C_p in the register-chained restoration's scratch
      woff += (long long)n1 * n2 * r2;
    }
    if (woff > INT32_MAX) return fail(TFMM_ERR_UNSUPPORTED, "TT-3D operator too large for the x-y product scratch");
    op->wtt_elems = (size_t)woff;
  } else if (op->fmt == TFMM_FMT_TUCKER4D || op->fmt == TFMM_FMT_HTUCKER4D) {
    const int r1 = r[0], r2 = r[1], r3 = r[2], r4 = r[3];
    long long oU1 = (op->fmt == TFMM_FMT_TUCKER4D) ? (long long)r1 * r2 * r3 * r4 : 0;
    long long oU2 = oU1 + (long long)n1 * r1, oU3 = oU2 + (long long)n2 * r2;
    for (int p = 0; p < nd; ++p) {
      int* d = &op->desc[8 * p];
      d[0] = p * r1 * r2 * r3;
      d[1] = (int)oU1; d[2] = (int)oU2; d[3] = (int)oU3;
      d[4] = r1; d[5] = r2; d[6] = r3;
    }
    a1 = (size_t)nd * r1 * r2 * r3;                                    // per-direction cores
    if (op->fmt == TFMM_FMT_HTUCKER4D) a1 += (size_t)nd * r3 * r[4];  // X2
    (void)r4;
  } else if (op->fmt == TFMM_FMT_TT4D) {
    const int r2 = r[1];
    for (int p = 0; p < nd; ++p) {
      int* d = &op->desc[8 * p];
      d[3] = p * n3 * r2;
      d[5] = r2;
    }
    a1 = (size_t)op->nq * r2 + (size_t)nd * n3 * r2;                  // T1 and V
  }
  op->a1_bytes = a1 * sizeof(float2);
  op->dev_bytes = h.size() * sizeof(float2);
  tfmm_status s = dev_alloc(c, (void**)&op->d_data, op->dev_bytes);
  if (s != TFMM_OK) return s;
  HIP_TRY(hipMemcpy(op->d_data, h.data(), op->dev_bytes, hipMemcpyHostToDevice));
  s = dev_alloc(c, (void**)&op->d_desc, op->desc.size() * sizeof(int));
  if (s != TFMM_OK) return s;
  op->dev_bytes += op->desc.size() * sizeof(int);
  HIP_TRY(hipMemcpy(op->d_desc, op->desc.data(), op->desc.size() * sizeof(int), hipMemcpyHostToDevice));
  // 3-D formats have per-direction ranks: launch the costliest restorations
  // first so the persistent grids finish evenly
  if (op->fmt == TFMM_FMT_TUCKER3D || op->fmt == TFMM_FMT_TT3D) {
    std::vector<double> cost(nd);
    for (int p = 0; p < nd; ++p) {
      const int* d = &op->desc[8 * p];
      const double r1 = d[4], r2 = d[5], r3 = d[6];
      cost[p] = op->fmt == TFMM_FMT_TUCKER3D
                    ? n1 * r1 * r2 * r3 + (double)n1 * n2 * r2 * r3 + (double)n1 * n2 * n3 * r3
                    : n1 * r1 * n2 * r2 + (double)n1 * n2 * n3 * r2;
    }
    std::vector<int> perm(nd);
    for (int p = 0; p < nd; ++p) perm[p] = p;
    std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    s = dev_alloc(c, (void**)&op->d_perm, (size_t)nd * sizeof(int));
    if (s != TFMM_OK) return s;
    op->dev_bytes += (size_t)nd * sizeof(int);
    HIP_TRY(hipMemcpy(op->d_perm, perm.data(), (size_t)nd * sizeof(int), hipMemcpyHostToDevice));
  }
  return plan_zstage(op);
}

// Scratch of one translation: the x-FFT'ed planes of a chunk of ndl directions
// (three-pass pipeline) and the per-direction cores of the 4-D formats.
struct ScratchPlan {
  int ndl = 1;
  int rhs_group = 1;
  size_t hbytes = 0, a1b = 0, w1b = 0;  // planes, per-call cores, x-mode products of a direction chunk
  size_t total() const { return hbytes + a1b + w1b; }
};

// x-mode product W1[fx][c][b] of one direction (4-D formats: uniform ranks)
size_t w1_elems_per_dir(const tfmm_op_s* op) {
  const auto& r = op->host.ranks;
  return (size_t)op->n[0] * r[1] * r[2];
}

ScratchPlan scratch_plan(const tfmm_op_s* op, int nr_total, size_t cap) {
  ScratchPlan sp;
  const int nd = op->ndir;
  // x-FFT'ed planes of one (RHS, direction): n1 x Ky x Kz complex64
  const size_t per_dir_rhs = (size_t)op->n[0] * op->K[1] * op->K[2] * sizeof(float2);
  const size_t w1_dir = op->use_w1 ? w1_elems_per_dir(op) * sizeof(float2) : 0;
  sp.rhs_group = std::max(1, std::min(nr_total, TFMM_MAX_RHS_PER_LAUNCH));
  sp.ndl = (int)std::max<size_t>(1, std::min<size_t>((size_t)nd, cap / (per_dir_rhs * sp.rhs_group + w1_dir)));
  sp.hbytes = op->fused ? 0 : per_dir_rhs * sp.rhs_group * sp.ndl;
  sp.hbytes = (sp.hbytes + 255) / 256 * 256;
  sp.a1b = (op->a1_bytes + 255) / 256 * 256;
  sp.w1b = (w1_dir * sp.ndl + 255) / 256 * 256;
  if (op->zfmt == tfmm::ZF_TT3D && op->tk2 && !op->fused) sp.w1b = (op->wtt_elems * sizeof(float2) + 255) / 256 * 256;
  return sp;
}

void fill_info(tfmm_op op, double setup_s) {
  tfmm_op_info& I = op->info;
  I = tfmm_op_info();
  I.fmt = op->fmt;
  I.prec = op->prec;
  for (int i = 0; i < 3; ++i) {
    I.K[i] = op->K[i];
    I.n[i] = op->n[i];
  }
  I.n_dir = op->ndir;
  I.L = op->L;
  I.bytes_full = (size_t)op->ndir * op->n[0] * op->n[1] * op->n[2] * 8;
  I.bytes_stored = op->stored_elems * 8;
  I.elems_stored = op->stored_elems;
  I.bytes_scratch = scratch_plan(op, 1, op->ctx->hcap).total();
  I.rel_err_fro = op->host.rel_err;
  I.max_dir_rel_err = op->host.max_dir_err;
  for (int i = 0; i < 8; ++i) I.ranks[i] = 0;
  const auto& r = op->host.ranks;
  if (op->fmt == TFMM_FMT_TUCKER3D || op->fmt == TFMM_FMT_TT3D) {
    const int k = (op->fmt == TFMM_FMT_TUCKER3D) ? 3 : 2;
    for (int p = 0; p < op->ndir; ++p)
      for (int i = 0; i < k; ++i) I.ranks[i] = std::max(I.ranks[i], r[(size_t)k * p + i]);
  } else {
    for (size_t i = 0; i < r.size() && i < 8; ++i) I.ranks[i] = r[i];
  }
  I.setup_seconds = setup_s;
}

tfmm_status check_problem(const tfmm_problem* P, int* ndir, int* L, int* nth, int* nph) {
  if (!P) return fail(TFMM_ERR_INVALID_ARG, "problem is NULL");
  tfmm_status s = validate_grid(P->K);
  if (s != TFMM_OK) return s;
  if ((int)P->fmt < 0 || (int)P->fmt > 5) return fail(TFMM_ERR_INVALID_ARG, "unknown format");
  if ((int)P->prec < 0 || (int)P->prec > 1) return fail(TFMM_ERR_INVALID_ARG, "unknown precision");
  int l = P->L;
  if (l <= 0) {
    const double kabs = std::hypot(P->k_re, P->k_im);
    if (!(P->digits > 0) || !(kabs > 0) || !(P->box_size > 0))
      return fail(TFMM_ERR_INVALID_ARG, "L == 0 needs positive digits, k and box_size");
    l = tfmm::multipole_order_ceil(kabs, P->box_size, P->digits);
  }
  if (l > 200) return fail(TFMM_ERR_INVALID_ARG, "multipole order too large");
  if (P->dirs) {
    // explicit direction list: unit vectors, the grid fields must be unset
    if (P->n_dir < 1 || P->n_dir > 100000) return fail(TFMM_ERR_INVALID_ARG, "n_dir out of range for dirs");
    if (P->n_theta > 0 || P->n_phi > 0) return fail(TFMM_ERR_INVALID_ARG, "dirs and n_theta/n_phi are exclusive");
    for (int p = 0; p < P->n_dir; ++p) {
      const double* d = P->dirs + 3 * (size_t)p;
      const double nn = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      if (!(std::fabs(nn - 1.0) <= 1e-9)) return fail(TFMM_ERR_INVALID_ARG, "dirs must hold unit vectors");
    }
    *L = l;
    *nth = 0;
    *nph = 0;
    *ndir = P->n_dir;
    return TFMM_OK;
  }
  int a = P->n_theta > 0 ? P->n_theta : l + 1;
  int b = P->n_phi > 0 ? P->n_phi : 2 * (l + 1);
  if ((P->n_theta > 0) != (P->n_phi > 0)) return fail(TFMM_ERR_INVALID_ARG, "set both n_theta and n_phi or neither");
  if (a < 1 || b < 1 || (long long)a * b > 100000) return fail(TFMM_ERR_INVALID_ARG, "bad direction grid");
  *L = l;
  *nth = a;
  *nph = b;
  *ndir = a * b;
  return TFMM_OK;
}

tfmm_op new_op(tfmm_ctx c, const tfmm_problem* P, int ndir, int L) {
  tfmm_op op = new tfmm_op_s();
  op->ctx = c;
  op->fmt = P->fmt;
  op->prec = P->prec;
  for (int i = 0; i < 3; ++i) {
    op->K[i] = P->K[i];
    op->n[i] = 2 * P->K[i];
  }
  op->ndir = ndir;
  op->L = L;
  return op;
}

void free_op(tfmm_ctx c, tfmm_op op) {
  if (op->d_full) dev_free(c, op->d_full, (size_t)op->ndir * op->n[0] * op->n[1] * op->n[2] * 8);
  if (op->d_data) dev_free(c, op->d_data, op->stored_elems * sizeof(float2));
  if (op->d_desc) dev_free(c, op->d_desc, op->desc.size() * sizeof(int));
  if (op->d_perm) dev_free(c, op->d_perm, (size_t)op->ndir * sizeof(int));
  for (auto& e : op->graphs) {
    (void)hipGraphExecDestroy(e.x);
    (void)hipGraphDestroy(e.g);
  }
  delete op;
}

// ---------------------------------------------------------------------------
// Translation orchestration
// ---------------------------------------------------------------------------

struct Launch {
  tfmm_ctx c;
  hipStream_t st;
  hipEvent_t a = nullptr;
  const char* name;
  Launch(tfmm_ctx c_, hipStream_t s, const char* n) : c(c_), st(s), name(n) {
    if (c->prof) {
      a = c->take_event();
      (void)hipEventRecord(a, st);
    }
  }
  void done() {
    if (c->prof) {
      hipEvent_t b = c->take_event();
      (void)hipEventRecord(b, st);
      c->pending.push_back({name, a, b});
    }
  }
};

// The per-call GEMMs (a1 and the formed products) of an operator restored in
// bf16x3 run in the same split arithmetic when it was compressed at gamma >=
// 1e-5: their rounding (a few 1e-6 relative) then stays an order below the
// compression error.  At smaller gamma, and for imported factors (no gamma),
// they run in FP32.
static bool gemm_bf16x3(const tfmm_op_s* op) { return op->prec == TFMM_PREC_BF16X3 && op->tol >= 1e-5; }

tfmm_status run_a1(tfmm_ctx c, tfmm_op op, float2* scr, hipStream_t st) {
  using tfmm::GOp;
  const int n1 = op->n[0], n2 = op->n[1], n3 = op->n[2], nd = op->ndir;
  const auto& r = op->host.ranks;
  const float2* D = op->d_data;
  const bool bfg = gemm_bf16x3(op);
  if (op->fmt == TFMM_FMT_TUCKER4D) {
    const int r1 = r[0], r2 = r[1], r3 = r[2], r4 = r[3];
    const int m = r1 * r2 * r3;
    const long long oU4 = (long long)m * r4 + (long long)n1 * r1 + (long long)n2 * r2 + (long long)n3 * r3;
    Launch L(c, st, "a1_tucker4d");
    HIP_TRY(tfmm::launch_cgemm(m, nd, r4, 1, GOp{D, r4, 1, 0}, GOp{D + oU4, 1, r4, 0}, scr, 1, m, 0, st, bfg));
    L.done();
  } else if (op->fmt == TFMM_FMT_HTUCKER4D) {
    const int r1 = r[0], r2 = r[1], r3 = r[2], r4 = r[3], r12 = r[4];
    const long long oU4 = (long long)n1 * r1 + (long long)n2 * r2 + (long long)n3 * r3;
    const long long oC12 = oU4 + (long long)nd * r4, oE = oC12 + (long long)r1 * r2 * r12;
    float2* Cp = scr;
    float2* X2 = Cp + (size_t)nd * r1 * r2 * r3;
    Launch L(c, st, "a1_htucker4d");
    // X2[p][a3][b] = sum_a4 E[a3][a4][b] U4[p][a4]   (Fig. 3(c): the (3,4) node, root
    // matrix absorbed at upload, times row p of U4)
    HIP_TRY(tfmm::launch_cgemm(r12, nd, r4, r3, GOp{D + oE, 1, r12, (long long)r4 * r12}, GOp{D + oU4, 1, r4, 0},
                               X2, 1, (long long)r3 * r12, r12, st, bfg));
    // Cp[p][a1 a2][a3] = sum_b C12[a1 a2][b] X2[p][a3][b]     (times C2)
    HIP_TRY(tfmm::launch_cgemm(r1 * r2, r3, r12, nd, GOp{D + oC12, r12, 1, 0}, GOp{X2, 1, r12, (long long)r3 * r12},
                               Cp, r3, 1, (long long)r1 * r2 * r3, st, bfg));
    L.done();
  } else if (op->fmt == TFMM_FMT_TT4D) {
    const int r1 = r[0], r2 = r[1], r3 = r[2];
    const long long oC1 = (long long)n1 * r1, oC2 = oC1 + (long long)r1 * n2 * r2,
                    oU3 = oC2 + (long long)r2 * n3 * r3;
    float2* T1 = scr;
    float2* V = T1 + (size_t)op->nq * r2;
    Launch L(c, st, "a1_tt4d");
    // T1[(x,y)][b] = sum_a U1[x][a] C1[a][y][b]               (Fig. 4(a) step 1, shared by all p)
    HIP_TRY(tfmm::launch_cgemm(n1, r2, r1, n2, GOp{D, r1, 1, 0}, GOp{D + oC1, (long long)n2 * r2, 1, r2}, T1,
                               (long long)n2 * r2, 1, r2, st, bfg));
    // V[p][z][b] = sum_c C2[b][z][c] U3[p][c]                  (Fig. 4(b) step 1, column p)
    // one GEMM per z (rows b, columns p), so each output column is a contiguous run of b
    HIP_TRY(tfmm::launch_cgemm(r2, nd, r3, n3, GOp{D + oC2, (long long)n3 * r3, 1, r3}, GOp{D + oU3, 1, r3, 0}, V,
                               1, (long long)n3 * r2, r2, st, bfg));
    L.done();
  }
  return TFMM_OK;
}

// Enqueue the translation of `nr` right-hand sides (pointer tables) on `st`
// with the scratch `scr` laid out by `sp`; `counter` = two ints of the
// persistent launches, zero on entry and left zero.  With side_slot >= 0 the
// per-call GEMMs go to that slot's side stream, forked from `st` here and
// joined back into `st` before the first z-stage (all later work, and the
// caller's completion event, stay on `st`).
tfmm_status enqueue_translate(tfmm_ctx c, tfmm_op op, const std::vector<const float2*>& As,
                              const std::vector<float2*>& Bs, hipStream_t st, void* scr, const ScratchPlan& sp,
                              int* counter, bool prof, int side_slot) {
  const int n1 = op->n[0], n2 = op->n[1], n3 = op->n[2], K3 = op->K[2], nd = op->ndir;
  const int nr_total = (int)As.size();
  const int rhs_group = sp.rhs_group, ndl = sp.ndl;
  const int lines = op->K[1] * K3;  // (y, z) lines of a box block
  float2* H = (float2*)scr;
  float2* a1 = (float2*)((char*)scr + sp.hbytes);
  float2* W1 = (float2*)((char*)scr + sp.hbytes + sp.a1b);
  const bool prof0 = c->prof;
  c->prof = prof0 && prof;
  struct Restore {
    tfmm_ctx c;
    bool v;
    ~Restore() { c->prof = v; }
  } restore{c, prof0};
  const bool tt3d_w = op->zfmt == tfmm::ZF_TT3D && op->tk2 && !op->fused;
  const bool w1_formed = op->use_w1 && !op->fused;
  // per-call GEMMs beside the first x pass (three-pass path only: the fused
  // kernel reads A itself)
  const bool split = side_slot >= 0 && !op->fused && (op->a1_bytes > 0 || tt3d_w || w1_formed);
  hipStream_t gs = st;
  if (split) {
    gs = c->side[side_slot];
    HIP_TRY(hipEventRecord(c->fork_ev[side_slot], st));
    HIP_TRY(hipStreamWaitEvent(gs, c->fork_ev[side_slot], 0));
  }
  bool joined = !split;
  auto join = [&]() -> hipError_t {
    if (joined) return hipSuccess;
    joined = true;
    hipError_t e = hipEventRecord(c->join_ev[side_slot], gs);
    return e == hipSuccess ? hipStreamWaitEvent(st, c->join_ev[side_slot], 0) : e;
  };
  if (op->a1_bytes) {
    tfmm_status s = run_a1(c, op, a1, gs);
    if (s != TFMM_OK) {
      (void)join();
      return s;
    }
  }
  if (tt3d_w) {
    // W_p[q][b] = sum_a U1_p[fx][a] C_p[a][fy][b] for every direction (Fig. 4(a) step 1)
    int r2max = 1;
    for (int p = 0; p < nd; ++p) r2max = std::max(r2max, op->desc[8 * p + 5]);
    Launch L(c, gs, "a1_tt3d_w");
    HIP_TRY(tfmm::launch_cgemm_tt3d(n1, n2, n2 * r2max, nd, op->d_desc, op->d_data, W1, gemm_bf16x3(op), gs));
    L.done();
  }
  float2* roots = op->d_roots_z;
  float2* twx = op->d_roots_x;
  tfmm::ZArgs z{};
  z.fmt = op->use_w1 && !op->fused ? tfmm::ZF_TUCKER_W1 : op->zfmt;
  z.n1 = n1; z.n2 = n2; z.n3 = n3; z.K3 = K3; z.nq = op->nq;
  z.H = H;
  z.Tfull = op->d_full;
  z.fbase = op->d_data;
  const bool four_d = op->fmt == TFMM_FMT_TUCKER4D || op->fmt == TFMM_FMT_HTUCKER4D;
  z.cbase = four_d ? a1 : op->d_data;
  if (z.fmt == tfmm::ZF_TUCKER_W1) {
    z.cbase = W1;
    z.w1dir = (long long)w1_elems_per_dir(op);
  }
  z.wbase = tt3d_w ? W1 : a1;
  z.vbase = a1 + (op->fmt == TFMM_FMT_TT4D ? (size_t)op->nq * op->host.ranks[1] : 0);
  z.desc = op->d_desc;
  z.roots = roots;
  z.KC = op->KC;
  z.cb = op->cb;
  z.lds_bytes = op->lds;
  z.bf = op->prec == TFMM_PREC_BF16X3 ? 1 : 0;
  z.tk2 = op->tk2 ? 1 : 0;
  z.rg = op->rg;
  z.perm = op->d_perm;
  z.counter = counter;
  z.ncu = c->ncu;
  const float scale = 1.0f / (float)((double)n1 * n2 * n3);
  if (op->fused) {
    z.KC = op->fKC;
    z.lds_bytes = op->flds;
    z.tk2 = op->ftk2 ? 1 : 0;
    z.p0 = 0;
    z.ndl = nd;
    for (int r0 = 0; r0 < nr_total; r0 += rhs_group) {
      const int nr = std::min(rhs_group, nr_total - r0);
      tfmm::RhsPtrs P{};
      for (int i = 0; i < nr; ++i) {
        P.a[i] = As[r0 + i];
        P.b[i] = Bs[r0 + i];
      }
      z.nrhs = nr;
      bool ok = false;
      Launch L(c, st, op->zfmt == tfmm::ZF_FULL ? "fused_full" : "fused_restore");
      HIP_TRY(tfmm::launch_fused(z, P, scale, st, &ok));
      L.done();
      if (!ok) return fail(TFMM_ERR_UNSUPPORTED, "fused translation size unsupported");
    }
    return TFMM_OK;
  }
  for (int r0 = 0; r0 < nr_total; r0 += rhs_group) {
    const int nr = std::min(rhs_group, nr_total - r0);
    tfmm::RhsPtrs P{};
    for (int i = 0; i < nr; ++i) {
      P.a[i] = As[r0 + i];
      P.b[i] = Bs[r0 + i];
    }
    for (int p0 = 0; p0 < nd; p0 += ndl) {
      const int nl = std::min(ndl, nd - p0);
      bool ok = false;
      {
        Launch L(c, st, "fwd_x");
        HIP_TRY(tfmm::launch_fwd_x(P, H, n1, lines, nr, p0, nl, op->d_perm, twx, st, &ok));
        L.done();
      }
      if (!ok) return fail(TFMM_ERR_UNSUPPORTED, "x-FFT size unsupported");
      if (z.fmt == tfmm::ZF_TUCKER_W1) {
        // W1[p][fx][b][c] = sum_a U1[fx][a] C_p[a][b][c] for the chunk's directions
        // (Fig. 3(a) step 1, the x-mode product, ahead of the z-stage); C_p is the
        // per-direction core a1 formed, [p][a][b][c].  The first chunk's runs on
        // the side stream (nothing has read W1 yet); later chunks' follow the
        // previous z-stage on `st`.
        const auto& r = op->host.ranks;
        const int r1 = r[0], r2 = r[1], r3 = r[2];
        const long long m = (long long)r1 * r2 * r3, r23 = (long long)r2 * r3;
        hipStream_t ws = joined ? st : gs;
        Launch L(c, ws, "a1_w1");
        HIP_TRY(tfmm::launch_cgemm(n1, (int)r23, r1, nl, tfmm::GOp{op->d_data + op->desc[1], r1, 1, 0},
                                   tfmm::GOp{a1 + (size_t)p0 * m, r23, 1, m}, W1, r23, 1, z.w1dir, ws,
                                   gemm_bf16x3(op)));
        L.done();
      }
      HIP_TRY(join());
      z.p0 = p0;
      z.nrhs = nr;
      z.ndl = nl;
      {
        Launch L(c, st, op->zfmt == tfmm::ZF_FULL ? "zstage_full" : "zstage_restore");
        HIP_TRY(tfmm::launch_zstage(z, st, &ok));
        L.done();
      }
      if (!ok) return fail(TFMM_ERR_UNSUPPORTED, "z-stage size unsupported");
      {
        Launch L(c, st, "inv_x");
        HIP_TRY(tfmm::launch_inv_x(P, H, n1, lines, nr, p0, nl, op->d_perm, scale, twx, st, &ok));
        L.done();
      }
      if (!ok) return fail(TFMM_ERR_UNSUPPORTED, "x-FFT size unsupported");
    }
  }
  return TFMM_OK;
}

// Translate `nr` right-hand sides given by pointer tables, using scratch slot
// `slot`.  The direction chunk starts at the context's chunk size and is
// halved (down to one direction) while the scratch does not fit the budget.
tfmm_status run_translate(tfmm_ctx c, tfmm_op op, const std::vector<const float2*>& As,
                          const std::vector<float2*>& Bs, hipStream_t st, int slot) {
  size_t cap = c->hcap;
  ScratchPlan sp = scratch_plan(op, (int)As.size(), cap);
  void* scr = nullptr;
  for (;;) {
    tfmm_status s = ensure_scratch(c, slot, sp.total(), &scr);
    if (s == TFMM_OK) break;
    if (s != TFMM_ERR_BUDGET || sp.ndl <= 1) return s;
    const int want = sp.ndl / 2;
    while (scratch_plan(op, (int)As.size(), cap).ndl > want && cap > 1) cap /= 2;
    sp = scratch_plan(op, (int)As.size(), cap);
  }
  return enqueue_translate(c, op, As, Bs, st, scr, sp, c->counters + 2 * slot, true, slot);
}

// ---------------------------------------------------------------------------
// Autotuner: tile configurations keyed by grid class, rank bucket, precision
// and RHS bucket.
// ---------------------------------------------------------------------------
std::string tune_key(tfmm_op op, int nrhs) {
  int rmax = 0;
  for (int32_t r : op->host.ranks) rmax = std::max(rmax, (int)r);
  const int nb = nrhs <= 1 ? 1 : (nrhs <= 4 ? 4 : (nrhs <= 16 ? 16 : 64));
  char buf[160];
  std::snprintf(buf, sizeof buf, "f%d|p%d|n%dx%dx%d|d%d|r%d|s%d", (int)op->fmt, (int)op->prec, op->n[0], op->n[1],
                op->n[2], op->ndir, (rmax + 7) / 8 * 8, nb);
  return buf;
}

bool same_choice(const TuneChoice& a, const TuneChoice& b) {
  return a.fused == b.fused && a.cb == b.cb && a.tk2 == b.tk2;
}

void drop_graphs(tfmm_op op) {
  for (auto& e : op->graphs) {
    (void)hipGraphExecDestroy(e.x);
    (void)hipGraphDestroy(e.g);
  }
  op->graphs.clear();
}

tfmm_status apply_choice(tfmm_op op, const TuneChoice& ch) {
  if (same_choice(op->choice, ch)) return TFMM_OK;
  const TuneChoice old = op->choice;
  op->choice = ch;
  tfmm_status s = plan_zstage(op);
  if (s != TFMM_OK) {
    op->choice = old;
    (void)plan_zstage(op);
    return s;
  }
  drop_graphs(op);
  op->info.bytes_scratch = scratch_plan(op, 1, op->ctx->hcap).total();
  return TFMM_OK;
}

// Use the tuned configuration for this RHS count if one is known.
void apply_tuned(tfmm_ctx c, tfmm_op op, int nrhs) {
  if (c->tune.empty()) return;
  auto it = c->tune.find(tune_key(op, nrhs));
  if (it != c->tune.end() && apply_choice(op, it->second) == TFMM_OK) op->tuned = true;
}

void load_tune_cache(tfmm_ctx c) {
  FILE* f = c->tune_path.empty() ? nullptr : std::fopen(c->tune_path.c_str(), "r");
  if (!f) return;
  char key[160];
  TuneChoice ch;
  while (std::fscanf(f, "%159s fused=%d cb=%d tk2=%d%*[^\n]", key, &ch.fused, &ch.cb, &ch.tk2) == 4)
    c->tune[key] = ch;
  std::fclose(f);
}

tfmm_status translate_contiguous(tfmm_ctx c, tfmm_op op, const void* A, void* B, int nrhs, hipStream_t st,
                                 int slot) {
  apply_tuned(c, op, nrhs);
  const size_t blk = (size_t)op->ndir * op->K[0] * op->K[1] * op->K[2];
  std::vector<const float2*> As(nrhs);
  std::vector<float2*> Bs(nrhs);
  for (int s = 0; s < nrhs; ++s) {
    As[s] = (const float2*)A + s * blk;
    Bs[s] = (float2*)B + s * blk;
  }
  return run_translate(c, op, As, Bs, st, slot);
}

// ---------------------------------------------------------------------------
// Scheduler: a worker thread admits queued jobs in arrival order against the
// device-memory budget, coalesces the ones on the same operator into one
// batched launch per stream slot, and a completer thread stamps completion
// when the slot's event fires and returns the jobs' memory to the budget.
//
// Admission charges each job's A and B (caller buffers, but device memory the
// job occupies) and the slot's translation scratch.  A job that does not fit is
// parked at the head of the queue until a running job completes; only a job
// that cannot fit even with nothing else running fails (TFMM_ERR_BUDGET).
// ---------------------------------------------------------------------------

size_t job_io_bytes(const Job& j) {
  return (size_t)2 * j.nrhs * j.op->ndir * j.op->K[0] * j.op->K[1] * j.op->K[2] * sizeof(float2);
}

// Bytes a batch needs beyond what is charged now: its A and B plus the growth of
// the slot's scratch for the smallest direction chunk.
size_t admission_need(tfmm_ctx c, tfmm_op op, int nr, size_t io, int slot) {
  const size_t scr = scratch_plan(op, nr, 1).total();
  const size_t have = c->scratch[1 + slot].bytes;
  return io + (scr > have ? scr : 0);
}

void worker_loop(tfmm_ctx c) {
  (void)hipSetDevice(c->device);
  for (;;) {
    std::vector<std::shared_ptr<Job>> batch;
    int slot = -1;
    {
      std::unique_lock<std::mutex> lk(c->qmu);
      c->qcv.wait(lk, [&] {
        return c->stop || (!c->queue.empty() && (c->slot_busy[0] == 0 || c->slot_busy[1] == 0));
      });
      if (c->stop && c->queue.empty()) return;
      slot = c->slot_busy[0] == 0 ? 0 : 1;
      // coalesce queued jobs on the operator of the oldest job (up to 4 x the
      // launch RHS cap), in arrival order
      tfmm_op op = c->queue.front()->op;
      int nr = 0;
      for (auto it = c->queue.begin(); it != c->queue.end();) {
        if ((*it)->op == op && nr + (*it)->nrhs <= 4 * TFMM_MAX_RHS_PER_LAUNCH) {
          nr += (*it)->nrhs;
          batch.push_back(*it);
          it = c->queue.erase(it);
        } else {
          ++it;
        }
      }
      c->slot_busy[slot] = 1;
    }
    tfmm_op op = batch.front()->op;
    // admission against the budget (the budget is guarded by c->mu)
    bool park = false;
    tfmm_status adm = TFMM_OK;
    {
      std::lock_guard<std::recursive_mutex> g(c->mu);
      auto need_of = [&](size_t njobs) {
        int nr = 0;
        size_t io = 0;
        for (size_t i = 0; i < njobs; ++i) {
          nr += batch[i]->nrhs;
          io += job_io_bytes(*batch[i]);
        }
        return admission_need(c, op, nr, io, slot);
      };
      size_t keep = batch.size();
      while (keep > 1 && c->used + need_of(keep) > c->budget) --keep;
      if (c->used + need_of(keep) > c->budget) {
        // the oldest job alone does not fit: free the idle slot's scratch and retry
        const int other = 1 - slot;
        bool other_idle;
        {
          std::lock_guard<std::mutex> lk(c->qmu);
          other_idle = c->slot_busy[other] == 0;
        }
        if (other_idle) release_scratch(c, 1 + other);
        if (c->used + need_of(keep) > c->budget) {
          release_scratch(c, 1 + slot);
          if (other_idle && c->used + need_of(keep) > c->budget) release_scratch(c, 0);
          if (c->used + need_of(keep) > c->budget) {
            if (other_idle) {
              // nothing else holds translation memory: the job can never fit
              adm = fail(TFMM_ERR_BUDGET, "job needs " + std::to_string(need_of(keep)) + " B, " +
                                              std::to_string(c->budget - std::min(c->budget, c->used)) +
                                              " B of the budget are not held by operators");
            } else {
              park = true;
            }
          }
        }
      }
      if (!park) {
        // jobs beyond `keep` (all but the oldest when it cannot fit) go back to
        // the head of the queue, in order
        if (adm != TFMM_OK) keep = 1;
        std::vector<std::shared_ptr<Job>> back(batch.begin() + keep, batch.end());
        batch.resize(keep);
        if (!back.empty()) {
          std::lock_guard<std::mutex> lk(c->qmu);
          c->queue.insert(c->queue.begin(), back.begin(), back.end());
        }
        if (adm == TFMM_OK)
          for (auto& j : batch) {
            j->charged = job_io_bytes(*j);
            c->used += j->charged;
          }
      }
    }
    if (park) {
      // back to the head of the queue; wait for a running job to complete
      std::unique_lock<std::mutex> lk(c->qmu);
      c->queue.insert(c->queue.begin(), batch.begin(), batch.end());
      c->n_parked += 1;
      c->slot_busy[slot] = 0;
      const int other = 1 - slot;
      c->fcv.wait(lk, [&] { return c->stop || c->slot_busy[other] == 0; });
      continue;
    }
    std::vector<const float2*> As;
    std::vector<float2*> Bs;
    const size_t blk = (size_t)op->ndir * op->K[0] * op->K[1] * op->K[2];
    for (auto& j : batch)
      for (int s = 0; s < j->nrhs; ++s) {
        As.push_back(j->A + s * blk);
        Bs.push_back(j->B + s * blk);
      }
    tfmm_status st = adm;
    hipEvent_t ev = nullptr;
    if (st == TFMM_OK) {
      std::lock_guard<std::recursive_mutex> g(c->mu);
      st = run_translate(c, op, As, Bs, c->streams[slot], 1 + slot);
      if (st == TFMM_OK) mark_slot(c, 1 + slot, c->streams[slot]);
      if (st == TFMM_OK && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess)
        (void)hipEventRecord(ev, c->streams[slot]);
    }
    InFlight f;
    f.ev = ev;
    f.jobs = batch;
    f.slot = slot;
    if (st == TFMM_OK) {
      std::lock_guard<std::mutex> lk(c->qmu);
      c->n_launch += 1;
    }
    if (st != TFMM_OK || !ev) {
      for (auto& j : batch) j->status = st != TFMM_OK ? st : TFMM_ERR_HIP;
      f.ev = nullptr;
    }
    {
      std::lock_guard<std::mutex> lk(c->qmu);
      c->inflight.push_back(std::move(f));
    }
    c->fcv.notify_all();
  }
}

void completer_loop(tfmm_ctx c) {
  (void)hipSetDevice(c->device);
  for (;;) {
    InFlight f;
    {
      std::unique_lock<std::mutex> lk(c->qmu);
      c->fcv.wait(lk, [&] { return c->stop || !c->inflight.empty(); });
      if (c->inflight.empty()) return;
      f = std::move(c->inflight.front());
      c->inflight.pop_front();
    }
    tfmm_status st = TFMM_OK;
    if (f.ev) {
      if (hipEventSynchronize(f.ev) != hipSuccess) st = TFMM_ERR_HIP;
      (void)hipEventDestroy(f.ev);
    }
    const double t = now_s();
    {
      std::lock_guard<std::recursive_mutex> g(c->mu);
      for (auto& j : f.jobs) {
        uncharge(c, j->charged);
        j->charged = 0;
      }
    }
    {
      std::lock_guard<std::mutex> lk(c->qmu);
      for (auto& j : f.jobs) {
        if (j->status == TFMM_OK) j->status = st;
        if (j->status == TFMM_OK)
          c->n_done += 1;
        else
          c->n_failed += 1;
        j->t_done = t;
        j->op->refs.fetch_sub(1);
        j->done.store(1);
      }
      c->slot_busy[f.slot] = 0;
    }
    c->qcv.notify_all();
    c->fcv.notify_all();
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* tfmm_status_str(tfmm_status s) {
  switch (s) {
    case TFMM_OK: return "ok";
    case TFMM_ERR_INVALID_ARG: return "invalid argument";
    case TFMM_ERR_UNSUPPORTED: return "unsupported";
    case TFMM_ERR_BUDGET: return "device-memory budget exhausted";
    case TFMM_ERR_OOM: return "out of memory";
    case TFMM_ERR_HIP: return "HIP error";
    case TFMM_ERR_BUSY: return "operator busy";
    case TFMM_ERR_UNKNOWN_TICKET: return "unknown ticket";
    case TFMM_ERR_QUEUE_FULL: return "queue full";
    case TFMM_ERR_INTERNAL: return "internal error";
    case TFMM_ERR_NO_DEVICE: return "no HIP device";
    case TFMM_ERR_NOT_CONVERGED: return "iterative solve did not converge";
  }
  return "unknown status";
}

const char* tfmm_last_error(void) { return g_last_error.c_str(); }

tfmm_status tfmm_ctx_create(int device, size_t budget, tfmm_ctx* out) {
  if (!out) return fail(TFMM_ERR_INVALID_ARG, "out is NULL");
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
    (void)hipGetLastError();
    return fail(TFMM_ERR_NO_DEVICE, "no HIP device visible");
  }
  if (device < 0 || device >= count) return fail(TFMM_ERR_INVALID_ARG, "device index out of range");
  HIP_TRY(hipSetDevice(device));
  size_t freeb = 0, total = 0;
  HIP_TRY(hipMemGetInfo(&freeb, &total));
  tfmm_ctx c = new tfmm_ctx_s();
  c->device = device;
  c->budget = budget ? budget : (size_t)(0.9 * (double)freeb);
  const char* nf = std::getenv("TFMM_NO_FUSED");
  c->no_fused = nf && nf[0] == '1';
  const char* nt = std::getenv("TFMM_NO_TK2");
  c->no_tk2 = nt && nt[0] == '1';
  const char* nw1 = std::getenv("TFMM_NO_W1");
  c->no_w1 = nw1 && nw1[0] == '1';
  const char* hc4 = std::getenv("TFMM_HOST_COMPRESS");
  c->host_compress = hc4 && hc4[0] == '1';
  // fewer, larger three-pass chunks are faster (one chunk for every direction of
  // the 24^3-box / 162-direction / 8-RHS workload: 1.91 -> 1.81 ms per step), so
  // the chunk takes an eighth of the budget, within [64 MiB, 1 GiB]
  c->hcap = std::min<size_t>((size_t)1 << 30, std::max<size_t>((size_t)64 << 20, c->budget / 8));
  if (const char* hc = std::getenv("TFMM_HCAP_MB")) {
    const long v = std::strtol(hc, nullptr, 10);
    if (v >= 1 && v <= 65536) c->hcap = (size_t)v << 20;
  }
  const char* tp = std::getenv("TFMM_TUNE_CACHE");
  if (tp && tp[0]) {
    c->tune_path = tp;
    load_tune_cache(c);
  }
  const char* gm = std::getenv("TFMM_GRAPH");
  if (gm && (gm[0] == '0' || gm[0] == '1')) c->graph_mode = gm[0] - '0';
  const char* ng = std::getenv("TFMM_NO_GRAPH");
  if (ng && ng[0] == '1') c->graph_mode = 0;
  if (hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c->ncu < 1)
    c->ncu = 1;
  // device address of this device's copy of the allocation-free entry point's
  // fixed scratch (looked up once per device; the device is current here)
  {
    const hipError_t e = tfmm::noalloc_scratch_init(device);
    if (e != hipSuccess) {
      // only the allocation-free entry point needs it; it reports this error
      c->noalloc_error = std::string("fixed scratch lookup failed: ") + hipGetErrorString(e);
      (void)hipGetLastError();
    }
  }
  if (hipMalloc((void**)&c->counters, 64 * sizeof(int)) != hipSuccess ||
      hipMemset(c->counters, 0, 64 * sizeof(int)) != hipSuccess ||
      hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    if (c->counters) (void)hipFree(c->counters);
    delete c;
    return fail(TFMM_ERR_HIP, "context resources could not be created");
  }
  for (int i = 0; i < 2; ++i)
    if (hipStreamCreateWithFlags(&c->streams[i], hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(TFMM_ERR_HIP, "stream creation failed");
    }
  for (auto& e : c->slot_ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      delete c;
      return fail(TFMM_ERR_HIP, "event creation failed");
    }
  for (int i = 0; i < tfmm_ctx_s::kSlots; ++i)
    if (hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->fork_ev[i], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->join_ev[i], hipEventDisableTiming) != hipSuccess) {
      delete c;
      return fail(TFMM_ERR_HIP, "side stream creation failed");
    }
  c->worker = std::thread(worker_loop, c);
  c->completer = std::thread(completer_loop, c);
  *out = c;
  return TFMM_OK;
}

tfmm_status tfmm_ctx_destroy(tfmm_ctx c) {
  if (!c) return fail(TFMM_ERR_INVALID_ARG, "ctx is NULL");
  {
    std::unique_lock<std::mutex> lk(c->qmu);
    c->fcv.wait(lk, [&] { return c->queue.empty() && c->inflight.empty() && !c->slot_busy[0] && !c->slot_busy[1]; });
    c->stop = true;
  }
  c->qcv.notify_all();
  c->worker.join();
  c->fcv.notify_all();
  c->completer.join();
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (auto& p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : c->event_pool) (void)hipEventDestroy(e);
  for (tfmm_basis b : c->bases) free_basis(c, b);
  for (tfmm_near m : c->nears) {
    (void)hipFree(m->d_rp);
    (void)hipFree(m->d_ci);
    (void)hipFree(m->d_val);
    delete m;
  }
  if (c->mv_buf) (void)hipFree(c->mv_buf);
  for (tfmm_op op : c->ops) free_op(c, op);
  for (auto& kv : c->roots) (void)hipFree(kv.second);
  for (auto& s : c->scratch)
    if (s.ptr) (void)hipFree(s.ptr);
  for (auto& s : c->streams) (void)hipStreamDestroy(s);
  for (auto& e : c->slot_ev) (void)hipEventDestroy(e);
  for (int i = 0; i < tfmm_ctx_s::kSlots; ++i) {
    (void)hipStreamDestroy(c->side[i]);
    (void)hipEventDestroy(c->fork_ev[i]);
    (void)hipEventDestroy(c->join_ev[i]);
  }
  (void)hipStreamDestroy(c->cap_stream);
  (void)hipFree(c->counters);
  delete c;
  return TFMM_OK;
}

tfmm_status tfmm_ctx_memory(tfmm_ctx c, size_t* used, size_t* budget) {
  if (!c) return fail(TFMM_ERR_INVALID_ARG, "ctx is NULL");
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (used) *used = c->used;
  if (budget) *budget = c->budget;
  return TFMM_OK;
}

tfmm_status tfmm_setup_compressed(tfmm_ctx c, const tfmm_problem* P, tfmm_op* out) {
  if (!c || !out) return fail(TFMM_ERR_INVALID_ARG, "ctx or out is NULL");
  int ndir, L, nth, nph;
  tfmm_status s = check_problem(P, &ndir, &L, &nth, &nph);
  if (s != TFMM_OK) return s;
  if (!(P->k_re > 0) || !(P->box_size > 0)) return fail(TFMM_ERR_INVALID_ARG, "k_re and box_size must be positive");
  if (!(P->k_im <= 0)) return fail(TFMM_ERR_INVALID_ARG, "k_im must be <= 0 (a passive medium)");
  if (P->fmt != TFMM_FMT_FULL && !(P->tol >= 0 && P->tol < 1)) return fail(TFMM_ERR_INVALID_ARG, "tol must be in [0, 1)");
  const double t0 = now_s();
  std::lock_guard<std::recursive_mutex> g(c->mu);
  HIP_TRY(hipSetDevice(c->device));
  std::vector<double> khat, w;
  if (P->dirs)
    khat.assign(P->dirs, P->dirs + 3 * (size_t)ndir);
  else
    tfmm::direction_grid(nth, nph, khat, w);
  const int n[3] = {2 * P->K[0], 2 * P->K[1], 2 * P->K[2]};
  const long long N = (long long)n[0] * n[1] * n[2];
  const size_t tbytes = (size_t)N * ndir * sizeof(double2);
  // FP64 sampling and FFT on the device (temporary buffers, not kept)
  double* d_khat = nullptr;
  double2* d_T = nullptr;
  HIP_TRY(hipMalloc(&d_khat, khat.size() * sizeof(double)));
  if (hipMalloc(&d_T, tbytes) != hipSuccess) {
    (void)hipFree(d_khat);
    (void)hipGetLastError();
    return fail(TFMM_ERR_OOM, "no device memory for operator sampling");
  }
  hipError_t e = hipMemcpy(d_khat, khat.data(), khat.size() * sizeof(double), hipMemcpyHostToDevice);
  const int near_rule = (int)P->near_rule;
  const double near_param = P->near_param > 0 ? P->near_param : (near_rule == 0 ? 1.0 : 4.0);
  const bool scale0 = P->scale_re == 0 && P->scale_im == 0;
  if (e == hipSuccess)
    e = tfmm::launch_sample(d_T, d_khat, ndir, P->K, P->box_size, P->k_re, P->k_im, L, near_rule, near_param,
                            scale0 ? 1.0 : P->scale_re, scale0 ? 0.0 : P->scale_im, 0);
  if (e == hipSuccess) e = hipStreamSynchronize(0);
  (void)hipFree(d_khat);
  if (e != hipSuccess) {
    (void)hipFree(d_T);
    return fail(TFMM_ERR_HIP, std::string("operator sampling: ") + hipGetErrorString(e));
  }
  std::string err = tfmm::fft3d_forward_device(d_T, n, ndir, 0);
  if (!err.empty()) {
    (void)hipFree(d_T);
    return fail(TFMM_ERR_HIP, "operator FFT: " + err);
  }
  // compression (Algorithms 1-3): the 4-D formats on the device, the
  // per-direction 3-D formats on the host
  tfmm_op op = new_op(c, P, ndir, L);
  op->tol = P->fmt == TFMM_FMT_FULL ? 0.0 : P->tol;
  const int nthreads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const bool four_d = P->fmt == TFMM_FMT_TUCKER4D || P->fmt == TFMM_FMT_TT4D || P->fmt == TFMM_FMT_HTUCKER4D;
  if (four_d && !c->host_compress) {
    err = tfmm::compress_4d_device(d_T, ndir, n, (int)P->fmt, P->tol, op->host, nthreads, 0);
    (void)hipFree(d_T);
  } else {
    std::vector<cd> T((size_t)N * ndir);
    e = hipMemcpy(T.data(), d_T, tbytes, hipMemcpyDeviceToHost);
    (void)hipFree(d_T);
    if (e != hipSuccess) {
      delete op;
      return fail(TFMM_ERR_HIP, std::string("operator copy: ") + hipGetErrorString(e));
    }
    err = tfmm::compress_operator(T, ndir, n, (int)P->fmt, P->fmt == TFMM_FMT_FULL ? 0.0 : P->tol, op->host,
                                  nthreads);
  }
  if (!err.empty()) {
    delete op;
    return fail(TFMM_ERR_INTERNAL, "compression: " + err);
  }
  s = build_device_op(c, op);
  if (s != TFMM_OK) {
    free_op(c, op);
    return s;
  }
  if (!P->dirs) {
    op->physical = true;
    op->khat = khat;
    op->wts = w;
    op->k_re = P->k_re;
    op->k_im = P->k_im;
    op->box = P->box_size;
  }
  fill_info(op, now_s() - t0);
  c->ops.push_back(op);
  *out = op;
  return TFMM_OK;
}

tfmm_status tfmm_op_import(tfmm_ctx c, const tfmm_problem* P, const int32_t* ranks, size_t nranks,
                           const double* data, size_t ndata, tfmm_op* out) {
  if (!c || !out) return fail(TFMM_ERR_INVALID_ARG, "ctx or out is NULL");
  int ndir, L, nth, nph;
  tfmm_problem Q = *P;
  if (Q.L <= 0 && Q.n_theta <= 0 && Q.n_dir <= 0)
    return fail(TFMM_ERR_INVALID_ARG, "import needs L, an explicit direction grid or a direction count");
  int count_only = 0;
  if (!Q.dirs && Q.n_dir > 0) {
    // a direction count alone: nothing is sampled, so no directions are needed
    if (Q.n_theta > 0 || Q.n_phi > 0) return fail(TFMM_ERR_INVALID_ARG, "n_dir and n_theta/n_phi are exclusive");
    if (Q.n_dir > 100000) return fail(TFMM_ERR_INVALID_ARG, "n_dir out of range");
    count_only = Q.n_dir;
    Q.n_theta = 1;
    Q.n_phi = Q.n_dir;
    if (Q.L <= 0) Q.L = 1;
  }
  tfmm_status s = check_problem(&Q, &ndir, &L, &nth, &nph);
  if (s != TFMM_OK) return s;
  if (count_only) L = P->L > 0 ? P->L : 0;
  if (nranks && !ranks) return fail(TFMM_ERR_INVALID_ARG, "ranks is NULL");
  if (!data) return fail(TFMM_ERR_INVALID_ARG, "data is NULL");
  const int n[3] = {2 * P->K[0], 2 * P->K[1], 2 * P->K[2]};
  std::vector<int32_t> r(ranks, ranks + nranks);
  const long long need = tfmm::factor_elems((int)P->fmt, n, ndir, r);
  if (need < 0) return fail(TFMM_ERR_INVALID_ARG, "ranks inconsistent with the format");
  if ((long long)ndata != 2 * need)
    return fail(TFMM_ERR_INVALID_ARG, "data holds " + std::to_string(ndata) + " doubles, format needs " +
                                          std::to_string(2 * need));
  std::lock_guard<std::recursive_mutex> g(c->mu);
  HIP_TRY(hipSetDevice(c->device));
  tfmm_op op = new_op(c, P, ndir, L);
  op->tol = P->fmt == TFMM_FMT_FULL || !(P->tol > 0 && P->tol < 1) ? 0.0 : P->tol;
  op->host.fmt = (int)P->fmt;
  for (int i = 0; i < 3; ++i) op->host.n[i] = n[i];
  op->host.ndir = ndir;
  op->host.ranks = r;
  op->host.data.resize((size_t)need);
  std::memcpy((void*)op->host.data.data(), data, ndata * sizeof(double));
  op->host.rel_err = -1.0;
  op->host.max_dir_err = -1.0;
  s = build_device_op(c, op);
  if (s != TFMM_OK) {
    free_op(c, op);
    return s;
  }
  fill_info(op, 0.0);
  c->ops.push_back(op);
  *out = op;
  return TFMM_OK;
}

tfmm_status tfmm_op_info_get(tfmm_op op, tfmm_op_info* out) {
  if (!op || !out) return fail(TFMM_ERR_INVALID_ARG, "op or out is NULL");
  *out = op->info;
  return TFMM_OK;
}

tfmm_status tfmm_op_ranks(tfmm_op op, int32_t* ranks, size_t cap, size_t* need) {
  if (!op) return fail(TFMM_ERR_INVALID_ARG, "op is NULL");
  const auto& r = op->host.ranks;
  if (need) *need = r.size();
  if (ranks) {
    if (cap < r.size()) return fail(TFMM_ERR_INVALID_ARG, "ranks buffer too small");
    std::copy(r.begin(), r.end(), ranks);
  }
  return TFMM_OK;
}

tfmm_status tfmm_op_export(tfmm_op op, double* buf, size_t cap, size_t* need) {
  if (!op) return fail(TFMM_ERR_INVALID_ARG, "op is NULL");
  const size_t n = op->host.data.size() * 2;
  if (need) *need = n;
  if (buf) {
    if (cap < n) return fail(TFMM_ERR_INVALID_ARG, "export buffer too small");
    std::memcpy(buf, (const void*)op->host.data.data(), n * sizeof(double));
  }
  return TFMM_OK;
}

tfmm_status tfmm_op_release(tfmm_ctx c, tfmm_op op) {
  if (!c || !op) return fail(TFMM_ERR_INVALID_ARG, "ctx or op is NULL");
  std::lock_guard<std::recursive_mutex> g(c->mu);
  auto it = std::find(c->ops.begin(), c->ops.end(), op);
  if (it == c->ops.end()) return fail(TFMM_ERR_INVALID_ARG, "operator does not belong to this context");
  if (op->refs.load() > 0) return fail(TFMM_ERR_BUSY, "operator has queued jobs");
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  c->ops.erase(it);
  free_op(c, op);
  return TFMM_OK;
}

static tfmm_status check_translate(tfmm_ctx c, tfmm_op op, const void* A, void* B, int32_t nrhs) {
  if (!c || !op) return fail(TFMM_ERR_INVALID_ARG, "ctx or op is NULL");
  if (op->ctx != c) return fail(TFMM_ERR_INVALID_ARG, "operator belongs to another context");
  if (!A || !B) return fail(TFMM_ERR_INVALID_ARG, "A or B is NULL");
  if (nrhs < 1) return fail(TFMM_ERR_INVALID_ARG, "nrhs must be >= 1");
  const size_t bytes = (size_t)nrhs * op->ndir * op->K[0] * op->K[1] * op->K[2] * 8;
  const char* a = (const char*)A;
  const char* b = (const char*)B;
  if (a < b + bytes && b < a + bytes) return fail(TFMM_ERR_INVALID_ARG, "A and B overlap");
  return TFMM_OK;
}

tfmm_status tfmm_translate(tfmm_ctx c, tfmm_op op, const void* A, void* B, int32_t nrhs, void* stream) {
  tfmm_status s = check_translate(c, op, A, B, nrhs);
  if (s != TFMM_OK) return s;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  // A single fused launch is cheaper to issue directly than as a graph;
  // multi-launch sequences (three-pass pipeline, per-call core contraction)
  // are captured once per (nrhs, A, B) and replayed.
  const bool multi = !op->fused || op->a1_bytes > 0;
  if (c->prof || c->graph_mode == 0 || (c->graph_mode == 2 && !multi)) {
    s = translate_contiguous(c, op, A, B, nrhs, st, 0);
    if (s == TFMM_OK) mark_slot(c, 0, st);
    return s;
  }
  // replay a captured translation of the same (nrhs, A, B) if its scratch is still in place
  auto& G = op->graphs;
  for (size_t i = 0; i < G.size(); ++i) {
    if (G[i].nrhs != nrhs || G[i].A != A || G[i].B != B) continue;
    tfmm_op_s::GraphEntry e = G[i];
    G.erase(G.begin() + i);
    if (e.gen == c->scratch_gen[0]) {
      G.push_back(e);
      HIP_TRY(hipGraphLaunch(e.x, st));
      mark_slot(c, 0, st);
      return TFMM_OK;
    }
    (void)hipGraphExecDestroy(e.x);
    (void)hipGraphDestroy(e.g);
    break;
  }
  // first use: run eagerly (this also sizes scratch and tables), then record the
  // same launch sequence on the capture stream for later calls
  s = translate_contiguous(c, op, A, B, nrhs, st, 0);
  if (s != TFMM_OK) return s;
  mark_slot(c, 0, st);
  const unsigned gen = c->scratch_gen[0];
  HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
  s = translate_contiguous(c, op, A, B, nrhs, c->cap_stream, 0);
  hipGraph_t gr = nullptr;
  const hipError_t ce = hipStreamEndCapture(c->cap_stream, &gr);
  if (s != TFMM_OK || ce != hipSuccess || gen != c->scratch_gen[0]) {
    if (gr) (void)hipGraphDestroy(gr);
    (void)hipGetLastError();
    return s;  // the eager result stands; capture is retried on the next call
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, gr, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(gr);
    (void)hipGetLastError();
    return TFMM_OK;
  }
  if (G.size() >= 4) {
    (void)hipGraphExecDestroy(G.front().x);
    (void)hipGraphDestroy(G.front().g);
    G.erase(G.begin());
  }
  G.push_back({nrhs, A, B, gen, gr, x});
  return TFMM_OK;
}

tfmm_status tfmm_translate_noalloc(tfmm_ctx c, tfmm_op op, const void* A, void* B, int32_t nrhs, void* stream) {
  tfmm_status s = check_translate(c, op, A, B, nrhs);
  if (s != TFMM_OK) return s;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  HIP_TRY(hipSetDevice(c->device));
  char* base = (char*)tfmm::noalloc_scratch(c->device);
  if (!base)
    return fail(TFMM_ERR_HIP, c->noalloc_error.empty() ? "fixed scratch of this device was not looked up"
                                                        : c->noalloc_error);
  const size_t room = tfmm::kNoAllocScratchBytes - tfmm::kNoAllocCounterBytes;
  // the direction chunk shrinks (down to one direction) until the scratch fits
  size_t cap = c->hcap;
  ScratchPlan sp = scratch_plan(op, nrhs, cap);
  while (sp.total() > room && sp.ndl > 1) {
    cap /= 2;
    sp = scratch_plan(op, nrhs, cap);
  }
  if (sp.total() > room)
    return fail(TFMM_ERR_UNSUPPORTED, "translation needs " + std::to_string(sp.total()) +
                                          " B of scratch, the fixed scratch holds " + std::to_string(room) + " B");
  hipStream_t st = (hipStream_t)stream;
  int* counter = (int*)base;
  // the persistent launches need their counters at zero; a kernel (not a
  // memset) so that the call may be captured
  HIP_TRY(tfmm::launch_zero(counter, 2, st));
  const size_t blk = (size_t)op->ndir * op->K[0] * op->K[1] * op->K[2];
  std::vector<const float2*> As(nrhs);
  std::vector<float2*> Bs(nrhs);
  for (int i = 0; i < nrhs; ++i) {
    As[i] = (const float2*)A + i * blk;
    Bs[i] = (float2*)B + i * blk;
  }
  return enqueue_translate(c, op, As, Bs, st, base + tfmm::kNoAllocCounterBytes, sp, counter, false, -1);
}

// ---------------------------------------------------------------------------
// Far-field matvec around the translation: patterns (Eq. (3)), aggregation
// (Eq. (4)), projection (Eq. (6))
// ---------------------------------------------------------------------------

static void free_basis(tfmm_ctx c, tfmm_basis b) {
  dev_free(c, b->d_pat, (size_t)b->ndir * b->N * sizeof(float4));
  dev_free(c, b->d_start, (size_t)(b->nbox + 1) * sizeof(int));
  dev_free(c, b->d_orig, (size_t)b->N * sizeof(int));
  dev_free(c, b->d_boxof, (size_t)b->N * sizeof(int));
  dev_free(c, b->d_w, (size_t)b->ndir * sizeof(float));
  delete b;
}

tfmm_status tfmm_basis_setup(tfmm_ctx c, tfmm_op op, int32_t n_basis, const double* pos, const double* orient,
                             tfmm_basis* out) {
  if (!c || !op || !out) return fail(TFMM_ERR_INVALID_ARG, "ctx, op or out is NULL");
  if (op->ctx != c) return fail(TFMM_ERR_INVALID_ARG, "operator belongs to another context");
  if (n_basis < 1 || !pos || !orient) return fail(TFMM_ERR_INVALID_ARG, "need n_basis >= 1, pos and orient");
  if (!op->physical)
    return fail(TFMM_ERR_UNSUPPORTED, "the operator carries no direction quadrature (imported or explicit directions)");
  const int K1 = op->K[0], K2 = op->K[1], K3 = op->K[2];
  const int nbox = K1 * K2 * K3, N = n_basis, nd = op->ndir;
  // box of every basis function (grid corner at the origin), sorted by box
  std::vector<int> box(N);
  for (int n = 0; n < N; ++n) {
    int v[3];
    for (int i = 0; i < 3; ++i) {
      const double x = pos[3 * (size_t)n + i] / op->box;
      if (!(x >= 0.0) || !(x < (double)op->K[i])) return fail(TFMM_ERR_INVALID_ARG, "basis position outside the box grid");
      v[i] = (int)std::floor(x);
    }
    const double un = orient[3 * (size_t)n] * orient[3 * (size_t)n] + orient[3 * (size_t)n + 1] * orient[3 * (size_t)n + 1] +
                      orient[3 * (size_t)n + 2] * orient[3 * (size_t)n + 2];
    if (!(std::fabs(un - 1.0) <= 1e-6)) return fail(TFMM_ERR_INVALID_ARG, "orientations must be unit vectors");
    box[n] = (v[0] * K2 + v[1]) * K3 + v[2];
  }
  std::vector<int> order(N);
  for (int n = 0; n < N; ++n) order[n] = n;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return box[a] < box[b]; });
  std::vector<int> start(nbox + 1, 0), boxof(N);
  std::vector<double> geo(6 * (size_t)N);
  for (int i = 0; i < N; ++i) {
    const int n = order[i], v = box[n];
    boxof[i] = v;
    start[v + 1] += 1;
    const int vx = v / (K2 * K3), vy = (v / K3) % K2, vz = v % K3;
    const double cen[3] = {(vx + 0.5) * op->box, (vy + 0.5) * op->box, (vz + 0.5) * op->box};
    for (int d = 0; d < 3; ++d) {
      geo[6 * (size_t)i + d] = pos[3 * (size_t)n + d] - cen[d];
      geo[6 * (size_t)i + 3 + d] = orient[3 * (size_t)n + d];
    }
  }
  for (int v = 0; v < nbox; ++v) start[v + 1] += start[v];
  std::vector<float> wf(nd);
  for (int p = 0; p < nd; ++p) wf[p] = (float)op->wts[p];
  std::lock_guard<std::recursive_mutex> g(c->mu);
  HIP_TRY(hipSetDevice(c->device));
  tfmm_basis b = new tfmm_basis_s();
  b->ctx = c;
  b->op = op;
  b->N = N;
  b->nbox = nbox;
  b->ndir = nd;
  tfmm_status s = dev_alloc(c, (void**)&b->d_pat, (size_t)nd * N * sizeof(float4));
  if (s == TFMM_OK) s = dev_alloc(c, (void**)&b->d_start, (size_t)(nbox + 1) * sizeof(int));
  if (s == TFMM_OK) s = dev_alloc(c, (void**)&b->d_orig, (size_t)N * sizeof(int));
  if (s == TFMM_OK) s = dev_alloc(c, (void**)&b->d_boxof, (size_t)N * sizeof(int));
  if (s == TFMM_OK) s = dev_alloc(c, (void**)&b->d_w, (size_t)nd * sizeof(float));
  if (s != TFMM_OK) {
    free_basis(c, b);
    return s;
  }
  b->bytes = (size_t)nd * N * sizeof(float4) + (size_t)(nbox + 1 + 2 * N) * sizeof(int) + nd * sizeof(float);
  double *d_khat = nullptr, *d_geo = nullptr;
  hipError_t e = hipMalloc(&d_khat, op->khat.size() * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&d_geo, geo.size() * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(d_khat, op->khat.data(), op->khat.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_geo, geo.data(), geo.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_start, start.data(), start.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_orig, order.data(), N * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_boxof, boxof.data(), N * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_w, wf.data(), nd * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = tfmm::launch_dipole_patterns(b->d_pat, d_khat, d_geo, N, nd, op->k_re, op->k_im, 0);
  if (e == hipSuccess) e = hipStreamSynchronize(0);
  if (d_khat) (void)hipFree(d_khat);
  if (d_geo) (void)hipFree(d_geo);
  if (e != hipSuccess) {
    free_basis(c, b);
    return fail(TFMM_ERR_HIP, std::string("basis patterns: ") + hipGetErrorString(e));
  }
  op->refs.fetch_add(1);
  c->bases.push_back(b);
  *out = b;
  return TFMM_OK;
}

tfmm_status tfmm_basis_release(tfmm_ctx c, tfmm_basis b) {
  if (!c || !b) return fail(TFMM_ERR_INVALID_ARG, "ctx or basis is NULL");
  std::lock_guard<std::recursive_mutex> g(c->mu);
  auto it = std::find(c->bases.begin(), c->bases.end(), b);
  if (it == c->bases.end()) return fail(TFMM_ERR_INVALID_ARG, "basis does not belong to this context");
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  c->bases.erase(it);
  b->op->refs.fetch_sub(1);
  free_basis(c, b);
  return TFMM_OK;
}

static tfmm_status check_basis(tfmm_ctx c, tfmm_basis b, const void* x, const void* y, int32_t nrhs) {
  if (!c || !b) return fail(TFMM_ERR_INVALID_ARG, "ctx or basis is NULL");
  if (b->ctx != c) return fail(TFMM_ERR_INVALID_ARG, "basis belongs to another context");
  if (!x || !y) return fail(TFMM_ERR_INVALID_ARG, "input or output is NULL");
  if (nrhs < 1 || nrhs > 4096) return fail(TFMM_ERR_INVALID_ARG, "nrhs out of range");
  return TFMM_OK;
}

tfmm_status tfmm_aggregate(tfmm_ctx c, tfmm_basis b, const void* I, void* A, int32_t nrhs, void* stream) {
  tfmm_status s = check_basis(c, b, I, A, nrhs);
  if (s != TFMM_OK) return s;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  HIP_TRY(hipSetDevice(c->device));
  Launch L(c, (hipStream_t)stream, "aggregate");
  HIP_TRY(tfmm::launch_aggregate(b->d_pat, b->d_start, b->d_orig, (const float2*)I, (float2*)A, b->N, b->nbox, b->ndir,
                                 nrhs, (hipStream_t)stream));
  L.done();
  return TFMM_OK;
}

tfmm_status tfmm_disaggregate(tfmm_ctx c, tfmm_basis b, const void* B, void* y, int32_t nrhs, void* stream) {
  tfmm_status s = check_basis(c, b, B, y, nrhs);
  if (s != TFMM_OK) return s;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  HIP_TRY(hipSetDevice(c->device));
  Launch L(c, (hipStream_t)stream, "disaggregate");
  HIP_TRY(tfmm::launch_disaggregate(b->d_pat, b->d_boxof, b->d_orig, b->d_w, (const float2*)B, (float2*)y, b->N,
                                    b->nbox, b->ndir, nrhs, (hipStream_t)stream));
  L.done();
  return TFMM_OK;
}

tfmm_status tfmm_farfield_matvec(tfmm_ctx c, tfmm_op op, tfmm_basis b, const void* I, void* y, int32_t nrhs,
                                 void* stream) {
  tfmm_status s = check_basis(c, b, I, y, nrhs);
  if (s != TFMM_OK) return s;
  if (!op || op != b->op) return fail(TFMM_ERR_INVALID_ARG, "op must be the operator the basis was set up with");
  if (2 * nrhs > 4096) return fail(TFMM_ERR_INVALID_ARG, "nrhs out of range");
  std::lock_guard<std::recursive_mutex> g(c->mu);
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  // A and B of the translation: 2 nrhs fields (theta, phi) per direction and box
  const size_t half = (size_t)2 * nrhs * op->ndir * b->nbox * sizeof(float2);
  const size_t need = (2 * half + 255) / 256 * 256;
  if (c->mv_bytes < need) {
    if (c->mv_buf) {
      (void)hipDeviceSynchronize();
      dev_free(c, c->mv_buf, c->mv_bytes);
      c->mv_buf = nullptr;
      c->mv_bytes = 0;
    }
    s = dev_alloc(c, &c->mv_buf, need);
    if (s != TFMM_OK) return s;
    c->mv_bytes = need;
  }
  float2* A = (float2*)c->mv_buf;
  float2* B = (float2*)((char*)c->mv_buf + half);
  {
    Launch L(c, st, "aggregate");
    HIP_TRY(tfmm::launch_aggregate(b->d_pat, b->d_start, b->d_orig, (const float2*)I, A, b->N, b->nbox, b->ndir,
                                   nrhs, st));
    L.done();
  }
  s = tfmm_translate(c, op, A, B, 2 * nrhs, stream);
  if (s != TFMM_OK) return s;
  Launch L(c, st, "disaggregate");
  HIP_TRY(tfmm::launch_disaggregate(b->d_pat, b->d_boxof, b->d_orig, b->d_w, B, (float2*)y, b->N, b->nbox, b->ndir,
                                    nrhs, st));
  L.done();
  return TFMM_OK;
}

// ---------------------------------------------------------------------------
// Near-field matrix (caller-supplied CSR) and the TFQMR solve (solver.cpp)
// ---------------------------------------------------------------------------

static void free_near(tfmm_ctx c, tfmm_near m) {
  dev_free(c, m->d_rp, (size_t)(m->n + 1) * sizeof(int));
  dev_free(c, m->d_ci, (size_t)m->nnz * sizeof(int));
  dev_free(c, m->d_val, (size_t)m->nnz * sizeof(float2));
  delete m;
}

tfmm_status tfmm_near_setup(tfmm_ctx c, int32_t n, const int32_t* row_ptr, const int32_t* cols, const double* vals,
                            tfmm_near* out) {
  if (!c || !out || !row_ptr) return fail(TFMM_ERR_INVALID_ARG, "ctx, out or row_ptr is NULL");
  if (n < 1) return fail(TFMM_ERR_INVALID_ARG, "n must be >= 1");
  if (row_ptr[0] != 0) return fail(TFMM_ERR_INVALID_ARG, "row_ptr[0] must be 0");
  for (int i = 0; i < n; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return fail(TFMM_ERR_INVALID_ARG, "row_ptr must be non-decreasing");
  const long long nnz = row_ptr[n];
  if (nnz > 0 && (!cols || !vals)) return fail(TFMM_ERR_INVALID_ARG, "cols or vals is NULL");
  for (long long j = 0; j < nnz; ++j)
    if (cols[j] < 0 || cols[j] >= n) return fail(TFMM_ERR_INVALID_ARG, "column index out of range");
  std::vector<float2> v((size_t)nnz);
  for (long long j = 0; j < nnz; ++j) v[j] = make_float2((float)vals[2 * j], (float)vals[2 * j + 1]);
  std::lock_guard<std::recursive_mutex> g(c->mu);
  HIP_TRY(hipSetDevice(c->device));
  tfmm_near m = new tfmm_near_s();
  m->ctx = c;
  m->n = n;
  m->nnz = std::max(1LL, nnz);
  tfmm_status s = dev_alloc(c, (void**)&m->d_rp, (size_t)(n + 1) * sizeof(int));
  if (s == TFMM_OK) s = dev_alloc(c, (void**)&m->d_ci, (size_t)std::max(1LL, nnz) * sizeof(int));
  if (s == TFMM_OK) s = dev_alloc(c, (void**)&m->d_val, (size_t)std::max(1LL, nnz) * sizeof(float2));
  if (s != TFMM_OK) {
    free_near(c, m);
    return s;
  }
  hipError_t e = hipMemcpy(m->d_rp, row_ptr, (size_t)(n + 1) * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess && nnz > 0) e = hipMemcpy(m->d_ci, cols, (size_t)nnz * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess && nnz > 0) e = hipMemcpy(m->d_val, v.data(), (size_t)nnz * sizeof(float2), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_near(c, m);
    return fail(TFMM_ERR_HIP, std::string("near-field upload: ") + hipGetErrorString(e));
  }
  c->nears.push_back(m);
  *out = m;
  return TFMM_OK;
}

tfmm_status tfmm_near_release(tfmm_ctx c, tfmm_near m) {
  if (!c || !m) return fail(TFMM_ERR_INVALID_ARG, "ctx or near is NULL");
  std::lock_guard<std::recursive_mutex> g(c->mu);
  auto it = std::find(c->nears.begin(), c->nears.end(), m);
  if (it == c->nears.end()) return fail(TFMM_ERR_INVALID_ARG, "near-field matrix does not belong to this context");
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  c->nears.erase(it);
  free_near(c, m);
  return TFMM_OK;
}

tfmm_status tfmm_near_matvec(tfmm_ctx c, tfmm_near m, const void* x, void* y, int32_t nrhs, void* stream) {
  if (!c || !m || !x || !y) return fail(TFMM_ERR_INVALID_ARG, "ctx, near, x or y is NULL");
  if (m->ctx != c) return fail(TFMM_ERR_INVALID_ARG, "near-field matrix belongs to another context");
  if (nrhs < 1) return fail(TFMM_ERR_INVALID_ARG, "nrhs must be >= 1");
  std::lock_guard<std::recursive_mutex> g(c->mu);
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(tfmm::launch_near_spmv(m->d_rp, m->d_ci, m->d_val, (const float2*)x, (float2*)y, m->n, nrhs,
                                 (hipStream_t)stream));
  return TFMM_OK;
}

tfmm_status tfmm_submit(tfmm_ctx c, tfmm_op op, const void* A, void* B, int32_t nrhs, tfmm_ticket* out) {
  tfmm_status s = check_translate(c, op, A, B, nrhs);
  if (s != TFMM_OK) return s;
  if (!out) return fail(TFMM_ERR_INVALID_ARG, "out is NULL");
  auto j = std::make_shared<Job>();
  j->id = c->next_ticket.fetch_add(1);
  j->op = op;
  j->A = (const float2*)A;
  j->B = (float2*)B;
  j->nrhs = nrhs;
  j->t_submit = now_s();
  op->refs.fetch_add(1);
  {
    std::lock_guard<std::mutex> lk(c->qmu);
    if (c->queue.size() >= 65536) {
      op->refs.fetch_sub(1);
      return fail(TFMM_ERR_QUEUE_FULL, "scheduler queue full");
    }
    c->jobs[j->id] = j;
    c->queue.push_back(j);
  }
  c->qcv.notify_all();
  *out = j->id;
  return TFMM_OK;
}

tfmm_status tfmm_poll(tfmm_ctx c, tfmm_ticket t, int32_t* done, tfmm_status* job_status, double* latency_us) {
  if (!c || !done) return fail(TFMM_ERR_INVALID_ARG, "ctx or done is NULL");
  std::lock_guard<std::mutex> lk(c->qmu);
  auto it = c->jobs.find(t);
  if (it == c->jobs.end()) return fail(TFMM_ERR_UNKNOWN_TICKET, "unknown ticket");
  const auto& j = it->second;
  *done = j->done.load();
  if (*done) {
    if (job_status) *job_status = j->status;
    if (latency_us) *latency_us = (j->t_done - j->t_submit) * 1e6;
    c->jobs.erase(it);
  }
  return TFMM_OK;
}

tfmm_status tfmm_wait(tfmm_ctx c, tfmm_ticket t, tfmm_status* job_status, double* latency_us) {
  if (!c) return fail(TFMM_ERR_INVALID_ARG, "ctx is NULL");
  std::shared_ptr<Job> j;
  {
    std::lock_guard<std::mutex> lk(c->qmu);
    auto it = c->jobs.find(t);
    if (it == c->jobs.end()) return fail(TFMM_ERR_UNKNOWN_TICKET, "unknown ticket");
    j = it->second;
  }
  {
    std::unique_lock<std::mutex> lk(c->qmu);
    c->fcv.wait(lk, [&] { return j->done.load() != 0; });
    c->jobs.erase(t);
  }
  if (job_status) *job_status = j->status;
  if (latency_us) *latency_us = (j->t_done - j->t_submit) * 1e6;
  return TFMM_OK;
}

tfmm_status tfmm_sched_stats(tfmm_ctx c, uint64_t* out, size_t cap) {
  if (!c || !out) return fail(TFMM_ERR_INVALID_ARG, "ctx or out is NULL");
  std::lock_guard<std::mutex> lk(c->qmu);
  const uint64_t v[5] = {c->n_launch, c->n_parked, c->n_done, c->n_failed, (uint64_t)c->queue.size()};
  for (size_t i = 0; i < cap && i < 5; ++i) out[i] = v[i];
  return TFMM_OK;
}

tfmm_status tfmm_set_profiling(tfmm_ctx c, int32_t on) {
  if (!c) return fail(TFMM_ERR_INVALID_ARG, "ctx is NULL");
  std::lock_guard<std::recursive_mutex> g(c->mu);
  c->prof = on != 0;
  return TFMM_OK;
}

tfmm_status tfmm_kernel_times(tfmm_ctx c, char* names, size_t names_cap, double* avg_ms, int32_t* launches,
                              int32_t cap, int32_t* count) {
  if (!c) return fail(TFMM_ERR_INVALID_ARG, "ctx is NULL");
  std::lock_guard<std::recursive_mutex> g(c->mu);
  for (auto& p : c->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->stats[p.name].total_ms += ms;
      c->stats[p.name].n += 1;
    }
    c->event_pool.push_back(p.a);
    c->event_pool.push_back(p.b);
  }
  c->pending.clear();
  int i = 0;
  const int lim = cap < 0 ? -cap : cap;
  std::string joined;
  for (auto& kv : c->stats) {
    if (i < lim) {
      if (avg_ms) avg_ms[i] = kv.second.n ? kv.second.total_ms / kv.second.n : 0.0;
      if (launches) launches[i] = kv.second.n;
    }
    joined += kv.first;
    joined += '\n';
    ++i;
  }
  if (count) *count = i;
  if (names && names_cap) {
    size_t n = std::min(names_cap - 1, joined.size());
    std::memcpy(names, joined.data(), n);
    names[n] = 0;
  }
  // a reset happens when the caller passes cap < 0
  if (cap < 0) c->stats.clear();
  return TFMM_OK;
}

}  // extern "C"

tfmm_status tfmm_op_plan(tfmm_op op, int32_t* out, size_t cap) {
  if (!op || !out) return fail(TFMM_ERR_INVALID_ARG, "op or out is NULL");
  const int32_t v[5] = {op->fused ? 1 : 0, op->cb, (op->fused ? op->ftk2 : op->tk2) ? 1 : 0, op->tuned ? 1 : 0,
                        op->use_w1 && !op->fused ? 1 : 0};
  for (size_t i = 0; i < cap && i < 5; ++i) out[i] = v[i];
  return TFMM_OK;
}

tfmm_status tfmm_autotune(tfmm_ctx c, tfmm_op op, int32_t nrhs, int32_t reps, int32_t* choice_out, double* best_ms) {
  if (!c || !op) return fail(TFMM_ERR_INVALID_ARG, "ctx or op is NULL");
  if (op->ctx != c) return fail(TFMM_ERR_INVALID_ARG, "operator belongs to another context");
  if (nrhs < 1 || nrhs > 4096) return fail(TFMM_ERR_INVALID_ARG, "nrhs out of range");
  if (reps < 1 || reps > 200) return fail(TFMM_ERR_INVALID_ARG, "reps must be in 1..200");
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (op->refs.load() > 0) return fail(TFMM_ERR_BUSY, "operator has queued jobs");
  HIP_TRY(hipSetDevice(c->device));
  // the operator's GEMMs (a1 and the formed products) measure their tile
  // configurations the first time they run in here
  struct GemmTuning {
    GemmTuning() { tfmm::set_gemm_tuning(true); }
    ~GemmTuning() { tfmm::set_gemm_tuning(false); }
  } gemm_tuning;
  const size_t bytes = (size_t)nrhs * op->ndir * op->K[0] * op->K[1] * op->K[2] * sizeof(float2);
  void *A = nullptr, *B = nullptr;
  tfmm_status s = dev_alloc(c, &A, bytes);
  if (s != TFMM_OK) return s;
  s = dev_alloc(c, &B, bytes);
  if (s != TFMM_OK) {
    dev_free(c, A, bytes);
    return s;
  }
  HIP_TRY(hipMemset(A, 0x3c, bytes));  // any finite pattern: the kernels' cost does not depend on values
  // candidates
  const int n1 = op->n[0], n2 = op->n[1], n3 = op->n[2], nq = n1 * n2;
  const bool tucker = op->zfmt != tfmm::ZF_FULL;  // register-chained or LDS-staged restoration
  const bool fusable = !c->no_fused && n1 == n2 && n2 == n3 && (n1 == 8 || n1 == 16 || n1 == 24 || n1 == 32);
  std::vector<TuneChoice> cand;
  for (int tk : tucker ? std::vector<int>{1, 0} : std::vector<int>{-1}) {
    if (fusable) cand.push_back({1, 0, tk});
    for (int cb = 1; cb <= 4; ++cb)
      if (cb_valid(cb, n2, nq, n3)) cand.push_back({0, cb, tk});
  }
  const bool prof = c->prof;
  c->prof = false;
  const TuneChoice start = op->choice;
  hipStream_t st = c->cap_stream;
  std::vector<hipEvent_t> ev(2 * reps);
  for (auto& e : ev) (void)hipEventCreate(&e);
  double best = 1e300;
  TuneChoice pick = start;
  for (const TuneChoice& ch : cand) {
    if (apply_choice(op, ch) != TFMM_OK) continue;
    bool ok = true;
    for (int w = 0; w < 2 && ok; ++w) ok = translate_contiguous(c, op, A, B, nrhs, st, 0) == TFMM_OK;
    for (int r = 0; r < reps && ok; ++r) {
      ok = hipEventRecord(ev[2 * r], st) == hipSuccess;
      ok = ok && translate_contiguous(c, op, A, B, nrhs, st, 0) == TFMM_OK;
      ok = ok && hipEventRecord(ev[2 * r + 1], st) == hipSuccess;
    }
    if (ok) mark_slot(c, 0, st);
    if (!ok || hipStreamSynchronize(st) != hipSuccess) {
      (void)hipGetLastError();
      continue;
    }
    std::vector<float> t(reps);
    for (int r = 0; r < reps; ++r) (void)hipEventElapsedTime(&t[r], ev[2 * r], ev[2 * r + 1]);
    std::nth_element(t.begin(), t.begin() + reps / 2, t.end());
    if (t[reps / 2] < best) {
      best = t[reps / 2];
      pick = ch;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  c->prof = prof;
  dev_free(c, A, bytes);
  dev_free(c, B, bytes);
  if (best >= 1e300) {
    (void)apply_choice(op, start);
    return fail(TFMM_ERR_INTERNAL, "no tile configuration ran");
  }
  s = apply_choice(op, pick);
  if (s != TFMM_OK) return s;
  op->tuned = true;
  const std::string key = tune_key(op, nrhs);
  c->tune[key] = pick;
  if (!c->tune_path.empty()) {
    if (FILE* f = std::fopen(c->tune_path.c_str(), "a")) {
      std::fprintf(f, "%s fused=%d cb=%d tk2=%d ms=%.6f\n", key.c_str(), pick.fused, pick.cb, pick.tk2, best);
      std::fclose(f);
    }
  }
  if (choice_out) {
    choice_out[0] = op->fused ? 1 : 0;
    choice_out[1] = op->cb;
    choice_out[2] = (op->fused ? op->ftk2 : op->tk2) ? 1 : 0;
  }
  if (best_ms) *best_ms = best;
  return TFMM_OK;
}
