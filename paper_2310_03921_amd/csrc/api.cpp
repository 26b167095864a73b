// C ABI of libgap: argument checks, workspace, and the order of kernel launches
// for each verb.  Every numerical step runs in the gfx950 kernels; this file
// only validates, lays out device workspace and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/gap.h"
#include "launch.h"

// Device scratch of the allocation-free entry point gap_forces_noalloc: one
// copy per GPU, held until the process ends.  Host code never passes this
// name to a kernel (on the host it is only a stand-in for the symbol); it
// looks up each device's address once, in gap_create, and uses that.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

struct gap_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  // Side stream (default priority) for work that overlaps the caller's stream
  // inside one call, forked and joined with the two events.
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::string err;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int* dev_err = nullptr;     // device status word
  double* dev_small = nullptr; // 64 doubles of small device scratch
  gapk::Timer timer;
  double tm_ms[gapk::TM_COUNT] = {};
  int64_t tm_n[gapk::TM_COUNT] = {};
  void* noalloc_scratch = nullptr;  // this device's address of `scratch`
  size_t ws_limit = 0;               // cap on optional workspace (0: none)
  bool fit_final_resid = true;       // gap_fit: residual after the last refinement step
};

namespace {

gap_status fail(gap_handle* h, gap_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (h) h->err = buf;
  return s;
}

#define HIP_TRY(h, expr)                                                              \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail((h), GAP_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

bool aligned32(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 31u) == 0; }

// Bump layout of the handle's device workspace (256-byte aligned slices).
struct Layout {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  }
};

gap_status ensure_ws(gap_handle* h, size_t bytes) {
  if (bytes <= h->ws_bytes) return GAP_OK;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  if (h->ws) HIP_TRY(h, hipFree(h->ws));
  h->ws = nullptr;
  h->ws_bytes = 0;
  const size_t want = bytes + bytes / 8;
  if (hipMalloc(&h->ws, want) != hipSuccess) {
    h->ws = nullptr;
    return fail(h, GAP_E_NOMEM, "workspace allocation of %zu bytes failed", want);
  }
  h->ws_bytes = want;
  return GAP_OK;
}

template <typename T>
T* at(gap_handle* h, size_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(h->ws) + off);
}

gap_status set_device(gap_handle* h) {
  HIP_TRY(h, hipSetDevice(h->device));
  return GAP_OK;
}

gap_status check_sparse(gap_handle* h, const gap_sparse* sp) {
  if (!sp) return fail(h, GAP_E_INVALID, "sparse points are NULL");
  if (sp->M < 1 || sp->D < 1) return fail(h, GAP_E_INVALID, "M and D must be >= 1");
  if (!sp->X) return fail(h, GAP_E_INVALID, "X is NULL");
  if (sp->ld_x < sp->D || sp->ld_x % 4 != 0)
    return fail(h, GAP_E_INVALID, "ld_x must be >= D and a multiple of 4");
  if (!aligned32(sp->X)) return fail(h, GAP_E_INVALID, "X must be 32-byte aligned");
  if (sp->zeta < 1 || sp->zeta > 64)
    return fail(h, GAP_E_UNSUPPORTED, "zeta must be an integer in [1, 64]");
  if (!std::isfinite(sp->delta)) return fail(h, GAP_E_INVALID, "delta must be finite");
  return GAP_OK;
}

gap_status check_atoms(gap_handle* h, const gap_atoms* a, const gap_sparse* sp, bool need_jac) {
  if (!a) return fail(h, GAP_E_INVALID, "atoms are NULL");
  if (a->n_cfg < 0 || a->n_atoms < 0 || a->n_pairs < 0)
    return fail(h, GAP_E_INVALID, "negative sizes");
  if (a->n_pairs > INT32_MAX || a->n_atoms > INT32_MAX)
    return fail(h, GAP_E_INVALID, "n_atoms and n_pairs must fit in int32");
  if (sp && a->D != sp->D) return fail(h, GAP_E_INVALID, "atoms.D != sparse.D");
  if (a->n_atoms > 0) {
    if (!a->desc) return fail(h, GAP_E_INVALID, "desc is NULL");
    if (a->desc_dt != GAP_DT_F32 && a->desc_dt != GAP_DT_F64)
      return fail(h, GAP_E_INVALID, "bad desc dtype");
    if (a->ld_desc < a->D || a->ld_desc % 4 != 0)
      return fail(h, GAP_E_INVALID, "ld_desc must be >= D and a multiple of 4");
    if (!aligned32(a->desc)) return fail(h, GAP_E_INVALID, "desc must be 32-byte aligned");
  }
  if (!a->cfg_ptr && a->n_cfg > 0) return fail(h, GAP_E_INVALID, "cfg_ptr is NULL");
  if (need_jac) {
    if (!a->pair_ptr || (a->n_pairs > 0 && !a->pair_j))
      return fail(h, GAP_E_INVALID, "pair_ptr / pair_j are NULL");
    if (a->n_pairs > 0) {
      if (!a->jac) return fail(h, GAP_E_INVALID, "jac is NULL");
      if (a->jac_dt != GAP_DT_F32 && a->jac_dt != GAP_DT_F64)
        return fail(h, GAP_E_INVALID, "bad jac dtype");
      if (a->ld_jac < a->D || a->ld_jac % 4 != 0)
        return fail(h, GAP_E_INVALID, "ld_jac must be >= D and a multiple of 4");
      if (!aligned32(a->jac)) return fail(h, GAP_E_INVALID, "jac must be 32-byte aligned");
    }
  }
  return GAP_OK;
}

gap_status drain_dev_err(gap_handle* h) {
  int v = 0;
  HIP_TRY(h, hipMemcpyAsync(&v, h->dev_err, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  if (v != 0) {
    int zero = 0;
    HIP_TRY(h, hipMemcpy(h->dev_err, &zero, sizeof(int), hipMemcpyHostToDevice));
  }
  if (v & GAP_DEVERR_NOT_PD)
    return fail(h, GAP_E_NOT_PD, "K_MM + jitter I is not positive definite (Cholesky pivot <= 0)");
  if (v & GAP_DEVERR_RANK)
    return fail(h, GAP_E_RANK, "least-squares matrix is rank deficient (zero pivot in R)");
  if (v & GAP_DEVERR_INDEX)
    return fail(h, GAP_E_INVALID, "index data out of range (pair target, pair_ptr or local-property atom index)");
  if (v & GAP_DEVERR_SYNC)
    return fail(h, GAP_E_HIP, "a grid barrier of the cooperative QR panel kernel timed out");
  return GAP_OK;
}

// Workspace slices of the pair transposition.
struct PairWs {
  size_t tgt_ptr, tgt_pair, src, order, scratch;
};
void layout_pairs(Layout& L, int64_t n_atoms, int64_t n_pairs, PairWs& p) {
  p.tgt_ptr = L.take(sizeof(int64_t) * (n_atoms + 1));
  p.tgt_pair = L.take(sizeof(int32_t) * std::max<int64_t>(n_pairs, 1));
  p.src = L.take(sizeof(int32_t) * std::max<int64_t>(n_pairs, 1));
  p.order = L.take(sizeof(int32_t) * std::max<int64_t>(n_atoms, 1));
  p.scratch = L.take(sizeof(int32_t) * (n_atoms + 2048));
}

void run_pairs(gap_handle* h, const gap_atoms* a, const PairWs& p, bool want_order,
               hipStream_t st = nullptr) {
  if (!st) st = h->stream;
  const hipStream_t timer_st = h->timer.st;
  h->timer.st = st;  // the stage is timed on the stream it runs on
  h->timer.begin(gapk::TM_PAIRS);
  gapk::pair_transpose(a->pair_ptr, a->pair_j, a->n_atoms, a->n_pairs, at<int64_t>(h, p.tgt_ptr),
                       at<int32_t>(h, p.tgt_pair), at<int32_t>(h, p.src),
                       want_order ? at<int32_t>(h, p.order) : nullptr, at<int32_t>(h, p.scratch),
                       h->dev_err, st);
  h->timer.end(gapk::TM_PAIRS);
  h->timer.st = timer_st;
}

bool f32(gap_dtype d) { return d == GAP_DT_F32; }

// Row strides of internal FP64 row-major buffers: a multiple of 4 doubles so
// that every row starts 32-byte aligned (vector loads).
int64_t ld4(int64_t n) { return (n + 3) & ~int64_t(3); }
int64_t ld8(int64_t n) { return (n + 7) & ~int64_t(7); }

// Split halves of X for the BF16x3 form.
struct SplitWs {
  size_t xh = 0, xl = 0, xth = 0, xtl = 0;
};
void layout_split(Layout& L, int64_t M, int64_t D, bool transposed, SplitWs& w) {
  const int64_t n = M * gapk::split_ld(D);
  w.xh = L.take(2 * n);
  w.xl = L.take(2 * n);
  if (transposed) {
    const int64_t nt = D * gapk::split_ld(M);
    w.xth = L.take(2 * nt);
    w.xtl = L.take(2 * nt);
  }
}
void run_split(gap_handle* h, const gap_sparse* sp, const SplitWs& w, bool transposed) {
  h->timer.begin(gapk::TM_SPLIT);
  gapk::split_x_bf16(sp->X, sp->ld_x, sp->M, sp->D, at<__bf16>(h, w.xh), at<__bf16>(h, w.xl),
                     transposed ? at<__bf16>(h, w.xth) : nullptr,
                     transposed ? at<__bf16>(h, w.xtl) : nullptr, h->stream);
  h->timer.end(gapk::TM_SPLIT);
}

// Predict internals shared by gap_predict and the refinement residual.
struct PredictWs {
  size_t W, e_atom, g, f_pair;
  size_t epart = 0;  // per-column-group energy partials of the P-stage
  PairWs pairs;
  SplitWs split;
};
void layout_predict(Layout& L, const gap_atoms* a, const gap_sparse* sp, bool need_g,
                    bool need_eatom, bool need_gbuf, bool need_forces, PredictWs& w,
                    bool bf16 = false) {
  const int64_t N = a->n_atoms, M = sp->M, D = sp->D;
  if (bf16) layout_split(L, M, D, true, w.split);
  // the BF16X3 P-stage writes an FP32 W, always (its epilogue forms W with the energies)
  w.W = (need_g || bf16) ? L.take((bf16 ? sizeof(float) : sizeof(double)) *
                                  std::max<int64_t>(N * ld4(M), 1))
                         : 0;
  w.e_atom = need_eatom ? L.take(sizeof(double) * std::max<int64_t>(N, 1)) : 0;
  w.epart = L.take(sizeof(double) *
                   std::max<int64_t>(N * std::max(gapk::pstage_groups(M),
                                                  gapk::gemm_b3_col_blocks(M)), 1));
  w.g = need_gbuf ? L.take(sizeof(double) * std::max<int64_t>(N * ld4(D), 1)) : 0;
  w.f_pair = need_forces ? L.take(sizeof(double) * std::max<int64_t>(3 * a->n_pairs, 1)) : 0;
  if (need_forces) layout_pairs(L, N, a->n_pairs, w.pairs);
}

void run_predict(gap_handle* h, const gap_atoms* a, const gap_sparse* sp, const double* c,
                 const PredictWs& w, double* e_atom, double* e_cfg, double* dEdd,
                 double* forces, bool bf16 = false, const int32_t* species = nullptr,
                 int32_t zsel = 0) {
  const int64_t N = a->n_atoms, M = sp->M, D = sp->D;
  const bool need_g = dEdd || forces;
  double* ea = e_atom ? e_atom : (e_cfg ? at<double>(h, w.e_atom) : nullptr);
  double* W = (need_g && !bf16) ? at<double>(h, w.W) : nullptr;
  float* W32 = bf16 ? at<float>(h, w.W) : nullptr;
  const int64_t ldw = ld4(M);
  auto wx = [&](double* out, int64_t ldo) {
    if (bf16)
      gapk::gemm_b3_wx(W32, ldw, N, M, at<__bf16>(h, w.split.xth), at<__bf16>(h, w.split.xtl), D,
                       out, ldo, h->stream);
    else
      gapk::gemm_wx_f64(W, ldw, N, M, sp->X, sp->ld_x, D, out, ldo, h->stream);
  };
  if (bf16) {
    run_split(h, sp, w.split, need_g);
    gapk::pstage_b3t(0, a->desc, f32(a->desc_dt), a->ld_desc, N, at<__bf16>(h, w.split.xh),
                     at<__bf16>(h, w.split.xl), M, D, sp->zeta, sp->delta, c, nullptr, W32, ldw,
                     at<double>(h, w.epart), nullptr, h->stream);
    if (ea)
      gapk::sum_parts_f64(at<double>(h, w.epart), gapk::gemm_b3_col_blocks(M), N, ea, 1, N, N,
                          h->stream);
  } else {
    gapk::pstage_f64(0, a->desc, f32(a->desc_dt), a->ld_desc, N, sp->X, sp->ld_x, M, D, sp->zeta,
                     sp->delta, c, nullptr, nullptr, 0, W, ldw, ea, nullptr, h->stream, nullptr, 0,
                     at<double>(h, w.epart));
  }
  if (species) gapk::mask_species_rows(species, zsel, N, ea, W, ldw, h->stream, W32);
  if (e_cfg) gapk::segment_sum_f64(ea, a->cfg_ptr, a->n_cfg, N, e_cfg, h->stream);
  if (forces) {
    double* g = at<double>(h, w.g);
    const int64_t ldg = ld4(D);
    wx(g, ldg);
    if (dEdd) gapk::copy_rows_f64(g, ldg, dEdd, D, N, D, h->stream);
    run_pairs(h, a, w.pairs, false);
    gapk::forces_f64(a->jac, f32(a->jac_dt), a->ld_jac, D, g, ldg, at<int32_t>(h, w.pairs.src), N,
                     a->n_pairs, at<int64_t>(h, w.pairs.tgt_ptr),
                     at<int32_t>(h, w.pairs.tgt_pair), at<double>(h, w.f_pair), forces,
                     h->stream);
  } else if (dEdd) {
    wx(dEdd, D);
  }
}

gap_status check_gfx950(gap_handle* h) {
  hipDeviceProp_t prop;
  HIP_TRY(h, hipGetDeviceProperties(&prop, h->device));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(h, GAP_E_HIP, "device %d is %s, this library is built for gfx950", h->device,
                prop.gcnArchName);
  return GAP_OK;
}

}  // namespace

extern "C" {

gap_status gap_create(gap_handle** out, int device, void* hip_stream) {
  if (!out) return GAP_E_INVALID;
  *out = nullptr;
  gap_handle* h = new gap_handle();
  h->device = device;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  h->timer.st = h->stream;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    delete h;
    return GAP_E_HIP;
  }
  if (hipSetDevice(device) != hipSuccess || check_gfx950(h) != GAP_OK) {
    delete h;
    return GAP_E_HIP;
  }
  {
    // this device's copy of the allocation-free scratch, looked up once
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device >= kMaxDevices) {
      delete h;
      return GAP_E_HIP;
    }
    if (!g_scratch_ptr[device]) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        delete h;
        return GAP_E_HIP;
      }
      g_scratch_ptr[device] = p;
    }
    h->noalloc_scratch = g_scratch_ptr[device];
  }
  if (hipMalloc(&h->dev_err, 256) != hipSuccess) {
    delete h;
    return GAP_E_NOMEM;
  }
  if (hipMalloc(&h->dev_small, 64 * sizeof(double)) != hipSuccess) {
    (void)hipFree(h->dev_err);
    delete h;
    return GAP_E_NOMEM;
  }
  int zero = 0;
  if (hipMemcpy(h->dev_err, &zero, sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) != hipSuccess) {
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->side) (void)hipStreamDestroy(h->side);
    (void)hipFree(h->dev_err);
    (void)hipFree(h->dev_small);
    delete h;
    return GAP_E_HIP;
  }
  *out = h;
  return GAP_OK;
}

gap_status gap_destroy(gap_handle* h) {
  if (!h) return GAP_OK;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  double ms[gapk::TM_COUNT];
  int64_t n[gapk::TM_COUNT];
  h->timer.collect(ms, n);
  if (h->side) (void)hipStreamSynchronize(h->side);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  if (h->side) (void)hipStreamDestroy(h->side);
  if (h->ws) (void)hipFree(h->ws);
  if (h->dev_err) (void)hipFree(h->dev_err);
  if (h->dev_small) (void)hipFree(h->dev_small);
  delete h;
  return GAP_OK;
}

const char* gap_last_error(const gap_handle* h) { return h ? h->err.c_str() : "null handle"; }

gap_status gap_sync(gap_handle* h) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  return drain_dev_err(h);
}

static const char* kTimerNames[gapk::TM_COUNT] = {
    "pair_transpose", "kmm", "energy_rows", "force_rows", "cholesky_stack", "qr_panel",
    "qr_update", "back_substitution", "predict", "predict_backward", "refinement", "split_bf16"};

gap_status gap_set_workspace_limit(gap_handle* h, size_t bytes) {
  if (!h) return GAP_E_INVALID;
  h->ws_limit = bytes;
  return GAP_OK;
}

gap_status gap_set_fit_report(gap_handle* h, int final_residual) {
  if (!h) return GAP_E_INVALID;
  h->fit_final_resid = final_residual != 0;
  return GAP_OK;
}

gap_status gap_timing(gap_handle* h, int enable) {
  if (!h) return GAP_E_INVALID;
  h->timer.on = enable != 0;
  return GAP_OK;
}

gap_status gap_timing_read(gap_handle* h, double* ms, int64_t* count, int reset) {
  if (!h || !ms || !count) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  h->timer.collect(h->tm_ms, h->tm_n);
  for (int i = 0; i < gapk::TM_COUNT; ++i) {
    ms[i] = h->tm_ms[i];
    count[i] = h->tm_n[i];
    if (reset) {
      h->tm_ms[i] = 0.0;
      h->tm_n[i] = 0;
    }
  }
  return GAP_OK;
}

const char* gap_timing_name(int i) { return (i >= 0 && i < gapk::TM_COUNT) ? kTimerNames[i] : ""; }

int gap_timing_count(void) { return gapk::TM_COUNT; }

gap_status gap_workspace_query(gap_handle* h, const gap_atoms* a, const gap_sparse* sp,
                               size_t* bytes) {
  if (!h || !bytes) return GAP_E_INVALID;
  gap_status s = check_sparse(h, sp);
  if (s != GAP_OK) return s;
  s = check_atoms(h, a, sp, false);
  if (s != GAP_OK) return s;
  const int64_t N = a->n_atoms, M = sp->M, D = sp->D;
  const int64_t n_rows = a->n_cfg + 3 * N;
  Layout L;
  PairWs p;
  layout_pairs(L, N, a->n_pairs, p);
  L.take(sizeof(double) * N * M);  // S
  size_t knm = L.off;
  Layout F;
  F.take(sizeof(double) * M * M);
  F.take(gapk::qr_workspace_bytes(n_rows + M, M));
  PredictWs pw;
  layout_predict(F, a, sp, true, true, true, true, pw);
  F.take(sizeof(double) * (3 * n_rows + 4 * M + 2 * N + N * D));
  *bytes = std::max(knm, F.off);
  return GAP_OK;
}

gap_status gap_pair_transpose(gap_handle* h, const gap_atoms* a, int64_t* tgt_ptr,
                              int32_t* tgt_pair) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  if (!a || !a->pair_ptr || (a->n_pairs > 0 && !a->pair_j) || !tgt_ptr ||
      (a->n_pairs > 0 && !tgt_pair))
    return fail(h, GAP_E_INVALID, "NULL argument");
  if (a->n_atoms < 0 || a->n_pairs < 0 || a->n_pairs > INT32_MAX || a->n_atoms > INT32_MAX)
    return fail(h, GAP_E_INVALID, "bad sizes");
  Layout L;
  const size_t src = L.take(sizeof(int32_t) * std::max<int64_t>(a->n_pairs, 1));
  const size_t scr = L.take(sizeof(int32_t) * (a->n_atoms + 2048));
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  gapk::pair_transpose(a->pair_ptr, a->pair_j, a->n_atoms, a->n_pairs, tgt_ptr, tgt_pair,
                       at<int32_t>(h, src), nullptr, at<int32_t>(h, scr), h->dev_err, h->stream);
  HIP_TRY(h, hipGetLastError());
  return GAP_OK;
}

gap_status gap_build_kmm(gap_handle* h, const gap_sparse* sp, double* Kmm, int64_t ld) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_sparse(h, sp);
  if (s != GAP_OK) return s;
  if (!Kmm || ld < sp->M) return fail(h, GAP_E_INVALID, "Kmm NULL or ld < M");
  h->timer.begin(gapk::TM_KMM);
  gapk::kmm_f64(sp->X, sp->ld_x, sp->M, sp->D, sp->zeta, sp->delta, Kmm, ld, h->stream);
  h->timer.end(gapk::TM_KMM);
  HIP_TRY(h, hipGetLastError());
  return GAP_OK;
}

}  // extern "C"

namespace {

// L-hat K_NM of gap_build_knm; with `species` non-null, the block of the
// per-species GP of species zsel (only atoms of that species are centres).
gap_status build_knm_impl(gap_handle* h, const gap_atoms* a, const gap_sparse* sp,
                          gap_precision prec, double* Knm, int64_t ld, const int32_t* species,
                          int32_t zsel) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_sparse(h, sp);
  if (s != GAP_OK) return s;
  s = check_atoms(h, a, sp, true);
  if (s != GAP_OK) return s;
  const int64_t N = a->n_atoms, M = sp->M, D = sp->D;
  const int64_t n_rows = a->n_cfg + 3 * N;
  if (!Knm || ld < n_rows) return fail(h, GAP_E_INVALID, "Knm NULL or ld < n_cfg + 3 n_atoms");
  if (prec != GAP_FP64 && prec != GAP_BF16X3) return fail(h, GAP_E_INVALID, "bad precision");
  Layout L;
  PairWs p;
  layout_pairs(L, N, a->n_pairs, p);
  const size_t S = L.take(sizeof(double) * std::max<int64_t>(N * ld4(M), 1));
  SplitWs sw;
  size_t jh = 0, jl = 0;
  bool presplit = false;
  if (prec == GAP_BF16X3) {
    layout_split(L, M, D, false, sw);
    const size_t jbytes = (size_t)3 * a->n_pairs * gapk::split_ld(D) * 2;
    // Pre-split the Jacobians once for descriptors of up to 256 entries (the
    // twelve-wave kernel then streams hi / lo halves with no split in its
    // loop) when both halves fit in the workspace with room to spare.  Longer
    // descriptors stream the FP32 / FP64 rows and split them in registers:
    // measured on the 576k-atom fit, the wide kernel on pre-split rows took
    // 6.7 s against 5.1 s on the original rows.
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
    double room = std::min(0.85 * (double)(free_b + h->ws_bytes), (double)((size_t)16 << 30));
    if (h->ws_limit > 0) room = std::min(room, (double)h->ws_limit);
    presplit = a->n_pairs > 0 && D <= 256 && (double)(L.off + 2 * jbytes) * 1.125 <= room;
    if (presplit) {
      jh = L.take(jbytes);
      jl = L.take(jbytes);
    }
  }
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  // The pair transpose (a chain of small kernels) runs on the side stream
  // while the splits and energy rows run here; the force rows wait for both.
  HIP_TRY(h, hipEventRecord(h->ev_fork, h->stream));
  HIP_TRY(h, hipStreamWaitEvent(h->side, h->ev_fork, 0));
  run_pairs(h, a, p, true, h->side);
  HIP_TRY(h, hipEventRecord(h->ev_join, h->side));
  if (prec == GAP_BF16X3) {
    run_split(h, sp, sw, false);
    if (presplit) {
      h->timer.begin(gapk::TM_SPLIT);
      gapk::split_j_bf16(a->jac, f32(a->jac_dt), a->ld_jac, a->n_pairs, D, at<__bf16>(h, jh),
                         at<__bf16>(h, jl), h->stream);
      h->timer.end(gapk::TM_SPLIT);
    }
    h->timer.begin(gapk::TM_ENERGY);
    gapk::energy_rows_bf16x3(a->desc, f32(a->desc_dt), a->ld_desc, a->cfg_ptr, a->n_cfg, N,
                             at<__bf16>(h, sw.xh), at<__bf16>(h, sw.xl), M, D, sp->zeta,
                             sp->delta, Knm, ld, at<float>(h, S), ld8(M), h->stream, species,
                             zsel);
    h->timer.end(gapk::TM_ENERGY);
    HIP_TRY(h, hipStreamWaitEvent(h->stream, h->ev_join, 0));
    h->timer.begin(gapk::TM_FORCE);
    bool done = false;
    if (presplit)
      done = gapk::force_rows_bf16x3_split(
          at<__bf16>(h, jh), at<__bf16>(h, jl), D, at<__bf16>(h, sw.xh), at<__bf16>(h, sw.xl), M,
          at<float>(h, S), ld8(M), at<int64_t>(h, p.tgt_ptr), at<int32_t>(h, p.tgt_pair),
          at<int32_t>(h, p.src), at<int32_t>(h, p.order), N, a->n_pairs, a->n_cfg, Knm, ld,
          h->stream);
    if (!done)
      gapk::force_rows_bf16x3(a->jac, f32(a->jac_dt), a->ld_jac, D, at<__bf16>(h, sw.xh),
                              at<__bf16>(h, sw.xl), M, at<float>(h, S), ld8(M),
                              at<int64_t>(h, p.tgt_ptr), at<int32_t>(h, p.tgt_pair),
                              at<int32_t>(h, p.src), at<int32_t>(h, p.order), N, a->n_pairs,
                              a->n_cfg, Knm, ld, h->stream);
    h->timer.end(gapk::TM_FORCE);
    HIP_TRY(h, hipGetLastError());
    return GAP_OK;
  }
  h->timer.begin(gapk::TM_ENERGY);
  gapk::energy_rows_f64(a->desc, f32(a->desc_dt), a->ld_desc, a->cfg_ptr, a->n_cfg, N, sp->X,
                        sp->ld_x, M, D, sp->zeta, sp->delta, Knm, ld, at<double>(h, S), ld4(M),
                        h->stream, species, zsel);
  h->timer.end(gapk::TM_ENERGY);
  HIP_TRY(h, hipStreamWaitEvent(h->stream, h->ev_join, 0));
  h->timer.begin(gapk::TM_FORCE);
  gapk::force_rows_f64(a->jac, f32(a->jac_dt), a->ld_jac, D, sp->X, sp->ld_x, M,
                       at<double>(h, S), ld4(M), at<int64_t>(h, p.tgt_ptr), at<int32_t>(h, p.tgt_pair),
                       at<int32_t>(h, p.src), at<int32_t>(h, p.order), N, a->n_pairs, a->n_cfg,
                       Knm, ld, h->stream);
  h->timer.end(gapk::TM_FORCE);
  HIP_TRY(h, hipGetLastError());
  return GAP_OK;
}

}  // namespace

extern "C" {

gap_status gap_build_knm(gap_handle* h, const gap_atoms* a, const gap_sparse* sp,
                         gap_precision prec, double* Knm, int64_t ld) {
  return build_knm_impl(h, a, sp, prec, Knm, ld, nullptr, 0);
}

gap_status gap_build_knm_species(gap_handle* h, const gap_atoms* a, const gap_sparse* sp,
                                 gap_precision prec, const int32_t* species, int32_t z,
                                 double* Knm, int64_t ld) {
  if (!h) return GAP_E_INVALID;
  if (!species && a && a->n_atoms > 0) return fail(h, GAP_E_INVALID, "species is NULL");
  return build_knm_impl(h, a, sp, prec, Knm, ld, species, z);
}

gap_status gap_lstsq(gap_handle* h, double* A, int64_t ld, int64_t m, int64_t n, double* x,
                     double* rdiag_minmax) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  if (!A || !x || n < 1 || m < n || ld < m || ld % 4 != 0 || !aligned32(A))
    return fail(h, GAP_E_INVALID, "need A, x, 1 <= n <= m <= ld, ld % 4 == 0, A 32-byte aligned");
  if (n > 8000) return fail(h, GAP_E_UNSUPPORTED, "n > 8000");
  Layout L;
  const size_t q = L.take(gapk::qr_workspace_bytes(m, n));
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  gapk::QrWork qw;
  gapk::qr_bind_workspace(at<char>(h, q), m, n, &qw);
  gapk::qr_factor(A, ld, m, n + 1, n, &qw, h->stream, h->dev_err, &h->timer);
  gapk::back_substitute(A, ld, n, A + n * ld, x, h->dev_small, h->dev_err, h->stream, qw.flags);
  HIP_TRY(h, hipGetLastError());
  double rd[2] = {0, 0};
  HIP_TRY(h, hipMemcpyAsync(rd, h->dev_small, 2 * sizeof(double), hipMemcpyDeviceToHost,
                            h->stream));
  s = drain_dev_err(h);
  if (rdiag_minmax) {
    rdiag_minmax[0] = rd[0];
    rdiag_minmax[1] = rd[1];
  }
  return s;
}

gap_status gap_build_local_rows(gap_handle* h, const gap_atoms* a, const gap_sparse* sp,
                                const int32_t* atom_idx, int64_t n_local, double* K,
                                int64_t ld) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_sparse(h, sp);
  if (s != GAP_OK) return s;
  s = check_atoms(h, a, sp, false);
  if (s != GAP_OK) return s;
  if (n_local < 0 || (n_local > 0 && (!atom_idx || !K)) || ld < n_local)
    return fail(h, GAP_E_INVALID, "need n_local >= 0, atom_idx and K, ld >= n_local");
  h->timer.begin(gapk::TM_ENERGY);
  gapk::local_rows_f64(a->desc, f32(a->desc_dt), a->ld_desc, a->n_atoms, atom_idx, n_local,
                       sp->X, sp->ld_x, sp->M, sp->D, sp->zeta, sp->delta, K, ld, h->dev_err,
                       h->stream);
  h->timer.end(gapk::TM_ENERGY);
  HIP_TRY(h, hipGetLastError());
  return GAP_OK;
}

gap_status gap_build_virial_rows(gap_handle* h, const gap_atoms* a, const gap_sparse* sp,
                                 const double* pair_r, double* Kv, int64_t ld) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_sparse(h, sp);
  if (s != GAP_OK) return s;
  s = check_atoms(h, a, sp, true);
  if (s != GAP_OK) return s;
  const int64_t N = a->n_atoms, M = sp->M, D = sp->D, nc = a->n_cfg;
  if ((a->n_pairs > 0 && !pair_r) || (nc > 0 && !Kv) || ld < 9 * nc)
    return fail(h, GAP_E_INVALID, "need pair_r, Kv and ld >= 9 n_cfg");
  if (nc == 0) return GAP_OK;
  Layout L;
  PairWs p;
  layout_pairs(L, N, a->n_pairs, p);
  const size_t S = L.take(sizeof(double) * std::max<int64_t>(N * ld4(M), 1));
  const size_t ke = L.take(sizeof(double) * nc * M);
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  run_pairs(h, a, p, false);  // pair sources (and the index checks)
  h->timer.begin(gapk::TM_ENERGY);
  gapk::energy_rows_f64(a->desc, f32(a->desc_dt), a->ld_desc, a->cfg_ptr, nc, N, sp->X,
                        sp->ld_x, M, D, sp->zeta, sp->delta, at<double>(h, ke), nc,
                        at<double>(h, S), ld4(M), h->stream);
  h->timer.end(gapk::TM_ENERGY);
  h->timer.begin(gapk::TM_FORCE);
  gapk::virial_rows_f64(a->jac, f32(a->jac_dt), a->ld_jac, D, sp->X, sp->ld_x, M,
                        at<double>(h, S), ld4(M), a->cfg_ptr, nc, a->pair_ptr,
                        at<int32_t>(h, p.src), pair_r, N, a->n_pairs, Kv, ld, h->stream);
  h->timer.end(gapk::TM_FORCE);
  HIP_TRY(h, hipGetLastError());
  return GAP_OK;
}

gap_status gap_predict_variance(gap_handle* h, const gap_atoms* a, const gap_sparse* sp,
                                const double* Kmm, double jitter, const double* R, int64_t ldr,
                                double* var) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_sparse(h, sp);
  if (s != GAP_OK) return s;
  s = check_atoms(h, a, sp, false);
  if (s != GAP_OK) return s;
  const int64_t N = a->n_atoms, M = sp->M, D = sp->D;
  if (!Kmm || !R || ldr < M || (N > 0 && !var))
    return fail(h, GAP_E_INVALID, "need Kmm, R with ldr >= M, and var");
  if (!(jitter >= 0.0) || !std::isfinite(jitter)) return fail(h, GAP_E_INVALID, "bad jitter");
  if (M > 8000) return fail(h, GAP_E_UNSUPPORTED, "M > 8000");
  if (N == 0) return GAP_OK;
  const int64_t ldm = ld4(M);
  Layout L;
  const size_t Lw = L.take(sizeof(double) * M * M);
  const size_t Ub = L.take(sizeof(double) * M * (M + 1));
  const size_t Yu = L.take(sizeof(double) * M * ldm);
  const size_t Yr = L.take(sizeof(double) * M * ldm);
  const size_t Ks = L.take(sizeof(double) * N * ldm);
  const size_t Zb = L.take(sizeof(double) * N * ldm);
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  h->timer.begin(gapk::TM_PREDICT);
  // U (K_MM + jitter I = U^T U) and the inverses of U and R
  gapk::cholesky_lower(at<double>(h, Lw), M, M, jitter, Kmm, M, h->dev_err, h->stream);
  gapk::stack_u(at<double>(h, Ub), M, 0, M, at<double>(h, Lw), M, h->stream);
  gapk::trinv_upper(at<double>(h, Ub), M, M, at<double>(h, Yu), ldm, h->dev_err, h->stream);
  gapk::trinv_upper(R, ldr, M, at<double>(h, Yr), ldm, h->dev_err, h->stream);
  // k_i rows, then var_i = k_ii - ||k_i^T U^-1||^2 + ||k_i^T R^-1||^2
  gapk::local_rows_f64(a->desc, f32(a->desc_dt), a->ld_desc, N, nullptr, N, sp->X, sp->ld_x, M,
                       D, sp->zeta, sp->delta, at<double>(h, Ks), ldm, h->dev_err, h->stream,
                       true);
  gapk::gemm_wx_f64(at<double>(h, Ks), ldm, N, M, at<double>(h, Yu), ldm, M, at<double>(h, Zb),
                    ldm, h->stream);
  gapk::var_rows(at<double>(h, Zb), ldm, N, M, -1.0, a->desc, f32(a->desc_dt), a->ld_desc, D,
                 sp->zeta, sp->delta, 1, var, h->stream);
  gapk::gemm_wx_f64(at<double>(h, Ks), ldm, N, M, at<double>(h, Yr), ldm, M, at<double>(h, Zb),
                    ldm, h->stream);
  gapk::var_rows(at<double>(h, Zb), ldm, N, M, 1.0, a->desc, f32(a->desc_dt), a->ld_desc, D,
                 sp->zeta, sp->delta, 0, var, h->stream);
  h->timer.end(gapk::TM_PREDICT);
  HIP_TRY(h, hipGetLastError());
  return drain_dev_err(h);
}

gap_status gap_select_cur(gap_handle* h, const gap_atoms* a, int64_t n_sparse, double jitter,
                          const double* u, int32_t* out_idx, double* leverage) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  if (!a || !a->desc || a->n_atoms < 0 || a->D < 1 || a->ld_desc < a->D)
    return fail(h, GAP_E_INVALID, "atoms: need desc with ld_desc >= D >= 1");
  if (a->desc_dt != GAP_DT_F32 && a->desc_dt != GAP_DT_F64)
    return fail(h, GAP_E_INVALID, "bad desc dtype");
  const int64_t N = a->n_atoms, D = a->D;
  if (n_sparse < 0 || n_sparse > N || (n_sparse > 0 && !out_idx))
    return fail(h, GAP_E_INVALID, "need 0 <= n_sparse <= n_atoms and out_idx");
  if (!(jitter >= 0.0) || !std::isfinite(jitter)) return fail(h, GAP_E_INVALID, "bad jitter");
  if (D > 8000) return fail(h, GAP_E_UNSUPPORTED, "D > 8000");
  if (N == 0) return GAP_OK;
  if (N > (int64_t(1) << 30)) return fail(h, GAP_E_UNSUPPORTED, "n_atoms > 2^30");
  const int64_t ldd = ld4(D), n_pad = gapk::cur_pad(N);
  Layout L;
  const size_t Dd = L.take(sizeof(double) * N * ldd);
  const size_t Gw = L.take(sizeof(double) * D * D);
  const size_t Lw = L.take(sizeof(double) * D * D);
  const size_t Ub = L.take(sizeof(double) * D * (D + 1));
  const size_t Yu = L.take(sizeof(double) * D * ldd);
  const size_t Zb = L.take(sizeof(double) * N * ldd);
  const size_t lv = L.take(sizeof(double) * N);
  const size_t ky = L.take(sizeof(double) * n_pad);
  const size_t ix = L.take(sizeof(int32_t) * n_pad);
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  double* dd = at<double>(h, Dd);
  double* lev = leverage ? leverage : at<double>(h, lv);
  // leverage l_i = ||d_i^T U^-1||^2 with U^T U = D^T D + jitter I
  gapk::desc_f64(a->desc, f32(a->desc_dt), a->ld_desc, N, D, dd, ldd, h->stream);
  gapk::gemm_wtd_f64(dd, ldd, N, D, dd, false, ldd, D, at<double>(h, Gw), D, h->stream);
  gapk::cholesky_lower(at<double>(h, Lw), D, D, jitter, at<double>(h, Gw), D, h->dev_err,
                       h->stream);
  gapk::stack_u(at<double>(h, Ub), D, 0, D, at<double>(h, Lw), D, h->stream);
  gapk::trinv_upper(at<double>(h, Ub), D, D, at<double>(h, Yu), ldd, h->dev_err, h->stream);
  gapk::gemm_wx_f64(dd, ldd, N, D, at<double>(h, Yu), ldd, D, at<double>(h, Zb), ldd, h->stream);
  gapk::var_rows(at<double>(h, Zb), ldd, N, D, 1.0, dd, false, ldd, D, 1, 1.0, 2, lev, h->stream);
  gapk::cur_select_sort(lev, u, N, at<double>(h, ky), at<int32_t>(h, ix), h->stream);
  if (n_sparse > 0)
    HIP_TRY(h, hipMemcpyAsync(out_idx, at<int32_t>(h, ix), sizeof(int32_t) * n_sparse,
                              hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(h, hipGetLastError());
  return drain_dev_err(h);
}

namespace {
gap_status check_se2b(gap_handle* h, const gap_se2b* k2) {
  if (!k2 || k2->M < 1 || !k2->x) return fail(h, GAP_E_INVALID, "se2b: need M >= 1 and x");
  if (!std::isfinite(k2->delta) || !(k2->theta > 0.0) || !std::isfinite(k2->theta) ||
      !(k2->r_cut > 0.0) || !std::isfinite(k2->r_cut) || !(k2->cut_width > 0.0) ||
      k2->cut_width > k2->r_cut)
    return fail(h, GAP_E_INVALID, "se2b: need finite delta, theta > 0, 0 < cut_width <= r_cut");
  return GAP_OK;
}
gap_status check_pairs_only(gap_handle* h, const gap_atoms* a, const double* pair_r) {
  if (!a || a->n_cfg < 0 || a->n_atoms < 0 || a->n_pairs < 0 || !a->cfg_ptr || !a->pair_ptr)
    return fail(h, GAP_E_INVALID, "atoms: need cfg_ptr and pair_ptr");
  if (a->n_pairs > 0 && (!a->pair_j || !pair_r))
    return fail(h, GAP_E_INVALID, "atoms: need pair_j and pair_r");
  if (a->n_pairs >= (int64_t(1) << 31)) return fail(h, GAP_E_UNSUPPORTED, "n_pairs >= 2^31");
  return GAP_OK;
}
}  // namespace

gap_status gap_build_2b_rows(gap_handle* h, const gap_atoms* a, const double* pair_r,
                             const gap_se2b* k2, double* K, int64_t ld) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_se2b(h, k2);
  if (s != GAP_OK) return s;
  s = check_pairs_only(h, a, pair_r);
  if (s != GAP_OK) return s;
  const int64_t n_rows = a->n_cfg + 3 * a->n_atoms;
  if (!K || ld < n_rows) return fail(h, GAP_E_INVALID, "K NULL or ld < n_cfg + 3 n_atoms");
  Layout L;
  PairWs p;
  layout_pairs(L, a->n_atoms, a->n_pairs, p);
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  run_pairs(h, a, p, false);
  h->timer.begin(gapk::TM_FORCE);
  gapk::se2b_rows_f64(pair_r, a->cfg_ptr, a->n_cfg, a->pair_ptr, at<int64_t>(h, p.tgt_ptr),
                      at<int32_t>(h, p.tgt_pair), a->n_atoms, a->n_pairs, k2->x, k2->M,
                      k2->delta, k2->theta, k2->r_cut, k2->cut_width, K, ld, h->stream);
  h->timer.end(gapk::TM_FORCE);
  HIP_TRY(h, hipGetLastError());
  return GAP_OK;
}

gap_status gap_build_kmm_2b(gap_handle* h, const gap_se2b* k2, double* Kmm, int64_t ld) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_se2b(h, k2);
  if (s != GAP_OK) return s;
  if (!Kmm || ld < k2->M) return fail(h, GAP_E_INVALID, "Kmm NULL or ld < M");
  gapk::se2b_kmm_f64(k2->x, k2->M, k2->delta, k2->theta, k2->r_cut, k2->cut_width, Kmm, ld,
                     h->stream);
  HIP_TRY(h, hipGetLastError());
  return GAP_OK;
}

gap_status gap_predict_2b(gap_handle* h, const gap_atoms* a, const double* pair_r,
                          const gap_se2b* k2, const double* c, double* e_cfg, double* forces) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_se2b(h, k2);
  if (s != GAP_OK) return s;
  s = check_pairs_only(h, a, pair_r);
  if (s != GAP_OK) return s;
  if (!c) return fail(h, GAP_E_INVALID, "c is NULL");
  Layout L;
  PairWs p;
  layout_pairs(L, a->n_atoms, a->n_pairs, p);
  const size_t ep = L.take(sizeof(double) * std::max<int64_t>(a->n_pairs, 1));
  const size_t gp = L.take(sizeof(double) * std::max<int64_t>(a->n_pairs, 1));
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  if (forces) run_pairs(h, a, p, false);
  h->timer.begin(gapk::TM_PREDICT);
  gapk::se2b_predict_f64(pair_r, a->cfg_ptr, a->n_cfg, a->pair_ptr, at<int64_t>(h, p.tgt_ptr),
                         at<int32_t>(h, p.tgt_pair), a->n_atoms, a->n_pairs, k2->x, c, k2->M,
                         k2->delta, k2->theta, k2->r_cut, k2->cut_width, at<double>(h, ep),
                         at<double>(h, gp), e_cfg, forces, h->stream);
  h->timer.end(gapk::TM_PREDICT);
  HIP_TRY(h, hipGetLastError());
  return GAP_OK;
}

// ------------------------------------------------------------ streamed fit
namespace {
gap_status check_fold_state(gap_handle* h, const double* T, int64_t ld, int64_t M,
                            int64_t n_rows) {
  if (!T || M < 1 || n_rows < 0 || ld < M + 1 + n_rows || ld % 4 != 0 || !aligned32(T))
    return fail(h, GAP_E_INVALID,
                "fold state needs M >= 1, ld >= M + 1 + n_rows, ld % 4 == 0, 32-byte alignment");
  if (M > 8000) return fail(h, GAP_E_UNSUPPORTED, "M > 8000");
  return GAP_OK;
}
}  // namespace

gap_status gap_fold_init(gap_handle* h, double* T, int64_t ld, int64_t M, const double* Kmm,
                         double jitter) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_fold_state(h, T, ld, M, 0);
  if (s != GAP_OK) return s;
  if (!Kmm) return fail(h, GAP_E_INVALID, "Kmm is NULL");
  if (!(jitter >= 0.0) || !std::isfinite(jitter)) return fail(h, GAP_E_INVALID, "bad jitter");
  Layout L;
  const size_t Lw = L.take(sizeof(double) * M * M);
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  double* Lm = at<double>(h, Lw);
  h->timer.begin(gapk::TM_CHOL);
  gapk::cholesky_lower(Lm, M, M, jitter, Kmm, M, h->dev_err, h->stream);
  gapk::stack_u(T, ld, 0, M, Lm, M, h->stream);  // rows [0, M): U, zero in column M
  gapk::fold_tidy(T, ld, M, true, h->stream);     // row M: zero
  h->timer.end(gapk::TM_CHOL);
  HIP_TRY(h, hipGetLastError());
  return drain_dev_err(h);
}

gap_status gap_fold_rows(gap_handle* h, double* T, int64_t ld, int64_t M, int64_t n_rows,
                         const double* y, const double* sigma) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_fold_state(h, T, ld, M, n_rows);
  if (s != GAP_OK) return s;
  if (n_rows == 0) return GAP_OK;
  if (!y || !sigma) return fail(h, GAP_E_INVALID, "y / sigma NULL");
  const int64_t m = M + 1 + n_rows;
  Layout L;
  const size_t q = L.take(gapk::qr_workspace_bytes(m, M));
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  gapk::QrWork qw;
  gapk::qr_bind_workspace(at<char>(h, q), m, M, &qw);
  h->timer.begin(gapk::TM_CHOL);
  gapk::scale_rows(T + M + 1, ld, n_rows, M, y, sigma, h->stream);
  h->timer.end(gapk::TM_CHOL);
  // [T ; block] = Q T': R of the first M columns, Q^T b in column M; what Q^T b
  // holds past row M - 1 is the residual, whose norm becomes the corner.
  gapk::qr_factor(T, ld, m, M + 1, M, &qw, h->stream, h->dev_err, &h->timer);
  gapk::norm2_f64(T + M + M * ld, n_rows + 1, T + M + M * ld, h->stream);
  gapk::fold_tidy(T, ld, M, false, h->stream);
  HIP_TRY(h, hipGetLastError());
  return GAP_OK;
}

gap_status gap_fold_solve(gap_handle* h, const double* T, int64_t ld, int64_t M, double* c,
                          double* lsq_resid, double* rdiag_minmax) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_fold_state(h, T, ld, M, 0);
  if (s != GAP_OK) return s;
  if (!c) return fail(h, GAP_E_INVALID, "c is NULL");
  Layout L;
  const size_t q = L.take(gapk::qr_workspace_bytes(M + 1, M));
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  gapk::QrWork qw;
  gapk::qr_bind_workspace(at<char>(h, q), M + 1, M, &qw);
  h->timer.begin(gapk::TM_TRSV);
  gapk::back_substitute(T, ld, M, T + M * ld, c, h->dev_small, h->dev_err, h->stream, qw.flags);
  h->timer.end(gapk::TM_TRSV);
  HIP_TRY(h, hipGetLastError());
  double rd[3] = {0, 0, 0};
  HIP_TRY(h, hipMemcpyAsync(rd, h->dev_small, 2 * sizeof(double), hipMemcpyDeviceToHost,
                            h->stream));
  HIP_TRY(h, hipMemcpyAsync(rd + 2, T + M + M * ld, sizeof(double), hipMemcpyDeviceToHost,
                            h->stream));
  s = drain_dev_err(h);
  if (rdiag_minmax) {
    rdiag_minmax[0] = rd[0];
    rdiag_minmax[1] = rd[1];
  }
  if (lsq_resid) *lsq_resid = std::fabs(rd[2]);
  return s;
}

// Matrix-free FP64 residual of a batch's observation rows (the refinement of
// a fit whose R came from approximate rows): workspace, the per-batch set-up,
// and one pass r = Sigma^-1/2 (y - K c), g = K^T Sigma^-1/2 r.
struct RefineWs {
  size_t kc = 0, rtop = 0, v = 0, hbuf = 0, gvec = 0, dcp = 0, ones = 0;
  PredictWs pw{};
};

void layout_refine(Layout& L, const gap_atoms* a, const gap_sparse* sp, RefineWs& w,
                   bool need_S = true) {
  const int64_t N = a->n_atoms, M = sp->M, D = sp->D;
  const int64_t n_rows = a->n_cfg + 3 * N;
  w.kc = L.take(sizeof(double) * std::max<int64_t>(n_rows, 1));
  w.rtop = L.take(sizeof(double) * std::max<int64_t>(n_rows, 1));
  w.v = L.take(sizeof(double) * std::max<int64_t>(n_rows, 1));
  w.hbuf = L.take(sizeof(double) * std::max<int64_t>(N * ld4(D), 1));
  w.gvec = L.take(sizeof(double) * M);
  w.dcp = L.take(sizeof(double) * std::max(gapk::pstage_row_blocks(N),
                                           gapk::resid_colsum_groups(N, M)) * M + 8);
  w.ones = L.take(sizeof(double) * M);
  // pw.W holds S = delta^2 zeta p^(zeta-1) unless the caller keeps it
  layout_predict(L, a, sp, need_S, false, true, true, w.pw);
}

// The exact FP64 kernel-gradient scale S[i][m] = delta^2 zeta (d_i . x_m)^(zeta-1)
// of a batch (row-major, ld4(M), padding zero): the P-stage with unit
// coefficients, whose weights W = S diag(c) are then S itself.
void refine_weights(gap_handle* h, const gap_atoms* a, const gap_sparse* sp, const RefineWs& w,
                    double* S, int64_t ldS) {
  const int64_t N = a->n_atoms, M = sp->M, D = sp->D;
  double* ones = at<double>(h, w.ones);
  gapk::fill_f64(ones, M, 1.0, h->stream);
  gapk::pstage_f64(0, a->desc, f32(a->desc_dt), a->ld_desc, N, sp->X, sp->ld_x, M, D, sp->zeta,
                   sp->delta, ones, nullptr, nullptr, 0, S, ldS, nullptr, nullptr, h->stream,
                   nullptr, 0, nullptr);
}

// rtop = Sigma^-1/2 (y - K c) over the batch's rows (energy rows, then three
// force rows per atom) and gvec = K^T Sigma^-1/2 rtop, K the exact FP64 rows,
// from the batch's S (ldS) and target-major pair view (run_pairs before):
//   g_i = (S diag c)_i X,  energy row c: sum_{i in c} d_i . g_i / zeta (Euler:
//   eps_i is homogeneous of degree zeta in d_i), force rows: -J^T g,
//   K^T v = -sum_i S_im (h~_i . x_m) with h~_i = J^T v_F (rows of atom i) -
//   (v_c(i) / zeta) d_i (k(d_i, x_m) = S_im (d_i . x_m) / zeta).
void refine_residual_rows(gap_handle* h, const gap_atoms* a, const gap_sparse* sp,
                          const RefineWs& w, const double* S, int64_t ldS, const double* c,
                          const double* y, const double* sigma) {
  const int64_t N = a->n_atoms, nc = a->n_cfg, M = sp->M, D = sp->D;
  const int64_t n_rows = nc + 3 * N;
  const int64_t ldg = ld4(D);
  double* g = at<double>(h, w.pw.g);
  double* kcp = at<double>(h, w.kc);
  double* vv = at<double>(h, w.v);
  double* gv = at<double>(h, w.gvec);
  double* hb = at<double>(h, w.hbuf);
  double* dcp = at<double>(h, w.dcp);
  if (N > 0) {
    gapk::gemm_wx_scaled_f64(S, ldS, N, M, c, sp->X, sp->ld_x, D, g, ldg, h->stream);
    gapk::cfg_energy_from_grad(a->desc, f32(a->desc_dt), a->ld_desc, g, ldg, a->cfg_ptr, nc, N, D,
                               sp->zeta, kcp, h->stream);
    gapk::forces_f64(a->jac, f32(a->jac_dt), a->ld_jac, D, g, ldg,
                     at<int32_t>(h, w.pw.pairs.src), N, a->n_pairs,
                     at<int64_t>(h, w.pw.pairs.tgt_ptr), at<int32_t>(h, w.pw.pairs.tgt_pair),
                     at<double>(h, w.pw.f_pair), kcp + nc, h->stream);
  } else {
    gapk::fill_f64(kcp, std::max<int64_t>(nc, 1), 0.0, h->stream);
  }
  gapk::residual_top(y, sigma, kcp, n_rows, at<double>(h, w.rtop), h->stream);
  gapk::div_sigma(at<double>(h, w.rtop), sigma, n_rows, vv, h->stream);
  if (N > 0) {
    gapk::jac_transpose_apply_f64(a->jac, f32(a->jac_dt), a->ld_jac, D, a->pair_ptr, a->pair_j,
                                  N, a->n_pairs, vv + nc, hb, ldg, h->stream);
    gapk::sub_cfg_desc(hb, ldg, a->desc, f32(a->desc_dt), a->ld_desc, vv, a->cfg_ptr, nc, N, D,
                       sp->zeta, h->stream);
    if (gapk::resid_colsum_f64(hb, ldg, N, D, sp->X, sp->ld_x, M, S, ldS, dcp, h->stream)) {
      gapk::reduce_rows_f64(dcp, gapk::resid_colsum_groups(N, M), M, gv, h->stream);
    } else {
      gapk::pstage_f64(3, nullptr, false, 0, N, sp->X, sp->ld_x, M, D, sp->zeta, sp->delta,
                       nullptr, nullptr, hb, ldg, nullptr, 0, nullptr, dcp, h->stream, S, ldS);
      gapk::reduce_rows_f64(dcp, gapk::pstage_row_blocks(N), M, gv, h->stream);
    }
  } else {
    gapk::fill_f64(gv, M, 0.0, h->stream);
  }
}

gap_status gap_fit(gap_handle* h, double* A, int64_t ld, int64_t n_rows, const double* Kmm,
                   const double* y, const double* sigma, double jitter, const gap_atoms* train,
                   const gap_sparse* sp, int refine_steps, double* c, gap_fit_info* info) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_sparse(h, sp);
  if (s != GAP_OK) return s;
  const int64_t M = sp->M, D = sp->D;
  const int64_t m = n_rows + M;
  if (!A || !Kmm || !y || !sigma || !c) return fail(h, GAP_E_INVALID, "NULL argument");
  if (n_rows < 0 || ld < m || ld % 4 != 0 || !aligned32(A))
    return fail(h, GAP_E_INVALID, "A needs ld >= n_rows + M, ld % 4 == 0, 32-byte alignment");
  if (!(jitter >= 0.0) || !std::isfinite(jitter)) return fail(h, GAP_E_INVALID, "bad jitter");
  if (M > 8000) return fail(h, GAP_E_UNSUPPORTED, "M > 8000");
  if (refine_steps < 0 || refine_steps > 7) return fail(h, GAP_E_INVALID, "refine_steps in [0,7]");
  if (refine_steps > 0) {
    s = check_atoms(h, train, sp, true);
    if (s != GAP_OK) return s;
    if (train->n_cfg + 3 * train->n_atoms != n_rows)
      return fail(h, GAP_E_INVALID, "train does not match n_rows");
    if (D > 2048) return fail(h, GAP_E_UNSUPPORTED, "refinement needs D <= 2048");
  }
  Layout L;
  const size_t Lw = L.take(sizeof(double) * M * M);
  const size_t q = L.take(gapk::qr_workspace_bytes(m, M));
  size_t rbot = 0;
  RefineWs rw;
  if (refine_steps > 0) {
    rbot = L.take(sizeof(double) * M);
    layout_refine(L, train, sp, rw);
  }
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  gapk::QrWork qw;
  gapk::qr_bind_workspace(at<char>(h, q), m, M, &qw);
  double* Lm = at<double>(h, Lw);
  h->timer.begin(gapk::TM_CHOL);
  // The Cholesky factor of K_MM (a chain of small latency-bound kernels) runs on
  // the side stream while the memory-bound row scaling of [K_NM | y] runs here;
  // U is stacked below once both are done.
  HIP_TRY(h, hipEventRecord(h->ev_fork, h->stream));
  HIP_TRY(h, hipStreamWaitEvent(h->side, h->ev_fork, 0));
  gapk::cholesky_lower(Lm, M, M, jitter, Kmm, M, h->dev_err, h->side);
  HIP_TRY(h, hipEventRecord(h->ev_join, h->side));
  gapk::scale_rows(A, ld, n_rows, M, y, sigma, h->stream);
  HIP_TRY(h, hipStreamWaitEvent(h->stream, h->ev_join, 0));
  gapk::stack_u(A, ld, n_rows, M, Lm, M, h->stream);
  h->timer.end(gapk::TM_CHOL);
  gapk::qr_factor(A, ld, m, M + 1, M, &qw, h->stream, h->dev_err, &h->timer);
  h->timer.begin(gapk::TM_TRSV);
  gapk::back_substitute(A, ld, M, A + M * ld, c, h->dev_small, h->dev_err, h->stream, qw.flags);
  h->timer.end(gapk::TM_TRSV);
  HIP_TRY(h, hipGetLastError());
  gap_fit_info inf;
  std::memset(&inf, 0, sizeof inf);
  for (double& r : inf.resid_norm) r = NAN;
  double rd[2];
  HIP_TRY(h, hipMemcpyAsync(rd, h->dev_small, 2 * sizeof(double), hipMemcpyDeviceToHost,
                            h->stream));
  s = drain_dev_err(h);
  inf.min_abs_rdiag = rd[0];
  inf.max_abs_rdiag = rd[1];
  if (s != GAP_OK) {
    if (info) *info = inf;
    return s;
  }
  if (refine_steps > 0) {
    double* gv = at<double>(h, rw.gvec);
    h->timer.begin(gapk::TM_REFINE);
    double* Sref = at<double>(h, rw.pw.W);
    refine_weights(h, train, sp, rw, Sref, ld4(M));
    run_pairs(h, train, rw.pw.pairs, false);
    // Each step contracts the error of c by about the same factor, estimated
    // from consecutive corrections, so the error left after step k is about
    // |dc_k|^2 / |dc_k-1| (relative to |c|); the steps stop once that is below
    // kRefineTol, and one more residual gives the reported |A^T r| (unless the
    // handle was told to skip it).
    constexpr double kRefineTol = 1e-14;
    int done = 0;
    bool stop = false;
    double prev = -1.0;
    for (int step = 0; step <= refine_steps; ++step) {
      if ((step == refine_steps || stop) && !h->fit_final_resid) break;
      // A^T r = K^T Sigma^-1/2 r_top + U^T r_bot with r = b - A_exact c
      refine_residual_rows(h, train, sp, rw, Sref, ld4(M), c, y, sigma);
      gapk::residual_bot(Lm, M, M, c, at<double>(h, rbot), h->stream);
      gapk::add_ut_r(Lm, M, M, at<double>(h, rbot), gv, h->stream);
      gapk::norm2_f64(gv, M, h->dev_small + 8 + step, h->stream);
      if (step == refine_steps || stop) break;
      // R^T R dc = A^T r ; c += dc
      gapk::seminormal_solve(A, ld, M, gv, h->stream, qw.flags, at<double>(h, rbot), h->dev_err);
      gapk::axpy_f64(M, 1.0, gv, c, h->stream);
      done = step + 1;
      if (step + 1 < refine_steps) {
        gapk::norm2_f64(gv, M, h->dev_small + 20, h->stream);
        gapk::norm2_f64(c, M, h->dev_small + 21, h->stream);
        double nn[2];
        HIP_TRY(h, hipMemcpyAsync(nn, h->dev_small + 20, 2 * sizeof(double),
                                  hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        const double rel = nn[1] > 0.0 ? nn[0] / nn[1] : 0.0;
        stop = rel == 0.0 || (prev > 0.0 && rel * rel / prev <= kRefineTol);
        prev = rel;
      }
    }
    h->timer.end(gapk::TM_REFINE);
    HIP_TRY(h, hipGetLastError());
    double rn[8];
    const int n_rn = h->fit_final_resid ? done + 1 : done;
    HIP_TRY(h, hipMemcpyAsync(rn, h->dev_small + 8, n_rn * sizeof(double),
                              hipMemcpyDeviceToHost, h->stream));
    s = drain_dev_err(h);
    for (int i = 0; i < n_rn && i < 8; ++i) inf.resid_norm[i] = rn[i];
    inf.refine_done = done;
  }
  if (info) *info = inf;
  return s;
}

}  // extern "C"

namespace {

// One batch's share of a refinement step, with S from the caller (S != null)
// or computed into the workspace.
gap_status refine_rows_impl(gap_handle* h, const gap_atoms* a, const gap_sparse* sp,
                            const double* S, int64_t ldS, const double* c, const double* y,
                            const double* sigma, double* g, double* rr) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_sparse(h, sp);
  if (s != GAP_OK) return s;
  s = check_atoms(h, a, sp, true);
  if (s != GAP_OK) return s;
  if (!c || !g) return fail(h, GAP_E_INVALID, "c / g are NULL");
  if (sp->M > 8000) return fail(h, GAP_E_UNSUPPORTED, "M > 8000");
  if (sp->D > 2048) return fail(h, GAP_E_UNSUPPORTED, "refinement needs D <= 2048");
  if (S && (ldS < sp->M || ldS % 4 != 0 || !aligned32(S)))
    return fail(h, GAP_E_INVALID, "S needs ldS >= M, ldS % 4 == 0 and 32-byte alignment");
  const int64_t n_rows = a->n_cfg + 3 * a->n_atoms;
  if (n_rows == 0) return GAP_OK;
  if (!y || !sigma) return fail(h, GAP_E_INVALID, "y / sigma are NULL");
  Layout L;
  RefineWs rw;
  layout_refine(L, a, sp, rw, S == nullptr);
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  h->timer.begin(gapk::TM_REFINE);
  if (!S) {
    S = at<double>(h, rw.pw.W);
    ldS = ld4(sp->M);
    refine_weights(h, a, sp, rw, at<double>(h, rw.pw.W), ldS);
  }
  run_pairs(h, a, rw.pw.pairs, false);
  refine_residual_rows(h, a, sp, rw, S, ldS, c, y, sigma);
  gapk::axpy_f64(sp->M, 1.0, at<double>(h, rw.gvec), g, h->stream);
  if (rr) gapk::sumsq_add_f64(at<double>(h, rw.rtop), n_rows, rr, h->stream);
  h->timer.end(gapk::TM_REFINE);
  HIP_TRY(h, hipGetLastError());
  return GAP_OK;
}

}  // namespace

extern "C" {

gap_status gap_refine_rows(gap_handle* h, const gap_atoms* a, const gap_sparse* sp,
                           const double* c, const double* y, const double* sigma, double* g,
                           double* rr) {
  return refine_rows_impl(h, a, sp, nullptr, 0, c, y, sigma, g, rr);
}

gap_status gap_refine_weights(gap_handle* h, const gap_atoms* a, const gap_sparse* sp, double* S,
                              int64_t ldS) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_sparse(h, sp);
  if (s != GAP_OK) return s;
  s = check_atoms(h, a, sp, false);
  if (s != GAP_OK) return s;
  if (!S && a->n_atoms > 0) return fail(h, GAP_E_INVALID, "S is NULL");
  if (ldS < sp->M || ldS % 4 != 0 || (S && !aligned32(S)))
    return fail(h, GAP_E_INVALID, "S needs ldS >= M, ldS % 4 == 0 and 32-byte alignment");
  if (a->n_atoms == 0) return GAP_OK;
  Layout L;
  RefineWs rw;
  rw.ones = L.take(sizeof(double) * sp->M);
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  h->timer.begin(gapk::TM_REFINE);
  refine_weights(h, a, sp, rw, S, ldS);
  h->timer.end(gapk::TM_REFINE);
  HIP_TRY(h, hipGetLastError());
  return GAP_OK;
}

gap_status gap_refine_rows_s(gap_handle* h, const gap_atoms* a, const gap_sparse* sp,
                             const double* S, int64_t ldS, const double* c, const double* y,
                             const double* sigma, double* g, double* rr) {
  if (!h) return GAP_E_INVALID;
  if (!S && a && a->n_atoms > 0) return fail(h, GAP_E_INVALID, "S is NULL");
  return refine_rows_impl(h, a, sp, S, ldS, c, y, sigma, g, rr);
}

gap_status gap_refine_solve(gap_handle* h, const double* R, int64_t ldr, int64_t M,
                            const double* Kmm, double jitter, double* g, double* c) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  if (!R || !Kmm || !g || !c) return fail(h, GAP_E_INVALID, "NULL argument");
  if (M < 1 || ldr < M) return fail(h, GAP_E_INVALID, "needs M >= 1 and ldr >= M");
  if (M > 8000) return fail(h, GAP_E_UNSUPPORTED, "M > 8000");
  if (!(jitter >= 0.0) || !std::isfinite(jitter)) return fail(h, GAP_E_INVALID, "bad jitter");
  Layout L;
  const size_t q = L.take(gapk::qr_workspace_bytes(M + 1, M));
  const size_t t1 = L.take(sizeof(double) * M);
  const size_t t2 = L.take(sizeof(double) * M);
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  gapk::QrWork qw;
  gapk::qr_bind_workspace(at<char>(h, q), M + 1, M, &qw);
  double* kc = at<double>(h, t1);
  h->timer.begin(gapk::TM_REFINE);
  // the regulariser rows U with zero targets: U^T (0 - U c) = -(K_MM + jitter I) c
  gapk::gemv_cm_f64(Kmm, M, M, M, c, kc, h->stream);
  gapk::axpy_f64(M, jitter, c, kc, h->stream);
  gapk::axpy_f64(M, -1.0, kc, g, h->stream);
  // R^T R dc = A^T r ; c += dc
  gapk::seminormal_solve(R, ldr, M, g, h->stream, qw.flags, at<double>(h, t2), h->dev_err);
  gapk::axpy_f64(M, 1.0, g, c, h->stream);
  h->timer.end(gapk::TM_REFINE);
  HIP_TRY(h, hipGetLastError());
  return drain_dev_err(h);
}

}  // extern "C"

namespace {

gap_status predict_impl(gap_handle* h, const gap_atoms* a, const gap_sparse* sp, const double* c,
                        gap_precision prec, double* e_atom, double* e_cfg, double* dEdd,
                        double* forces, const int32_t* species, int32_t zsel) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_sparse(h, sp);
  if (s != GAP_OK) return s;
  s = check_atoms(h, a, sp, forces != nullptr);
  if (s != GAP_OK) return s;
  if (!c) return fail(h, GAP_E_INVALID, "c is NULL");
  if (prec != GAP_FP64 && prec != GAP_BF16X3) return fail(h, GAP_E_INVALID, "bad precision");
  const bool bf = prec == GAP_BF16X3;
  Layout L;
  PredictWs pw;
  layout_predict(L, a, sp, dEdd || forces, e_cfg && !e_atom, forces != nullptr, forces != nullptr,
                 pw, bf);
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  h->timer.begin(gapk::TM_PREDICT);
  run_predict(h, a, sp, c, pw, e_atom, e_cfg, dEdd, forces, bf, species, zsel);
  h->timer.end(gapk::TM_PREDICT);
  HIP_TRY(h, hipGetLastError());
  return GAP_OK;
}

}  // namespace

extern "C" {

gap_status gap_predict(gap_handle* h, const gap_atoms* a, const gap_sparse* sp, const double* c,
                       gap_precision prec, double* e_atom, double* e_cfg, double* dEdd,
                       double* forces) {
  return predict_impl(h, a, sp, c, prec, e_atom, e_cfg, dEdd, forces, nullptr, 0);
}

gap_status gap_predict_species(gap_handle* h, const gap_atoms* a, const gap_sparse* sp,
                               const double* c, gap_precision prec, const int32_t* species,
                               int32_t z, double* e_atom, double* e_cfg, double* dEdd,
                               double* forces) {
  if (!h) return GAP_E_INVALID;
  if (!species && a && a->n_atoms > 0) return fail(h, GAP_E_INVALID, "species is NULL");
  return predict_impl(h, a, sp, c, prec, e_atom, e_cfg, dEdd, forces, species, z);
}

gap_status gap_predict_backward(gap_handle* h, const gap_atoms* a, const gap_sparse* sp,
                                const double* c, gap_precision prec, const double* g_e,
                                double* d_desc, double* d_c, double* d_X) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_sparse(h, sp);
  if (s != GAP_OK) return s;
  s = check_atoms(h, a, sp, false);
  if (s != GAP_OK) return s;
  if (!c || !g_e) return fail(h, GAP_E_INVALID, "c or g_e is NULL");
  if (prec != GAP_FP64 && prec != GAP_BF16X3) return fail(h, GAP_E_INVALID, "bad precision");
  const bool bf = prec == GAP_BF16X3;
  const int64_t N = a->n_atoms, M = sp->M, D = sp->D;
  Layout L;
  const bool needW = d_desc || d_X;
  const int64_t ldw = ld4(M);
  if (bf) {
    // tiled BF16X3 path: FP32 W from the P-stage, then W X and W^T D (W and the
    // descriptors read as column views)
    const size_t W32 = L.take(sizeof(float) * std::max<int64_t>(N * ldw, 1));
    const size_t dcp = L.take(sizeof(double) * (gapk::gemm_b3_row_blocks(N) * M + 8));
    // W^T D splits its k = atom range into nz slices so that the grid holds about
    // one 128 KB-LDS block per compute unit (256); more slices only add FP64
    // partials (nz M D values written, then summed) to the HBM stream
    const int64_t base = gapk::gemm_b3_col_blocks(M) * gapk::gemm_b3_col_blocks(D);
    const int nz = (int)std::max<int64_t>(
        1, std::min<int64_t>({32, (256 + base - 1) / base, std::max<int64_t>(N / 512, 1)}));
    const size_t part = d_X ? L.take(sizeof(double) * std::max<int64_t>(nz * M * D, 1)) : 0;
    SplitWs sw;
    layout_split(L, M, D, true, sw);
    s = ensure_ws(h, L.off);
    if (s != GAP_OK) return s;
    h->timer.begin(gapk::TM_BACKWARD);
    run_split(h, sp, sw, d_desc != nullptr);
    gapk::pstage_b3t(1, a->desc, f32(a->desc_dt), a->ld_desc, N, at<__bf16>(h, sw.xh),
                     at<__bf16>(h, sw.xl), M, D, sp->zeta, sp->delta, c, g_e, at<float>(h, W32),
                     ldw, nullptr, at<double>(h, dcp), h->stream);
    if (d_c)
      gapk::sum_parts_f64(at<double>(h, dcp), gapk::gemm_b3_row_blocks(N), M, d_c, 1, M, M,
                          h->stream);
    if (d_desc)
      gapk::gemm_b3_wx(at<float>(h, W32), ldw, N, M, at<__bf16>(h, sw.xth),
                       at<__bf16>(h, sw.xtl), D, d_desc, D, h->stream);
    if (d_X)
      gapk::gemm_b3_wtd(at<float>(h, W32), ldw, M, N, a->desc, f32(a->desc_dt), a->ld_desc, D,
                        at<double>(h, part), nz, d_X, D, h->stream);
    h->timer.end(gapk::TM_BACKWARD);
    HIP_TRY(h, hipGetLastError());
    return GAP_OK;
  }
  const size_t W = needW ? L.take(sizeof(double) * std::max<int64_t>(N * ldw, 1)) : 0;
  const size_t dcp = L.take(sizeof(double) * (gapk::pstage_row_blocks(N) * M + 8));
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  double* Wp = needW ? at<double>(h, W) : nullptr;
  h->timer.begin(gapk::TM_BACKWARD);
  {
    gapk::pstage_f64(1, a->desc, f32(a->desc_dt), a->ld_desc, N, sp->X, sp->ld_x, M, D, sp->zeta,
                     sp->delta, c, g_e, nullptr, 0, Wp, ldw, nullptr, at<double>(h, dcp),
                     h->stream);
  }
  if (d_c) gapk::reduce_rows_f64(at<double>(h, dcp), gapk::pstage_row_blocks(N), M, d_c, h->stream);
  if (d_desc) gapk::gemm_wx_f64(Wp, ldw, N, M, sp->X, sp->ld_x, D, d_desc, D, h->stream);
  if (d_X)
    gapk::gemm_wtd_f64(Wp, ldw, N, M, a->desc, f32(a->desc_dt), a->ld_desc, D, d_X, D, h->stream);
  h->timer.end(gapk::TM_BACKWARD);
  HIP_TRY(h, hipGetLastError());
  return GAP_OK;
}

gap_status gap_forces(gap_handle* h, const gap_atoms* a, const double* dEdd, double* forces) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_atoms(h, a, nullptr, true);
  if (s != GAP_OK) return s;
  if (!dEdd || !forces) return fail(h, GAP_E_INVALID, "dEdd or forces is NULL");
  const bool direct = aligned32(dEdd) && a->D % 4 == 0;
  Layout L;
  PairWs p;
  layout_pairs(L, a->n_atoms, a->n_pairs, p);
  const size_t fp = L.take(sizeof(double) * std::max<int64_t>(3 * a->n_pairs, 1));
  const size_t gp = direct ? 0 : L.take(sizeof(double) * std::max<int64_t>(a->n_atoms * ld4(a->D), 1));
  s = ensure_ws(h, L.off);
  if (s != GAP_OK) return s;
  const double* g = dEdd;
  int64_t ldg = a->D;
  if (!direct) {
    ldg = ld4(a->D);
    gapk::copy_rows_f64(dEdd, a->D, at<double>(h, gp), ldg, a->n_atoms, a->D, h->stream);
    g = at<double>(h, gp);
  }
  run_pairs(h, a, p, false);
  gapk::forces_f64(a->jac, f32(a->jac_dt), a->ld_jac, a->D, g, ldg, at<int32_t>(h, p.src),
                   a->n_atoms, a->n_pairs, at<int64_t>(h, p.tgt_ptr), at<int32_t>(h, p.tgt_pair),
                   at<double>(h, fp), forces, h->stream);
  HIP_TRY(h, hipGetLastError());
  return GAP_OK;
}

gap_status gap_split_bf16x3(gap_handle* h, const void* x, gap_dtype dt, int64_t rows,
                            int64_t cols, int64_t ld, uint16_t* hi, uint16_t* lo, uint16_t* hi_t,
                            uint16_t* lo_t) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  if (rows < 0 || cols < 1) return fail(h, GAP_E_INVALID, "rows must be >= 0 and cols >= 1");
  if (dt != GAP_DT_F32 && dt != GAP_DT_F64) return fail(h, GAP_E_INVALID, "bad dtype");
  if (rows == 0) return GAP_OK;
  if (!x || !hi || !lo) return fail(h, GAP_E_INVALID, "x, hi or lo is NULL");
  if (ld < cols || ld % 4 != 0 || !aligned32(x))
    return fail(h, GAP_E_INVALID, "ld must be >= cols and a multiple of 4, x 32-byte aligned");
  if ((reinterpret_cast<uintptr_t>(hi) | reinterpret_cast<uintptr_t>(lo)) & 15u)
    return fail(h, GAP_E_INVALID, "hi and lo must be 16-byte aligned");
  if ((hi_t == nullptr) != (lo_t == nullptr))
    return fail(h, GAP_E_INVALID, "give both transposed halves or neither");
  if (hi_t) {
    if (dt != GAP_DT_F64)
      return fail(h, GAP_E_INVALID, "the transposed halves are produced from FP64 input only");
    gapk::split_x_bf16(static_cast<const double*>(x), ld, rows, cols,
                       reinterpret_cast<__bf16*>(hi), reinterpret_cast<__bf16*>(lo),
                       reinterpret_cast<__bf16*>(hi_t), reinterpret_cast<__bf16*>(lo_t), h->stream);
  } else {
    gapk::split_rows_bf16(x, f32(dt), ld, rows, cols, reinterpret_cast<__bf16*>(hi),
                          reinterpret_cast<__bf16*>(lo), h->stream);
  }
  HIP_TRY(h, hipGetLastError());
  return GAP_OK;
}

gap_status gap_forces_noalloc(gap_handle* h, const gap_atoms* a, const double* dEdd,
                              double* forces) {
  if (!h) return GAP_E_INVALID;
  gap_status s = set_device(h);
  if (s != GAP_OK) return s;
  s = check_atoms(h, a, nullptr, true);
  if (s != GAP_OK) return s;
  if (!dEdd || !forces) return fail(h, GAP_E_INVALID, "dEdd or forces is NULL");
  if (!h->noalloc_scratch) return fail(h, GAP_E_HIP, "no allocation-free scratch on this device");
  // the same slices as gap_forces, laid out in the static scratch
  const bool direct = aligned32(dEdd) && a->D % 4 == 0;
  Layout L;
  PairWs p;
  layout_pairs(L, a->n_atoms, a->n_pairs, p);
  const size_t fp = L.take(sizeof(double) * std::max<int64_t>(3 * a->n_pairs, 1));
  const size_t gp = direct ? 0 : L.take(sizeof(double) * std::max<int64_t>(a->n_atoms * ld4(a->D), 1));
  if (L.off > kNoAllocScratchBytes)
    return fail(h, GAP_E_INVALID,
                "gap_forces_noalloc needs %zu bytes of scratch for %lld atoms and %lld pairs; "
                "its static scratch holds %zu (use gap_forces)",
                L.off, (long long)a->n_atoms, (long long)a->n_pairs, kNoAllocScratchBytes);
  char* base = static_cast<char*>(h->noalloc_scratch);
  const double* g = dEdd;
  int64_t ldg = a->D;
  if (!direct) {
    ldg = ld4(a->D);
    gapk::copy_rows_f64(dEdd, a->D, reinterpret_cast<double*>(base + gp), ldg, a->n_atoms, a->D,
                        h->stream);
    g = reinterpret_cast<const double*>(base + gp);
  }
  gapk::pair_transpose(a->pair_ptr, a->pair_j, a->n_atoms, a->n_pairs,
                       reinterpret_cast<int64_t*>(base + p.tgt_ptr),
                       reinterpret_cast<int32_t*>(base + p.tgt_pair),
                       reinterpret_cast<int32_t*>(base + p.src), nullptr,
                       reinterpret_cast<int32_t*>(base + p.scratch), h->dev_err, h->stream);
  gapk::forces_f64(a->jac, f32(a->jac_dt), a->ld_jac, a->D, g, ldg,
                   reinterpret_cast<int32_t*>(base + p.src), a->n_atoms, a->n_pairs,
                   reinterpret_cast<int64_t*>(base + p.tgt_ptr),
                   reinterpret_cast<int32_t*>(base + p.tgt_pair),
                   reinterpret_cast<double*>(base + fp), forces, h->stream);
  HIP_TRY(h, hipGetLastError());
  return GAP_OK;
}

}  // extern "C"
