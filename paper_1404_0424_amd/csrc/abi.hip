// Public C entry points (include/mimo_cg.h): argument validation, kernel
// selection and launch.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "../../include/mimo_cg.h"
#include "launch.hpp"

namespace {

thread_local char g_last_error[512] = "";

mimo_status fail(int status, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return static_cast<mimo_status>(status);
}

mimo_status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return MIMO_OK;
  return fail(MIMO_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// Calls with U > MIMO_MAX_USERS_COMMON run the four-wavefront kernels, built
// for complex64 storage.
mimo_status check_wide(int U, int in_dtype) {
  if (U > MIMO_MAX_USERS_COMMON && in_dtype != MIMO_C32)
    return fail(MIMO_EUNSUPPORTED, "U=%d > %d needs complex64 storage", U,
                MIMO_MAX_USERS_COMMON);
  return MIMO_OK;
}

// max_u: the entry point's largest U (MIMO_MAX_USERS for the CG detection
// and precoding calls, MIMO_MAX_USERS_COMMON for the others).
mimo_status check_shape(const mimo_shape* s, bool need_k, int max_u = MIMO_MAX_USERS_COMMON) {
  if (!s) return fail(MIMO_EINVAL, "shape is NULL");
  if (s->U < 1) return fail(MIMO_EINVAL, "U=%d < 1", s->U);
  if (s->U > max_u)
    return fail(MIMO_EUNSUPPORTED, "U=%d > %d (U up to %d: CG detection with the approximate "
                "SINR and CG precoding, complex64 storage)", s->U, max_u, MIMO_MAX_USERS);
  if (s->B < s->U) return fail(MIMO_EINVAL, "B=%d < U=%d", s->B, s->U);
  if (s->B > MIMO_MAX_ANTENNAS)
    return fail(MIMO_EUNSUPPORTED, "B=%d > %d", s->B, MIMO_MAX_ANTENNAS);
  if (s->S < 1) return fail(MIMO_EINVAL, "S=%d < 1", s->S);
  // Kernels address one subcarrier's arrays through buffer descriptors with
  // 32-bit byte offsets, and mark masked lanes with the offset 2^31: every
  // per-subcarrier byte range (Y and Q: 8 B S, LLRs up to 32 U S) must stay
  // below 2^31.
  const int64_t per_rhs = 8 * (int64_t)(s->B > 4 * s->U ? s->B : 4 * s->U);
  if ((int64_t)s->S * per_rhs >= MIMO_MAX_SPAN_BYTES)
    return fail(MIMO_EUNSUPPORTED, "S=%d too large for B=%d, U=%d (per-subcarrier arrays of "
                "%lld bytes; the limit is %lld)", s->S, s->B, s->U,
                (long long)((int64_t)s->S * per_rhs), (long long)MIMO_MAX_SPAN_BYTES);
  if (s->n_sc < 0) return fail(MIMO_EINVAL, "n_sc=%lld < 0", (long long)s->n_sc);
  if (need_k && (s->K < 1 || s->K > 1024)) return fail(MIMO_EINVAL, "K=%d outside [1, 1024]", s->K);
  return MIMO_OK;
}

mimo_status check_dtype(int in_dtype, int B) {
  if (in_dtype != MIMO_C32 && in_dtype != MIMO_C16 && in_dtype != MIMO_CBF16)
    return fail(MIMO_EINVAL, "in_dtype=%d unknown", in_dtype);
  if (in_dtype != MIMO_C32 && (B % 8) != 0)
    return fail(MIMO_EINVAL, "16-bit storage needs B %% 8 == 0 (B=%d)", B);
  return MIMO_OK;
}

mimo_status check_ptr(const void* p, const char* name, bool required) {
  if (!p) return required ? fail(MIMO_EINVAL, "%s is NULL", name) : MIMO_OK;
  if (!aligned16(p)) return fail(MIMO_EINVAL, "%s is not 16-byte aligned", name);
  return MIMO_OK;
}

// ---------------------------------------------------------------- schedules
// Process-wide table of kernel schedules, indexed by operation, user class
// (U <= 16, U <= 32) and storage type; written by mimo_tune_set (the
// autotuner), read at every launch.  Each entry packs variant | blocks << 8.
constexpr int kOps = 4, kUClasses = 2, kDtypes = 3;
std::atomic<int> g_sched[kOps][kUClasses][kDtypes];
std::atomic<bool> g_sched_init{false};

int pack(int variant, int blocks) { return (variant & 0xff) | (blocks << 8); }

void sched_defaults() {
  bool expect = false;
  if (!g_sched_init.compare_exchange_strong(expect, true)) return;
  for (int o = 0; o < kOps; ++o)
    for (int u = 0; u < kUClasses; ++u)
      for (int d = 0; d < kDtypes; ++d) g_sched[o][u][d].store(pack(0, 0));
  // measured defaults on MI355X (128x16 and 256x32 workloads); the
  // autotuner overrides them per process
  for (int u = 0; u < kUClasses; ++u)
    for (int d = 0; d < kDtypes; ++d) {
      g_sched[MIMO_OP_DETECT][u][d].store(pack(mimo::kDetectStream, 0));
      g_sched[MIMO_OP_PRECODE][u][d].store(pack(mimo::kPrecodeResident, 8));
      g_sched[MIMO_OP_GRAM_MF][u][d].store(pack(mimo::kGramStream, 0));
      g_sched[MIMO_OP_SLOT][u][d].store(pack(mimo::kSlotFused, 0));
    }
}

mimo::Schedule get_sched(int op, int U, int dt) {
  sched_defaults();
  const int v = g_sched[op][U <= 16 ? 0 : 1][dt].load(std::memory_order_relaxed);
  return mimo::Schedule{v & 0xff, v >> 8};
}

int variant_count(int op) {
  switch (op) {
    case MIMO_OP_DETECT: return mimo::kDetectVariants;
    case MIMO_OP_PRECODE: return mimo::kPrecodeVariants;
    case MIMO_OP_GRAM_MF: return mimo::kGramVariants;
    case MIMO_OP_SLOT: return mimo::kSlotVariants;
  }
  return 0;
}

// Level unit of square 2^qam_bits-QAM with average energy es.
float qam_scale(float es, int qam_bits) {
  const int M = 1 << qam_bits;
  return std::sqrt(es * 3.0f / (2.0f * (float)(M - 1)));
}

#define CHECK(x)              \
  do {                        \
    const mimo_status st_ = (x); \
    if (st_ != MIMO_OK) return st_; \
  } while (0)

}  // namespace

namespace mimo {
void set_last_error(const char* msg) { std::snprintf(g_last_error, sizeof(g_last_error), "%s", msg); }

int num_compute_units() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v <= 0) {
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        v <= 0)
      v = 256;
    cache[dev].store(v, std::memory_order_relaxed);
  }
  return v;
}
}  // namespace mimo

extern "C" {

int mimo_tune_variant_count(int op) { return variant_count(op); }

const char* mimo_tune_variant_name(int op, int variant) {
  if (op == MIMO_OP_DETECT) {
    switch (variant) {
      case mimo::kDetectGeneric: return "generic";
      case mimo::kDetectStream: return "stream";
      case mimo::kDetectStreamSmall: return "stream-small";
      case mimo::kDetectPlain: return "plain";
      case mimo::kDetectRing: return "ring";
      case mimo::kDetectSplit: return "split";
      case mimo::kDetectValu: return "stream-valu";
      case mimo::kDetectX3: return "stream-x3";
    }
  } else if (op == MIMO_OP_PRECODE) {
    switch (variant) {
      case mimo::kPrecodeGeneric: return "generic";
      case mimo::kPrecodeStream: return "stream";
      case mimo::kPrecodeStreamSmall: return "stream-small";
      case mimo::kPrecodeResident: return "resident";
      case mimo::kPrecodeSplit: return "split";
      case mimo::kPrecodeX3: return "x3";
    }
  } else if (op == MIMO_OP_GRAM_MF) {
    switch (variant) {
      case mimo::kGramGeneric: return "generic";
      case mimo::kGramStream: return "stream";
    }
  } else if (op == MIMO_OP_SLOT) {
    switch (variant) {
      case mimo::kSlotSeparate: return "separate";
      case mimo::kSlotFused: return "fused";
      case mimo::kSlotFusedX3: return "fused-x3";
    }
  }
  return nullptr;
}

mimo_status mimo_tune_set(int op, int user_class, int in_dtype, int variant, int blocks_per_cu) {
  g_last_error[0] = 0;
  if (op < 0 || op >= kOps) return fail(MIMO_EINVAL, "op=%d unknown", op);
  if (user_class < 0 || user_class >= kUClasses)
    return fail(MIMO_EINVAL, "user_class=%d outside [0, %d)", user_class, kUClasses);
  if (in_dtype < 0 || in_dtype >= kDtypes) return fail(MIMO_EINVAL, "in_dtype=%d unknown", in_dtype);
  if (variant < 0 || variant >= variant_count(op))
    return fail(MIMO_EINVAL, "variant=%d outside [0, %d)", variant, variant_count(op));
  if (blocks_per_cu < 0 || blocks_per_cu > 64)
    return fail(MIMO_EINVAL, "blocks_per_cu=%d outside [0, 64]", blocks_per_cu);
  sched_defaults();
  g_sched[op][user_class][in_dtype].store(pack(variant, blocks_per_cu));
  return MIMO_OK;
}

mimo_status mimo_tune_get(int op, int user_class, int in_dtype, int* variant, int* blocks_per_cu) {
  g_last_error[0] = 0;
  if (op < 0 || op >= kOps || user_class < 0 || user_class >= kUClasses || in_dtype < 0 ||
      in_dtype >= kDtypes || !variant || !blocks_per_cu)
    return fail(MIMO_EINVAL, "bad tune_get arguments");
  const mimo::Schedule s = get_sched(op, user_class == 0 ? 16 : 32, in_dtype);
  *variant = s.variant;
  *blocks_per_cu = s.blocks_per_cu;
  return MIMO_OK;
}


const char* mimo_version(void) { return "mimo_cg 0.1 gfx950"; }

const char* mimo_last_error(void) { return g_last_error; }

const char* mimo_status_string(mimo_status status) {
  switch (status) {
    case MIMO_OK: return "ok";
    case MIMO_EINVAL: return "invalid argument";
    case MIMO_EUNSUPPORTED: return "unsupported configuration";
    case MIMO_EWORKSPACE: return "workspace missing or too small";
    case MIMO_EHIP: return "HIP runtime error";
  }
  return "unknown status";
}

size_t mimo_workspace_bytes(const mimo_shape* shape, int op, int sinr_mode) {
  (void)shape;
  (void)op;
  (void)sinr_mode;
  return 0;   // every kernel keeps its per-subcarrier state in LDS / registers
}

mimo_status mimo_gram_mf(const mimo_shape* shape, const void* H, const void* Y, int in_dtype, float reg,
                 void* A, void* b, void* stream) {
  g_last_error[0] = 0;
  CHECK(check_shape(shape, false, MIMO_MAX_USERS));
  CHECK(check_dtype(in_dtype, shape->B));
  CHECK(check_wide(shape->U, in_dtype));
  if (!(reg >= 0.f) || !std::isfinite(reg)) return fail(MIMO_EINVAL, "reg=%g must be >= 0", reg);
  CHECK(check_ptr(H, "H", true));
  CHECK(check_ptr(Y, "Y", false));
  CHECK(check_ptr(A, "A", true));
  CHECK(check_ptr(b, "b", false));
  if (b && !Y) return fail(MIMO_EINVAL, "b requested without Y");
  if (shape->n_sc == 0) return MIMO_OK;
  mimo::GramParams p{H, Y, shape->B, shape->U, shape->S, shape->n_sc, reg, (float2*)A, (float2*)b};
  if (shape->U > MIMO_MAX_USERS_COMMON)
    return hip_status(mimo::launch_gram_mf_wide(p, (hipStream_t)stream), "gram_mf launch");
  return hip_status(mimo::launch_gram_mf(p, in_dtype, get_sched(MIMO_OP_GRAM_MF, shape->U, in_dtype),
                                         (hipStream_t)stream),
                    "gram_mf launch");
}

mimo_status mimo_detect_cg(const mimo_shape* shape, const void* H, const void* Y, int in_dtype, float n0,
                   float es, int qam_bits, int sinr_mode, int scalar_prec, float* llr, void* xhat,
                   float* mu, float* sinr, void* workspace, size_t workspace_bytes,
                   void* stream) {
  g_last_error[0] = 0;
  CHECK(check_shape(shape, true, MIMO_MAX_USERS));
  CHECK(check_dtype(in_dtype, shape->B));
  CHECK(check_wide(shape->U, in_dtype));
  if (!(n0 > 0.f) || !std::isfinite(n0)) return fail(MIMO_EINVAL, "n0=%g must be > 0", n0);
  if (!(es > 0.f) || !std::isfinite(es)) return fail(MIMO_EINVAL, "es=%g must be > 0", es);
  if (qam_bits != 2 && qam_bits != 4 && qam_bits != 6 && qam_bits != 8)
    return fail(MIMO_EUNSUPPORTED, "qam_bits=%d not in {2,4,6,8}", qam_bits);
  if (sinr_mode != MIMO_SINR_APPROX && sinr_mode != MIMO_SINR_EXACT)
    return fail(MIMO_EINVAL, "sinr_mode=%d unknown", sinr_mode);
  if (sinr_mode == MIMO_SINR_EXACT && shape->U > MIMO_MAX_USERS_COMMON)
    return fail(MIMO_EUNSUPPORTED, "exact SINR with U=%d > %d", shape->U, MIMO_MAX_USERS_COMMON);
  if (scalar_prec != MIMO_SCALAR_F32 && scalar_prec != MIMO_SCALAR_F64)
    return fail(MIMO_EINVAL, "scalar_prec=%d unknown", scalar_prec);
  CHECK(check_ptr(H, "H", true));
  CHECK(check_ptr(Y, "Y", true));
  CHECK(check_ptr(llr, "llr", true));
  CHECK(check_ptr(xhat, "xhat", false));
  CHECK(check_ptr(mu, "mu", false));
  CHECK(check_ptr(sinr, "sinr", false));
  const size_t need = mimo_workspace_bytes(shape, MIMO_OP_DETECT, sinr_mode);
  if (need > 0 && (!workspace || workspace_bytes < need))
    return fail(MIMO_EWORKSPACE, "workspace needs %zu bytes", need);
  if (shape->n_sc == 0) return MIMO_OK;
  const float scale = qam_scale(es, qam_bits);
  mimo::DetectParams p{H, Y, shape->B, shape->U, shape->S, shape->K, shape->n_sc,
                       n0 / es, n0, es, scale, 1.0f / scale,
                       llr, (float2*)xhat, mu, sinr};
  const int f64 = scalar_prec == MIMO_SCALAR_F64;
  hipError_t e = sinr_mode == MIMO_SINR_EXACT
                     ? mimo::launch_detect_exact(p, in_dtype, f64, qam_bits, (hipStream_t)stream)
                 : shape->U > MIMO_MAX_USERS_COMMON
                     ? mimo::launch_detect_wide(p, f64, qam_bits, (hipStream_t)stream)
                     : mimo::launch_detect_approx(p, in_dtype, f64, qam_bits,
                                                  get_sched(MIMO_OP_DETECT, shape->U, in_dtype),
                                                  (hipStream_t)stream);
  return hip_status(e, "detect_cg launch");
}

mimo_status mimo_precode_cg(const mimo_shape* shape, const void* H, const void* T, int in_dtype,
                    float beta, int normalize, int scalar_prec, void* Q, float* qnorm,
                    void* workspace, size_t workspace_bytes, void* stream) {
  g_last_error[0] = 0;
  CHECK(check_shape(shape, true, MIMO_MAX_USERS));
  CHECK(check_dtype(in_dtype, shape->B));
  CHECK(check_wide(shape->U, in_dtype));
  if (!(beta >= 0.f) || !std::isfinite(beta)) return fail(MIMO_EINVAL, "beta=%g must be >= 0", beta);
  if (scalar_prec != MIMO_SCALAR_F32 && scalar_prec != MIMO_SCALAR_F64)
    return fail(MIMO_EINVAL, "scalar_prec=%d unknown", scalar_prec);
  CHECK(check_ptr(H, "H", true));
  CHECK(check_ptr(T, "T", true));
  CHECK(check_ptr(Q, "Q", true));
  CHECK(check_ptr(qnorm, "qnorm", false));
  const size_t need = mimo_workspace_bytes(shape, MIMO_OP_PRECODE, 0);
  if (need > 0 && (!workspace || workspace_bytes < need))
    return fail(MIMO_EWORKSPACE, "workspace needs %zu bytes", need);
  if (shape->n_sc == 0) return MIMO_OK;
  mimo::PrecodeParams p{H, (const float2*)T, shape->B, shape->U, shape->S, shape->K,
                        shape->n_sc, beta, normalize ? 1 : 0, (float2*)Q, qnorm};
  if (shape->U > MIMO_MAX_USERS_COMMON)
    return hip_status(mimo::launch_precode_wide(p, scalar_prec == MIMO_SCALAR_F64,
                                                (hipStream_t)stream),
                      "precode_cg launch");
  return hip_status(mimo::launch_precode(p, in_dtype, scalar_prec == MIMO_SCALAR_F64,
                                         get_sched(MIMO_OP_PRECODE, shape->U, in_dtype),
                                         (hipStream_t)stream),
                    "precode_cg launch");
}

mimo_status mimo_detect_precode_cg(const mimo_shape* ul, const mimo_shape* dl, const void* H,
                           const void* Y, const void* T, int in_dtype, float n0, float es,
                           int qam_bits, float beta, int normalize, int scalar_prec,
                           float* llr, void* xhat, float* mu, float* sinr, void* Q,
                           float* qnorm, void* stream) {
  g_last_error[0] = 0;
  CHECK(check_shape(ul, true, MIMO_MAX_USERS));
  CHECK(check_shape(dl, true, MIMO_MAX_USERS));
  if (ul->B != dl->B || ul->U != dl->U || ul->n_sc != dl->n_sc)
    return fail(MIMO_EINVAL, "uplink (B=%d, U=%d, n_sc=%lld) and downlink (B=%d, U=%d, "
                "n_sc=%lld) shapes must share the channel", ul->B, ul->U, (long long)ul->n_sc,
                dl->B, dl->U, (long long)dl->n_sc);
  CHECK(check_dtype(in_dtype, ul->B));
  CHECK(check_wide(ul->U, in_dtype));
  if (!(n0 > 0.f) || !std::isfinite(n0)) return fail(MIMO_EINVAL, "n0=%g must be > 0", n0);
  if (!(es > 0.f) || !std::isfinite(es)) return fail(MIMO_EINVAL, "es=%g must be > 0", es);
  if (qam_bits != 2 && qam_bits != 4 && qam_bits != 6 && qam_bits != 8)
    return fail(MIMO_EUNSUPPORTED, "qam_bits=%d not in {2,4,6,8}", qam_bits);
  if (!(beta >= 0.f) || !std::isfinite(beta)) return fail(MIMO_EINVAL, "beta=%g must be >= 0", beta);
  if (scalar_prec != MIMO_SCALAR_F32 && scalar_prec != MIMO_SCALAR_F64)
    return fail(MIMO_EINVAL, "scalar_prec=%d unknown", scalar_prec);
  CHECK(check_ptr(H, "H", true));
  CHECK(check_ptr(Y, "Y", true));
  CHECK(check_ptr(T, "T", true));
  CHECK(check_ptr(llr, "llr", true));
  CHECK(check_ptr(xhat, "xhat", false));
  CHECK(check_ptr(mu, "mu", false));
  CHECK(check_ptr(sinr, "sinr", false));
  CHECK(check_ptr(Q, "Q", true));
  CHECK(check_ptr(qnorm, "qnorm", false));
  if (ul->n_sc == 0) return MIMO_OK;
  const float scale = qam_scale(es, qam_bits);
  mimo::SlotParams p{
      mimo::DetectParams{H, Y, ul->B, ul->U, ul->S, ul->K, ul->n_sc, n0 / es, n0, es, scale,
                         1.0f / scale, llr, (float2*)xhat, mu, sinr},
      mimo::PrecodeParams{H, (const float2*)T, dl->B, dl->U, dl->S, dl->K, dl->n_sc, beta,
                          normalize ? 1 : 0, (float2*)Q, qnorm}};
  const int f64 = scalar_prec == MIMO_SCALAR_F64;
  if (ul->U > MIMO_MAX_USERS_COMMON) {
    CHECK(hip_status(mimo::launch_detect_wide(p.ul, f64, qam_bits, (hipStream_t)stream),
                     "detect_precode_cg: detection launch"));
    return hip_status(mimo::launch_precode_wide(p.dl, f64, (hipStream_t)stream),
                      "detect_precode_cg: precoding launch");
  }
  const mimo::Schedule sch = get_sched(MIMO_OP_SLOT, ul->U, in_dtype);
  if ((sch.variant == mimo::kSlotFused || sch.variant == mimo::kSlotFusedX3) &&
      mimo::slot_eligible(p, in_dtype))
    return hip_status(mimo::launch_slot(p, in_dtype, f64, qam_bits, sch, (hipStream_t)stream),
                      "detect_precode_cg launch");
  CHECK(hip_status(mimo::launch_detect_approx(p.ul, in_dtype, f64, qam_bits,
                                              get_sched(MIMO_OP_DETECT, ul->U, in_dtype),
                                              (hipStream_t)stream),
                   "detect_precode_cg: detection launch"));
  return hip_status(mimo::launch_precode(p.dl, in_dtype, f64,
                                         get_sched(MIMO_OP_PRECODE, dl->U, in_dtype),
                                         (hipStream_t)stream),
                    "detect_precode_cg: precoding launch");
}

// ---------------------------------------------------------------- Sec. III-F
// Shared validation of the detection entry points; fills p on success.
static mimo_status detect_args(const mimo_shape* shape, bool need_k, const void* H, const void* Y,
                       int in_dtype, float n0, float es, int qam_bits, float* llr, void* xhat,
                       float* mu, float* sinr, mimo::DetectParams& p) {
  CHECK(check_shape(shape, need_k));
  CHECK(check_dtype(in_dtype, shape->B));
  if (!(n0 > 0.f) || !std::isfinite(n0)) return fail(MIMO_EINVAL, "n0=%g must be > 0", n0);
  if (!(es > 0.f) || !std::isfinite(es)) return fail(MIMO_EINVAL, "es=%g must be > 0", es);
  if (qam_bits != 2 && qam_bits != 4 && qam_bits != 6 && qam_bits != 8)
    return fail(MIMO_EUNSUPPORTED, "qam_bits=%d not in {2,4,6,8}", qam_bits);
  CHECK(check_ptr(H, "H", true));
  CHECK(check_ptr(Y, "Y", true));
  CHECK(check_ptr(llr, "llr", true));
  CHECK(check_ptr(xhat, "xhat", false));
  CHECK(check_ptr(mu, "mu", false));
  CHECK(check_ptr(sinr, "sinr", false));
  const float scale = qam_scale(es, qam_bits);
  p = mimo::DetectParams{H, Y, shape->B, shape->U, shape->S, need_k ? shape->K : 1, shape->n_sc,
                         n0 / es, n0, es, scale, 1.0f / scale,
                         llr, (float2*)xhat, mu, sinr};
  return MIMO_OK;
}

static mimo_status precode_args(const mimo_shape* shape, bool need_k, const void* H, const void* T,
                        int in_dtype, float beta, int normalize, void* Q, float* qnorm,
                        mimo::PrecodeParams& p) {
  CHECK(check_shape(shape, need_k));
  CHECK(check_dtype(in_dtype, shape->B));
  if (!(beta >= 0.f) || !std::isfinite(beta)) return fail(MIMO_EINVAL, "beta=%g must be >= 0", beta);
  CHECK(check_ptr(H, "H", true));
  CHECK(check_ptr(T, "T", true));
  CHECK(check_ptr(Q, "Q", true));
  CHECK(check_ptr(qnorm, "qnorm", false));
  p = mimo::PrecodeParams{H, (const float2*)T, shape->B, shape->U, shape->S,
                          need_k ? shape->K : 1, shape->n_sc, beta, normalize ? 1 : 0,
                          (float2*)Q, qnorm};
  return MIMO_OK;
}

static mimo_status detect_inverse(const mimo_shape* shape, int method, const void* H, const void* Y,
                          int in_dtype, float n0, float es, int qam_bits, float* llr, void* xhat,
                          float* mu, float* sinr, void* stream) {
  g_last_error[0] = 0;
  mimo::DetectParams p;
  CHECK(detect_args(shape, method == mimo::kInvNeumann, H, Y, in_dtype, n0, es, qam_bits, llr,
                    xhat, mu, sinr, p));
  if (shape->n_sc == 0) return MIMO_OK;
  return hip_status(mimo::launch_detect_inverse(p, method, in_dtype, qam_bits,
                                                (hipStream_t)stream),
                    method == mimo::kInvCholesky ? "detect_cholesky launch"
                                                 : "detect_neumann launch");
}

static mimo_status precode_inverse(const mimo_shape* shape, int method, const void* H, const void* T,
                           int in_dtype, float beta, int normalize, void* Q, float* qnorm,
                           void* stream) {
  g_last_error[0] = 0;
  mimo::PrecodeParams p;
  CHECK(precode_args(shape, method == mimo::kInvNeumann, H, T, in_dtype, beta, normalize, Q,
                     qnorm, p));
  if (shape->n_sc == 0) return MIMO_OK;
  return hip_status(mimo::launch_precode_inverse(p, method, in_dtype, (hipStream_t)stream),
                    method == mimo::kInvCholesky ? "precode_cholesky launch"
                                                 : "precode_neumann launch");
}

mimo_status mimo_detect_cholesky(const mimo_shape* shape, const void* H, const void* Y, int in_dtype,
                         float n0, float es, int qam_bits, float* llr, void* xhat, float* mu,
                         float* sinr, void* stream) {
  return detect_inverse(shape, mimo::kInvCholesky, H, Y, in_dtype, n0, es, qam_bits, llr, xhat,
                        mu, sinr, stream);
}

mimo_status mimo_detect_neumann(const mimo_shape* shape, const void* H, const void* Y, int in_dtype,
                        float n0, float es, int qam_bits, float* llr, void* xhat, float* mu,
                        float* sinr, void* stream) {
  return detect_inverse(shape, mimo::kInvNeumann, H, Y, in_dtype, n0, es, qam_bits, llr, xhat,
                        mu, sinr, stream);
}

mimo_status mimo_precode_cholesky(const mimo_shape* shape, const void* H, const void* T, int in_dtype,
                          float beta, int normalize, void* Q, float* qnorm, void* stream) {
  return precode_inverse(shape, mimo::kInvCholesky, H, T, in_dtype, beta, normalize, Q, qnorm,
                         stream);
}

mimo_status mimo_precode_neumann(const mimo_shape* shape, const void* H, const void* T, int in_dtype,
                         float beta, int normalize, void* Q, float* qnorm, void* stream) {
  return precode_inverse(shape, mimo::kInvNeumann, H, T, in_dtype, beta, normalize, Q, qnorm,
                         stream);
}

// ---------------------------------------------------------------- Sec. III-E
// CGLS keeps antenna-length vectors of 16 right-hand sides in LDS.
static mimo_status check_cgls_lds(int B, bool precode) {
  int dev = 0, limit = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&limit, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
      limit <= 0)
    limit = 65536;
  const size_t need = mimo::cgls_lds_bytes(B, precode) + 8192;   // + static LDS
  if (need > (size_t)limit)
    return fail(MIMO_EUNSUPPORTED, "CGLS %s with B=%d needs %zu bytes of LDS per block (limit %d)",
                precode ? "precoding" : "detection", B, need, limit);
  return MIMO_OK;
}

mimo_status mimo_detect_cgls(const mimo_shape* shape, const void* H, const void* Y, int in_dtype,
                     float n0, float es, int qam_bits, int scalar_prec, float* llr, void* xhat,
                     float* mu, float* sinr, void* stream) {
  g_last_error[0] = 0;
  mimo::DetectParams p;
  CHECK(detect_args(shape, true, H, Y, in_dtype, n0, es, qam_bits, llr, xhat, mu, sinr, p));
  if (scalar_prec != MIMO_SCALAR_F32 && scalar_prec != MIMO_SCALAR_F64)
    return fail(MIMO_EINVAL, "scalar_prec=%d unknown", scalar_prec);
  if (shape->n_sc == 0) return MIMO_OK;
  CHECK(check_cgls_lds(shape->B, false));
  return hip_status(mimo::launch_detect_cgls(p, in_dtype, scalar_prec == MIMO_SCALAR_F64,
                                             qam_bits, (hipStream_t)stream),
                    "detect_cgls launch");
}

mimo_status mimo_precode_cgls(const mimo_shape* shape, const void* H, const void* T, int in_dtype,
                      float beta, int normalize, int scalar_prec, void* Q, float* qnorm,
                      void* stream) {
  g_last_error[0] = 0;
  mimo::PrecodeParams p;
  CHECK(precode_args(shape, true, H, T, in_dtype, beta, normalize, Q, qnorm, p));
  if (scalar_prec != MIMO_SCALAR_F32 && scalar_prec != MIMO_SCALAR_F64)
    return fail(MIMO_EINVAL, "scalar_prec=%d unknown", scalar_prec);
  if (shape->n_sc == 0) return MIMO_OK;
  CHECK(check_cgls_lds(shape->B, true));
  return hip_status(mimo::launch_precode_cgls(p, in_dtype, scalar_prec == MIMO_SCALAR_F64,
                                              (hipStream_t)stream),
                    "precode_cgls launch");
}

// ---------------------------------------------------------------- cached Gram
mimo_status mimo_detect_cg_gram(const mimo_shape* shape, const void* G, const void* H,
                                const void* Y, int in_dtype, float n0, float es, int qam_bits,
                                int scalar_prec, float* llr, void* xhat, float* mu, float* sinr,
                                void* stream) {
  g_last_error[0] = 0;
  mimo::DetectParams p;
  CHECK(detect_args(shape, true, H, Y, in_dtype, n0, es, qam_bits, llr, xhat, mu, sinr, p));
  if (scalar_prec != MIMO_SCALAR_F32 && scalar_prec != MIMO_SCALAR_F64)
    return fail(MIMO_EINVAL, "scalar_prec=%d unknown", scalar_prec);
  CHECK(check_ptr(G, "G", true));
  if (shape->n_sc == 0) return MIMO_OK;
  p.gram = (const float2*)G;
  return hip_status(mimo::launch_detect_approx(p, in_dtype, scalar_prec == MIMO_SCALAR_F64,
                                               qam_bits, get_sched(MIMO_OP_DETECT, shape->U,
                                                                   in_dtype),
                                               (hipStream_t)stream),
                    "detect_cg_gram launch");
}

mimo_status mimo_precode_cg_gram(const mimo_shape* shape, const void* G, const void* H,
                                 const void* T, int in_dtype, float beta, int normalize,
                                 int scalar_prec, void* Q, float* qnorm, void* stream) {
  g_last_error[0] = 0;
  mimo::PrecodeParams p;
  CHECK(precode_args(shape, true, H, T, in_dtype, beta, normalize, Q, qnorm, p));
  if (scalar_prec != MIMO_SCALAR_F32 && scalar_prec != MIMO_SCALAR_F64)
    return fail(MIMO_EINVAL, "scalar_prec=%d unknown", scalar_prec);
  CHECK(check_ptr(G, "G", true));
  if (shape->n_sc == 0) return MIMO_OK;
  p.gram = (const float2*)G;
  return hip_status(mimo::launch_precode(p, in_dtype, scalar_prec == MIMO_SCALAR_F64,
                                         get_sched(MIMO_OP_PRECODE, shape->U, in_dtype),
                                         (hipStream_t)stream),
                    "precode_cg_gram launch");
}

// Prefix the message of a failed check with the frame index.
static mimo_status frame_fail(int status, int i) {
  char msg[sizeof(g_last_error)];
  std::memcpy(msg, g_last_error, sizeof(msg));
  return fail(status, "frame %d: %s", i, msg);
}

static mimo_status check_frame(const mimo_frame& f, int i, int in_dtype, bool detect) {
  mimo_shape sh{f.B, f.U, f.S, f.K, f.n_sc};
  mimo_status st = check_shape(&sh, true);
  if (st == MIMO_OK) st = check_dtype(in_dtype, f.B);
  if (st == MIMO_OK) st = check_ptr(f.H, "H", true);
  if (st == MIMO_OK) st = check_ptr(f.Y, detect ? "Y" : "T", true);
  if (st == MIMO_OK) st = check_ptr(f.out, detect ? "llr" : "Q", true);
  if (st == MIMO_OK) st = check_ptr(f.out2, "out2", false);
  if (st == MIMO_OK) st = check_ptr(f.gram, "gram", false);
  if (st != MIMO_OK) return frame_fail(st, i);
  if (detect) {
    if (!(f.n0 > 0.f) || !std::isfinite(f.n0) || !(f.es > 0.f) || !std::isfinite(f.es))
      return fail(MIMO_EINVAL, "frame %d: n0=%g es=%g must be > 0", i, f.n0, f.es);
  } else if (!(f.beta >= 0.f) || !std::isfinite(f.beta)) {
    return fail(MIMO_EINVAL, "frame %d: beta=%g must be >= 0", i, f.beta);
  }
  return MIMO_OK;
}

static mimo_status build_batch(const mimo_frame* frames, int n_frames, int in_dtype, bool detect,
                       int qam_bits, mimo::BatchArgs& a, int& max_u) {
  if (!frames && n_frames > 0) return fail(MIMO_EINVAL, "frames is NULL");
  if (n_frames < 0 || n_frames > MIMO_MAX_BATCH)
    return fail(MIMO_EINVAL, "n_frames=%d outside [0, %d]", n_frames, MIMO_MAX_BATCH);
  std::memset(&a, 0, sizeof(a));
  max_u = 1;
  for (int i = 0; i < n_frames; ++i) {
    const mimo_frame& f = frames[i];
    CHECK(check_frame(f, i, in_dtype, detect));
    if (f.n_sc == 0) continue;
    mimo::FrameArgs& d = a.f[a.n++];
    d.H = f.H;
    d.Y = f.Y;
    d.out = f.out;
    d.out2 = f.out2;
    d.gram = f.gram;
    d.sc_begin = a.total;
    d.n_sc = f.n_sc;
    d.B = f.B;
    d.U = f.U;
    d.S = f.S;
    d.K = f.K;
    if (detect) {
      d.n0 = f.n0;
      d.es = f.es;
      d.reg = f.n0 / f.es;
      d.scale = qam_scale(f.es, qam_bits);
      d.inv_scale = 1.0f / d.scale;
    } else {
      d.beta = f.beta;
      d.normalize = f.normalize ? 1 : 0;
    }
    a.total += f.n_sc;
    if (f.U > max_u) max_u = f.U;
  }
  return MIMO_OK;
}

mimo_status mimo_detect_cg_batch(const mimo_frame* frames, int n_frames, int in_dtype, int qam_bits,
                         int scalar_prec, void* stream) {
  g_last_error[0] = 0;
  if (qam_bits != 2 && qam_bits != 4 && qam_bits != 6 && qam_bits != 8)
    return fail(MIMO_EUNSUPPORTED, "qam_bits=%d not in {2,4,6,8}", qam_bits);
  if (scalar_prec != MIMO_SCALAR_F32 && scalar_prec != MIMO_SCALAR_F64)
    return fail(MIMO_EINVAL, "scalar_prec=%d unknown", scalar_prec);
  static thread_local mimo::BatchArgs a;
  int max_u = 1;
  CHECK(build_batch(frames, n_frames, in_dtype, true, qam_bits, a, max_u));
  if (a.n == 0) return MIMO_OK;
  return hip_status(mimo::launch_detect_batch(a, max_u, in_dtype,
                                              scalar_prec == MIMO_SCALAR_F64, qam_bits,
                                              get_sched(MIMO_OP_DETECT, max_u, in_dtype),
                                              (hipStream_t)stream),
                    "detect_cg_batch launch");
}

mimo_status mimo_precode_cg_batch(const mimo_frame* frames, int n_frames, int in_dtype,
                          int scalar_prec, void* stream) {
  g_last_error[0] = 0;
  if (scalar_prec != MIMO_SCALAR_F32 && scalar_prec != MIMO_SCALAR_F64)
    return fail(MIMO_EINVAL, "scalar_prec=%d unknown", scalar_prec);
  static thread_local mimo::BatchArgs a;
  int max_u = 1;
  CHECK(build_batch(frames, n_frames, in_dtype, false, 0, a, max_u));
  if (a.n == 0) return MIMO_OK;
  return hip_status(mimo::launch_precode_batch(a, max_u, in_dtype,
                                               scalar_prec == MIMO_SCALAR_F64,
                                               get_sched(MIMO_OP_PRECODE, max_u, in_dtype),
                                               (hipStream_t)stream),
                    "precode_cg_batch launch");
}

mimo_status mimo_convert(const void* src, void* dst, int dst_dtype, int64_t n, int32_t R, int32_t C,
                 void* stream) {
  g_last_error[0] = 0;
  if (dst_dtype != MIMO_C16 && dst_dtype != MIMO_CBF16)
    return fail(MIMO_EINVAL, "dst_dtype=%d must be MIMO_C16 or MIMO_CBF16", dst_dtype);
  if (n < 0 || R < 8 || (R % 8) != 0 || C < 1)
    return fail(MIMO_EINVAL, "bad extents n=%lld R=%d C=%d (R must be a positive multiple of 8)",
                (long long)n, R, C);
  CHECK(check_ptr(src, "src", true));
  CHECK(check_ptr(dst, "dst", true));
  if (n == 0) return MIMO_OK;
  return hip_status(mimo::launch_convert((const float2*)src, (uint16_t*)dst, dst_dtype, n, R, C,
                                         (hipStream_t)stream),
                    "convert launch");
}

}  // extern "C"
