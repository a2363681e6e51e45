/*
 * mimo_serve.h -- C ABI of the native serving runtime on top of mimo_cg.h:
 * continuous batching of uplink (detection) and downlink (precoding) frames
 * of mixed shapes on one MI355X, admitted by an HBM budget.
 *
 * A frame is one OFDM frame of one channel: n_sc subcarrier systems of the
 * paper's problem statement (Sec. II-A uplink y = H_u x + n, Sec. II-B
 * downlink with H_d = H_u^H), each solved by Algorithm 1 exactly as the
 * mimo_cg.h entry points do (the server calls them).  Nothing here changes
 * the arithmetic: a frame's outputs are bitwise those of a single
 * mimo_detect_cg / mimo_precode_cg call on the same inputs (a GPU test
 * checks this alone and in a mix), also when the channel was registered with
 * its Gram matrix (mimo_server_register_channel_gram).
 *
 * Memory.  mimo_server_create allocates one device pool of cfg.hbm_budget
 * bytes; the server allocates nothing else on the device.  Registered
 * channels are the caller's device arrays; their bytes count against the
 * budget while registered.  Each admitted request takes its output buffers
 * (and, for 16-bit channels, a scratch copy of Y in the channel's storage
 * type) from the pool; the scratch returns at completion, the outputs when
 * the caller releases the request (mimo_server_release, or the deleter of a
 * DLPack tensor from mimo_server_dlpack).  Admission waits while
 * pool bytes in use + the new request's bytes + registered channel bytes
 * would exceed the budget, so device memory held by the server stays within
 * it.  Inputs (Y, T) are the caller's and must stay valid and unchanged
 * until the request completes.
 *
 * Scheduling.  Requests are admitted in arrival order.  When the queue head
 * fits, later queued requests of the same kernel class (direction, U <= 16
 * or U <= 32, storage type, QAM order, scalar precision, xhat requested)
 * that also fit join it, up to cfg.max_batch frames within cfg.lookahead
 * queue entries, in one batched launch on one of cfg.n_slots HIP streams
 * (default priority).  Exact-SINR uplink requests launch alone.  A
 * scheduler thread owns every launch; calls from other threads only queue
 * requests, read completions and release outputs.
 *
 * Times are seconds on the host's steady clock since mimo_server_create.
 * t_done is the completion of the request's launch, read from a HIP event
 * aligned to that clock at creation (best of several round trips).
 *
 * All functions return a mimo_status (mimo_cg.h); on failure
 * mimo_last_error() of the calling thread names the cause.
 */
#ifndef MIMO_SERVE_H
#define MIMO_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "mimo_cg.h"

#ifdef __cplusplus
extern "C" {
#endif

#define MIMO_SERVE_MAX_SLOTS 16

typedef struct mimo_server mimo_server;

typedef struct mimo_server_config {
  int64_t hbm_budget;  /* bytes: registered channels + pool in use; > 0 */
  int32_t n_slots;     /* launches in flight (HIP streams), 1 .. MIMO_SERVE_MAX_SLOTS */
  int32_t max_batch;   /* frames per launch, 1 .. MIMO_MAX_BATCH */
  int32_t lookahead;   /* queue entries scanned to fill a launch, >= 1 */
  int32_t paused;      /* 1: queue submissions until mimo_server_resume */
  int32_t keep_outputs;/* 1: completed requests hold their outputs until released;
                          0: outputs return to the pool at completion (completions
                          then carry NULL output pointers) */
} mimo_server_config;

typedef struct mimo_uplink_req {
  int64_t ch_id;       /* registered channel */
  const void* Y;       /* complex64 [n_sc][B][S], device, caller-owned */
  int32_t S, qam_bits, K;
  int32_t sinr_mode;   /* MIMO_SINR_APPROX (batched) or MIMO_SINR_EXACT (alone) */
  int32_t scalar_prec; /* MIMO_SCALAR_F32 / MIMO_SCALAR_F64 */
  int32_t want_xhat;   /* 1: also return xhat */
  float n0, es;        /* noise power N0 > 0 and symbol energy E_s > 0 */
} mimo_uplink_req;

typedef struct mimo_downlink_req {
  int64_t ch_id;
  const void* T;       /* complex64 [n_sc][U][S], device, caller-owned */
  int32_t S, K;
  int32_t normalize;   /* 1: s = q / ||q|| per vector (Sec. II-B) */
  int32_t scalar_prec;
  float beta;          /* regularization >= 0 (0: zero-forcing) */
} mimo_downlink_req;

typedef struct mimo_completion {
  int64_t req_id;
  int32_t status;      /* MIMO_OK, or the failed launch's status */
  int32_t kind;        /* 0 uplink, 1 downlink */
  double t_submit, t_admit, t_done;
  void* out;           /* uplink: float llr [n_sc][U][S][qam_bits]; downlink: complex64 Q [n_sc][B][S] */
  void* out2;          /* uplink: complex64 xhat [n_sc][U][S] or NULL; downlink: float qnorm [n_sc][S] */
  int64_t n_sc;
  int32_t B, U, S, qam_bits;
  int64_t solves;      /* n_sc * S subcarrier solves */
  int64_t llr_bits;    /* LLRs produced (uplink) */
} mimo_completion;

typedef struct mimo_server_stats {
  int64_t frames;              /* completed requests counted */
  double p50_ms, p99_ms, mean_ms;   /* latency t_done - max(t_submit, t_resume) */
  double frames_per_s, solves_per_s, llr_gbit_s;
  int64_t peak_bytes;          /* largest pool bytes in use + channel bytes seen */
  int64_t budget_waits;        /* queue heads that waited for budget */
  int64_t launches;            /* batched launches so far */
  double mean_batch;           /* frames per launch */
} mimo_server_stats;

/* Create a server on `device` (its HIP device index).  Allocates the pool,
 * the slot streams and a scheduler thread. */
int mimo_server_create(const mimo_server_config* cfg, int device, mimo_server** out);
/* Wait for every submitted request, stop the thread, free the pool.  Outputs
 * not yet released are freed with the pool. */
int mimo_server_destroy(mimo_server* s);

/* H: [n_sc][B][U] in storage type in_dtype (complex64, or the blocked
 * 16-bit layout of mimo_convert), device, caller-owned while registered.
 * Registering an id again replaces its channel; requests already submitted
 * keep the arrays registered when they were submitted, which must stay valid
 * until those requests complete. */
int mimo_server_register_channel(mimo_server* s, int64_t ch_id, const void* H, int in_dtype,
                                 int64_t n_sc, int32_t B, int32_t U);
/* The same with the channel's Gram matrix G = H^H H (Sec. II-A; the downlink's
 * H_d H_d^H by reciprocity, Sec. II-B): complex64 [n_sc][U][U] as
 * mimo_gram_mf writes it with reg = 0 from this H, device, caller-owned and
 * complete (like H) before the first request on the channel is submitted.
 * Uplink frames with the approximate SINR and downlink frames of channels
 * with U > 8 then run as mimo_detect_cg_gram / mimo_precode_cg_gram, which
 * skip the Gram's products; their outputs are bitwise those of the direct
 * calls.  Exact-SINR frames and channels with U <= 8 ignore G.  G's bytes
 * count against the budget with H's.  G = NULL is mimo_server_register_channel. */
int mimo_server_register_channel_gram(mimo_server* s, int64_t ch_id, const void* H,
                                      const void* G, int in_dtype, int64_t n_sc, int32_t B,
                                      int32_t U);
int mimo_server_unregister_channel(mimo_server* s, int64_t ch_id);

/* Queue a request; *req_id receives its id (> 0).  `ready_stream` (a
 * hipStream_t, or NULL): the inputs are complete once the work queued on it
 * so far is; the launch waits for that.  Requests that can never fit the
 * budget are refused with MIMO_EUNSUPPORTED. */
int mimo_server_submit_uplink(mimo_server* s, const mimo_uplink_req* r, void* ready_stream,
                              int64_t* req_id);
int mimo_server_submit_downlink(mimo_server* s, const mimo_downlink_req* r, void* ready_stream,
                                int64_t* req_id);

/* Up to `max` completions not yet returned, waiting up to timeout_us
 * microseconds for the first (0: do not wait).  Returns the count (>= 0) or
 * a negative status. */
int mimo_server_poll(mimo_server* s, mimo_completion* out, int max, int64_t timeout_us);
/* Return a completed request's output buffers to the pool (cfg.keep_outputs). */
int mimo_server_release(mimo_server* s, int64_t req_id);
/* A DLPack tensor (DLManagedTensor*, device type ROCm) over output `which`
 * (0: out, 1: out2) of a completed request.  The request's buffers return
 * to the pool when every tensor handed out has been deleted and, if no
 * tensor was requested, at mimo_server_release. */
int mimo_server_dlpack(mimo_server* s, int64_t req_id, int which, void** managed);

int mimo_server_pause(mimo_server* s);
int mimo_server_resume(mimo_server* s);
/* Block until the queue is empty and nothing is in flight (timeout_us < 0:
 * no limit); MIMO_EINVAL on timeout. */
int mimo_server_drain(mimo_server* s, int64_t timeout_us);
/* Statistics of completed requests, leaving out the first `skip` by
 * submission order; reset = 1 clears the records afterwards. */
int mimo_server_stats_get(mimo_server* s, int64_t skip, int reset, mimo_server_stats* out);
/* Bytes of registered channels and of pool memory in use. */
int mimo_server_memory(mimo_server* s, int64_t* channel_bytes, int64_t* pool_bytes);

#ifdef __cplusplus
}
#endif

#endif /* MIMO_SERVE_H */
