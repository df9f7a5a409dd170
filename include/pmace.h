/*
 * pmace.h -- C ABI of the MI355X PMACE library (libpmace.so).
 *
 * PMACE (Projected Multi-Agent Consensus Equilibrium) reconstructs a complex
 * object x (N1 x N2) from ptychographic intensities z_j (Np x Np, one per
 * scan position j = 0..J-1) measured through a known complex probe d
 * (Np x Np), Sec. II eq. (1).  One iteration of the library is one pass of
 * the loop body of Alg. 1 over all J positions:
 *     w <- F(v);   z <- G(2w - v);   v <- v + 2 rho (z - w)
 * with the data agent F_j of eq. (9) and the consensus operator G of
 * eq. (11) (weights |d|^kappa, normaliser Lambda = sum_j P_j^t |d|^kappa).
 *
 * Conventions shared by every entry point:
 *   - Complex arrays are interleaved (re, im) float32 ("c64"), row-major.
 *   - Array arguments are DEVICE pointers unless stated otherwise.
 *   - Calls are stream-ordered on the HIP stream given to pmace_init and
 *     return as soon as the work is queued; device-side failures (a fault,
 *     a non-finite state) surface at the next pmace_sync().
 *   - All persistent state lives in a caller-owned device workspace of
 *     pmace_footprint() bytes; the library never allocates device memory.
 *     It keeps a small host-side context (malloc) per reconstruction.
 *   - No C++ exception crosses this boundary; every call returns a status.
 *   - A context is not thread-safe; distinct contexts are.
 */
#ifndef PMACE_H
#define PMACE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PMACE_OK = 0,
  PMACE_EINVAL = 1,        /* bad argument: size, range, NaN/Inf, negative intensity, position */
  PMACE_EUNSUPPORTED = 2,  /* valid per the paper but not built here (an Np without a transform here) */
  PMACE_ENOMEM = 3,        /* workspace smaller than pmace_footprint() */
  PMACE_EDEVICE = 4,       /* a HIP call failed (launch, copy, sync) */
  PMACE_ESTATE = 5,        /* call out of order (e.g. NULL or destroyed context) */
  PMACE_EDIVERGED = 6      /* the consensus image became non-finite */
} pmace_status;

/* Intensities are stored with the zero frequency at the array centre
 * (fftshift layout); they are reordered once at init. */
#define PMACE_CENTERED_DC 0x1u
/* Agent variant (all are exact algebra of eq. (9) and Alg. 1, and their
 * results agree to rounding, except in spectral bins that are exactly zero in
 * exact arithmetic, e.g. a probe symmetric about its half-pixel centre seen
 * through the flat start: the whole-patch and three-pass transforms return
 * those zeros exactly, the split agent's leave rounding noise there, and
 * eq. (9)'s "0 where W = 0" then does not act).  np <= 128 runs the
 * whole-patch agent; np = 160, 192, 256 the three-pass agent, which stages
 * each chunk's spectra through memory twice, or:
 *   - np = 160, 192 or 256: each state kept as the DFTs of its rows
 *     ("row-spectrum" agent): the column pass writes the new state itself,
 *     and the consensus inverts the rows it sums, so each chunk's spectra are
 *     staged once instead of twice (PMACE with a probe without exact zeros,
 *     where eq. (9)'s d = 0 rule acts per pixel; SHARP+ with any probe);
 *   - np = 128, 192 or 256, PMACE with a probe without exact zeros: each
 *     state kept as the four coset blocks of the top radix-2 step of its 2-D
 *     DFT ("split" agent): every agent then runs on (np/2)^2 blocks held on
 *     chip and no spectrum is staged, at the price of reading the probe and
 *     the consensus window once per block.
 * Which sides use which by default is a build choice (timed by the tuner).
 *   PMACE_STAGED_AGENT:  the three-pass agent (np > 128), never the split one.
 *   PMACE_SPLIT_AGENT:   the split agent wherever it applies.
 *   PMACE_ROWSPEC_AGENT: the row-spectrum agent wherever it applies.
 * Setting more than one of them is EINVAL. */
#define PMACE_STAGED_AGENT 0x2u
#define PMACE_SPLIT_AGENT 0x4u
#define PMACE_ROWSPEC_AGENT 0x8u

/* Iteration run by a context (pmace_params.method). */
#define PMACE_METHOD_PMACE 0      /* Alg. 1: Mann iteration of T = (2G - I)(2F - I) */
#define PMACE_METHOD_SHARP_PLUS 1 /* Alg. 2: SHARP+ on frames s_j = D P_j x (Sec. III-B) */

typedef struct {
  int32_t n1, n2;     /* object grid N1 x N2 (Sec. II); n1, n2 >= np */
  int32_t np;         /* probe / patch side Np; this build runs 32, 48, 64, 96, 128, 160, 192,
                         256 (radix 2, 3 and 5 transforms) */
  int32_t num_pos;    /* J >= 1 scan positions */
  float alpha;        /* >= 0: noise-to-signal weight of the agent, eq. (9) */
  float kappa;        /* >= 0: probe exponent of the consensus weights, eq. (11) */
  float rho;          /* 0 < rho < 1: Mann averaging parameter, eq. (13) */
  uint32_t flags;     /* PMACE_CENTERED_DC and at most one of PMACE_STAGED_AGENT,
                         PMACE_SPLIT_AGENT, PMACE_ROWSPEC_AGENT; or 0 */
  int32_t chunk;      /* Np > 128 only: at most this many positions per staging chunk
                         (>= 1, capped at J; the chunks are then evened out),
                         0 = the build's tuned default for Np = 256, scaled by
                         256^2/Np^2 so that every side stages about as many bytes */
  int32_t method;     /* PMACE_METHOD_PMACE (alpha, kappa, rho used) or PMACE_METHOD_SHARP_PLUS */
  float beta;         /* SHARP+ relaxation, 0 <= beta <= 1 (Alg. 2); ignored by PMACE */
  int32_t ppw;        /* patches per workgroup of the whole-patch agent (Np <= 128): a power
                         of two up to 8 within 1024 threads per workgroup (np 32: up to 8,
                         48: 4, 64: 2 with this build's line splits; 96 and 128: 1), or 0 =
                         the build's tuned default.  Other sides: 0 or 1.  A batch's merged
                         launch for one patch side takes its first such member's value.
                         Anything else is EINVAL.  Results do not depend on it. */
} pmace_params;

typedef struct pmace_ctx pmace_ctx;      /* one reconstruction */
typedef struct pmace_batch pmace_batch;  /* several reconstructions stepped together */

/* Bytes of device workspace one reconstruction needs (0 if params are invalid).
 * Layout: agent states J*Np^2*8, amplitudes J*Np^2*4, object images N1*N2*36,
 * probe tables Np^2*48, positions J*8, a staging buffer of chunk*Np^2*8
 * bytes (Np > 128: the chunk's spectra; SHARP+ with Np <= 128: all J frames;
 * PMACE with Np <= 128: none), data-fit partials and the consensus tile
 * tables; each section 256-byte aligned. */
size_t pmace_footprint(const pmace_params* params);

/* Alg. 1 initialisation: v_j = P_j x0 for every j.  Also computes
 * y = sqrt(z) (eq. (2)), the weights |d|^kappa and Lambda^{-1} of eq. (11)
 * (Lambda^{-1} := 0 where Lambda = 0) and D^{-1} (in FP64 on the host from a
 * copy of the probe), and the starting reconstruction x0 restricted to the
 * covered pixels.
 *   probe_d     np*np c64, the known probe d (Sec. II)
 *   pos_d       num_pos x 2 int32 (row, col) top-left patch offsets, each in
 *               [0, n1-np] x [0, n2-np]  (P_j, Sec. II)
 *   intensity_d num_pos*np*np float32 z_j >= 0, finite; DC at [0,0] unless
 *               PMACE_CENTERED_DC
 *   x0_d        n1*n2 c64 initial object, or NULL for 1+0i everywhere
 *   workspace_d device buffer of ws_bytes >= pmace_footprint(params), owned
 *               by the caller and kept alive until pmace_destroy
 *   hip_stream  hipStream_t the context queues all its work on (NULL = the
 *               null stream)
 * Inputs are read during this call's stream work; this call synchronises the
 * stream before returning, so the caller may free them afterwards.
 * Errors: EINVAL (bad sizes/ranges, non-finite or negative intensity, position
 * outside the object), EUNSUPPORTED (np), ENOMEM (ws_bytes too small),
 * EDEVICE.  On error *out is NULL. */
pmace_status pmace_init(const pmace_params* params, const void* probe_d,
                        const int32_t* pos_d, const float* intensity_d,
                        const void* x0_d, void* workspace_d, size_t ws_bytes,
                        void* hip_stream, pmace_ctx** out);

/* Run n_iter >= 0 iterations of the Alg. 1 loop body (stream-ordered, async).
 * Each iteration reads and rewrites every agent state once. */
pmace_status pmace_iterate(pmace_ctx* ctx, int32_t n_iter);

/* Alg. 1 output: xhat = Lambda^{-1} sum_j P_j^t |d|^kappa v_j, written to
 * xhat_d (n1*n2 c64, device).  Stream-ordered. */
pmace_status pmace_reconstruct(pmace_ctx* ctx, void* xhat_d);

/* Copy the stacked agent states v (num_pos*np*np c64, device) out / in.
 * set_state also recomputes the reconstruction as the weighted average of
 * the new v (checkpoint resume; one-step parity checks).  PMACE keeps each
 * state multiplied by the probe (as it is where d == 0); get_state divides by
 * d again, so v there carries the conditioning of d^{-1}, as the agent's own
 * output does (eq. (9)). */
pmace_status pmace_get_state(pmace_ctx* ctx, void* v_d);
pmace_status pmace_set_state(pmace_ctx* ctx, const void* v_d);

/* Wait for the context's queued work; reports EDEVICE for a failed HIP call
 * and EDIVERGED if the consensus image became NaN/Inf. */
pmace_status pmace_sync(pmace_ctx* ctx);

/* Queue the context's later work on hip_stream instead (synchronises the old
 * stream first).  A serving loop initialises a new reconstruction on a side
 * stream, so its host-side set-up overlaps the running batch, then moves it
 * to the batch's stream.  Not for a context that a live batch holds (the
 * batch keeps launching on the stream it was created with). */
pmace_status pmace_set_stream(pmace_ctx* ctx, void* hip_stream);

/* Which agent a context runs (see the agent flags above): a host query. */
#define PMACE_AGENT_WHOLE_PATCH 0  /* np <= 128: one workgroup per patch */
#define PMACE_AGENT_THREE_PASS 1   /* np > 128: rows, columns, inverse rows, spectra staged */
#define PMACE_AGENT_SPLIT 2        /* coset blocks of (np/2)^2, states in the split layout */
#define PMACE_AGENT_ROWSPEC 3      /* np > 128: rows, columns, states kept as row spectra */
int32_t pmace_agent_kind(const pmace_ctx* ctx);  /* -1 for NULL */

/* Release the host context (not the caller's workspace).  NULL is a no-op. */
void pmace_destroy(pmace_ctx* ctx);

const char* pmace_status_str(pmace_status s);

/* NRMSE tracking (eq. (17)): a reference object xref_d (n1*n2 c64, device)
 * and an optional region mask_d (n1*n2 bytes, nonzero = inside; NULL = every
 * pixel).  Both stay owned by the caller and must stay alive while the
 * context (or a batch holding it) may read them; xref_d = NULL turns tracking
 * off.  Resets the context's NRMSE history and stop flag; synchronises. */
pmace_status pmace_set_reference(pmace_ctx* ctx, const void* xref_d, const uint8_t* mask_d);

/* NRMSE of the current reconstruction against the reference:
 * min over theta of ||xhat - e^{i theta} xref|| / ||xref|| over the region,
 * with theta = arg sum conj(xref) xhat.  Synchronises; *out on the host.
 * ESTATE if no reference is set. */
pmace_status pmace_nrmse(pmace_ctx* ctx, double* out);

/* Data-fit cost of eq. (4) at the current reconstruction, with sigma_n = 1:
 *   sum_j 1/2 || y_j - |F D P_j xhat| ||^2,  y_j = sqrt(z_j),
 * F the orthonormal 2-D DFT.  Needs no reference object.  Uses the context's
 * staging buffer (stream-ordered with its iterations); does not change the
 * stop rule's history.  Synchronises; *out on the host. */
pmace_status pmace_data_fit(pmace_ctx* ctx, double* out);

/* Batches: several reconstructions on one device and stream advanced
 * together; from the third pmace_batch_step call on, one HIP graph launch per
 * iteration (a batch rebuilt every few steps, as in a serving loop, launches
 * eagerly instead of paying for capture).  Positions of members with
 * Np <= 128 share merged launches per patch size; Np > 128 members run as
 * parallel branches beside them.  Every iteration counts towards max_iter; after every
 * check_every-th iteration of the batch the stop rule is evaluated on the
 * device, and a member stops (its kernels return at once) when
 *   PMACE_STOP_NRMSE:    its NRMSE against its reference (set before
 *                        pmace_batch_create) changed by less than tol,
 *                        |e_k - e_{k-1}| < tol (eq. (17)); members without a
 *                        reference stop only at max_iter;
 *   PMACE_STOP_DATA_FIT: its data-fit cost C of eq. (4) (as pmace_data_fit)
 *                        changed by at most tol relative to the previous
 *                        evaluation, |C_k - C_{k-1}| <= tol C_{k-1}; needs no
 *                        reference (the paper leaves its stopping test open);
 * once at least min_iter iterations have run, or after max_iter iterations. */
#define PMACE_STOP_NRMSE 0
#define PMACE_STOP_DATA_FIT 1
typedef struct {
  float tol;           /* threshold of the criterion (e.g. 1e-4) */
  int32_t min_iter;    /* >= 0 */
  int32_t max_iter;    /* >= 1 */
  int32_t criterion;   /* PMACE_STOP_NRMSE or PMACE_STOP_DATA_FIT */
  int32_t check_every; /* >= 0: evaluate every this many iterations (0 = 1) */
} pmace_stop_rule;

/* Device workspace bytes a batch of these members needs (0 if invalid). */
size_t pmace_batch_footprint(pmace_ctx* const* ctxs, int32_t n);
/* Members must be distinct, on one device and stream, and stay alive until
 * the batch is destroyed (pmace_batch_destroy first, then pmace_destroy).
 * pmace_set_reference on a member also updates the batch's copy of it.  The
 * workspace is owned by the caller.  A member's stop flag and NRMSE history belong to the member
 * (reset by pmace_set_reference), so a member moved into a new batch carries
 * on where it stopped; pmace_iterate clears the stop flag. */
pmace_status pmace_batch_create(pmace_ctx* const* ctxs, int32_t n, const pmace_stop_rule* rule,
                                void* workspace_d, size_t ws_bytes, pmace_batch** out);
/* n_iter iterations of every member still running (stream-ordered, async). */
pmace_status pmace_batch_step(pmace_batch* batch, int32_t n_iter);
/* Synchronise and read back per member: stop flag, last NRMSE, iterations
 * counted by the stop rule.  Host arrays of n entries; any may be NULL.
 * Np > 128 members found stopped are left out of the batch's later launches
 * (the graphs are captured again on the next step); a member whose stop flag
 * the host clears (pmace_iterate, pmace_set_reference) is launched again from
 * the next pmace_batch_step on.  Results are the same either way. */
pmace_status pmace_batch_poll(pmace_batch* batch, int32_t* done, double* nrmse, int32_t* iters);
/* As pmace_batch_poll, plus the last data-fit cost the stop rule evaluated
 * (infinity before the first evaluation). */
pmace_status pmace_batch_poll_fit(pmace_batch* batch, int32_t* done, double* nrmse, int32_t* iters,
                                  double* data_fit);
void pmace_batch_destroy(pmace_batch* batch);

/* Simulated measurements (Sec. II eq. (1); Sec. IV eq. (16)) for synthetic
 * problems made on the device:  I_j = |F D P_j x|^2  for every position and,
 * when peak_photons > 0, z_j = Pois(I_j * peak_photons / max I) with the
 * maximum over all positions and pixels (one scale per experiment); else
 * z = I.  Poisson variates come from the counter-based generator
 * Philox4x32-10 keyed by `seed` and counted by element index, so the output
 * depends only on the inputs and the seed.
 *   probe_d np*np c64; pos_d num_pos x 2 int32 (inside the object, else
 *   EINVAL); x_d n1*n2 c64; z_d num_pos*np*np float32 (output, DC at [0,0]);
 *   workspace_d >= pmace_simulate_footprint(np, num_pos) bytes (caller-owned);
 *   scale_out (host, may be NULL) receives peak_photons / max I (1 if
 *   noise-free): multiply the probe by sqrt(scale) to keep the object's units.
 * Synchronises (positions are validated on the host). */
size_t pmace_simulate_footprint(int32_t np, int32_t num_pos);
pmace_status pmace_simulate(int32_t n1, int32_t n2, int32_t np, int32_t num_pos,
                            const void* probe_d, const int32_t* pos_d, const void* x_d,
                            double peak_photons, uint64_t seed, float* z_d, void* workspace_d,
                            size_t ws_bytes, double* scale_out, void* hip_stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * simulation as pmace_simulate, with the same arguments minus the workspace,
 * and the same results bit for bit.  Its scratch memory (the maximum, a
 * position flag and, for np > 128, the row transforms of the frames) is one
 * static device array per GPU, held from the first call on that GPU until the
 * process ends; nothing is allocated per call.  Limit: np > 128 needs
 * num_pos*np*np*8 <= pmace_simulate_static_max_bytes() (64 MiB - 256 B, e.g.
 * 127 positions of 256 x 256), else ENOMEM; np <= 128 has no such limit.
 * Positions are validated on the device (EINVAL if a patch leaves the
 * object).  Every call on one GPU shares that GPU's array: calls that overlap
 * on one GPU (other streams, other threads) race; serialise them.
 * Synchronises hip_stream (the position check; and scale_out as in
 * pmace_simulate). */
size_t pmace_simulate_static_max_bytes(void);
pmace_status pmace_simulate_static(int32_t n1, int32_t n2, int32_t np, int32_t num_pos,
                                   const void* probe_d, const int32_t* pos_d, const void* x_d,
                                   double peak_photons, uint64_t seed, float* z_d, double* scale_out,
                                   void* hip_stream);
/* Exposes the generator behind pmace_simulate for known-answer checks: io_d
 * holds n records of 6 uint32 (counter[4], key[2]); the counter words are
 * replaced by Philox4x32-10(counter, key). */
pmace_status pmace_philox4x32_10(uint32_t* io_d, int32_t n, void* hip_stream);
/* The Poisson sampler behind pmace_simulate on given means lam_d[n] (FP64):
 * element i draws from the stream of element index i under `seed`. */
pmace_status pmace_poisson(const double* lam_d, float* out_d, int32_t n, uint64_t seed,
                           void* hip_stream);

/* Batched 2-D orthonormal DFT of `count` np x np c64 arrays (the operator F
 * of Sec. II, or F^* when inverse != 0), in_d and out_d may alias.
 * np in {32, 48, 64, 96, 128, 160, 192, 256}.  Stream-ordered on hip_stream. */
pmace_status pmace_fft2(int32_t np, int32_t count, const void* in_d, void* out_d,
                        int32_t inverse, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* PMACE_H */
