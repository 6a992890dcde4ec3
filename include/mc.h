/*
 * mc.h -- C interface of libmc, an MI355X (gfx950) simulator of the
 * deliver/update simulation cycle of leaky integrate-and-fire networks with
 * explicitly stored synapses (Kurth, Senk, Terhorst, Finnerty, Diesmann,
 * "Sub-realtime simulation of a neuronal network of natural density").
 *
 * What the paper fixes and this interface follows:
 *   - the problem statement of the Methods section: instantiate the network
 *     (not timed), then simulate a span of model time T_model on a fixed grid
 *     of h = 0.1 ms after a presimulation, and report the realtime factor
 *     RTF = T_wall / T_model (the one equation of the Methods section);
 *   - the simulation cycle named in the Fig. 1 caption: "update" advances the
 *     state of every neuron, "deliver" distributes each spike to its targets;
 *   - the observable of Supplementary Fig. 1: the spike raster;
 *   - synaptic events = transmitted spikes (Methods, energy per event);
 *   - explicit per-synapse weights (Discussion), which makes per-synapse
 *     gradients well defined (mc_adjoint).
 *
 * Conventions for every function:
 *   - returns MC_OK (0) or a negative mc_status; no C++ exception crosses the
 *     boundary; mc_last_error() returns a message for the calling thread's
 *     most recent failure;
 *   - pointers named *_host are host memory, *_dev device memory; every
 *     output buffer is owned by the caller; the library owns all memory that
 *     belongs to an mc_net until mc_free;
 *   - one host thread may use an mc_net at a time;
 *   - neuron ids are global and dense: instance b of a batched network holds
 *     ids [inst_off[b], inst_off[b+1]) (mc_get_instance_offsets), and inside
 *     an instance the populations follow in configuration order;
 *   - "step" counts grid steps of h since the network was built (step 0 is
 *     the first step simulated).
 */
#ifndef MC_H
#define MC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MC_ABI_VERSION 1
#define MC_MAX_POPS 16
#define MC_RING_SLOTS 128        /* input ring depth; delays are 1..MC_RING_SLOTS-28 steps */

typedef enum mc_status {
  MC_OK = 0,
  MC_ERR_INVALID_ARG = -1,       /* a NULL or malformed argument, or an inconsistent configuration */
  MC_ERR_RANGE = -2,             /* a value outside what the representation holds (weight, delay, size) */
  MC_ERR_OOM = -3,               /* host or device allocation failed; the handle stays valid */
  MC_ERR_HIP = -4,               /* a HIP runtime call failed */
  MC_ERR_STATE = -5,             /* handle in the wrong state (freed, host-only, failed, or not fresh) */
  MC_ERR_BUFFER_TOO_SMALL = -6,  /* *count_out holds the required element count */
  MC_ERR_NO_DEVICE = -7,         /* no usable gfx950 device */
  MC_ERR_MISMATCH = -8,          /* adjoint recomputation did not reproduce the recorded spikes */
  MC_ERR_TIMEOUT = -9            /* the persistent kernel's wait for a step's spike records exceeded its
                                    time limit (a workgroup never published); the handle is marked failed */
} mc_status;

enum { MC_RULE_FIXED_INDEGREE = 0, MC_RULE_BERNOULLI = 1 };
enum { MC_GRAD_F64 = 0, MC_GRAD_F32 = 1 };
enum {
  MC_FLAG_HOST_ONLY = 1u,       /* build the network on the host only (no device memory) */
  MC_FLAG_DEVICE_CONNECT = 2u   /* draw the connections on the device: the pair tests of
                                   MC_RULE_BERNOULLI and the source draws of MC_RULE_FIXED_INDEGREE
                                   (integer Philox draws) run as HIP kernels; the sort into rows,
                                   weights, delays and everything else stay on the host; the network is
                                   bit-identical to the host build.  INVALID_ARG with
                                   MC_FLAG_HOST_ONLY. */
};

typedef struct mc_net mc_net;

/*
 * Network description.  Populations: n_pops (<= MC_MAX_POPS) of sizes
 * pop_size; instance b holds max(1, rint(inst_scale[b] * pop_size[a]))
 * neurons of population a.  Matrices are [post * n_pops + pre].
 *
 * Connectivity: MC_RULE_FIXED_INDEGREE -- conn = number of sources per target
 * drawn from population pre uniformly with replacement (autapses and
 * multapses allowed); MC_RULE_BERNOULLI -- conn = probability that a given
 * (source, target) pair is connected (autapses allowed, no multapses).
 * Weights: N(w_mean, (w_rel_sd*|w_mean|)^2) pA, stored as signed integers in
 * units of 2^-16 pA (round to nearest even).  Delays: N(d_mean[pre],
 * (d_rel_sd*d_mean[pre])^2) ms, rounded to the step h and clipped to
 * [d_min_steps, d_max_steps] (1 <= d_min_steps, d_max_steps <= 100).
 * Drive: a Poisson number of inputs per neuron and step with mean
 * nu_ext_hz * k_ext[pop] * h, each of weight w_ext_pA.
 * Neuron: leaky integrate-and-fire with exponentially decaying current
 * (tau_m_ms, c_m_pF, e_l_mV, v_reset_mV, v_th_mV, t_ref_ms, tau_syn_ms,
 * constant current i_e_pA), exact integration at step h_ms; initial
 * membrane potential uniform in [v0_lo_mV, v0_hi_mV).
 * All random draws are counter-based (Philox4x64-10) keyed by the instance
 * seed, so results do not depend on launch configuration, batching or
 * thread counts.
 */
typedef struct mc_config {
  uint32_t struct_size;          /* sizeof(mc_config); guards the ABI */
  int32_t n_pops;
  const int32_t* pop_size;       /* [n_pops] */
  int32_t rule;
  const double* conn;            /* [n_pops*n_pops] */
  const double* w_mean_pA;       /* [n_pops*n_pops], signed */
  double w_rel_sd;
  const double* d_mean_ms;       /* [n_pops], by presynaptic population */
  double d_rel_sd;
  int32_t d_min_steps, d_max_steps;
  const double* k_ext;           /* [n_pops] */
  double nu_ext_hz, w_ext_pA;
  double tau_m_ms, c_m_pF, e_l_mV, v_reset_mV, v_th_mV, t_ref_ms, tau_syn_ms, i_e_pA, h_ms;
  double v0_lo_mV, v0_hi_mV;
  int32_t n_instances;           /* >= 1 */
  const double* inst_scale;      /* [n_instances]; NULL means 1.0 for every instance */
  const uint64_t* inst_seed;     /* [n_instances]; required */
  void* hip_stream;              /* hipStream_t to run on; NULL: a stream owned by the library */
  uint32_t flags;                /* MC_FLAG_* */
  /* Optional device allocator (e.g. a framework's caching allocator): every
   * device buffer that belongs to the network (synapse store, state, ring,
   * tables, raster, adjoint buffers, probe buffers) comes from
   * dev_alloc(bytes, alloc_ctx), which must return device memory of the
   * current device aligned to 256 bytes, or NULL (the call then fails with
   * OOM); it is returned with dev_free(ptr, alloc_ctx) after the network's
   * stream has finished with it.  Both NULL: hipMalloc / hipFree.  Giving
   * one without the other is INVALID_ARG.  Temporary buffers of the device
   * connection draws during mc_build_network use hipMalloc. */
  void* (*dev_alloc)(size_t bytes, void* alloc_ctx);
  void (*dev_free)(void* ptr, void* alloc_ctx);
  void* alloc_ctx;
} mc_config;

/* Launch configuration of the simulation loop (see mc_set_launch). */
enum { MC_SCHEME_STEP_KERNELS = 0,   /* one kernel per step (update, then source-owner delivery with device
                                        atomics), replayed from a HIP graph */
       MC_SCHEME_PERSISTENT_LDS = 1,  /* one persistent kernel per chunk; near-future input held in LDS */
       MC_SCHEME_TARGET_OWNER = 2,    /* two kernels per step: update, then target-owner delivery combined
                                        in LDS (no device atomics); replayed from a HIP graph */
       MC_SCHEME_PERSISTENT_BUCKETS = 3 };  /* one persistent kernel per chunk; workgroups own target blocks of
                                        one instance and exchange spikes with their own instance only;
                                        events go to per-workgroup buckets by arrival step (batches of
                                        instances, networks too large for the LDS window) */
typedef struct mc_launch {
  uint32_t struct_size;
  int32_t scheme;
  int32_t block;                 /* threads per workgroup: 64..1024, multiple of 64 */
  int32_t neurons_per_wg;        /* neurons updated by one workgroup: multiple of 4, <= 4*block, <= 1024
                                    (persistent: <= block; target owner: the targets of one delivery block,
                                    its update kernel takes one quad per thread; buckets: <= min(4092,
                                    64*block)); 0: automatic */
  int32_t steps_per_graph;       /* steps captured per graph replay / per persistent launch (>= 1) */
  int32_t rows_per_wave;         /* step kernels' delivery: 0 = all threads of a workgroup walk each
                                    spiking row in turn; 1 = each wavefront walks whole rows (short rows);
                                    ignored by the other schemes */
} mc_launch;

typedef struct mc_counters {
  int64_t step;                  /* next step to simulate */
  int64_t spikes;                /* spikes emitted since build */
  int64_t events;                /* synaptic events delivered since build (sum of out-degrees of spikes) */
  int64_t spikes_per_pop[MC_MAX_POPS];   /* summed over instances */
} mc_counters;

typedef struct mc_adjoint_config {
  uint32_t struct_size;
  int64_t window_steps;          /* S >= 1 */
  int64_t ckpt_every;            /* K >= 1: forward state kept every K steps, recomputed in between */
  double v_target_mV;            /* loss target V* */
  int32_t grad_dtype;            /* MC_GRAD_F64 or MC_GRAD_F32 */
  int32_t input_mode;            /* how a segment's synaptic input is recovered for the recompute:
                                    MC_ADJ_INPUT_AUTO, _RECORD (the forward stores every neuron's whole
                                    integer input, drive included: 8 B per neuron-step), _REPLAY (the
                                    ring is kept with every checkpoint, the recorded spikes are
                                    delivered again and the drive is redrawn) */
} mc_adjoint_config;
enum { MC_ADJ_INPUT_AUTO = 0, MC_ADJ_INPUT_RECORD = 1, MC_ADJ_INPUT_REPLAY = 2 };

/* --- the four calls of the simulation --------------------------------- */

/* Builds the network on the host (OpenMP; with MC_FLAG_DEVICE_CONNECT the
 * connection draws on the device), derives propagators and drive
 * tables, uploads everything to the current HIP device.  Untimed
 * instantiation of the Methods section.  *out receives the handle (NULL on
 * failure).  Errors: INVALID_ARG (inconsistent config), RANGE (a quantised
 * weight beyond int32, a delay range beyond the ring, too many neurons),
 * OOM, HIP, NO_DEVICE. */
int mc_build_network(const mc_config* cfg, mc_net** out);

/* Advances the network by `steps` grid steps (update, then deliver, per
 * step: the simulation cycle of the Fig. 1 caption; the Methods time such a
 * call over T_model after a presimulation), recording every spike.  Asynchronous on the network's stream;
 * getters synchronize.  Resumable: consecutive calls continue the same
 * trajectory bit for bit.  Errors: STATE (host-only or failed handle), HIP,
 * OOM (raster growth).  Test hook: the environment variable
 * MC_PERSIST_LIST_CAP = k (1..1024) makes the persistent scheme, in the
 * steps that mc_profile_phases runs, list every step of more than k spikes
 * in producer order after the wait (the path of a step beyond its LDS
 * list); results are unchanged. */
int mc_simulate(mc_net* net, int64_t steps);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): mc_simulate for the
 * persistent scheme (mc_set_launch scheme 1) without any allocation -- no
 * hipMalloc or hipFree, no graph instantiation, no raster drain.  The
 * kernels' spike records and side array (the scratch mc_simulate keeps in
 * library-allocated memory) come from a file-scope device array of about
 * 4.1 MiB (room for 512 workgroups of 512 targets) that each GPU holds until
 * the process ends.  The records are cleared by a kernel at the start of
 * every call.  Every call on one GPU shares that GPU's array, so calls that
 * overlap on one GPU (two networks on concurrent streams) race: serialize
 * them.  Same trajectory, raster and counters as mc_simulate(steps).
 * Errors: STATE (another scheme, or a host-only/failed handle), RANGE (a
 * persistent shape beyond the scratch, step count beyond int32),
 * BUFFER_TOO_SMALL (more steps than the raster holds without a drain: call
 * mc_reserve first), INVALID_ARG (steps < 0, or the network's device is not
 * the current one), HIP.  Asynchronous on the network's stream. */
int mc_simulate_noalloc(mc_net* net, int64_t steps);

/* Copies the recorded spikes (the raster of Supplementary Fig. 1) with step
 * in [step_begin, step_end) into caller-owned host arrays, sorted by step,
 * then neuron id.  If more than
 * `capacity` spikes fall in the range, writes nothing, sets *count_out to the
 * number required and returns BUFFER_TOO_SMALL. */
int mc_get_spikes(mc_net* net, int64_t step_begin, int64_t step_end,
                  int32_t* step_out_host, int32_t* id_out_host, int64_t capacity, int64_t* count_out);

/* Gradient of L = 1/(N S) sum_i sum_{n0<=n<n0+S} (V_i(n+1) - V*)^2 over the
 * window of S steps that starts at the current step n0, with respect to every
 * synaptic weight in pA, with the spike pattern of the window held fixed
 * (Discussion: explicit per-synapse weights; reverse-time adjoint with the
 * transposed exact-integration propagators, gathered over the outgoing
 * synapse rows of every recorded spike).  N counts real neurons of all
 * instances.  The state at n0, including inputs still pending from spikes
 * before n0, is the fixed initial condition.  The network advances by S
 * steps exactly as mc_simulate(S) would (same spikes, same raster).  The
 * forward state (y, I, r) is kept every ckpt_every steps and recomputed per
 * segment; the segment's input comes either from a record of every
 * neuron's whole integer input made by the forward (8 B per neuron-step: the
 * default up to 16 GiB) or from the ring kept with each checkpoint (about
 * 8 B x 128 x N) plus a second delivery of the recorded spikes and the
 * redrawn drive.  A recompute that does not reproduce the recorded spikes
 * returns MISMATCH.  grad_dev: caller-owned device array of
 * mc_get_sizes().n_synapses elements (double for MC_GRAD_F64; float for
 * MC_GRAD_F32, accumulated as
 * g = f32(g + f32(term)) from FP64 adjoint states), in the canonical synapse
 * order of mc_get_synapses; overwritten.  *loss_out (host): L.
 * Synchronizes the stream.  Errors: INVALID_ARG (NULL pointers, S outside
 * [1, 1e6], ckpt_every outside [1, 4096], unknown grad_dtype), STATE, RANGE,
 * OOM, HIP, MISMATCH. */
int mc_adjoint(mc_net* net, const mc_adjoint_config* acfg, void* grad_dev, double* loss_out);

void mc_free(mc_net* net);
const char* mc_strerror(int code);
const char* mc_last_error(void);
int mc_abi_version(void);

/* --- introspection and control (same conventions) ---------------------- */

int mc_get_sizes(mc_net* net, int64_t* n_neurons, int64_t* n_synapses, int32_t* n_instances);
int mc_get_instance_offsets(mc_net* net, int64_t* off_host /* [n_instances+1] */);
/* Population offsets of instance b in global ids: [n_pops+1]. */
int mc_get_pop_offsets(mc_net* net, int32_t instance, int64_t* off_host);
/* The explicit synapse store (Discussion: every synapse's weight stored) in
 * canonical order: rows by source id, ascending target inside a row
 * (multapses in draw order).  row_ptr [N+1], tgt/w_q/dly [M]. */
int mc_get_synapses(mc_net* net, int64_t* row_ptr_host, int32_t* tgt_host, int32_t* w_q_host, uint8_t* dly_host);
/* State of the leaky integrate-and-fire neurons with exponential currents
 * (Supplementary Fig. 1 caption) after the last simulated step: y = V - E_L
 * (mV), I (pA), refractory steps left.  set: replaces it (r in [0, 255]). */
int mc_get_state(mc_net* net, double* y_host, double* i_host, int32_t* r_host);
int mc_set_state(mc_net* net, const double* y_host, const double* i_host, const int32_t* r_host);
/* Logical input ring: pending[k*N + i] = integer input (2^-16 pA) neuron i
 * reads at step (current step + k), k in [0, depth), depth <= MC_RING_SLOTS. */
int mc_get_ring(mc_net* net, int64_t depth, int64_t* pending_host);
/* Adds `value` (2^-16 pA) to the input neuron i reads at step current+k. */
int mc_inject(mc_net* net, int64_t k, int64_t neuron, int64_t value);
/* Propagators P11, P21, P22, P20 of the exact integration step of h
 * (Supplementary Fig. 1 caption: h = 0.1 ms, tau_m, tau_syn). */
int mc_get_propagators(mc_net* net, double* p_host /* [4] */);
/* Poisson inverse-CDF tables [n_pops][64] of the external drive, instance 0
 * (the tables are the same for every instance). */
int mc_get_drive_tables(mc_net* net, uint64_t* t_host);
/* Step, spikes and synaptic events (Methods: transmitted spikes, the
 * denominator of the energy per synaptic event) since the build. */
int mc_get_counters(mc_net* net, mc_counters* out);
/* Launch configuration of the cycle (how its update and delivery map onto
 * the GPU; the paper's counterpart is the thread placement of its Results);
 * a change never changes results (integer sums).  A
 * shape the device cannot run (RANGE, INVALID_ARG) leaves the current one;
 * a failure while the new shape's tables are built (OOM, HIP) marks the
 * handle failed. */
int mc_set_launch(mc_net* net, const mc_launch* l);
int mc_get_launch(mc_net* net, mc_launch* l);
/* Times candidate launch configurations on copies of the current state for
 * `steps` steps each, keeps the fastest (state and raster are restored).
 * If the environment variable MC_TUNE_CACHE names a file, the choice is
 * kept there keyed by the network's shape (neurons, instance and population
 * sizes, and the synapse count to an eighth of an octave, so that networks
 * drawn with other seeds share the key) and the device (name and compute
 * units); a later call for the same key applies the stored choice without
 * timing anything.  *best_out: the launch chosen. */
int mc_tune(mc_net* net, int64_t steps, mc_launch* best_out);
/* Shape of the persistent scheme in use: workgroups, target neurons per
 * workgroup and steps of pending input held in LDS (the bucket scheme: 0
 * steps; all 0 under the step kernels). */
int mc_get_persist_shape(mc_net* net, int32_t* workgroups_out, int32_t* targets_per_wg_out, int32_t* lds_steps_out);
/* The time per phase of the cycle (Fig. 1b splits the run time into update,
 * deliver, communicate and other): simulates `steps` steps with per-phase
 * device timestamps (persistent schemes only) and returns the mean time per
 * step in microseconds, averaged
 * over workgroups: us_out[0] update, [1] compaction+publication, [2] wait
 * for every workgroup's spikes, [3] spike-list gather, [4] delivery (LDS
 * window: the delay-1 events; buckets: every event of the step), [5] the
 * sum of [0..4]; overlapping parts of [2]: [6] drive of the next step (and,
 * in the LDS window, pending delivery of the previous one; first
 * wavefront), [7] polling (first polling thread).  The trajectory is the
 * one mc_simulate would produce. */
int mc_profile_phases(mc_net* net, int64_t steps, double* us_out_host);
/* The per-workgroup times behind the last mc_profile_phases, [G][8] us per
 * step (columns 0..4 as us_out[0..4], 5: drive + pending delivery of
 * wavefront 0, 6: polling of the first poller, 7: unused); *workgroups_out =
 * G (0 before any profile).  BUFFER_TOO_SMALL if capacity < 8*G. */
int mc_get_phase_table(mc_net* net, double* out_host, int64_t capacity, int32_t* workgroups_out);
/* Throughput form of the deliver phase (Fig. 1 caption): every synapse of every recorded spike
 * with step in [step_begin, step_end) (< current step) is delivered in ONE
 * launch into a scratch ring of S = step_end - step_begin + 101 slots with
 * device int64 atomics (slot k = input read at step step_begin + k).
 * *ms_out: kernel time (HIP events); *events_out: synapses delivered.  If
 * ring_out_host is not NULL it receives the ring as [S][N] int64 (capacity
 * in elements; BUFFER_TOO_SMALL if < S*N).  The network state is untouched. */
int mc_replay_delivery(mc_net* net, int64_t step_begin, int64_t step_end, int64_t* ring_out_host,
                       int64_t ring_capacity, double* ms_out, int64_t* events_out);
/* Measured rate (1e9 per second) of uniformly random device-scope int64
 * atomic adds into a table of `entries` elements: the achievable peak the
 * delivery's atomics are compared with. */
int mc_atomic_rate(mc_net* net, int64_t entries, double* gops_out);
/* Achievable memory rates the delivery is measured against (Methods: the
 * simulation's time goes to updating neurons and delivering spikes; here
 * the delivery streams the synapse records and adds into a slot-major ring):
 *   mc_probe_stream   -- streaming read of `bytes` (>= 1 MiB, rounded down to
 *                        16 B) of device memory it allocates; *gbs_out GB/s
 *                        (1e9 B/s) of the second of two launches;
 *   mc_probe_atomics  -- int64 atomic adds into a table of slots x (the
 *                        network's ring stride) entries it allocates;
 *                        pattern 0: uniformly random (slot, target);
 *                        pattern 1: the delivery's own pattern (chunks of 256
 *                        events of a row: ascending targets at the store's
 *                        mean spacing N/mean out-degree, delays drawn from the
 *                        store's delay histogram, spike steps advancing over
 *                        the table); *gops_out 1e9 adds per second, of
 *                        the fastest of three timed launches of 2^27 adds;
 *   mc_probe_exchange -- the persistent scheme in use with nothing but its
 *                        exchange: its workgroups publish and poll one record
 *                        per step; *us_per_step_out the time per step, the
 *                        floor of the persistent kernel's step (STATE under
 *                        another scheme; TIMEOUT if a record never arrived).
 * Each synchronizes and leaves the network untouched. */
int mc_probe_stream(mc_net* net, int64_t bytes, double* gbs_out);
int mc_probe_atomics(mc_net* net, int64_t slots, int32_t pattern, double* gops_out);
int mc_probe_exchange(mc_net* net, int64_t steps, double* us_per_step_out);
/* Wall time (ms) of the GPU work of the most recent mc_simulate, from HIP events. */
int mc_last_simulate_ms(mc_net* net, double* ms_out);
/* Persistent schemes: the summed durations (ms) of the persistent kernel's
 * launches in the most recent mc_simulate (or mc_simulate_noalloc), how many
 * launches were timed (at most 64) and the steps they covered.  Every launch,
 * direct or replayed from a graph, is timed by HIP events recorded on the
 * simulation stream right before and after it; an mc_simulate call that is a
 * single launch is timed by the call's own two events instead (each event on
 * the stream lengthens the call by a few microseconds), so then the result
 * equals mc_last_simulate_ms.  Zero launches under the other schemes.
 * Synchronizes on that call. */
int mc_last_kernel_ms(mc_net* net, double* ms_out, int64_t* launches_out, int64_t* steps_out);
/* GPU time (ms, HIP events) of the most recent mc_adjoint: its forward
 * (S steps with checkpoints) and its reverse pass (recompute, adjoint,
 * gather). */
int mc_last_adjoint_ms(mc_net* net, double* forward_ms_out, double* reverse_ms_out);
/* Makes room for the spikes of `steps` further steps (at most 2e6) so that
 * mc_simulate allocates nothing for them; the room is the worst-case bound
 * (one spike per refractory period per neuron).  OOM leaves the room there
 * was, and the handle usable. */
int mc_reserve(mc_net* net, int64_t steps);
/* Full dynamic state (step, y, I, r, ring, counters) to/from a host blob,
 * so that a run can resume or restart from any step (a simulation resumes
 * bit for bit; the Methods' presimulation is such a prefix). */
int mc_save_state(mc_net* net, void* blob_host, size_t capacity, size_t* used_out);
int mc_load_state(mc_net* net, const void* blob_host, size_t size);
/* Replaces every weight by rint(w_pA_dev[k] * 2^16) (device array of
 * mc_get_sizes().n_synapses doubles in pA, canonical order; round to nearest
 * even).  RANGE if a value is not finite or its quantised weight does not fit
 * int32 (|w| >= 32768 pA): then the store is unchanged.  Synchronizes. */
int mc_set_weights(mc_net* net, const double* w_pA_dev);
/* One gradient-descent step on the stored weights (Discussion: explicit
 * per-synapse weights keep plasticity and learning possible; with the
 * gradient of mc_adjoint this is learning on the store itself): every weight
 * becomes rint((w_q[k] 2^-16 - eta g[k]) 2^16) in units of 2^-16 pA (round to
 * nearest even), the difference evaluated in FP64 as fl(w - fl(eta g)).
 * grad_dev: device array of n_synapses elements in canonical order, double
 * for MC_GRAD_F64, float for MC_GRAD_F32 (as mc_adjoint writes it); eta: pA
 * per unit of g.  RANGE (store unchanged) if a new weight is not finite or
 * does not fit int32; INVALID_ARG for a NULL gradient, an unknown dtype or a
 * non-finite eta.  Synchronizes. */
int mc_apply_gradient(mc_net* net, const void* grad_dev, int32_t grad_dtype, double eta);
int mc_stream(mc_net* net, void** hip_stream_out);

#ifdef __cplusplus
}
#endif
#endif /* MC_H */
