/*
 * pmc.h - C ABI of the MI355X (gfx950) proton-transport Monte Carlo engine.
 *
 * The engine computes dose by condensed-history Monte Carlo transport of
 * proton histories through a voxelised CT, following Wan Chan Tseung, Ma &
 * Beltran, "A fast GPU-based Monte Carlo simulation of proton transport with
 * detailed modeling of non-elastic interactions" (arXiv:1409.8336):
 *   - geometry from HU via a piecewise material table (Sec. II.A.1);
 *   - stopping power with water scaling, Eq. 1, and range scaling, Eq. 2
 *     (Sec. II.A.2); titanium-like bins use their own tables;
 *   - Highland multiple scattering x F (Sec. II.A.2), Gaussian straggling;
 *   - steps limited by the nuclear distance, the voxel boundary and the
 *     residual range, with a random hinge (Sec. II.A.3);
 *   - nuclear elastic scattering, Eq. 3 (Sec. II.A.5), and non-elastic events
 *     emitting secondary protons from a per-nucleus table (Sec. II.A.4);
 *   - N histories in K statistical groups, dose and its variance
 *     (Sec. II.B.2).
 *
 * Every entry point is a plain C function taking plain pointers and sizes and
 * returning a pmc_status; no C++ exception crosses this boundary.  On error
 * the outputs are left untouched and pmc_last_error() returns a message.
 *
 * Conventions used throughout:
 *   - 3-D arrays (HU, dose, variance) are [nz][ny][nx], x fastest.
 *   - The grid spans [0,nx*dx) x [0,ny*dy) x [0,nz*dz) cm.  Beam spots start
 *     on the z = 0 face, travelling along +z, with zero divergence.
 *   - Element order of every per-element array: H, C, N, O, P, Ca, Ti.
 *   - Tabulated nuclear data live on the energy grid
 *     E_i = 0.1 * 2500^(i/999) MeV, i = 0..999, linear in ln E between points.
 *   - Dose is dose to medium in Gy per unit primary weight; variance is the
 *     variance of that estimate from the K groups, in Gy^2.
 *   - Random numbers: Philox4x32-10 keyed by the run seed, counter =
 *     (particle uid, step index, tag); results depend only on the seed and the
 *     inputs, not on launch shape, up to the order of floating-point sums.
 *   - Threading: a context may be used by one host thread at a time.
 */
#ifndef PMC_H
#define PMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PMC_OK = 0,
    PMC_ERR_ARG = -1,            /* NULL pointer, bad size or inconsistent table */
    PMC_ERR_RANGE = -2,          /* spot energy outside (0.1, 250] MeV, negative weight or width */
    PMC_ERR_NOMEM = -3,          /* device or host allocation failed */
    PMC_ERR_DEVICE = -4,         /* HIP runtime error (message in pmc_last_error) */
    PMC_ERR_QUEUE_OVERFLOW = -5, /* secondary queue full: dose incomplete, energy counted as overflow */
    PMC_ERR_STATE = -6           /* call order: physics and geometry must be loaded first */
} pmc_status;

/* Test switches: the closed-form special cases of the method; and the
 * straggling and multiple-scattering models. */
enum {
    PMC_NO_STRAGGLE = 1u,  /* mean energy loss only */
    PMC_NO_MCS = 2u,       /* no angular deflection */
    PMC_NO_NUCLEAR = 4u,   /* no elastic or non-elastic nuclear events */
    PMC_VAVILOV = 8u,      /* Vavilov-Gaussian straggling (Sec. II.A.2): the loss of a step
                              is <Delta> + sigma W, sigma^2 Bohr's variance, W the
                              standardised Vavilov variable of the step's kappa = xi/T_max
                              and beta^2 when kappa is in [0.01, 10), else standard normal;
                              W drawn by mapping the step's normal score through the
                              quantile table pmc_vavilov_table returns (trilinear).
                              Default (flag clear): W standard normal */
    PMC_MOLIERE = 16u,     /* Molière multiple scattering (Sec. II.A.2's full Molière option)
                              instead of the scaled Highland Gaussian, on steps where
                              Bethe's B (B - ln B = ln(chi_c^2 / 1.167 chi_a^2)) is at
                              least 4.5; chi_c^2 = K m_e c^2 rho s sum w Z(Z+1)/A / (p beta)^2,
                              the screening angle from the Z(Z+1)/A-weighted logs of the
                              elements' chi_0^2 (1.13 + 3.76 (Z alpha / beta)^2); polar
                              angle chi_c sqrt(B) v with v^2 = q R(q, 1/B), q = -ln u, from
                              the table pmc_moliere_table returns (bilinear), at most pi.
                              Steps with B < 4.5 keep the Highland Gaussian (f_mcs applies
                              there only) */
    PMC_INC = 64u          /* non-elastic events by the intranuclear cascade and evaporation
                              of Sec. II.A.4 (pmc_inc_events describes the model) instead of
                              the per-nucleus secondary tables of pmc_nuclear_data: the
                              transport lists each event and stops the proton; after each
                              transport generation a cascade kernel works the list (FP64),
                              queues the protons it emits above 0.1 MeV for the next
                              generation, deposits the kinetic energy of heavier fragments
                              and sub-cut-off protons in the event's voxel and books
                              neutrons, separation energies and the residual excitation as
                              neutral.  The event list holds queue_capacity events per
                              generation (0: max(65536, N)); beyond it the event's energy is
                              overflow and the run returns PMC_ERR_QUEUE_OVERFLOW */
};

typedef struct {
    double f_mcs;            /* Highland width multiplier; 1.07 in the paper (Sec. II.A.2) */
    double s_min_cm;         /* shortest step unless range-limited; 1e-4 cm */
    int32_t k_batches;       /* statistical groups; 10 in the paper (Sec. II.B.2), 2..64 */
    uint32_t flags;          /* PMC_NO_* */
    uint32_t queue_capacity; /* secondary-queue entries per generation; 0 = automatic */
    int32_t block_threads;   /* transport workgroup size (64..1024, multiple of 64); 0 = tuned */
    int32_t blocks_per_cu;   /* resident workgroups per CU for the persistent grid; 0 = occupancy */
    int32_t refill_lanes;    /* a wave refills when at least this many of its 64 lanes are idle; 0 = tuned */
    int32_t batch_events;    /* a wave handles pending nuclear events once this many lanes wait; 0 = tuned */
    int32_t tally_cache;     /* LDS deposit cache per workgroup: slots, 512..16384; 0 = automatic
                                (the tuner may turn it off, else sized from the LDS left by the
                                tables); -1 = off (every deposit is a global FP64 atomic) */
    int32_t epoch_steps;     /* loop iterations between epoch ends (cache flush, own-queue
                                publication); 0 = 32 */
    int32_t cache_probes;    /* cache slots tried per deposit (linear probing), 1..16; 0 = 3 */
    int32_t claim_run_log2;  /* a workgroup claims primaries in runs of up to 2^claim_run_log2
                                consecutive histories (a pencil's worth for the cache), 4..16;
                                0 = 10 */
    int32_t local_queue;     /* secondary protons a workgroup queues for its own lanes within a
                                launch (entries of 48 B per workgroup), 1..65536; 0 = up to
                                65536 within 1 GiB for the grid;
                                -1 = off (every secondary waits for the next generation launch) */
} pmc_params;
/* Autotuning: when any of block_threads, refill_lanes, batch_events is 0 and
 * a run has at least 2e5 histories, the first run of each workload signature
 * (single/batched, plan count, log2 of histories and voxels) times the
 * candidate launch shapes (workgroup size, refill and event thresholds, LDS
 * deposit cache on or off) on the first spots of every plan, a fifth of the
 * run (2e5 to 2e6 histories), times the three fastest twice more, and keeps
 * the one with the best of its times for that signature.  Results do not
 * depend on the shape. */

/* Fill *p with the defaults above.  Never fails for a non-NULL p. */
pmc_status pmc_default_params(pmc_params* p);

typedef struct {
    float x_cm, y_cm;          /* spot centre on the z = 0 face */
    float e_mev;               /* kinetic energy, (0.1, 250] */
    float sigma_x_cm, sigma_y_cm; /* Gaussian lateral widths (>= 0) */
    float weight;              /* relative weight (>= 0); histories are shared in proportion */
} pmc_spot;

/* HU -> material conversion (Sec. II.A.1).  Bin b covers HU in
 * [hu_lo[b], hu_lo[b+1]) (the last bin ends at 3000); density rises linearly
 * from rho_lo[b] to rho_hi[b] across the bin; composition and mean excitation
 * energy are constant within a bin.  own_table[b] != 0 marks a bin (at most
 * one, titanium in the paper) whose stopping power comes from its own
 * Bethe-Bloch table instead of water scaling.  HU outside [-1000, 3000] is
 * clipped.  All arrays hold n_bins entries (mass_frac n_bins x 7, rows sum to
 * 1); hu_lo ascending with hu_lo[0] <= -1000; 1 <= n_bins <= 16. */
typedef struct {
    int32_t n_bins;
    const int16_t* hu_lo;
    const float* rho_lo;     /* g/cm^3 */
    const float* rho_hi;     /* g/cm^3 */
    const float* mass_frac;  /* n_bins x 7 */
    const float* i_ev;       /* mean excitation energy, eV */
    const int32_t* own_table;
} pmc_material_table;

/* Nuclear data (Sec. II.A.4-5).  Cross sections per element on the energy
 * grid; non-elastic secondaries per nucleus C..Ti (6) and incident-energy bin
 * of 10 MeV (25 bins):
 *   mult_cdf[n][j][m]  P(secondary protons <= m), m = 0..4, last entry 1
 *   f_local[n][j]      fraction of the incident energy deposited locally
 *   x_cdf[n][j][i]     CDF of E_secondary/E_incident at i/32, i = 0..32
 *   mu_cdf[n][j][i]    CDF of the polar cosine at -1 + 2i/32, i = 0..32 */
typedef struct {
    const float* sigma_ne_barn;   /* 7 x 1000 */
    const float* sigma_el_barn;   /* 7 x 1000 */
    const float* mult_cdf;        /* 6 x 25 x 5 */
    const float* f_local;         /* 6 x 25 */
    const float* x_cdf;           /* 6 x 25 x 33 */
    const float* mu_cdf;          /* 6 x 25 x 33 */
} pmc_nuclear_data;

/* Run ledger and counters.  Energies are weighted MeV; the identity
 * incident = deposited + escaped + neutral + overflow holds to rounding. */
typedef struct {
    double incident, deposited, escaped, neutral, overflow;
    uint64_t histories, steps, secondaries, n_elastic, n_nonelastic, n_overflow;
                           /* secondaries: protons emitted by nuclear events (taken by the
                              emitting workgroup, this plan, plus those that went through the
                              generation queues, whole run) */
    uint64_t n_short_steps; /* steps lengthened to s_min (sub-micron boundary approaches) */
    uint64_t tally_atomics; /* energy deposits scored (one per step, event or termination;
                               with LET_d scoring also its own deposits) */
    double total_weight;   /* sum of primary weights (dose normalisation) */
    double device_ms;      /* device time of the run, HIP events */
    double transport_ms;   /* sum over transport launches of their HIP-event durations */
    int32_t generations;   /* generations run: the primaries' and each secondary generation
                              that had work (with the workgroup queues on, usually 1) */
    int32_t launches;      /* transport launches issued (generations are launched in groups;
                              launches past the empty generation exit at once) */
    uint64_t global_atomics; /* FP64 atomic adds that reached the tally in device memory
                                (deposits that missed the LDS cache plus cache flushes) */
    int32_t block_threads;   /* launch shape used: workgroup size, */
    int32_t grid_blocks;     /* workgroups in the persistent grid, */
    int32_t cache_slots;     /* deposit-cache slots per workgroup (0 = off), */
    int32_t epoch_steps;     /* loop iterations between epoch ends (cache flush, own-queue
                                publication) */
    uint64_t cache_flush_atomics; /* of global_atomics, those the epoch flushes issued (the rest
                                     are deposits that found no cache slot) */
    int32_t refill_lanes;    /* launch shape used (continued): refill and event thresholds */
    int32_t batch_events;
    double first_launch_ms;  /* HIP-event duration of the first transport launch (generation 0;
                                with the workgroup queues on it holds the whole transport, the
                                following launch only confirms that nothing overflowed) */
    uint64_t inc_events;     /* PMC_INC: non-elastic events worked by the cascade kernel, */
    uint64_t inc_secondaries; /* the protons it queued (also counted in secondaries), */
    uint64_t inc_collisions; /* the allowed nucleon-nucleon collisions of their cascades */
    double inc_ms;           /* PMC_INC: sum of the cascade launches' HIP-event durations */
} pmc_summary;

typedef struct pmc_ctx pmc_ctx;

/* Create a context on HIP device `device` with params p (NULL = defaults).
 * *out receives the context, owned by the caller until pmc_destroy.
 * Errors: PMC_ERR_ARG (out NULL, params out of range), PMC_ERR_DEVICE. */
pmc_status pmc_create(pmc_ctx** out, int device, const pmc_params* p);

/* Release every device buffer of the context.  NULL is accepted. */
pmc_status pmc_destroy(pmc_ctx* c);

/* Message for the last error on this context (never NULL; "" if none).
 * With c == NULL: the last error of pmc_create on this thread. */
const char* pmc_last_error(const pmc_ctx* c);

/* Upload nuclear data (copied; the caller keeps ownership of nd).
 * Errors: PMC_ERR_ARG (NULL arrays, negative cross sections, CDFs that do
 * not start at 0 and end at 1), PMC_ERR_NOMEM, PMC_ERR_DEVICE. */
pmc_status pmc_load_physics(pmc_ctx* c, const pmc_nuclear_data* nd);

/* Build the voxel records (density, material) of an HU grid and the
 * per-material tables (Sec. II.A.1-2, Eq. 1-2).  hu has nx*ny*nz int16 in
 * [nz][ny][nx] order, copied to the device; dx,dy,dz voxel size in cm.
 * Replaces the previous geometry.  Errors: PMC_ERR_ARG (dims <= 0, voxel
 * size <= 0, bad material table), PMC_ERR_NOMEM, PMC_ERR_DEVICE. */
pmc_status pmc_load_geometry(pmc_ctx* c, const int16_t* hu, int nx, int ny, int nz,
                             float dx_cm, float dy_cm, float dz_cm,
                             const pmc_material_table* mt);

/* Transport n_histories primaries shared over the spots in proportion to
 * their weights (largest remainder), seed = Philox key, and write dose and
 * variance (host arrays of nx*ny*nz doubles) and the ledger (summary may be
 * NULL).  Errors: PMC_ERR_STATE (no physics/geometry), PMC_ERR_ARG (NULL
 * outputs, n_spots <= 0 with n_histories > 0), PMC_ERR_RANGE (spot values),
 * PMC_ERR_QUEUE_OVERFLOW (outputs written, dose incomplete), PMC_ERR_NOMEM,
 * PMC_ERR_DEVICE.  n_histories == 0 writes zeros. */
pmc_status pmc_run_spots(pmc_ctx* c, const pmc_spot* spots, int n_spots, uint64_t n_histories,
                         uint64_t seed, double* dose_out, double* var_out, pmc_summary* summary);

/* As pmc_run_spots, with dose and variance written into caller-owned device
 * buffers (nx*ny*nz doubles each; var may be NULL) in stream order on
 * `hip_stream` (a hipStream_t; NULL = the null stream).  spots is a host
 * array.  The call returns after the run has completed on the stream. */
pmc_status pmc_run_spots_dev(pmc_ctx* c, const pmc_spot* spots, int n_spots, uint64_t n_histories,
                             uint64_t seed, double* d_dose, double* d_var, void* hip_stream,
                             pmc_summary* summary);

/* As pmc_run_spots_dev, and the dose-averaged LET (LET_d, Sec. III and its
 * LET_d maps) of every voxel in keV/um into the caller-owned device buffer
 * d_let (nx*ny*nz doubles, [nz][ny][nx]), computed in the same transport:
 *   LET_d(v) = sum(w eps L) / sum(w eps)
 * over the proton steps (primaries and secondary protons) that start in v,
 * eps the step's deposit (with straggling; the whole energy on a step the
 * range ends) and L the stopping power of v's medium averaged over the
 * step's mean energy loss (over the residual range when the range ends the
 * step).  Energy deposited outside any step (recoil nuclei and the local
 * share of nuclear events, sub-cut-off secondaries and track rests) is not
 * scored, as the paper's LET_d leaves out heavy recoils.  0 where no step
 * deposited.  Dose and variance are those pmc_run_spots_dev gives.  The
 * tally holds two extra FP64 planes (16 bytes per voxel).  Errors: as
 * pmc_run_spots_dev; PMC_ERR_ARG also for d_let NULL. */
pmc_status pmc_run_spots_let_dev(pmc_ctx* c, const pmc_spot* spots, int n_spots, uint64_t n_histories,
                                 uint64_t seed, double* d_dose, double* d_var, double* d_let,
                                 void* hip_stream, pmc_summary* summary);

/* As pmc_run_spots with LET_d (keV/um) into the host array let_out as well. */
pmc_status pmc_run_spots_let(pmc_ctx* c, const pmc_spot* spots, int n_spots, uint64_t n_histories,
                             uint64_t seed, double* dose_out, double* var_out, double* let_out,
                             pmc_summary* summary);

/* Load a further geometry for batched runs (configurations with many CTs).
 * Same arguments as pmc_load_geometry, which must have been called first; the
 * material table must equal the one already loaded.  *geometry_id_out
 * receives the slot (>= 1; slot 0 is pmc_load_geometry's).  At most 64 slots.
 * Errors: PMC_ERR_STATE (no base geometry), PMC_ERR_ARG, PMC_ERR_NOMEM,
 * PMC_ERR_DEVICE. */
pmc_status pmc_load_geometry_slot(pmc_ctx* c, int* geometry_id_out, const int16_t* hu, int nx, int ny,
                                  int nz, float dx_cm, float dy_cm, float dz_cm,
                                  const pmc_material_table* mt);

/* One plan of a batched run: n_histories over its spots on geometry slot
 * geometry_id, dose and variance into caller-owned device buffers of that
 * geometry's voxel count (d_var may be NULL), optional host summary, and
 * optionally LET_d as pmc_run_spots_let_dev gives it (d_let NULL = not
 * wanted; when any plan of a batch asks for it, the whole launch scores it). */
typedef struct {
    int32_t geometry_id;
    int32_t n_spots;
    const pmc_spot* spots;     /* host array */
    uint64_t n_histories;      /* < 2^32 per plan */
    double* d_dose;
    double* d_var;
    pmc_summary* summary;      /* host, may be NULL */
    double* d_let;             /* LET_d, keV/um, or NULL */
} pmc_plan;

/* Transport every plan in one persistent launch per secondary generation:
 * the histories of all plans form one work list shared by all waves, each
 * with its plan's geometry, tally and random key seed + plan index, so plan p
 * gives exactly the result of pmc_run_spots_dev on its geometry with seed + p
 * (up to floating-point summation order).  Plans must use distinct geometry
 * slots; 1 <= n_plans <= 64.  Runs on hip_stream and returns when done.
 * The device/transport times and generation count in the summaries are those
 * of the whole batch.  Errors: as pmc_run_spots_dev. */
pmc_status pmc_run_plans(pmc_ctx* c, const pmc_plan* plans, int n_plans, uint64_t seed, void* hip_stream);

/* Host-side tables the engine built for the loaded physics and geometry, for
 * inspection (no device work).  out_lnr_water/out_lnr_own receive the 1000
 * float32 ln(range) entries (entry 0 is -inf: zero range at 0.1 MeV) of water
 * and of the own-table bin (zeros if none); out_sigma_per_g receives n_bins x
 * 1000 float32 total nuclear cross sections per gram (cm^2/g);
 * out_material receives n_bins x 4 doubles (water-equivalence factor f of
 * Eq. 1, radiation length g/cm^2, Z/A, own-table flag).  Any output may be
 * NULL.  Errors: PMC_ERR_STATE before both loads. */
pmc_status pmc_inspect_tables(const pmc_ctx* c, float* out_lnr_water, float* out_lnr_own,
                              float* out_sigma_per_g, double* out_material, int32_t* out_n_bins);

/* Measurement aid for the dose tally (no physics): time n_atomics FP64
 * atomic adds of zero into the loaded geometry's [voxel][group] tally along
 * straight z tracks started inside the central 40x40-voxel window, issued by
 * a grid of 4 workgroups of 256 lanes per CU on hip_stream.  *ms_out receives
 * the device time scaled to exactly n_atomics.  The tally contents are
 * unchanged.  Errors: PMC_ERR_ARG, PMC_ERR_STATE (no geometry),
 * PMC_ERR_DEVICE. */
pmc_status pmc_atomic_probe(pmc_ctx* c, uint64_t n_atomics, void* hip_stream, double* ms_out);

/* Roofline measurement of the transport on the loaded geometry (single
 * plan, same spots, histories and seed as pmc_run_spots_dev).  The
 * transport's memory work per condensed-history step is one voxel-record
 * gather and one FP64 dose-tally add (Sec. II.A.3 steps, Sec. II.B.2
 * tallies).  This call runs the workload once as a normal run (autotuned
 * shape; transport_ms = its first transport launch), once more with an
 * address trace (the same launch shape; every loop iteration each lane
 * records the tally element its step deposited into), then replays that
 * address stream with the same grid, workgroups, lanes and epochs and none
 * of the physics: the trace alone, the gathers, the deposits as
 * device-memory FP64 atomics, the deposits through the workgroup LDS cache
 * as the transport issues them, and gathers plus cached deposits.  Each
 * replay time includes streaming the trace (4 bytes per lane and
 * iteration; trace_only_ms).  Deposits outside a step (nuclear events,
 * terminations below the cut-off) are not traced: steps_traced of the
 * run's deposits.  Results are written to the context's dose and variance
 * buffers and discarded; the tally is left as the run made it (replays add
 * zero).  Needs about 4 B x lanes x iterations of device memory (8 GB for
 * the 1e7-history field), released on return.  Errors: PMC_ERR_ARG,
 * PMC_ERR_RANGE, PMC_ERR_STATE, PMC_ERR_NOMEM, PMC_ERR_DEVICE. */
typedef struct {
    double transport_ms;      /* the untraced run's first transport launch */
    double trace_only_ms;     /* replay streaming the trace only */
    double gather_ms;         /* + every step's voxel-record gather (8 B) */
    double atomic_ms;         /* + every step's deposit as a device-memory FP64 atomic */
    double cached_atomic_ms;  /* + every step's deposit through the LDS cache, epoch flushes */
    double combined_ms;       /* + gathers and cached deposits together */
    uint64_t steps;           /* steps of the untraced run */
    uint64_t steps_traced;    /* trace entries holding a step (generation 0) */
    uint64_t deposits;        /* deposits of the untraced run (steps and local deposits) */
    uint64_t trace_iters;     /* loop iterations recorded per lane */
    int32_t grid_blocks, block_threads, cache_slots, epoch_steps;
} pmc_replay_result;

pmc_status pmc_roofline_replay(pmc_ctx* c, const pmc_spot* spots, int n_spots, uint64_t n_histories,
                               uint64_t seed, void* hip_stream, pmc_replay_result* out);

/* Memory-bandwidth references on hip_stream: a plain read of `bytes` of
 * device memory (16-byte loads over a grid of 8 workgroups of 256 lanes per
 * CU) and a plain copy of `bytes` to another buffer (`bytes` read and
 * `bytes` written), each the best of three launches; the copy is the
 * reference of known size for HBM byte counters.  Allocates 2 x bytes and
 * frees them on return.  Errors: PMC_ERR_ARG (bytes < 1 MiB or not a
 * multiple of 16, NULL outputs), PMC_ERR_NOMEM, PMC_ERR_DEVICE. */
pmc_status pmc_stream_probe(pmc_ctx* c, uint64_t bytes, void* hip_stream, double* read_ms, double* copy_ms);

/* Mass density (g/cm^3, float32) of every voxel of geometry geometry_id
 * (0 = pmc_load_geometry's) as the transport uses it (the HU calibration of
 * Sec. II.A.1), written to the device array d_rho ([nz][ny][nx]) on
 * hip_stream.  Errors: PMC_ERR_ARG (NULL, unknown id), PMC_ERR_STATE (no
 * geometry), PMC_ERR_DEVICE. */
pmc_status pmc_geometry_density(pmc_ctx* c, int32_t geometry_id, float* d_rho, void* hip_stream);

/* The Vavilov straggling table used with PMC_VAVILOV (host only, no device
 * work): 5 x 31 x 97 floats into out, [beta^2 = k/10, k < 5][log10 kappa =
 * -2 + j/10, j < 31][z = -6 + i/8, i < 97], the quantile G(z) = F_W^-1(Phi(z))
 * of the standardised loss W = (Delta - <Delta>) / sqrt(xi T_max (1 -
 * beta^2/2)) in Vavilov's model (free-electron collisions with transfer
 * density kappa (1 - beta^2 v)/v^2, v = eps/T_max in (0, 1]), from the
 * inversion of its characteristic function.  Built once per process (about
 * a second).  Errors: PMC_ERR_ARG (out NULL or n_floats < 15035). */
pmc_status pmc_vavilov_table(float* out, int32_t n_floats);

/* The Molière sampling table used with PMC_MOLIERE (host only, no device
 * work): 13 x 161 floats into out, [1/B = 1/20 + j (2/9 - 1/20)/12, j < 13]
 * [q = k/8, k < 161], ln(v^2 / q) where P(V > v) = e^-q for the reduced angle
 * V of Bethe's expansion f0 + f1/B + f2/B^2 (1/B clamped to the table's
 * range by the transport).  Built once per process.  Errors: PMC_ERR_ARG
 * (out NULL or n_floats < 2093). */
pmc_status pmc_moliere_table(float* out, int32_t n_floats);

/* Launch layout of the transport kernel, host only (no device work, usable
 * without a GPU).  The run driver lays out and checks every launch with the
 * same code: the workgroup's LDS (Sec. II.B.3 keeps the hot tables in fast
 * on-chip memory; here the table blob, a batch's plan descriptors, the
 * deposit cache's sums, keys and LET numerators, the control words, the
 * staged arguments and a batch's per-plan ledgers and counters) and the
 * sizes of the device buffers the kernel indexes (tally planes, generation
 * and workgroup queues, claim counters, the primary work list). */
typedef struct {
    int32_t block_threads;      /* workgroup size, multiple of 64 in [64, 1024] */
    int32_t grid_blocks;        /* workgroups of the launch; 0 = not yet known
                                   (then the grid-dependent sizes stay 0) */
    int32_t n_plans;            /* [1, 64]; 1 for a single-plan launch */
    int32_t batched;            /* nonzero: the batched-plan kernel */
    int32_t score_let;          /* nonzero: LET_d planes and numerators */
    int32_t k_batches;          /* statistical groups, [2, 64] */
    int32_t n_mat;              /* material bins, [1, 16] */
    int32_t tally_cache;        /* as pmc_params.tally_cache: -1 off, 0 sized from the LDS left */
    int32_t local_queue;        /* as pmc_params.local_queue */
    int32_t n_spots;            /* all plans */
    uint64_t queue_capacity;    /* as pmc_params.queue_capacity (0 = max(65536, N)) */
    uint64_t n_histories;       /* all plans */
    uint64_t max_plan_histories;
    uint64_t max_nvox;          /* largest plan grid, voxels */
} pmc_launch_query;

typedef struct {
    uint64_t lds_bytes;         /* dynamic LDS per workgroup */
    /* LDS regions, 32-bit word offsets from the start of the allocation */
    int32_t blob_words, plan_desc_off, cache_off, key_off, num_off, ctl_off, args_off,
        ledger_off, counter_off, end_words;
    int32_t cache_slots, key_words, tally_planes, local_queue_cap, args_bytes, reserved;
    uint64_t queue_cap;         /* generation queue entries (12 u32 planes each) */
    uint64_t local_queue_words; /* all workgroup queues (12 u32 per entry) */
    uint64_t claim_words;       /* per-generation claim counters (u64) */
    uint64_t order_words;       /* primary work list (u64) */
} pmc_launch_layout;

/* Fills *out for *q and checks it: every LDS region aligned, disjoint and
 * inside the allocation, the allocation within a CU's 160 KiB, every cache
 * key below the free-slot marker, every queue, claim and work-list index
 * inside its buffer.  Returns PMC_OK, or PMC_ERR_ARG with the reason in why
 * (why_len bytes, NUL-terminated; may be NULL) and *out as far as computed.
 * Errors: PMC_ERR_ARG (NULL q/out, or the launch does not fit). */
pmc_status pmc_plan_launch(const pmc_launch_query* q, pmc_launch_layout* out, char* why, int32_t why_len);

/* ---- Intranuclear cascade and evaporation (Sec. II.A.4; flag PMC_INC) ----
 * Targets: element 1..6 = C-12, N-14, O-16, P-31, Ca-40, Ti-48 (the
 * material compositions' C, N, O, P, Ca, Ti).  The model, with the readings
 * taken where the paper is silent or its models' parameters are absent:
 *   - nucleus: Woods-Saxon density, R = 1.16 A^(1/3) (1 - 1.16 A^(-2/3)) fm,
 *     diffuseness 0.55 fm, cut at R + 5 a into 15 equal-thickness shells at
 *     the profile's mean density, normalised to A; protons Z/A of it,
 *     neutrons N/A; a two-component Fermi gas per shell (Fermi momentum
 *     (3 pi^2 rho)^(1/3) hbar c), well depth = Fermi energy + 7 MeV;
 *   - the proton enters at an impact parameter uniform over the outer disc,
 *     refracted at every shell boundary (energy conserved, tangential
 *     momentum kept; total reflection where the normal component would be
 *     imaginary); free paths from free elastic NN cross sections (like
 *     nucleons 22 + 1000/T mb, unlike 30 + 3000/T mb; stand-ins for
 *     Cugnon's) on the partners not yet exhausted; partner momentum uniform
 *     in the shell's Fermi sphere; CM angle from exp(B t), B = 5.5 p^8 /
 *     (7.7 + p^8) (GeV/c)^-2; Pauli blocking: both products above their
 *     Fermi energies; the entry is repeated (at most 64 times) until the
 *     cascade has an allowed collision, else the proton is absorbed;
 *   - excitation of the residual = incident energy - emitted kinetic energy
 *     - 7 MeV per emitted nucleon beyond the first; Weisskopf-Ewing
 *     evaporation of n, p, d, t, 3He, alpha (Weizsaecker binding energies,
 *     Coulomb barriers at R = 1.5 (A_d^(1/3) + a^(1/3)) fm, level density
 *     exp(2 sqrt(A_d U / 8))), isotropic, until no channel is open or A <= 4;
 *   - at most 96 emitted particles per event; FP64 throughout.
 * Random numbers: Philox4x32-10 keyed by seed, counter (uid, ks, tag):
 * cascade particle j's m-th block of entry attempt e uses tag 0x40000000 |
 * e << 20 | j << 12 | m; evaporation step i tag 0x50000000 | i << 8 | r;
 * the uid of an emitted proton with child id is the first two words of the
 * block with tag 0xC0000000 | id. */
typedef struct {
    int32_t n_out;           /* emitted particles in particles[i * 96 ...] */
    int32_t n_coll;          /* allowed NN collisions of the final entry attempt */
    int32_t n_blocked;       /* Pauli-blocked (or no-room) collision candidates, all attempts */
    int32_t attempts;        /* entry attempts (64 and compound = 1: absorbed) */
    int32_t n_esc;           /* nucleons that left the nucleus in the cascade */
    int32_t compound;
    int32_t z_res, a_res;    /* residual after the cascade */
    int32_t z_fin, a_fin;    /* after evaporation */
    int32_t n_flights;       /* flights (to a collision or a shell boundary) of all cascade particles */
    int32_t reserved;
    double e_star;           /* residual excitation from the energy balance, MeV */
    double e_star_sum;       /* the same from the holes and trapped particles (a check) */
    double e_star_fin;       /* excitation left after evaporation (photons, not followed) */
    double binding;          /* 7 MeV per extra cascade nucleon + evaporation separation energies */
} pmc_inc_result;

typedef struct {
    int32_t kind;            /* 0 n, 1 p, 2 d, 3 t, 4 3He, 5 alpha */
    int32_t stage;           /* 0 cascade, 1 evaporation */
    uint32_t id;             /* child id: 0x100 + cascade particle, 0x400 + evaporation step */
    int32_t reserved;
    double t_mev;            /* kinetic energy */
    double dir[3];           /* direction; the incident proton moves along +z */
} pmc_inc_particle;

/* Runs n non-elastic events on the GPU, event i a proton of t_mev[i] on
 * element[i] with random stream (uid[i], ks[i]) under key seed; evaporate =
 * 0 stops after the cascade.  Host buffers: results[n], particles[n * 96]
 * (entries beyond results[i].n_out unspecified).  Device memory is
 * allocated and released inside the call (an inspection entry point; the
 * transport uses the same kernel code on its event lists).  Errors:
 * PMC_ERR_ARG (NULL arrays with n > 0, n < 0, element outside 1..6),
 * PMC_ERR_RANGE (t_mev outside (0, 1000]), PMC_ERR_NOMEM, PMC_ERR_DEVICE. */
pmc_status pmc_inc_events(pmc_ctx* c, const int32_t* element, const double* t_mev, const uint64_t* uid,
                          const uint32_t* ks, int32_t n, uint64_t seed, int32_t evaporate,
                          pmc_inc_result* results, pmc_inc_particle* particles);

/* The cascade's target nucleus, host only: out[0..15] shell boundaries (fm),
 * out[16..30] proton and out[31..45] neutron densities (fm^-3), out[46..60]
 * proton and out[61..75] neutron Fermi kinetic energies (MeV), out[76] the
 * Woods-Saxon radius R (fm), out[77] A.  Errors: PMC_ERR_ARG (out NULL,
 * n_doubles < 78, element outside 1..6). */
pmc_status pmc_inc_nucleus(int32_t element, double* out, int32_t n_doubles);

/* Relative evaporation width of ejectile kind (0..5) from nucleus (z, a) at
 * excitation e_star (MeV), host only, in closed form; *sep and *barrier (may
 * be NULL) get the channel's separation energy and Coulomb barrier.  0 for a
 * closed channel, a kind outside 0..5, or a nucleus beyond the cascade's
 * range (z outside 0..23, a outside 1..49). */
double pmc_inc_width(int32_t z, int32_t a, double e_star, int32_t kind, double* sep, double* barrier);

/* Library version string, e.g. "pmc 0.1 gfx950". */
const char* pmc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PMC_H */
