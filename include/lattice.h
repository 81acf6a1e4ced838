/*
 * lattice.h -- C-ABI of liblattice.so: the coupled-pair Metropolis sweep with an
 * exact charge constraint on an L x L periodic lattice of four-state sites,
 * on one MI355X (gfx950).
 *
 * Method: Budrin, Ulitko, Chikov, Panov, Moskvin, arXiv:2301.11735.
 *   Model and energy: section 2.1, eq. (1) and the sigma form eq. (3)
 *     E = Delta sum S_i^2 + V sum_<ij> S_i S_j + (J/4) sum_<ij> sigma_i sigma_j.
 *   Constraint: eq. (2), sum S_i = nN, held exactly at every step.
 *   Update: section 3.1 ("Algorithm"): a coupled pair keeps its charge and
 *     takes a random configuration of the same-charge set, accepted by the
 *     classical Metropolis rule.
 *   Parallel form: section 3.2: only pairs that do not interact are updated
 *     together; partners are long-range random.
 *
 * Site codes (one per site in the canonical layout, row-major, site (x,y) at
 * index y*L + x): 0 = spin up (S=0, sigma=+1), 1 = spin down (S=0, sigma=-1),
 * 2 = charge S=+1, 3 = charge S=-1.
 *
 * Conventions for every call:
 *   - Device pointers are HIP device memory (e.g. from torch.empty on a ROCm
 *     device); host pointers are ordinary host memory.  The caller owns all
 *     memory; the library never allocates or frees device memory.
 *   - Return value 0 on success, or a negative LAT_E* code.  The text of the
 *     last error of the calling thread is returned by lattice_last_error().
 *     No C++ exception crosses this interface: host memory exhaustion inside
 *     a call is returned as LAT_ENOMEM, any other internal failure as
 *     LAT_EHIP.
 *   - A handle is not thread-safe; all of its work is ordered on the stream
 *     given at creation.  Calls that return data to the host synchronise
 *     that stream.
 */
#ifndef PAPER_2301_11735_LATTICE_H
#define PAPER_2301_11735_LATTICE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LAT_OK 0
#define LAT_EINVAL (-1) /* invalid argument (geometry, parameters, codes, null pointer) */
#define LAT_ENOMEM (-2) /* a caller buffer is smaller than required, or host memory ran out */
#define LAT_EHIP (-3)   /* a HIP runtime call failed; see lattice_last_error() */
#define LAT_ESTATE (-4) /* misuse: null or destroyed handle */

/* State encodings of the device buffer.
 *   LAT_ENC_INT8: one code per byte, canonical row-major layout; L % 4 == 0.
 *   LAT_ENC_2BIT: 2 bits per site, N/4 bytes; L % 64 == 0.  Sites are stored
 *     by sublattice class: class c = 4*(y mod 2) + (x mod 4) holds the
 *     (L/4) x (L/2) sites x = 4X + (x mod 4), y = 2Y + (y mod 2); class c
 *     starts at 32-bit word c*(L/2)*(L/64); class row Y is L/64 words; site X
 *     of the row is bits 2*(X mod 16) of word X/16 (little-endian). */
#define LAT_ENC_INT8 0
#define LAT_ENC_2BIT 1

typedef struct lattice lattice; /* opaque host-side handle */

typedef struct {
    int32_t L;            /* side; >= 4 and L % 4 == 0 (int8) or L % 64 == 0 (2-bit) */
    int32_t encoding;     /* LAT_ENC_INT8 or LAT_ENC_2BIT */
    double n;             /* target charge density of eq. (2); |n| <= 1 */
    double Delta, V, J;   /* couplings of eq. (3); finite */
    double T;             /* temperature (k = 1); finite and > 0 */
    uint64_t seed;        /* Philox4x32-10 key */
    int64_t n_charged;    /* number of charged sites at init; -1 = max(N/4, |Q|) */
    uint64_t start_sweep; /* index of the first sweep (0, or a resume point) */
    const int8_t *init_codes; /* NULL: seeded init; else N host codes (row-major)
                                 used verbatim, and Q, Nc are taken from them */
} lat_params;

typedef struct {
    uint64_t sweep;      /* sweeps done so far, counted from start_sweep */
    int64_t sum_S;       /* sum S_i (eq. 2; constant) */
    int64_t n_charged;   /* sum S_i^2 */
    int64_t bond_SS;     /* sum over the 2N bonds of S_i S_j */
    int64_t bond_ss;     /* sum over the 2N bonds of sigma_i sigma_j */
    int64_t M;           /* sum sigma_i */
    int64_t M_stag;      /* sum (-1)^(x+y) sigma_i */
    int64_t C_stag;      /* sum (-1)^(x+y) S_i */
    int64_t track_nD;    /* sum over accepted moves of the change of n_charged */
    int64_t track_nV;    /* ... of bond_SS */
    int64_t track_nJ;    /* ... of bond_ss */
    double E;            /* Delta*n_charged + V*bond_SS + 0.25*J*bond_ss (FP64) */
} lat_obs;

/* Bytes of the device state buffer for side L: N (int8) or N/4 (2-bit).
 * Returns 0 if L is not valid for the encoding. */
size_t lattice_state_bytes(int32_t L, int32_t encoding);

/* Bytes of the device scratch buffer a lattice needs: threshold and
 * transition tables, energy tracker, reduction slots (88 KiB), plus, for an
 * int8 lattice with L % 64 == 0, N/4 bytes for the 2-bit copy its sweeps
 * run on when it is swept by the multi-block kernels. */
size_t lattice_scratch_bytes(int32_t L, int32_t encoding);

/* Charge target of eq. (2) for side L and density n (Q rounded to the
 * parity of the charged count; n_charged = -1 picks max(N/4, |Q|)).
 * Writes Q and the charged count; LAT_EINVAL if none exists. */
int lattice_charge_target(int32_t L, double n, int64_t n_charged, int64_t *Q, int64_t *Nc);

/* Create a lattice: validate p, compute the charge target (eq. 2), build the
 * initial configuration (stage 1 of section 3.1) and the Metropolis threshold
 * table (section 3.1, eq. 3), and copy both to the caller's device buffers on
 * hip_stream (a hipStream_t, or NULL for the default stream).  d_state must
 * hold lattice_state_bytes(), d_scratch lattice_scratch_bytes(); both must
 * stay valid until lattice_destroy.  The copies are asynchronous; host
 * memory of p->init_codes may be reused once the call returns.
 * Errors: LAT_EINVAL (bad geometry, |Q| > Nc, Nc > N, n_charged of the wrong
 * parity, non-finite parameters, T <= 0, codes outside 0..3, null pointers),
 * LAT_ENOMEM (a buffer too small), LAT_EHIP. */
int lattice_create(const lat_params *p, void *d_state, size_t state_bytes, void *d_scratch,
                   size_t scratch_bytes, void *hip_stream, lattice **out);

/* Advance by `sweeps` sweeps (section 3.1 update, section 3.2 parallel form):
 * each sweep is four phases of N/8 non-interacting coupled pairs, so every
 * site is updated once per sweep.  Asynchronous on the handle's stream.
 * Lattices with L % 64 == 0 and 256 < L <= 1024 advance in one cooperative
 * launch per call, whose blocks must all be resident at once, with a
 * device-wide barrier after every phase: kernels of other streams running
 * at the same time can delay it, and a barrier that waits longer than about
 * 0.2 s (LATTICE_BARRIER_TICKS: another bound, in 10 ns ticks of the device
 * clock) marks the state invalid, which the next read (lattice_observables,
 * lattice_observables_batch, lattice_series_read) reports as LAT_EHIP.
 * LATTICE_WORDS_PERSISTENT=0 in the environment at the call selects one
 * launch per phase instead; set it for calls captured into a HIP graph,
 * whose kernel nodes do not guarantee that all blocks are resident at once.
 * Errors: LAT_ESTATE, LAT_EHIP. */
int lattice_sweep(lattice *h, uint32_t sweeps);

/* Reduce the current configuration to its integer observables, read the
 * incremental energy tracker, and fill *out (E in FP64 on the host).
 * Synchronises the handle's stream.  Errors: LAT_ESTATE, LAT_EINVAL, LAT_EHIP. */
int lattice_observables(lattice *h, lat_obs *out);

/* An observation series kept on the device: `intervals` times, advance the
 * lattice by `every` sweeps and write its observables (the values
 * lattice_observables would return) into record k of d_series, with no host
 * synchronisation in between.  Lattices on the persistent multi-block path
 * take the records from the sums before the series plus the tracked moves
 * (integers, equal to a reduction of the configuration); the others reduce
 * the configuration after each interval.  Record k is 88 bytes at byte 88k: 11 int64,
 * the tracker (nD, nV, nJ), the 7 sums in lat_obs order from sum_S to
 * C_stag, and the sweep index after the interval (start_sweep + sweeps
 * done).  d_series is caller-owned device memory of at least 88*intervals
 * bytes.  Asynchronous on the handle's stream; read the records with
 * lattice_series_read.  Errors: LAT_ESTATE, LAT_EINVAL (every == 0, null
 * d_series), LAT_ENOMEM (d_series too small), LAT_EHIP. */
int lattice_sweep_series(lattice *h, uint32_t intervals, uint32_t every, void *d_series, size_t series_bytes);
/* Synchronise the handle's stream and convert `intervals` records of
 * d_series (written by lattice_sweep_series on this handle) into out.
 * Errors: LAT_ESTATE, LAT_EINVAL, LAT_EHIP. */
int lattice_series_read(lattice *h, const void *d_series, uint32_t intervals, lat_obs *out);

/* Copy the configuration to N host codes in the canonical row-major layout.
 * Synchronises the handle's stream.  Errors: LAT_ESTATE, LAT_EINVAL, LAT_EHIP. */
int lattice_read_state(lattice *h, int8_t *host_codes);

/* Advance `count` lattices by `sweeps` sweeps each, on hip_stream (section
 * 3.2: several lattice copies processed together).  Lattices may differ in
 * L, encoding, parameters and seed; results are identical to calling
 * lattice_sweep on each.  Lattices on the on-chip path (L <= 256 with
 * L % 64 == 0, L <= 512 otherwise) advance together in one launch per 256 of
 * them, each resident in on-chip memory for all the sweeps; those with
 * L % 64 == 0 up to 2048 advance together on the multi-block word kernel (one
 * cooperative launch per 64 of them up to L = 1024, as lattice_sweep, else
 * one launch per phase); larger ones one after another.  The caller orders hip_stream
 * after any pending work of the lattices' own streams.  A lattice may appear
 * only once.  Errors: LAT_EINVAL, LAT_ESTATE, LAT_EHIP. */
int lattice_sweep_batch(lattice *const *hs, int32_t count, uint32_t sweeps, void *hip_stream);

/* Observables of `count` lattices (as lattice_observables) with one reduction
 * launch per 256 lattices and one device-to-host copy.  d_out is caller-owned
 * device scratch of at least 80*count bytes; out receives `count` records.
 * Synchronises hip_stream.  Errors: LAT_EINVAL, LAT_ENOMEM, LAT_ESTATE,
 * LAT_EHIP. */
int lattice_observables_batch(lattice *const *hs, int32_t count, void *d_out, size_t out_bytes, lat_obs *out,
                              void *hip_stream);

/* lattice_observables_batch for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * allocation): the same records, with the device staging taken from a
 * static array inside the library instead of a caller buffer.  The array
 * holds 1024 records (80 KiB) on each device the library runs on, for the
 * life of the process; the current device of the calling thread must be the
 * lattices' device.  The call allocates no device memory and keeps its host
 * staging on the stack.  Every call on a device shares that device's array:
 * calls that overlap on one device (other threads, other streams) race and
 * must be serialised by the caller.  Synchronises hip_stream.
 * Errors: LAT_EINVAL (count < 0 or > 1024, null pointers), LAT_ESTATE,
 * LAT_EHIP. */
int lattice_observables_batch_noalloc(lattice *const *hs, int32_t count, lat_obs *out, void *hip_stream);

/* Batched observation intervals captured once into a HIP graph (section 3.2,
 * lattice copies advanced together).  One replay runs `intervals` intervals;
 * each advances the `count` lattices by `sweeps` sweeps and reduces their
 * observables into its own slot of the device buffer d_out (slot k at byte
 * 80*count*k, 80 bytes per lattice, as lattice_observables_batch), so a whole
 * observable series is produced with one graph launch and read with one copy.
 * Every lattice must take the on-chip batched path (L <= 256 with
 * L % 64 == 0, L <= 512 otherwise) or the multi-block word path (L % 64 == 0
 * up to 2048, one launch per phase in the graph).  The capture runs on a
 * private stream and launches nothing; replays run on hip_stream, which the
 * caller orders after the lattices' other work.  The lattices and d_out must
 * outlive the graph.
 * Errors: LAT_EINVAL (empty or duplicate batch, sweeps == 0, intervals == 0,
 * a lattice on neither path, null pointers), LAT_ENOMEM (d_out smaller than
 * 80*count*intervals bytes), LAT_ESTATE, LAT_EHIP. */
typedef struct lat_batch_graph lat_batch_graph;
int lattice_batch_graph_create(lattice *const *hs, int32_t count, uint32_t sweeps, uint32_t intervals, void *d_out,
                               size_t out_bytes, void *hip_stream, lat_batch_graph **out);
/* Enqueue `times` replays on the graph's stream (asynchronous).  Errors:
 * LAT_ESTATE, LAT_EHIP. */
int lattice_batch_graph_launch(lat_batch_graph *g, uint32_t times);
/* Synchronise the graph's stream and convert d_out, as written by the last
 * replay, into intervals*count records (interval-major: record k*count + i is
 * lattice i after interval k).  Errors: LAT_ESTATE, LAT_EINVAL, LAT_EHIP. */
int lattice_batch_graph_read(lat_batch_graph *g, lat_obs *out);
/* Synchronise the graph's stream and release the graph (caller memory
 * untouched).  Errors: LAT_ESTATE, LAT_EHIP. */
int lattice_batch_graph_destroy(lat_batch_graph *g);

/* ---------------------------------------------------------------------------
 * Serving: simulation requests that arrive while others run.  The server
 * admits queued requests, in arrival order, into the caller's device pool when
 * a slot and pool memory are free; every call of lat_server_step advances all
 * resident requests together (section 3.2: lattice copies processed
 * together), then harvests the finished ones and frees their memory, so new
 * requests join between steps.  Lattices that fit one compute unit's on-chip
 * memory by default (L <= 256, or L % 64 != 0) share one batched launch on
 * the server's stream, each by about the same time on its compute unit:
 * max(1, quantum_updates / (N + 11000)) sweeps, capped by what the request
 * still needs (a sweep costs about N + 11000 site-update times, the constant
 * being its fixed per-phase cost).  The others (L = 320 .. 512, L % 64 == 0)
 * advance on a second stream of the server at its own pace, spread over many
 * compute units (one launch per phase holds all of them): a thread of the
 * server keeps up to three chunks in flight there, each of
 * max(1, quantum_updates / 50000) sweeps of every such lattice, and a step
 * harvests them once the chunk holding their last sweep has completed.
 * The server's calls must come from one thread at a time.  A request's result is bit-identical to
 * running it alone with lattice_create/lattice_sweep.  Served lattices need
 * L <= 512.  Timestamps are seconds of the monotonic clock (CLOCK_MONOTONIC).
 */
typedef struct lat_server lat_server;

#define LAT_REQ_QUEUED 0
#define LAT_REQ_RESIDENT 1
#define LAT_REQ_FINISHED 2
#define LAT_REQ_FAILED 3 /* could not be set up on the device; `error` says why */

typedef struct {
    uint64_t id;
    int32_t status;          /* LAT_REQ_* */
    int32_t error;           /* LAT_E* code of a failed request, else 0 */
    uint32_t sweeps_total;
    uint32_t sweeps_done;
    double t_submit, t_admit, t_finish;
    lat_obs obs;             /* valid once finished */
} lat_request_info;

typedef struct {
    int32_t queued, resident;
    uint64_t pool_used;      /* bytes of the pool held by resident lattices and the reserved slot */
    uint64_t steps;          /* lat_server_step calls that launched work */
    uint64_t site_updates;   /* site updates launched so far */
} lat_server_counters;

/* d_pool: caller-owned device memory the server carves lattices from (each
 * takes lattice_state_bytes + lattice_scratch_bytes, 256-byte aligned; the
 * first 80*max_slots bytes, rounded up, are reserved for observables).
 * Errors: LAT_EINVAL, LAT_ENOMEM. */
int lat_server_create(void *d_pool, size_t pool_bytes, int32_t max_slots, uint64_t quantum_updates,
                      void *hip_stream, lat_server **out);
/* Queue a request to run `sweeps` sweeps of the lattice p describes (p is
 * copied).  keep_state != 0 keeps the final codes for lat_server_poll.  The
 * parameters get lattice_create's checks here, so a request that could never
 * be set up is refused at once instead of reaching the queue.
 * Errors: LAT_ESTATE, LAT_EINVAL (as lattice_create, or L > 512). */
int lat_server_submit(lat_server *s, const lat_params *p, uint32_t sweeps, int32_t keep_state, uint64_t *id);
/* Admit, advance every resident request once, harvest finished ones.  A
 * request whose set-up fails at admission is marked LAT_REQ_FAILED (with its
 * error code) and the queue moves on.  Synchronises the server's stream when
 * requests are admitted or finish.  Errors: LAT_ESTATE, LAT_EHIP. */
int lat_server_step(lat_server *s, int32_t *n_finished);
/* State of a request; final_codes (N host codes, may be NULL) is filled for a
 * finished request submitted with keep_state.  Errors: LAT_ESTATE, LAT_EINVAL. */
int lat_server_poll(lat_server *s, uint64_t id, lat_request_info *out, int8_t *final_codes);
/* Forget a finished or failed request.  Errors: LAT_ESTATE, LAT_EINVAL. */
int lat_server_release(lat_server *s, uint64_t id);
int lat_server_stats(lat_server *s, lat_server_counters *out);
/* Destroy the server and any resident lattices (caller memory untouched). */
int lat_server_destroy(lat_server *s);

/* Map mode (section 3.2 as the paper builds it): apply maps first_map ..
 * first_map + n_maps - 1.  Map m of a lattice is a list of non-interacting
 * coupled pairs built with the paper's sequential algorithm from the
 * lattice's seed.  Draw k of map m is the word w = word k mod 4 of
 * Philox4x32-10 at counter (m_lo, 0x400, k / 4, m_hi) with the seed as key.
 *   partner = LAT_MAP_ANY (the paper's algorithm): max(1, N/10) pairs; a
 *     draw gives site floor(w N / 2^32); draw until an unmarked site comes up
 *     (site a, marked), the same for its partner b, record (a, b), mark the
 *     neighbours of both, repeat.  a and b may be neighbours; the bond
 *     between them then enters the energy change once.
 *   partner = LAT_MAP_NEIGHBOUR (the paper's first version, kept to show its
 *     loss of ergodicity): max(1, N/20) pairs; a draw gives a; if a is marked
 *     the next draw starts over, else the next draw picks b = neighbour
 *     w >> 30 of a (order x+1, x-1, y+1, y-1); if b is marked the pair is
 *     dropped, else a, b and the neighbours of both are marked and (a, b)
 *     is recorded.
 * No two pairs of a map interact, so they are updated concurrently.  Pair i
 * of the map takes words 2(i mod 2) (configuration) and 2(i mod 2)+1
 * (acceptance) of Philox at counter (m_lo, 0x500, i / 2, m_hi).  Maps are
 * built on the device; the lattice must have L <= 256.  The sweep counter of
 * the handle is not changed.  Asynchronous on the handle's stream.
 * Errors: LAT_ESTATE, LAT_EINVAL (L > 256, unknown partner rule), LAT_EHIP. */
#define LAT_MAP_ANY 0
#define LAT_MAP_NEIGHBOUR 1
int lattice_map_steps(lattice *h, uint64_t first_map, uint32_t n_maps, int32_t partner);
/* The same for `count` lattices in one launch (one block per lattice, up to
 * 256 per launch), on hip_stream.  Each lattice uses its own seed, so its
 * maps are its own.  Errors: LAT_EINVAL (bad batch, duplicate, L > 256,
 * unknown partner rule), LAT_ESTATE, LAT_EHIP. */
int lattice_map_steps_batch(lattice *const *hs, int32_t count, uint64_t first_map, uint32_t n_maps,
                            int32_t partner, void *hip_stream);

/* Penalty mode (section 2.2): the prior method the paper replaces, kept to
 * show why.  The energy gets the term -mu * sum_i S_i and sites are updated
 * one at a time (checkerboard colours c = (x+y) mod 2, c = 0 first), so the
 * charge is free to change; after every sweep mu is adjusted by the
 * proportional controller mu += kappa * (Q - sum S) / N (Q: the handle's
 * target charge; the paper says only that mu is adjusted automatically).
 * Site k of colour c (row k / (L/2), column 2 (k mod L/2) + ((row + c) & 1))
 * in sweep s proposes code w >> 30 from word 2(k mod 2) of Philox at counter
 * (s_lo, 0x600 + c, k / 2, s_hi), the next word being its acceptance draw;
 * thresholds of dE = Delta nD + V nV + (J/4) nJ - mu dS follow the convention
 * of the coupled-pair mode.  Runs sweeps first_sweep .. first_sweep +
 * n_sweeps - 1 and synchronises the handle's stream after each (the
 * controller needs sum S).  *mu is the starting mu on entry and the next
 * sweep's mu on return; mu_series / sumS_series (each n_sweeps long, may be
 * null) receive the mu of every sweep and sum S after it.  The tracker keeps
 * counting the physical energy (without the penalty term).  Int8 lattices
 * only.  Errors: LAT_ESTATE, LAT_EINVAL (2-bit lattice, null or non-finite
 * mu, non-finite kappa), LAT_EHIP. */
int lattice_mu_sweeps(lattice *h, uint64_t first_sweep, uint32_t n_sweeps, double kappa, double *mu,
                      double *mu_series, int64_t *sumS_series);

/* Release the handle (host memory only; caller buffers are untouched). */
int lattice_destroy(lattice *h);

/* Text of the last error on the calling thread ("" if none). */
const char *lattice_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_2301_11735_LATTICE_H */
