/*
 * lgf.h -- C ABI of the MI355X (gfx950) lattice Landau gauge-fixing library.
 *
 * The library runs the checkerboard SU(3) relaxation of M. Schroeck and
 * H. Vogt, "Gauge fixing in lattice QCD with multi-GPUs" (arXiv:1305.3440):
 * for every site of one parity it gathers the 8 links touching the site into
 * K(x) (Eq. (8)), maximises Re tr[g(x) K(x)] (Eq. (7)) through the three
 * Cabibbo-Marinari SU(2) subgroups (Eq. (9), Sec. 3) with overrelaxation
 * (Sec. 3.1) or stochastic relaxation (Sec. 3.2), applies g(x) to the 8 links
 * (Eq. (3)), and measures the functional F (Eq. (2)) and the precision theta
 * (Eqs. (4)-(5)), repeating until theta reaches a target (Sec. 4).
 *
 * Conventions shared by every entry point
 *  - dims = {Lt, Lz, Ly, Lx}, each even and >= 2 (the checkerboard needs even
 *    periodic extents), V = Lt*Lz*Ly*Lx <= 2^31.  Direction mu = 0 is t, 1 z,
 *    2 y, 3 x.  Site index s = ((t*Lz + z)*Ly + y)*Lx + x; parity of a site is
 *    (t+z+y+x) mod 2.
 *  - Canonical link array (host or device): double[V][4][3][3][2]
 *    (site, mu, row, column, re/im), 72 doubles per site, 4*V links.
 *  - Device layouts are private to the library; only the canonical array
 *    crosses the boundary.
 *  - Every call enqueues its GPU work on the handle's stream.  Calls that
 *    return host values (measure, store, peek, gauge_fix, ...) synchronise that
 *    stream before returning.  A handle must not be used from two host threads
 *    at once.
 *  - Errors: every entry point returns an lgf_status and never throws;
 *    lgf_last_error() gives a message for the calling thread's last failure.
 */
#ifndef LGF_H
#define LGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LGF_OK = 0,
    LGF_EINVAL = 1,   /* bad argument: null pointer, odd extent, omega/p out of range, size mismatch */
    LGF_ENOMEM = 2,   /* device or host allocation failed */
    LGF_EHIP = 3,     /* a HIP runtime call failed; lgf_last_error() has its message */
    LGF_ENOTCONV = 4, /* gauge_fix reached max_sweeps; the result is still filled in */
    LGF_ENUMERIC = 5, /* F or theta came out NaN or infinite */
    LGF_ESTATE = 6    /* the operation is not valid in the handle's current state */
} lgf_status;

/* Link storage formats.  FP64_18 / FP32_18 store all 9 complex entries;
 * the _12 formats store rows 0 and 1 and rebuild row 2 = conj(row0 x row1)
 * in registers (exact for SU(3)).  Arithmetic is done in the storage
 * precision, except reunitarization and the F/theta reductions, which are FP64
 * for every format. */
typedef enum {
    LGF_FP64_18 = 0,
    LGF_FP32_18 = 1,
    LGF_FP32_12 = 2,
    LGF_FP64_12 = 3,
    /* Sweep format of the fixed-link form only (bulk_format / finish_format
     * of lgf_gauge_fix, lgf_coulomb_gauge_fix and lgf_ensemble_gauge_fix with
     * fixed_links set, and the fixed-link tuning calls), never a storage
     * format of a handle: FP64 arithmetic with g in FP64-12, the read-only
     * links in a split copy -- every real entry x of rows 0 and 1 as hi =
     * fl32(x) plus a 16-bit integer q = round((x - hi) 2^40), read back as
     * hi + q 2^-40, within 2^-40 of x for |x| <= 1 (every SU(3) entry): 72 B
     * per link against 96 B in FP64-12.  Links are re-split from the
     * handle's FP64 field at the start of each gauge fixing, at the precision
     * switch when the finish uses this format. */
    LGF_FP64_12S = 4
} lgf_format;

typedef struct lgf_lattice lgf_lattice;   /* opaque handle: one lattice on one GPU */

/* Parameters of lgf_gauge_fix (Sec. 4: sweep the two parities in turn and
 * iterate until the requested precision).  Defaults: lgf_fix_params_default. */
typedef struct {
    double omega;          /* overrelaxation parameter, [1, 2] (Sec. 3.1) */
    double p_sr;           /* stochastic-relaxation probability, [0, 1] (Sec. 3.2) */
    double theta_target;   /* stop at the first measurement with theta < target */
    double theta_switch;   /* mixed precision: leave bulk_format once theta < switch (0 = never) */
    int bulk_format;       /* format of the bulk sweeps (lgf_format); the handle's own when equal */
    int check_every;       /* sweeps between reunitarize + measure, >= 1 (default 20) */
    int use_graph;         /* capture each chunk of check_every sweeps in a hipGraph (default 1) */
    int finish_format;     /* format of the sweeps after the switch (-1 = the handle's own) */
    int accumulate_g;      /* mixed precision without orbit drift: the FP32 bulk also accumulates
                              g(x) and the FP64 links are rebuilt at the switch as
                              g(x) U(x) g(x+mu)^dag from the untouched FP64 input (needs an FP32
                              bulk, an FP64 finish and an FP64 handle) */
    int separate_measure;  /* 1: reunitarize and measure in two passes of their own after each
                              chunk; 0 (default): inside the chunk's last half-sweep plus one
                              read-only pass over the other parity, where the sweep allows it
                              (overrelaxation, non-temporal, not the t-slice pipeline).  The links
                              are the same; F and theta differ only in the summation order */
    int fixed_links;       /* 1: the sweeps keep the links at their input values and update the
                              gauge transformation g instead (a site field in the sweep format),
                              forming each link g(x) U_mu(x) g(x+mu)^dag (Eq. (3)) in registers;
                              K(x) = g(x) M(x) with M(x) = sum_mu U_mu(x) g(x+mu)^dag +
                              [g(x-mu) U_mu(x-mu)]^dag gives the update of Sec. 3 unchanged.  A
                              half-sweep reads the 8 links and writes only g(x).  Every check_every
                              sweeps each g is reunitarized as it is stored; at the precision switch
                              g is handed over (reunitarized in FP64) and the finish runs on the
                              FP64 links; at the end the handle's links become g U g^dag from the
                              untouched input, an exact gauge transformation of it.  Needs an FP64
                              handle; accumulate_g is implied.  The sweep formats may include
                              LGF_FP64_12S; when the last sweeps ran in it, the result's F and theta
                              (and the stopping test) come from one more measurement on the
                              transformed FP64 links (one more history entry); if that one is not
                              below theta_target, the sweeps go on in FP64-12 from the transformed
                              links (g restarting at 1) while max_sweeps allows.  FP64-12 and
                              LGF_FP64_12S may be paired as bulk and finish in either order.  In
                              FP32-12, FP64-12 and LGF_FP64_12S the sweeps read the links from per-site records
                              by default (an exact copy laid out for the access pattern; see
                              lgf_set_fixed_tuning), built when the run starts and at the switch.
                              0 (default): the sweeps rewrite the links. */
    int64_t max_sweeps;    /* give up after this many full sweeps (default 100000) */
    uint64_t seed;         /* key of the stochastic-relaxation Philox stream */
    uint64_t sweep_offset; /* counter value of the first sweep (for resumed runs) */
} lgf_fix_params;

/* Outcome of lgf_gauge_fix.  Times are in milliseconds, taken with HIP events
 * on the handle's stream. */
typedef struct {
    int64_t sweeps;        /* full sweeps done (a multiple of check_every unless max_sweeps cut it) */
    int64_t sweeps_bulk;   /* of which in bulk_format */
    double theta;          /* last measured theta (Eq. (5)) */
    double F;              /* last measured F (Eq. (2)) */
    int status;            /* LGF_OK or LGF_ENOTCONV / LGF_ENUMERIC */
    int n_history;         /* measurements written to the history buffer */
    double t_total_ms;     /* wall time of the whole call (host clock, links resident) */
    double t_sweep_bulk_ms;   /* sweep kernels in bulk_format */
    double t_sweep_finish_ms; /* sweep kernels in finish_format */
    double t_measure_ms;   /* reunitarize + measure */
    double t_convert_ms;   /* format conversions */
} lgf_fix_result;

/* Message of the calling thread's last failed call ("" if none). */
const char *lgf_last_error(void);

/* Library version string. */
const char *lgf_version(void);

/* Fill *p with the defaults: omega 1.7, p_sr 0, theta_target 1e-14,
 * theta_switch 0, bulk_format -1 and finish_format -1 (= handle's format),
 * accumulate_g 0, check_every 20, use_graph 1, max_sweeps 100000, seed 0,
 * sweep_offset 0. */
lgf_status lgf_fix_params_default(lgf_fix_params *p);

/* Device bytes of a link field of the given dims in the given format
 * (4*V links of 18 or 12 reals); 0 for invalid arguments. */
size_t lgf_required_bytes(const int dims[4], int format);

/* Create a handle for a lattice.
 *  stream:     hipStream_t the handle enqueues on; NULL makes the library
 *              create its own (blocking, default-priority) stream.
 *  device_buf: NULL makes the library allocate the link field; otherwise a
 *              device buffer of at least lgf_required_bytes(dims, format) bytes
 *              that the handle borrows (the caller keeps it alive until
 *              lgf_destroy, and the library never frees it).
 * The links are uninitialised until lgf_load_links or lgf_generate_links. */
lgf_status lgf_create(const int dims[4], int format, void *stream, void *device_buf,
                      size_t buf_bytes, lgf_lattice **out);

/* Release the handle and everything it owns (never a borrowed buffer).
 * NULL is allowed and does nothing. */
lgf_status lgf_destroy(lgf_lattice *h);

/* Current storage format and dims of a handle. */
lgf_status lgf_get_info(const lgf_lattice *h, int dims[4], int *format);

/* Copy a canonical host array (n_doubles == 72*V) into the handle's layout and
 * format (rounding to FP32 and dropping row 2 where the format says so).  The
 * host pointer is read only during the call. */
lgf_status lgf_load_links(lgf_lattice *h, const double *host_canon, size_t n_doubles);

/* Copy the links out to a canonical host array (n_doubles == 72*V); _12
 * formats have row 2 rebuilt. */
lgf_status lgf_store_links(lgf_lattice *h, double *host_canon, size_t n_doubles);

/* Gather the 4 links U_mu(s) of each listed site (host array of n_sites site
 * indices, each in [0, V)) into host_out, n_sites*72 doubles in canonical
 * order.  For spot checks of large lattices without copying the whole field. */
lgf_status lgf_peek_links(lgf_lattice *h, const int64_t *sites, int64_t n_sites,
                          double *host_out);

/* Fill the field with the seeded synthetic links: for every link
 * U = exp(i eps sum_j a_j lambda_j) with a_j ~ N(0,1) (Gell-Mann lambda_j,
 * tr lambda_a lambda_b = 2 delta_ab), projected onto SU(3); if haar != 0 each
 * link is then gauge transformed, U_mu(x) <- g(x) U_mu(x) g(x+mu)^dag
 * (Eq. (3)), by a Haar-random g(x).  Normals come from Philox4x32-10 keyed by
 * the seed, counter (s, mu, call, 1) for a_j and (s, 0, call, 2) for g(s),
 * through Box-Muller with uniforms (w + 1/2) 2^-32.  eps >= 0. */
lgf_status lgf_generate_links(lgf_lattice *h, uint64_t seed, double eps, int haar);

/* Change the storage format of the handle (allocates the new field, converts,
 * frees the old one).  Conversions into an FP64 format reunitarize in FP64.
 * LGF_ESTATE for a handle with a borrowed buffer. */
lgf_status lgf_convert(lgf_lattice *h, int format);

/* One half-sweep (parity 0 or 1) or a full sweep (parity 2: parity 0 then 1)
 * of the relaxation (Sec. 3, Sec. 4): every site x of the parity gets
 * K = sum_mu U_mu(x) + U_mu(x-mu)^dag (Eq. (8) with the neighbour g's already
 * applied to the links), then for the subgroups (0,1), (0,2), (1,2) the SU(2)
 * maximum of Eq. (9), overrelaxed to first order as N[(1-omega) + omega r]
 * (Sec. 3.1), or squared with probability p_sr (Sec. 3.2), and finally
 * U_mu(x) <- G U_mu(x), U_mu(x-mu) <- U_mu(x-mu) G^dag.
 * The stochastic choices use Philox4x32-10 keyed by seed with counter
 * (s, sweep_index, 0, 3); subgroup k squares when word k < floor(p_sr 2^32).
 * omega in [1, 2], p_sr in [0, 1]. */
lgf_status lgf_sweep(lgf_lattice *h, int parity, double omega, double p_sr, uint64_t seed,
                     uint64_t sweep_index);

/* Project every link back onto SU(3) in FP64: normalise row 0, orthogonalise
 * and normalise row 1, row 2 = conj(row0 x row1). */
lgf_status lgf_reunitarize(lgf_lattice *h);

/* F = (1/(3*4*V)) sum_{x,mu} Re tr U_mu(x) (Eq. (2) at g = 1) and
 * theta = (1/(3V)) sum_x tr[Delta(x) Delta(x)^dag] (Eq. (5)) with
 * Delta(x) = sum_mu A_mu(x) - A_mu(x-mu) (Eq. (4)) and
 * A_mu = [(U - U^dag)/(2i)]_traceless, accumulated in FP64 for every format.
 * Either output pointer may be NULL.  Synchronises. */
lgf_status lgf_measure(lgf_lattice *h, double *F, double *theta);

/* Average plaquette (1/(18 V)) sum_x sum_{mu<nu} Re tr[U_mu(x) U_nu(x+mu)
 * U_mu(x+nu)^dag U_nu(x)^dag], accumulated in FP64: gauge invariant, so it
 * tracks how far a run has left the gauge orbit of its input.  Synchronises. */
lgf_status lgf_plaquette(lgf_lattice *h, double *P);

/* Iterate full sweeps until theta < theta_target (Sec. 4).  Every
 * check_every sweeps the links are reunitarized and F, theta measured (also
 * once before the first sweep).  Mixed precision: when bulk_format differs
 * from finish_format (theta_switch > 0 required), the sweeps run on a copy in
 * bulk_format until a measurement gives theta < theta_switch; the copy is then
 * converted to finish_format (reunitarized in FP64) and the sweeps go on
 * until theta < theta_target.  The links end up in the handle's own format.
 * history (may be NULL) receives up to history_cap (sweeps, F, theta)
 * triples.  Returns LGF_OK when converged, LGF_ENOTCONV at max_sweeps,
 * LGF_ENUMERIC when theta or F is not finite; the result struct is filled in
 * every case. */
lgf_status lgf_gauge_fix(lgf_lattice *h, const lgf_fix_params *params, lgf_fix_result *result,
                         double *history, int history_cap);

/* Stepwise gauge fixing in the fixed-link form, for callers that drive the
 * iteration of Sec. 4 themselves (sweep the two parities in turn, check theta
 * of Eq. (5) every few sweeps, stop at a precision of their choosing).
 * lgf_fix_begin opens a session on an FP64 handle: the gauge transformation
 * g (a site field owned by the handle, in the sweep format's precision;
 * FP64-12 for LGF_FP64_12S) is set to 1 and the read-only links are prepared
 * in `format` (any format of lgf_fix_params.fixed_links, LGF_FP64_12S
 * included); it allocates what the session needs on the first call
 * (LGF_ENOMEM).  lgf_fix_chunk runs n full sweeps (parity 0, then 1) with
 * overrelaxation omega in [1, 2] or stochastic relaxation p_sr in [0, 1]
 * (Philox key `seed`, counters sweep0 .. sweep0+n-1), captured in a hipGraph
 * when use_graph is set; its last sweep stores every g reunitarized, and F
 * (Eq. (2)) and theta (Eq. (5)) of the links g(x) U(x) g(x+mu)^dag are
 * measured in FP64 (for LGF_FP64_12S on the split links, within 2^-40 of the
 * FP64 ones) and returned; *sweep_ms (may be NULL) gets the time of the n
 * sweeps from HIP events on the handle's stream.  Synchronises.  LGF_ENUMERIC
 * when F or theta is not finite.  lgf_fix_end writes g U g^dag (from the
 * untouched input) into the handle's field and closes the session.  Any call
 * that loads, generates, converts, reunitarizes, sweeps, anneals, autotunes,
 * sets the fixed-link tuning or gauge-fixes the handle closes the session
 * without applying g; lgf_fix_chunk and lgf_fix_end then return LGF_ESTATE. */
lgf_status lgf_fix_begin(lgf_lattice *h, int format);
lgf_status lgf_fix_chunk(lgf_lattice *h, int n, double omega, double p_sr, uint64_t seed, uint64_t sweep0,
                         int use_graph, double *F, double *theta, double *sweep_ms);
lgf_status lgf_fix_end(lgf_lattice *h);

/* Simulated annealing.  The paper names it among the supported methods
 * (Sec. 1) and leaves its heat bath and schedule to a reference; the reading
 * implemented here: the site update of Sec. 3 (K(x) of Eq. (8), the three
 * Cabibbo-Marinari subgroups in order, G applied to the 8 links) with the
 * SU(2) step of each subgroup drawn from the Boltzmann weight
 * exp(Re tr[s(r) w] / T) against the SU(2) Haar measure, a heat bath for the
 * local functional of Eq. (7) at temperature T.  As T -> 0 the draw becomes
 * the maximum of Eq. (9).  The draw writes r = x b with b that maximum,
 * x0 = <r, b> of density sqrt(1 - x0^2) exp(alpha x0), alpha = 2|a|/T (a the
 * quaternion projection of the block): Kennedy-Pendleton above alpha = 0.7, a
 * uniform proposal below, at most 64 trials (then x = 1); (x1, x2, x3)
 * uniform on the sphere.  Random words: Philox4x32-10 keyed by `seed`, counter
 * (site index, sweep, 0, ((k + 1) << 16) | trial) for subgroup k, trial 0xFFFF
 * for the direction.  FP64 arithmetic; FP64 handles only (LGF_EINVAL
 * otherwise).
 * lgf_anneal_sweep: one heat-bath half-sweep (parity 0 or 1) or full sweep
 * (2: parity 0, then 1) at temperature T > 0 with counter sweep_index;
 * *trials (may be NULL; then the call does not synchronise) receives the
 * accept-reject trials of the call.
 * lgf_anneal: n_sweeps >= 1 full sweeps with T falling linearly from T_start
 * (first sweep) to T_end (last), sweep n taking counter sweep0 + n; the links
 * are reunitarized after every 20 sweeps and after the last one.  *trials and
 * *ms (each may be NULL) receive the trials and the time of the sweeps (HIP
 * events on the handle's stream).  Synchronises.  Anneal first, then fix the
 * gauge with lgf_gauge_fix (overrelaxation to the target precision). */
lgf_status lgf_anneal_sweep(lgf_lattice *h, int parity, double T, uint64_t seed, uint64_t sweep_index,
                            uint64_t *trials);
lgf_status lgf_anneal(lgf_lattice *h, int64_t n_sweeps, double T_start, double T_end, uint64_t seed,
                      uint64_t sweep0, uint64_t *trials, double *ms);

/* F and theta of the handle's links, as lgf_measure computes them (the same
 * kernels and summation order, so the same bits), written to d_out[0] = F,
 * d_out[1] = theta in device memory on the handle's device; enqueued on the
 * handle's stream and not synchronised.  For callers that cannot allocate
 * device memory -- code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc: this call allocates nothing.  Its
 * per-workgroup partial sums go to a 4 MiB device array of the library (one
 * per GPU, held until the process ends), so it serves lattices of at most
 * 2^26 sites (LGF_EINVAL beyond).  Calls that overlap on one GPU (several
 * streams or threads) share that array and race; the caller orders them.
 * Every call writes all the partial sums it reads, so nothing carries over
 * from one call to the next. */
lgf_status lgf_measure_noalloc(lgf_lattice *h, double *d_out);

/* Block until all work queued on the handle's stream has finished. */
lgf_status lgf_synchronize(lgf_lattice *h);

/* Kernel tuning of a handle, per storage format (the autotuner sets it too):
 * lanes_per_site in {1, 2, 4} (lanes that share one site update),
 * sites_per_thread in {1, 2, 4} (tiles of `block` lanes per workgroup,
 * strided over the launch), block (threads per workgroup: 64, 128 or 256),
 * xcd_remap (0/1: give each XCD a contiguous range of workgroups),
 * nontemporal (0/1: stream the links past the caches), schedule of a full
 * sweep: 0 = parity 0 then parity 1, each updating the links in place;
 * 1 = t-slice pipeline, parity 1 of slice k-1 right after parity 0 of slice k,
 * so that parity 1 reads what parity 0 wrote from the last-level cache;
 * 2 = out of place, parity 0 reads the field and writes every link into a
 * second buffer of the same size, parity 1 writes them back (needs
 * nontemporal = 1; the library allocates the buffer here, LGF_ENOMEM if it
 * cannot).  Every schedule gives bit-identical links; single half-sweeps
 * (lgf_sweep with parity 0 or 1) always run in place.  A new handle starts at 1
 * lane, 1 tile, 128 lanes, no remap, non-temporal, in place -- except FP64-12,
 * which starts out of place (its second buffer allocated before its first full
 * sweep; without memory for it the format falls back to in place).
 * lgf_set_tuning copies *tuning (LGF_EINVAL on a value outside these sets);
 * lgf_get_tuning fills *tuning with the current values. */
typedef struct {
    int lanes_per_site;
    int sites_per_thread;
    int block;
    int xcd_remap;
    int nontemporal;
    int schedule;
} lgf_sweep_tuning;

lgf_status lgf_set_tuning(lgf_lattice *h, int format, const lgf_sweep_tuning *tuning);
lgf_status lgf_get_tuning(const lgf_lattice *h, int format, lgf_sweep_tuning *tuning);

/* Time the sweep variants (lanes per site, sites per thread, block, XCD
 * remap, non-temporal, schedule in place or out of place; the t-slice
 * pipeline is left to lgf_set_tuning) for a format on this handle's lattice
 * and keep the fastest.  The variants sweep the buffer that lgf_gauge_fix
 * sweeps in that format (the handle's field, saved to a temporary copy first
 * and restored afterwards, or the handle's working copy in another format), so
 * the links are left as they were.  trials = timed full sweeps per variant in
 * the first round (>= 1); the fastest few are re-timed over longer runs. */
lgf_status lgf_autotune(lgf_lattice *h, int format, int trials);

/* Tuning of the fixed-link sweep (lgf_fix_params.fixed_links) per sweep
 * format (LGF_FP64_12S included):
 *  lanes_per_site 2 or 4, or 1 in the FP32 formats (in FP64 one lane per site
 *    takes all 512 registers and runs slower);
 *  block 64, 128 or 256;
 *  xcd_remap = tile order: 0 lexicographic tiles; 1 contiguous ranges per
 *    XCD; 2 each XCD takes blocks of 8, 4 or 2 t-slices x z-planes, walked z,
 *    t, then y, so that the neighbouring g a site update reads were read by a
 *    nearby workgroup of the same XCD; 3 every XCD walks the (t, z) planes in
 *    lexicographic order taking its own eighth of each plane, so that the
 *    neighbouring g were read by the same XCD one plane or one t-slice
 *    earlier while the 8 XCDs stream through the same region of memory
 *    (orders 2 and 3 fall back to 0 where the lattice does not divide into
 *    such blocks or planes of a multiple of 8 tiles);
 *  schedule = layout of the read-only links: 0 the link field (the handle's
 *    own, or its copy in the sweep format); 1 (FP32-12, FP64-12 and
 *    LGF_FP64_12S only) per-site link records -- for each parity and tile of
 *    32 consecutive sites the 8 links of each site (U_mu(x), then
 *    U_mu(x-mu)), so that a wavefront reads one contiguous block (in
 *    LGF_FP64_12S each link's FP32 part, then its remainders); a copy of
 *    twice the link field's size (of the split storage's), rebuilt from the
 *    field whenever a gauge fixing or session starts
 *    (Landau and Coulomb gauge; a Coulomb update reads the 6 spatial slots of
 *    its record).  The records hold the field's values, and neither layout nor tile
 *    order changes a bit of the result; without device memory for the
 *    records the format falls back to layout 0;
 *  sites_per_thread must be 1 and nontemporal 1 (links and g(x) are streamed,
 *  the neighbouring g go through the caches).
 * Default: FP64-12 and LGF_FP64_12S 2 lanes, 128-lane workgroups, order 2,
 * records; FP32-12 1 lane, 128-lane workgroups, order 0, records (all three
 * on the link field for lattices of fewer than 2^18 sites); FP64-18 2
 * lanes, 64-lane workgroups, order 2, layout 0; FP32-18 2 lanes, 256-lane
 * workgroups, order 0, layout 0.  LGF_EINVAL on other values.  Setting a
 * tuning closes an open stepwise session (lgf_fix_begin) without applying g. */
lgf_status lgf_set_fixed_tuning(lgf_lattice *h, int format, const lgf_sweep_tuning *tuning);
lgf_status lgf_get_fixed_tuning(const lgf_lattice *h, int format, lgf_sweep_tuning *tuning);

/* Pick the fastest fixed-link sweep variant for `format` on this lattice
 * (lanes 1 (FP32 formats)/2/4 x block 64/128/256 x tile order 0-3 x link
 * layout 0/1 (FP32-12, FP64-12, LGF_FP64_12S); the FP64 formats keep tile order 2
 * wherever the lattice admits it; orders the lattice does not admit are
 * left out): each timed over `trials` full sweeps, the fastest again over ten
 * times as many in five interleaved rounds; the default stays unless another
 * is 1 % faster.  The sweeps read the handle's links (or their copy in
 * `format`, and its per-site records) and write only the gauge
 * transformation, which lgf_gauge_fix resets: the links are untouched.  Needs
 * an FP64 handle.  Synchronises. */
lgf_status lgf_autotune_fixed(lgf_lattice *h, int format, int trials);

/* Average duration in ms of the last n_launches sweep kernels enqueued through
 * lgf_time_sweeps: runs n full sweeps (2n launches) with the given omega/p_sr
 * and returns the per-launch mean measured with HIP events on the handle's
 * stream. */
lgf_status lgf_time_sweeps(lgf_lattice *h, int n, double omega, double p_sr, uint64_t seed,
                           uint64_t sweep_index, double *ms_per_launch);

/* The bandwidth of a plain device copy, the practical ceiling of a streaming
 * kernel: allocates two buffers of `bytes` (a multiple of 16) on the current
 * device, copies one into the other reps times on hip_stream (NULL = default)
 * with one 16-byte vector per lane and non-temporal access, and returns the
 * read + write rate *GBs = 2 * bytes * reps / time (1e9 bytes/s).  Frees the
 * buffers before returning.  LGF_ENOMEM if they cannot be allocated. */
lgf_status lgf_copy_bandwidth(size_t bytes, int reps, void *hip_stream, double *GBs);

/* ------------------------------------------------------------------------ */
/* Coulomb gauge.  The paper names Coulomb gauge among the supported gauges   */
/* (abstract, Sec. 1) without its definitions; the reading used here: each     */
/* timeslice t has the functional F_C(t) = (1/(3*3*V3)) sum_{x in t, i=1..3}   */
/* Re tr U_i(x) and precision theta_C(t) = (1/(3*V3)) sum_{x in t}             */
/* tr[Delta_C Delta_C^dag] with Delta_C(x) = sum_i A_i(x) - A_i(x-i), so K(x)  */
/* holds the 6 spatial links; the gauge transformation still acts on all 8     */
/* links, temporal ones included.  All timeslices are relaxed by one launch   */
/* per (4-D) parity.                                                           */
/* ------------------------------------------------------------------------ */

/* One Coulomb half-sweep (parity 0, 1) or full sweep (2) of every timeslice
 * whose flag in slice_active (host array of Lt bytes; NULL = all) is nonzero;
 * other arguments as lgf_sweep. */
lgf_status lgf_sweep_coulomb(lgf_lattice *h, int parity, double omega, double p_sr, uint64_t seed,
                             uint64_t sweep_index, const unsigned char *slice_active);

/* F_C(t) and theta_C(t) of every timeslice (host arrays of Lt doubles, either
 * may be NULL), accumulated in FP64.  Synchronises. */
lgf_status lgf_measure_coulomb(lgf_lattice *h, double *F_t, double *theta_t);

/* Coulomb gauge fixing, as lgf_gauge_fix with per-timeslice convergence: a
 * timeslice stops being updated at its first measurement with theta_C(t) <
 * theta_target; the mixed-precision switch happens once every live timeslice
 * is below theta_switch.  result: sweeps (total), theta = largest theta_C(t),
 * F = mean F_C(t); sweeps_t, F_t, theta_t (host arrays of Lt doubles, may be
 * NULL) receive per-timeslice sweeps, F_C and theta_C.  accumulate_g and
 * fixed_links work as in lgf_gauge_fix (in the fixed-link form a site update
 * reads only its 6 spatial links; the temporal links enter only the final
 * g(x) U_mu(x) g(x+mu)^dag; with LGF_FP64_12S last, every timeslice's F_C
 * and theta_C of the result, and the stopping test, come from one more
 * measurement of the transformed FP64 links); separate_measure is ignored
 * (two measurement passes). */
lgf_status lgf_coulomb_gauge_fix(lgf_lattice *h, const lgf_fix_params *params, lgf_fix_result *result,
                                 double *sweeps_t, double *F_t, double *theta_t);

/* ------------------------------------------------------------------------ */
/* Ensembles: many independent lattices (sizes may differ) swept and measured */
/* by one persistent launch per parity.                                       */
/* ------------------------------------------------------------------------ */

typedef struct lgf_ensemble lgf_ensemble;   /* opaque handle: n lattices on one GPU */

/* Create an ensemble of n configurations; dims holds n*4 extents (each
 * configuration as in lgf_create), format is the home storage format of all
 * of them.  The library allocates every field; stream as in lgf_create.  The
 * links are uninitialised until loaded or generated. */
lgf_status lgf_ensemble_create(int n, const int *dims, int format, void *stream, lgf_ensemble **out);

/* Release the ensemble and everything it owns; NULL is allowed. */
lgf_status lgf_ensemble_destroy(lgf_ensemble *e);

/* Per configuration i in [0, n): generate (as lgf_generate_links), load or
 * store the canonical host array (72*V_i doubles). */
lgf_status lgf_ensemble_generate(lgf_ensemble *e, int i, uint64_t seed, double eps, int haar);
lgf_status lgf_ensemble_load_links(lgf_ensemble *e, int i, const double *host_canon, size_t n_doubles);
lgf_status lgf_ensemble_store_links(lgf_ensemble *e, int i, double *host_canon, size_t n_doubles);

/* One half-sweep (parity 0, 1) or full sweep (2) of every configuration in the
 * home format, as lgf_sweep, in one persistent launch per parity; the
 * stochastic-relaxation counter of configuration i is (s, sweep_index, i, 3). */
lgf_status lgf_ensemble_sweep(lgf_ensemble *e, int parity, double omega, double p_sr, uint64_t seed,
                              uint64_t sweep_index);

/* F[i], theta[i] of every configuration (as lgf_measure); either output may be
 * NULL.  Synchronises. */
lgf_status lgf_ensemble_measure(lgf_ensemble *e, double *F, double *theta);

/* Gauge-fix every configuration (as lgf_gauge_fix, one lgf_fix_params for all)
 * with per-configuration state: each configuration leaves the bulk format when
 * its own theta < theta_switch and stops sweeping when its own theta <
 * theta_target; the others go on.  All live configurations share each
 * persistent launch, whatever their phase.  results[i] (n entries) gets each
 * configuration's sweeps, theta, F and status; its time fields hold the
 * ensemble totals (chunks holding any bulk configuration count as bulk time),
 * except t_total_ms, the time at which that configuration finished.
 * fixed_links works as in lgf_gauge_fix (2 lanes per site, so a tile of
 * `tile` lanes covers tile/2 sites; FP64 home format; bulk/finish FP32-12 /
 * FP64-12 or FP64-12S, or one of them, or FP64-18 alone: LGF_EINVAL
 * otherwise; a configuration whose last sweeps ran in FP64-12S gets its F,
 * theta and status from one more measurement of its FP64 home links; in
 * FP32-12, FP64-12 and FP64-12S the launches read each configuration's links
 * from its per-site records (see lgf_set_fixed_tuning), built when its links
 * are prepared in that format and kept, twice the links' size, until
 * lgf_ensemble_destroy; without device memory for them the link fields:
 * the same bits either way); accumulate_g is rejected. */
lgf_status lgf_ensemble_gauge_fix(lgf_ensemble *e, const lgf_fix_params *params,
                                  lgf_fix_result *results);

/* Average ms per persistent launch (one parity of every configuration) of n
 * full sweeps in the given format, on copies of the links (the home fields are
 * untouched). */
lgf_status lgf_ensemble_time_sweeps(lgf_ensemble *e, int format, int n, double omega, double p_sr,
                                    double *ms_per_launch);

/* The same for the fixed-link form (lgf_fix_params.fixed_links): average ms
 * per persistent launch of n full fixed-link sweeps of every configuration in
 * `format` (FP32-12, FP64-12, LGF_FP64_12S or FP64-18; an FP64 ensemble), the
 * links read as lgf_ensemble_gauge_fix reads them (copies in `format` and
 * per-site records where the format has them; the home links are only read),
 * each configuration's gauge transformation starting at 1 and left as the
 * sweeps leave it (the next gauge fixing resets it).  LGF_EINVAL for other
 * formats or an FP32 ensemble. */
lgf_status lgf_ensemble_time_fixed_sweeps(lgf_ensemble *e, int format, int n, double omega, double p_sr,
                                          double *ms_per_launch);

/* Tuning of the persistent ensemble launches: tile = sites per work-list tile
 * and lanes per workgroup (64, 128 or 256), grid_mult = persistent workgroups
 * as a multiple (1, 2 or 4) of what fits on the GPU at once, nontemporal
 * (0/1) link access.  Results do not depend on it.  lgf_ensemble_autotune
 * times the 12 variants for `format` on scratch copies of the links (trials =
 * timed full sweeps per variant, >= 1), re-times the fastest, and keeps the
 * winner; the links are untouched. */
lgf_status lgf_ensemble_set_tuning(lgf_ensemble *e, int tile, int grid_mult, int nontemporal);
lgf_status lgf_ensemble_get_tuning(const lgf_ensemble *e, int *tile, int *grid_mult, int *nontemporal);
lgf_status lgf_ensemble_autotune(lgf_ensemble *e, int format, int trials);

#ifdef __cplusplus
}
#endif

#endif /* LGF_H */
