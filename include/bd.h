/*
 * bd.h -- C ABI of the MI355X Brownian hard-disk library.
 *
 * The library advances N hard disks in a square box with hard walls by the
 * time step of Carter, Hitschfeld, Navarro and Soto, "GPU parallel simulation
 * algorithm of Brownian particles with excluded volume using Delaunay
 * triangulations" (arXiv:1703.02484), Algorithm 1: pair forces, an
 * Euler-Maruyama move with Brownian noise (Sec. 2.2, 2.4), repair of the
 * Delaunay triangulation by edge flips (Sec. 4.1, 4.3), and overlap
 * correction over Delaunay edges (Sec. 2.3, 4.4, Algorithm 2).  The
 * triangulation and all particle state stay resident in device memory.
 *
 * Conventions shared by every entry point:
 *   - Host arrays are caller-owned.  Inputs are copied before the call
 *     returns; outputs are written before it returns.
 *   - Particle arrays are in caller order (the order given to bd_init).
 *     Positions are interleaved (x0, y0, x1, y1, ...).
 *   - Every call returns BD_OK (0) or a negative BD_ERR_* code; no C++
 *     exception crosses this interface.  bd_strerror() names a code and
 *     bd_last_error() gives the detail of the last failure on a handle.
 *   - A handle is used by one host thread at a time.
 */
#ifndef BD_H
#define BD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BD_MAX_SPECIES 8

enum bd_error {
    BD_OK = 0,
    BD_ERR_INVALID_ARG = -1,     /* NULL pointer, n < 3, NaN or out-of-range parameter */
    BD_ERR_BAD_INPUT = -2,       /* initial disks overlap or lie outside the walls */
    BD_ERR_NO_CONVERGENCE = -3,  /* overlap rounds exceeded max_overlap_rounds */
    BD_ERR_TRIANGULATION = -4,   /* the triangulation could not be built or repaired */
    BD_ERR_DEVICE = -5,          /* a HIP runtime call failed */
    BD_ERR_OOM = -6              /* device or pinned host allocation failed */
};

enum bd_force_kind {
    BD_FORCE_POWER = 0,     /* g(d) = d^-q: q = 2 is the paper's long-range law r/r^3, q = 6 its r/r^7 */
    BD_FORCE_SCREENED = 1   /* g(d) = A exp(-d / lambda) / d */
};

enum bd_overlap_method {
    BD_OVERLAP_DELAUNAY = 0,  /* overlap rounds over the edges of the Delaunay triangulation (Sec. 4.4) */
    BD_OVERLAP_VERLET = 1     /* overlap rounds over the neighbour lists, no triangulation (the paper's
                                 short-range algorithm, Sec. 5); needs cutoff > 0 */
};

enum bd_precision {
    BD_PREC_FP64 = 0,       /* forces computed and summed in FP64 */
    BD_PREC_FP32 = 1        /* forces in FP32 from FP32 copies of the positions; everything else FP64 */
};

/*
 * Pair force F_i = sum_{j != i} K[s_i][s_j] g(d_ij) (r_i - r_j) / d_ij
 * (Sec. 2.2: the two-charge model mu_i alpha_k generalised to an S x S
 * strength matrix; positive K repels).  With cutoff > 0 only pairs with
 * d_ij <= cutoff contribute (Sec. 2.2 cutoff rule, no force shift).
 */
typedef struct bd_force_params {
    int32_t kind;        /* bd_force_kind */
    int32_t S;           /* number of species, 1..BD_MAX_SPECIES */
    double q;            /* power-law exponent of g (kind POWER) */
    double A;            /* screened amplitude (kind SCREENED) */
    double lambda;       /* screening length (kind SCREENED) */
    double cutoff;       /* <= 0: all pairs */
    double skin;         /* cutoff > 0: Verlet lists hold pairs within cutoff + skin, rebuilt when a
                            disk has moved more than skin / 2 since the last build */
    const double *K;     /* S*S row-major, K[a*S + b] acts on species a from species b; copied */
} bd_force_params;

/*
 * Step parameters.  Positions advance by
 *   x <- x + (F + v0 (cos th, sin th)) dt + sqrt(2 D dt) xi       (Sec. 2.2, Sec. 7)
 *   th <- th + sqrt(2 Dr dt) n                                   (Sec. 7)
 * with xi two standard normals clamped to [-noise_clip, noise_clip]
 * (Sec. 2.4, truncation method) and n one standard normal, drawn from
 * Philox4x32-10 keyed by (seed, step, particle id, stream).
 */
typedef struct bd_params {
    double L;                    /* box [0, L]^2, hard walls */
    double D;                    /* translational diffusion coefficient */
    double dt;                   /* time step */
    double v0;                   /* self-propulsion speed */
    double Dr;                   /* rotational diffusion coefficient */
    uint64_t seed;               /* noise key */
    int64_t step0;               /* index of the first step (noise counter), for resume */
    double overlap_factor;       /* Sec. 2.3: 1.0 moves each disk by the overlap ("bounce"), 0.5 to contact */
    double cap_frac;             /* Sec. 4.4: summed correction truncated to cap_frac * r_i (0.5 = sigma/4) */
    double noise_clip;           /* Sec. 2.4: clamp of each normal component (3.0) */
    double contact_tol;          /* a pair overlaps when d < (r_i + r_j)(1 - contact_tol) (1e-9) */
    int32_t max_overlap_rounds;  /* cap on overlap rounds per step (10000) */
    int32_t max_flip_rounds;     /* cap on flip rounds per repair before the host rebuild (200) */
    int32_t force_precision;     /* bd_precision */
    int32_t force_chunk;         /* all-pairs force: j per chunk (64..65536); 0 lets the library choose,
                                    by timing the candidate tilings once per workload shape when the pair
                                    count is large (see bd_get_force_config); -1 / -2 / -3: the symmetric
                                    form (inverse-square law only) with chunks of at most 1024 (4 per
                                    lane) / 512 (2 per lane) / 1024 (8 per lane, 2 wavefronts) */
    int32_t force_per_lane;      /* with force_chunk > 0: particles i per lane, 2 or 4 (0: 4); a tile holds
                                    256 * force_per_lane particles i */
    int32_t force_launch;        /* with force_chunk > 0: 0 one workgroup per tile, j as wave-uniform scalar
                                    loads; 1 a resident grid taking the tiles from a queue (the autotuner's
                                    two launch forms); 2 one workgroup per tile with j staged through LDS
                                    (the shared-memory broadcast of the paper's n-body kernel, Sec. 6;
                                    inverse-square law without cutoff; same sums as 0, bitwise) */
    int32_t overlap_method;      /* bd_overlap_method.  BD_OVERLAP_VERLET finds overlapping pairs in the
                                    neighbour lists (radius cutoff + skin); they hold every pair closer than
                                    contact while no disk moved more than (cutoff + skin - 2 r_max) / 2 since
                                    the build, and are rebuilt inside the step when one did.  No reversal
                                    count and no triangulation (bd_get_triangulation fails) */
    int32_t max_dt_halvings;     /* Sec. 4.3 edge reversal (a Delaunay edge whose vector reversed in a move):
                                    0 counts it only; k in 1..12 discards the move and redoes the step as
                                    two halves, each split again on a reversal, down to 2^-k of dt.  The
                                    halves' noise is a Brownian bridge of the step's own draws (Philox,
                                    keyed by step, disk, level and interval), so a trajectory stays a
                                    function of the seed.  Delaunay overlap method only */
    int32_t periodic;            /* 0: hard walls.  1: periodic box [0, L)^2 (the paper's domain, Sec. 2.1):
                                    positions folded into [0, L) after every move, every separation taken
                                    from the nearest image (minimum-image convention, ties to even) in the
                                    forces, the neighbour lists and the overlap rounds.  The Delaunay
                                    overlap method keeps the triangulation of the flat torus (2n triangles,
                                    no frame points, no infinite vertex), whose predicates read a triangle
                                    or a quad at the nearest images of its vertices.  One system per
                                    handle; all-pairs forces in the one-workgroup-per-tile form
                                    (force_chunk >= 0, force_launch 0); no adjoint */
} bd_params;

/* Counters accumulated since bd_init (the paper reports rounds and flips per step, Sec. 6). */
typedef struct bd_stats {
    int64_t steps;
    int64_t overlap_rounds_total;   /* overlap-correction rounds that moved disks */
    int64_t overlap_rounds_max;     /* most rounds in one step */
    int64_t overlap_edges_total;    /* overlapping Delaunay edges corrected, summed over rounds */
    int64_t cap_hits;               /* per-disk corrections truncated by the cap */
    int64_t reversals;              /* Delaunay edges whose vector reversed in a move (Sec. 4.3) */
    int64_t noise_clamps;           /* clamped normal components */
    int64_t flips_total;            /* edge flips performed on the device */
    int64_t inversion_flips;        /* of which decided by the inverted-triangle rule (Sec. 4.3) */
    int64_t flip_rounds_total;      /* parallel flip rounds that flipped at least one edge */
    int64_t kinetic_repairs;        /* repairs redone on the device in sub-steps (multi-edge crossings) */
    int64_t host_rebuilds;          /* repairs that fell back to a host triangulation */
    int64_t verlet_rebuilds;        /* neighbour-list rebuilds (cutoff > 0) */
    int64_t host_continued;         /* steps whose enqueued rounds ran out and the host finished */
    int64_t dt_halvings;            /* moves discarded after an edge reversal and redone as two halves */
    int64_t reserved;
} bd_stats;

typedef struct bd_sim bd_sim;
/* A batch of independent systems (bd_batch_init) is a handle of the same type. */
typedef struct bd_sim bd_batch;

/* Name of an error code (static string). */
const char *bd_strerror(int code);

/* Detail of the last failure on sim (static per handle; never NULL; "" if none). */
const char *bd_last_error(const bd_sim *sim);

/* Fills p with the defaults named in the field comments; L must still be set. */
void bd_params_default(bd_params *p);

/*
 * Creates a simulation of n >= 3 disks (Algorithm 1 initial state).
 *   xy       2n doubles, centres; each must satisfy r_i <= x, y <= L - r_i
 *   radii    n doubles > 0
 *   species  n int32 in [0, S)
 *   theta    n doubles (initial director angles) or NULL for zeros
 * Disks may touch but not overlap (d_ij >= r_i + r_j), else BD_ERR_BAD_INPUT.
 * Builds the Delaunay triangulation on the host once (Sec. 4.1) and uploads
 * it; all later repairs run on the device.  Uses the calling thread's current
 * HIP device and creates its own stream (see bd_set_stream).
 * On success *out owns all device memory until bd_destroy.
 */
int bd_init(bd_sim **out, int32_t n, const double *xy, const double *radii, const int32_t *species,
            const double *theta, const bd_force_params *fp, const bd_params *p);

/*
 * Creates R >= 1 independent systems advanced together (batched replicas; not
 * in the paper: each system on its own follows Algorithm 1 exactly as a
 * handle from bd_init would).  System r holds n_per[r] >= 3 disks in a box
 * [0, L_per[r]]^2 with noise key seed_per[r]; the arrays xy (2 per disk),
 * radii, species and theta (or NULL) hold the systems one after another
 * (disk offsets are the prefix sums of n_per).  p->L and p->seed are ignored;
 * every other field of p and fp applies to all systems.  Noise is keyed by
 * (seed_per[r], step, index of the disk inside its system), so a system's
 * trajectory does not depend on the others; forces act only inside a system.
 * The all-pairs force of all systems is one launch over a tile list ordered
 * longest first.  Short-range forces (fp->cutoff > 0) need R == 1.
 * bd_step, bd_forces, bd_get_state, bd_set_positions, bd_get_frame and
 * bd_get_triangulation then act on the concatenation; bd_batch_layout gives
 * the offsets.
 */
int bd_batch_init(bd_sim **out, int32_t R, const int32_t *n_per, const double *xy, const double *radii,
                  const int32_t *species, const double *theta, const double *L_per, const uint64_t *seed_per,
                  const bd_force_params *fp, const bd_params *p);

/*
 * Layout of the systems of a handle: *R_out systems; disk_off[r] (R+1
 * entries, may be NULL) is the first disk of system r in caller order and
 * frame_off[r] (R+1 entries, may be NULL) the first frame point of system r
 * in bd_get_frame order.  Triangulation ids: disk i is i, frame point k is
 * n + k with n = disk_off[R].
 */
int bd_batch_layout(bd_sim *sim, int32_t *R_out, int32_t *disk_off, int32_t *frame_off);

/* Tiling of the all-pairs force kernel in use (measurement and reproducibility). */
typedef struct bd_force_config {
    int32_t chunk;        /* j per chunk (results depend on it at rounding level) */
    int32_t per_lane;     /* i per lane; a tile holds 256 * per_lane particles i */
    int32_t persistent;   /* launch form: 0 one workgroup per tile (i-block x chunk); 1 a fixed grid taking
                             those tiles from a queue; 2 symmetric: one workgroup per pair of chunks,
                             each pair of disks evaluated once and both sums written; 3 one workgroup
                             per tile with j staged through LDS (force_launch 2) */
    int32_t tiles;        /* tiles per force evaluation */
    int32_t grid;         /* workgroups launched per force evaluation */
    int32_t tuned;        /* 1: chosen by timing, 2: taken from the tuning cache, 0: fixed rule */
    double tuned_ms;      /* force + partial-sum reduction time of the chosen tiling when timed, else 0 */
} bd_force_config;
int bd_get_force_config(bd_sim *sim, bd_force_config *out);

/*
 * Advances nsteps >= 0 steps of Algorithm 1: forces, move, walls, flip repair
 * of the triangulation, then overlap rounds (each followed by a repair) until
 * no Delaunay edge overlaps.  On return the triangulation is the Delaunay
 * triangulation of the current positions.  On error the state is that of the
 * last completed step.
 */
int bd_step(bd_sim *sim, int64_t nsteps);

/* Forces at the current positions in caller order, 2n doubles.  Does not advance time. */
int bd_forces(bd_sim *sim, double *f_out);

/*
 * Pair forces of the Sec. 2.2 law for positions the caller holds in device
 * memory, without a handle:
 *   F_i = sum_{j != i} K[s_i][s_j] g(d_ij) (r_i - r_j) / d_ij
 * with g and the cutoff from fp (fp->skin is ignored; all pairs are
 * evaluated, no neighbour lists).
 *   n          number of particles, >= 1
 *   xy         device, 2n doubles, x and y interleaved (caller order)
 *   species    device, n int32 in 0..fp->S-1 (not checked on the device)
 *   fp         host; fp->K (S*S doubles, host) is copied before the call returns
 *   precision  BD_PREC_FP64 or BD_PREC_FP32 (pair sums in FP32 from FP32
 *              copies of the positions; the final sum over j splits in FP64)
 *   f_out      device, 2n doubles (Fx, Fy interleaved), written
 *   stream     hipStream_t of the current device to run on (NULL: the null stream)
 * All device pointers belong to the current device.  The call allocates its
 * working memory (the per-split sums, J * n * 16 bytes at most, J <= 64),
 * runs on `stream`, synchronises it, frees the memory and returns.  Two
 * distinct particles at the same position give non-finite forces.
 * BD_ERR_INVALID_ARG for bad arguments, BD_ERR_OOM if the working memory
 * cannot be allocated, BD_ERR_DEVICE if a launch fails.
 */
int bd_pair_forces_dev(int32_t n, const double *xy, const int32_t *species, const bd_force_params *fp,
                       int32_t precision, double *f_out, void *stream);

/*
 * bd_pair_forces_dev for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, same kernels and bitwise the same forces.  It
 * allocates nothing: the per-split sums use a fixed 32 MiB device array, one
 * per GPU, held from the first call on that GPU until the process ends.
 * Limit: J * n * (16 bytes for FP64, 8 for FP32) <= 32 MiB, i.e. n up to
 * 2,097,152 (FP64) or 4,194,304 (FP32); larger n returns BD_ERR_INVALID_ARG.
 * The call only enqueues the work on `stream` and returns; f_out is ready
 * when the stream reaches that point.  All calls on one GPU share the array:
 * calls that overlap in time on one GPU (other streams, other threads) race;
 * order them on one stream.
 */
int bd_pair_forces_dev_noalloc(int32_t n, const double *xy, const int32_t *species, const bd_force_params *fp,
                               int32_t precision, double *f_out, void *stream);

/*
 * Copies the state out: xy_out (2n doubles, may be NULL), theta_out (n
 * doubles, may be NULL), step_out (may be NULL), stats_out (may be NULL).
 * Synchronises the library's stream.
 */
int bd_get_state(const bd_sim *sim, double *xy_out, double *theta_out, int64_t *step_out, bd_stats *stats_out);

/*
 * Positions (2n doubles, x and y interleaved, caller order) and angles (n
 * doubles) into device memory of the handle's GPU (either may be NULL);
 * returns when they are written.
 */
int bd_get_state_dev(bd_sim *sim, double *xy_out, double *theta_out);

/*
 * Finite triangles of the resident triangulation, counter-clockwise: 3 int32
 * per triangle into tri_out (room for cap triangles; 2 (n + m) is always
 * enough), count into *ntri_out.  Ids 0..n-1 are disks in caller order; ids
 * n..n+m-1 are the frame points of bd_get_frame.  BD_ERR_INVALID_ARG if cap
 * is short.  In a periodic box: the 2n triangles of the flat torus, each
 * counter-clockwise at the nearest images of its vertices.
 */
int bd_get_triangulation(const bd_sim *sim, int32_t *tri_out, int32_t cap, int32_t *ntri_out);

/*
 * The triangulated point set is the disks plus m fixed frame points outside
 * the walls, which play the role of the paper's boundary-free periodic
 * triangulation (Sec. 2.1) for a box with walls: they keep the triangles
 * along the walls well shaped, and no frame point can lie in the diametral
 * circle of an overlapping pair, so the closest overlapping pair stays a
 * Delaunay edge.  Frame: four arcs at 2 r_max beyond the wall lines, one point
 * per 2 r_max, bowed outwards by at most r_max / 2 (strictly convex), the
 * bottom, right, top and left sides holding K, K+1, K+2, K+3 points with
 * K = ceil((L + 4 r_max) / (2 r_max)).  *m_out receives m; with xy_out non-NULL
 * (room for cap points) the 2m coordinates are written in vertex-id order.
 */
int bd_get_frame(bd_sim *sim, double *xy_out, int32_t cap, int32_t *m_out);

/*
 * Replaces the positions (2n doubles, caller order, inside the walls) and
 * restores the Delaunay triangulation by the device flip repair (inverted-
 * triangle flips, Sec. 4.3, with Lawson flips, Sec. 4.1).  When a disk crossed
 * more than one edge, which the inverted-triangle rule cannot untangle
 * (Sec. 4.3, two-flip figure), the repair restarts from the previous
 * triangulation and replays the move in 2, 4, ... 64 equal sub-steps, each
 * repaired by the same rule; only if that fails is the triangulation rebuilt
 * on the host.  No overlap correction and no time advance.
 */
int bd_set_positions(bd_sim *sim, const double *xy);

/*
 * Graph mode (enable != 0; off after bd_init): each step's device work is
 * replayed from HIP graphs captured on first use (one set per round-budget
 * setting) instead of being launched kernel by kernel; the step counter and
 * the round stamps are read from device memory, so replays need no new
 * arguments.  Results are identical to the launch-by-launch mode.
 */
int bd_set_graph_mode(bd_sim *sim, int enable);

/*
 * How the overlap rounds of a step after its first detection are launched:
 * mode 0 one launch per phase (detection, gather, apply, each flip-round
 * phase, validation), mode 1 all of them in one workgroup separated by
 * barriers, mode 2 the first flip rounds of each repair and the overlap
 * rounds that recently queued many disks launched per phase and the rest in
 * one workgroup, -1 (default) the library's choice: mode 1 for handles of at
 * most 16,384 disks (measured equal or up to 2 % faster there), else mode 2
 * (6-18 % faster on 32,768, faster on 65,536 and on 1M).  With overlap
 * rounds over the neighbour lists (Sec. 5): mode 0 every round a launch over
 * all disks, mode 1 every round after the first in one workgroup over the
 * disks near those the round before moved, mode 2 the rounds after one that
 * recently moved more than 512 disks launched over all disks, the rest in one
 * workgroup.  Results are identical.
 */
int bd_set_tail_mode(bd_sim *sim, int mode);

/*
 * Device memory of handles created after this call comes from alloc_fn /
 * free_fn (called with the handle's stream and ctx), e.g. a framework's
 * caching allocator; NULL for both restores hipMalloc / hipFree.  A handle
 * keeps the allocator it was created with.  Pinned host staging buffers are
 * always hipHostMalloc'd.  BD_ERR_INVALID_ARG if only one function is given.
 */
int bd_set_allocator(void *(*alloc_fn)(size_t bytes, void *stream, void *ctx),
                     void (*free_fn)(void *ptr, void *stream, void *ctx), void *ctx);

/* Runs later work on hip_stream (a hipStream_t; NULL = the library's own stream). */
int bd_set_stream(bd_sim *sim, void *hip_stream);

/*
 * Per-kernel timing for measurement: with enable != 0 the library records HIP
 * events on its stream around each launch of the all-pairs force kernel.
 * bd_kernel_time() returns the summed milliseconds and launch count since
 * timing was enabled (it synchronises the stream).
 */
int bd_enable_kernel_timing(bd_sim *sim, int enable);
int bd_kernel_time(bd_sim *sim, double *force_ms, int64_t *force_launches);

/*
 * Adjoint of the step (not in the paper): gradients of a scalar loss of the
 * positions after nsteps steps with respect to the positions before them and
 * to the strength matrix K.  The step is differentiated as written with every
 * discrete choice of the forward pass held fixed: the overlapping partners of
 * each correction round (the correction acts as a projection onto that
 * round's contact set, Sec. 2.3 displacement and Sec. 4.4 Jacobi sum and
 * cap), the cap branch, the wall branches.  Noise and director angles do not
 * depend on the positions.  All-pairs inverse-square force only (kind POWER,
 * q = 2, no cutoff); BD_ERR_INVALID_ARG otherwise.
 *
 * bd_adjoint_begin advances nsteps >= 1 steps exactly like bd_step while
 * keeping a device copy of the state every checkpoint_every >= 1 steps; the
 * handle is then at the final step (read it with bd_get_state).
 *
 * bd_adjoint_backward takes grad_xy = dL/dx at the final step (2n doubles,
 * caller order) and writes grad_xy0 = dL/dx at the first step through the
 * dynamics (2n doubles, may be NULL) and grad_K = dL/dK (S*S doubles,
 * row-major, may be NULL).  It replays each segment between checkpoints
 * from its checkpoint (recomputation instead of storing every step), records
 * what the reverse sweep needs, and sweeps it backwards; the handle is left
 * at the final step with its counters unchanged.  It may be called again
 * with another grad_xy.  Device memory: one checkpoint per segment, the
 * positions of one segment and, when they fit in 8 GiB, the force partial
 * sums of one segment (otherwise the sweep recomputes them).
 */
int bd_adjoint_begin(bd_sim *sim, int64_t nsteps, int32_t checkpoint_every);
int bd_adjoint_backward(bd_sim *sim, const double *grad_xy, double *grad_xy0, double *grad_K);
/* The same with all three arrays in device memory of the handle's GPU; returns when they are written. */
int bd_adjoint_backward_dev(bd_sim *sim, const double *grad_xy, double *grad_xy0, double *grad_K);

/* Frees everything; accepts NULL. */
void bd_destroy(bd_sim *sim);

/*
 * Batch and adjoint calls under the names of the interface specification of
 * this library.  Each has the contract of the call it names:
 *   bd_batch_step(b, n)                 = bd_step(b, n)
 *   bd_batch_get_state(b, xy, th, s, st)= bd_get_state(b, xy, th, s, st), all
 *                                         systems concatenated (bd_batch_layout)
 *   bd_batch_destroy(b)                 = bd_destroy(b)
 *   bd_rollout(sim, n, every)           = bd_adjoint_begin(sim, n, every);
 *                                         every must fit in int32
 *   bd_backward(sim, gT, gK, g0)        = bd_adjoint_backward(sim, gT, g0, gK)
 *                                         (note the order: dL/dK before dL/dx0)
 *   bd_backward_dev(sim, gT, gK, g0)    = bd_adjoint_backward_dev(sim, gT, g0, gK)
 */
int bd_batch_step(bd_batch *b, int64_t nsteps);
int bd_batch_get_state(const bd_batch *b, double *xy_out, double *theta_out, int64_t *step_out, bd_stats *stats_out);
void bd_batch_destroy(bd_batch *b);
int bd_rollout(bd_sim *sim, int64_t nsteps, int64_t checkpoint_every);
int bd_backward(bd_sim *sim, const double *grad_xy, double *grad_K, double *grad_xy0);
int bd_backward_dev(bd_sim *sim, const double *grad_xy, double *grad_K, double *grad_xy0);

#ifdef __cplusplus
}
#endif

#endif /* BD_H */
