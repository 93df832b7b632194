/*
 * dr.h — C ABI of the Diffusion Restore chain-step library for MI355X (gfx950).
 *
 * The library runs the many-chain step of the Diffusion Restore process: a
 * Jump Restore process on the primary-sample-space torus (Def. 4.1) whose
 * local moves are unadjusted Euler-Maruyama Langevin steps with an optional
 * rotational drift (Sec. 5, Eq. local-dynamics, Alg. 5.1), with holding rate
 * 1/dt (Eq. diffusion-restore-holding-rate), killing rate k0/p
 * (Eq. modified-killing-rate with uniform regeneration), regeneration from the
 * uniform distribution, and Rao-Blackwellised holding-time splats into a
 * frame buffer (Alg. 4.1-4.3).
 *
 * Conventions for every entry point:
 *  - Every function returns dr_status; DR_OK on success.  On failure nothing
 *    is changed and dr_last_error() returns a message (thread-local, valid
 *    until the next dr_* call on the same thread).
 *  - "host" pointers are ordinary CPU memory, "device" pointers are HIP device
 *    memory on the device the object was created on.  Pointers passed in are
 *    borrowed: the library never frees them, and device pointers must stay
 *    valid until the stream work that uses them has completed.
 *  - hip_stream arguments are hipStream_t values (NULL = the legacy default
 *    stream).  Calls documented as asynchronous only enqueue work.
 *  - Arrays of chain state are planar ("structure of arrays"): coordinate i
 *    of chain c is at [i * n_chains + c].
 *  - Handles are not thread-safe; use one thread (and one stream) per handle.
 */
#ifndef DR_H
#define DR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DR_OK = 0,
    DR_ERR_INVALID_ARG = 1,
    DR_ERR_OUT_OF_MEMORY = 2,
    DR_ERR_DEVICE = 3,
    DR_ERR_BAD_STATE = 4,
    DR_ERR_UNSUPPORTED = 5
} dr_status;

/* Message for the last failed call on this thread ("" if none). */
const char* dr_last_error(void);

/* Library version string. */
const char* dr_version(void);

/* ------------------------------------------------------------------------
 * Scene (the integrand f of Sec. 3 is the path contribution of this scene).
 * ------------------------------------------------------------------------ */
enum { DR_MAT_LAMBERT = 0, DR_MAT_GGX_CONDUCTOR = 1, DR_MAT_SMOOTH_CONDUCTOR = 2, DR_MAT_SMOOTH_DIELECTRIC = 3 };

/* Parallelogram light p0 + a e1 + b e2 (a, b in [0,1]) emitting radiance Le
 * on the side of e1 x e2 (the paper's lights are diffuse area lights, Sec. 6
 * test scenes).  Each light must also be present in the triangle list as two
 * triangles wound like e1 x e2 with an emissive material. */
typedef struct { float p0[3], e1[3], e2[3], Le[3]; } dr_quad_light;

/* The material set of the paper's test scenes (Sec. 6: diffuse, conductor,
 * dielectric):
 *   DR_MAT_LAMBERT            albedo/pi;
 *   DR_MAT_GGX_CONDUCTOR      Trowbridge-Reitz D with alpha = roughness,
 *                             separable Smith G, Schlick F with normal
 *                             reflectance f0;
 *   DR_MAT_SMOOTH_CONDUCTOR   perfect mirror weighted by Schlick's F (f0);
 *   DR_MAT_SMOOTH_DIELECTRIC  Fresnel-weighted choice of mirror reflection or
 *                             Snell refraction; eta is the index of refraction
 *                             on the side opposite e1 x e2 (the outside is
 *                             the e1 x e2 side, index 1), finite and > 0.
 * The two smooth kinds have delta lobes: no next-event estimate is taken at
 * their vertices, and emission is counted at a vertex reached through them.
 * Le is emitted radiance for emitter triangles; eta is read only for the
 * dielectric. */
typedef struct {
    uint32_t kind;
    float albedo[3];
    float roughness;
    float f0[3];
    float Le[3];
    float eta;
} dr_material;

/* Binary BVH node as built on the host: a >= 0 is an inner node with children
 * a and b; a < 0 is a leaf holding bvh_prim_order[~a .. ~a + b).  Node 0 is the
 * root.  lo/hi bound every triangle below the node. */
typedef struct { float lo[3]; float hi[3]; int32_t a; int32_t b; } dr_bvh_node;

/* Pinhole camera; the film point (u0, u1) in [0,1)^2 maps to the ray through
 * ((2 u0 - 1) tan(fov/2) W/H, (1 - 2 u1) tan(fov/2)) in the camera frame, row
 * 0 at the top. */
typedef struct {
    float eye[3], at[3], up[3];
    float vfov_deg;
    uint32_t width, height;
} dr_camera;

typedef struct {
    const float* vertices; uint32_t n_vertices;        /* host, xyz per vertex */
    const uint32_t* indices; uint32_t n_triangles;      /* host, 3 per triangle */
    const uint32_t* tri_material;                       /* host, n_triangles */
    const dr_material* materials; uint32_t n_materials; /* host */
    const dr_quad_light* lights; uint32_t n_lights;     /* host, 1..127 */
    const dr_bvh_node* bvh; uint32_t n_nodes;           /* host; NULL: the library builds one */
    const uint32_t* bvh_prim_order;                     /* host, n_triangles (with bvh) */
    dr_camera camera;
} dr_scene_desc;

typedef struct dr_scene dr_scene;
typedef struct dr_chains dr_chains;

/* Build a binned-SAH BVH on the host (no device work).  nodes_out must hold
 * 2*n_triangles nodes and prim_order_out n_triangles entries; leaves hold at
 * most max_leaf (1..16) triangles and the tree depth is kept <= 40.
 * Fails with DR_ERR_INVALID_ARG on empty input or an index out of range. */
dr_status dr_bvh_build(const float* vertices, uint32_t n_vertices, const uint32_t* indices, uint32_t n_triangles,
                       uint32_t max_leaf, dr_bvh_node* nodes_out, uint32_t* n_nodes_out, uint32_t* prim_order_out);

/* Validate and deep-copy a scene to device `device` (the caller's arrays may be
 * freed on return).  Converts the host BVH to the device node layout.
 * Errors: DR_ERR_INVALID_ARG (index/material/node out of range, no lights,
 * more than 2^24-1 triangles or 127 lights, BVH deeper than 64),
 * DR_ERR_UNSUPPORTED (a tree whose traversal could need more than 64 stack
 * entries),
 * DR_ERR_OUT_OF_MEMORY, DR_ERR_DEVICE.  Synchronous. */
dr_status dr_scene_create(const dr_scene_desc* desc, int device, dr_scene** out);

/* Replace the camera (a scene change: chains built on this scene must be
 * re-initialised with dr_chains_reinit before the next dr_step, Sec. 4.3).
 * Waits for the device to finish the work in flight, then updates the camera
 * in device memory.  The image size cannot change. */
dr_status dr_scene_set_camera(dr_scene* s, const dr_camera* cam);

/* Device memory hooks, for callers whose framework owns device memory (a
 * caching allocator): alloc(bytes, hip_stream, user) returns device memory
 * aligned to 256 bytes, or NULL; free_(ptr, bytes, hip_stream, user) returns
 * it.  hip_stream is the stream the buffer is used on (NULL for scene data,
 * which is uploaded synchronously).  Buffers allocated after the call (scenes,
 * chain sets, the scratch of dr_eval_logp_grad) use the hooks, and each buffer
 * is released through the hooks that allocated it: chain sets and scenes at
 * destroy after the device is idle, the evaluation scratch right after its
 * kernels are enqueued, so free_ must be stream-ordered (the memory may be
 * reused only by work ordered after that stream's).  Both NULL restores
 * hipMalloc/hipFree; one NULL is DR_ERR_INVALID_ARG.  The hooks must stay
 * callable while any buffer they allocated exists, also after other hooks are
 * installed.  Process-wide; not to be called while other dr_* calls run. */
typedef void* (*dr_alloc_fn)(size_t bytes, void* hip_stream, void* user);
typedef void (*dr_free_fn)(void* ptr, size_t bytes, void* hip_stream, void* user);
dr_status dr_set_allocator(dr_alloc_fn alloc, dr_free_fn free_, void* user);

/* Device layout of a created scene: triangles, 4-wide BVH nodes (128 B
 * each), and the traversal stack a lane needs (the exact worst case over the
 * tree's root-to-leaf paths, at most 64 entries of 4 bytes).  Kernels that
 * trace rays reserve that many LDS bytes per lane, which bounds how many
 * wavefronts a compute unit can hold. */
typedef struct {
    uint32_t n_triangles;
    uint32_t n_nodes;
    uint32_t stack_entries;
    uint32_t stack_bytes_per_lane;
} dr_scene_stats;
dr_status dr_scene_get_stats(const dr_scene* s, dr_scene_stats* out);

void dr_scene_destroy(dr_scene* s);

/* ------------------------------------------------------------------------
 * Chains
 * ------------------------------------------------------------------------ */
enum { DR_MODE_FUSED = 0, DR_MODE_PLAIN = 1 };

typedef struct {
    uint32_t n_chains;       /* N >= 1 */
    uint32_t max_path_len;   /* L in 2..16 path segments; dimension d = 4(L-1) */
    float stddev;            /* sqrt(dt) sigma, paper 5e-3 (Sec. 6) */
    float dt;                /* Euler-Maruyama step, paper 1e-5; holding rate 1/dt */
    float gamma;             /* rotational drift scale, gamma~ = dt gamma / 2 (Alg. 5.1) */
    float m;                 /* mean steps per tour, k0 = p_lambda/(m dt), paper 64 */
    float eps;               /* target penalty, paper 1e-8 (Sec. 5) */
    float k0;                /* > 0: use it; <= 0: estimate p_lambda in the init pass */
    uint32_t rao_blackwell;  /* 1: splat weight 1/(h+k); 0: the sampled holding time */
    uint32_t mode;           /* DR_MODE_FUSED or DR_MODE_PLAIN */
    const float* sigma_diag; /* device, d x N per-chain stddev (overrides stddev), borrowed, nullable */
} dr_params;

/* Allocate the chain buffers for scene s and run the initialise pass of frame
 * `frame` (Alg. 4.1): x ~ uniform, f(x), p_lambda estimate and k0 unless
 * given, hold/kill, splat, and the score of the survivors.  Asynchronous on
 * hip_stream.  Errors: DR_ERR_INVALID_ARG (see dr_params ranges),
 * DR_ERR_OUT_OF_MEMORY. */
dr_status dr_chains_init(dr_scene* s, const dr_params* p, uint64_t seed, uint32_t frame, void* hip_stream,
                         dr_chains** out);

/* Re-run the initialise pass of frame `frame` on existing buffers (clears the
 * frame buffer and tour count; required after a scene change).  Asynchronous. */
dr_status dr_chains_reinit(dr_chains* c, uint32_t frame, void* hip_stream);

/* Advance every chain by n_steps evolve steps (Alg. 4.2 with Alg. 5.1).
 * Asynchronous.  DR_ERR_BAD_STATE if the scene camera changed since init. */
dr_status dr_step(dr_chains* c, uint32_t n_steps, void* hip_stream);

/* Resolve pass (Alg. 4.3): image_dev[ch * W*H + pix] = W H k0 accum / tourCount
 * (0 while tourCount is 0); planar RGB float, device.  Asynchronous; no host
 * synchronisation, so it can sit in a captured graph. */
dr_status dr_resolve(dr_chains* c, float* image_dev, void* hip_stream);

/* Resolve pass (Alg. 4.3, as dr_resolve) into the library's own image
 * buffer, copy it to host_rgb (3*W*H planar floats, host, caller-owned) and
 * the tour count to *tour_count (nullable), then synchronise hip_stream.
 * Errors: DR_ERR_INVALID_ARG (null chains or host_rgb), DR_ERR_DEVICE. */
dr_status dr_image_read(dr_chains* c, float* host_rgb, uint64_t* tour_count, void* hip_stream);

dr_status dr_chains_destroy(dr_chains* c);

/* Host view of the chain state.  Any pointer may be NULL (skipped).
 *  x, score      d x N float (planar)
 *  killed        N uint32 (0/1)
 *  accum         3 x W*H float: sum of (w/dt) f/p per pixel (planar RGB)
 *  last-step record (valid only while recording is on):
 *  p, weight     N float: p(x) and the splat weight w of the last accumulate
 *  pixel         N uint32
 *  f_over_p      3 x N float
 *  path_rec      (L-1) x N uint32 per vertex: (triangle << 8 | light << 1 |
 *                next-event contribution) or 0xFFFFFFFF for no vertex; the
 *                triangle is the original (input) index; at a smooth
 *                conductor or dielectric vertex the light field holds the
 *                lobe (0 reflection, 1 refraction) and the contribution
 *                bit is 0
 *  step          next global step index; tour_count; k0; p_lambda_hat */
typedef struct {
    float* x; float* score; uint32_t* killed; float* accum;
    float* p; float* weight; uint32_t* pixel; float* f_over_p; uint32_t* path_rec;
    uint64_t step; uint64_t tour_count; double k0; double p_lambda_hat;
} dr_state;

/* Copy the state to the host (synchronises hip_stream). */
dr_status dr_chains_read_state(dr_chains* c, dr_state* out, void* hip_stream);

/* Overwrite x, score, killed (non-NULL ones), the step counter and, if
 * k0 > 0, the killing constant; accum and tour_count are set when accum is
 * non-NULL.  Synchronous. */
dr_status dr_chains_write_state(dr_chains* c, const dr_state* in, void* hip_stream);

/* Turn the per-chain last-step record on or off (off by default). */
dr_status dr_chains_set_record(dr_chains* c, int enable);

/* Counters (chain-steps, rays, BVH nodes visited, triangles tested, kills)
 * accumulate only while enabled (off by default: a uniform branch). */
typedef struct {
    uint64_t chain_steps, rays, node_visits, tri_tests, kills, tours, adjoints;
    double k0, p_lambda_hat;
} dr_counters;
dr_status dr_chains_set_counters(dr_chains* c, int enable);
dr_status dr_stats(dr_chains* c, dr_counters* out, void* hip_stream);

/* Launch configuration of the fused persistent kernel: threads per block
 * (64, 128, 192 or 256), resident blocks per compute unit of the persistent
 * grid, the number of consecutive chains a lane (or lane pair) takes per pop
 * of the device work queue (1..64), lanes per chain (1, or 2: the two lanes
 * trace a path's continuation and shadow rays concurrently), and
 * sort_by_length (1: before each launch, order the chains by the number of
 * path vertices of their last step so the chains of a wavefront finish
 * together; 2: off), and refill (1: the ray-refill form of the fused kernel,
 * one lane per chain, where a lane whose ray query finishes shades and issues
 * its next ray, or finishes its step and starts the next, while the other
 * lanes of its wavefront keep traversing; 2: off) with its two thresholds:
 * a wavefront runs the shading events once refill_event_pct percent of its
 * lanes with rays wait for one, and the step-finishing code once
 * refill_advance_pct percent of its busy lanes do (1..100).  grab and
 * lanes_per_chain do not apply to the refill form.  sort_by_tile (1: before
 * each launch, order the chains by the screen tile of their film coordinates,
 * 64 x 64 tiles in Morton order, killed chains last, so a wavefront's camera
 * rays and the shadow rays from their hits are coherent; takes precedence
 * over sort_by_length; 2: off), and
 * wavefront (1: the initialise pass evaluates its paths as ray waves -
 * alternating launches of a traversal kernel whose persistent lanes take
 * the next pending ray as theirs finishes, and an event kernel that shades
 * each path's vertex and issues its next ray - instead of one lane
 * following one path; 2: off; turning it on allocates its buffers the first
 * time, about 180 bytes per chain, DR_ERR_OUT_OF_MEMORY if that fails, with
 * no field changed), and init_refill (1: the initialise pass
 * evaluates its paths with the ray-refill state machine - a lane whose ray or
 * path ends takes its next event or chain while the others keep traversing,
 * events run once three quarters of the busy lanes wait for one; takes
 * precedence over wavefront; 2: off).
 * Zeros keep the current
 * value.  Defaults: 256 threads, 4 blocks per compute unit, 1 chain per pop,
 * 2 lanes per chain when n_chains is below two wavefronts per SIMD
 * (n_cu * 512) else 1, sorting off (it pays only when chains outnumber the
 * resident lanes several times over), refill off, thresholds 50 and 50,
 * tile ordering off, straight-line initialise pass
 * (init_refill off), ray waves off (on the scenes
 * measured here the state round trips between the two kernels cost more than
 * the denser traversal saves).  The form, the ray waves and the order in which chains are processed never change results. */
typedef struct {
    uint32_t block;
    uint32_t blocks_per_cu;
    uint32_t grab;
    uint32_t lanes_per_chain;
    uint32_t sort_by_length;
    uint32_t refill;
    uint32_t refill_event_pct;
    uint32_t refill_advance_pct;
    uint32_t sort_by_tile;
    uint32_t wavefront;
    uint32_t init_refill;
} dr_launch_cfg;
dr_status dr_chains_set_launch(dr_chains* c, const dr_launch_cfg* cfg);
dr_status dr_chains_get_launch(dr_chains* c, dr_launch_cfg* cfg);

/* ------------------------------------------------------------------------
 * Captured frames (the real-time loop of Sec. 4.3 and 6: scene change ->
 * re-initialise, evolve, resolve once per displayed frame)
 * ------------------------------------------------------------------------ */
typedef struct dr_frame dr_frame;

/* Capture one frame as a HIP graph on hip_stream (must not be the default
 * stream): if reinit, the initialise pass of the next frame (the device frame
 * counter advances by one per launch, starting after the last dr_chains_init
 * or dr_chains_reinit frame); then n_steps evolve steps; then the resolve into
 * image_dev (3*W*H floats, device, borrowed for the frame's lifetime).  Step
 * and frame counters and the camera are read from device memory, so every
 * launch continues the chains and sees dr_scene_set_camera updates.  Record
 * and counter switches are fixed at capture time.  The capture enqueues no
 * memset and no allocation. */
dr_status dr_frame_capture(dr_chains* c, uint32_t n_steps, int reinit, float* image_dev, void* hip_stream,
                           dr_frame** out);
/* Launch a captured frame (asynchronous).  DR_ERR_BAD_STATE if the scene
 * changed and the frame does not re-initialise. */
dr_status dr_frame_launch(dr_frame* f, void* hip_stream);
dr_status dr_frame_destroy(dr_frame* f);

/* ------------------------------------------------------------------------
 * Path-space evaluation (differentiation surface)
 * ------------------------------------------------------------------------ */
/* For n points u_dev (n x d row-major, d = 4(L-1), device) evaluate f (n x 3),
 * log(p + eps) (n) and, if grad_dev is non-NULL, the score grad_u log(p + eps)
 * (n x d) by the reverse-mode adjoint over the taken path (discrete choices
 * held fixed).  The score is the gradient the Langevin drift of Sec. 5
 * (Eq. langevin-drift, with p penalised by eps) moves a chain along; p is the
 * luminance of f (Sec. 3, the target density proportional to f).  rec_dev (n x (L-1), nullable) receives the path record as in
 * dr_state.path_rec.  f_dev and logp_dev are nullable too.  Without grad_dev
 * the points are evaluated by the ray-refill form (lanes take the next point
 * or ray as theirs finish), with results bit-identical to the form that also
 * computes the score.  Allocates a scratch buffer of 4(L-1)n bytes from the
 * stream-ordered pool.  Asynchronous. */
dr_status dr_eval_logp_grad(dr_scene* s, uint32_t L, const float* u_dev, uint32_t n, float eps, float* f_dev,
                            float* logp_dev, float* grad_dev, uint32_t* rec_dev, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as dr_eval_logp_grad, same arguments and results, with the
 * scratch taken from a 16 MiB buffer the library holds in device memory on
 * each GPU it runs on (until the process ends) instead of allocated per call.
 * Calls no hipMalloc/hipFree or any other allocating routine.  With grad_dev
 * the scratch holds 4 (L-1) n bytes of path records, so n (L-1) may be at
 * most 4,194,304 (e.g. n <= 599,186 at L = 8); larger inputs are rejected
 * with DR_ERR_INVALID_ARG before any device work (forward-only calls need
 * 4 bytes and have no limit).  Every call on one GPU shares that GPU's
 * buffer, which keeps the last call's contents: calls that overlap in time
 * on one GPU (other streams, other threads) race, so the caller serialises
 * them (one stream, or events between streams).  The buffer's device
 * address is resolved on the first call on each device.  Asynchronous. */
dr_status dr_eval_logp_grad_noalloc(dr_scene* s, uint32_t L, const float* u_dev, uint32_t n, float eps,
                                    float* f_dev, float* logp_dev, float* grad_dev, uint32_t* rec_dev,
                                    void* hip_stream);

/* Independent path tracing: spp samples per pixel, u0 = (px + U)/W,
 * u1 = (py + U)/H, other coordinates U; img_dev = per-pixel mean of f
 * (3 x W*H planar, device).  Asynchronous. */
dr_status dr_pt_render(dr_scene* s, uint32_t L, uint64_t seed, uint32_t spp, float* img_dev, void* hip_stream);

/* ------------------------------------------------------------------------
 * Analytic target: the chain step on a wrapped Gaussian mixture
 * ------------------------------------------------------------------------ */
/* p(x) = c0 + sum_j w_j prod_i N_wrap(x_i; m_ji, s_j^2) on the torus T^d, and
 * f = p g with the test functions g = (1, cos 2 pi x_0, sin 2 pi x_0, ...,
 * cos 2 pi x_{d-1}, sin 2 pi x_{d-1}) (1 + 2d of them).  The Restore
 * estimator k0 accum / tourCount of Alg. 4.3 converges to lambda(p g), whose
 * components are c0 + sum_j w_j and sum_j w_j exp(-2 pi^2 s_j^2)
 * cos / sin(2 pi m_ji) (Sec. 3: the ergodic and importance identities behind
 * Restore; Sec. 5 for the drift).  The chains use the same regeneration,
 * Euler-Maruyama move, hold/kill draws and random streams as dr_step. */
typedef struct {
    uint32_t d;            /* even, 2..16 */
    uint32_t n_modes;      /* 0..16 */
    const float* weights;  /* host, n_modes, finite, >= 0 */
    const float* means;    /* host, n_modes x d, on [0,1) */
    const float* stds;     /* host, n_modes, in (0, 0.25] */
    float c0;              /* constant floor, >= 0; c0 + sum of weights > 0 */
} dr_mixture_desc;

/* Initialise pass of frame `frame` (Alg. 4.1: x ~ uniform, p_lambda
 * estimate and k0 = p_lambda/(m dt) unless p->k0 > 0, hold/kill/splat,
 * scores) and n_steps evolve steps (Alg. 4.2 with Alg. 5.1) of
 * p->n_chains chains (p->max_path_len and p->mode are ignored;
 * p->sigma_diag, if set, is a device d x N per-chain stddev).  Chains are
 * grouped into n_batches batches (the chains of each 256-chain block go to
 * batch block % n_batches); batch_accum (host, n_batches x (1 + 2d) doubles)
 * receives each batch's sum of (w/dt) g over all its accumulate events and
 * batch_tours (host, n_batches) its completed tours, so the estimate is
 * k0 dt sum(accum) / sum(tours) and the batches give its spread.  *k0_out and
 * *p_lambda_out (nullable) receive k0 and p_lambda.  Allocates its working
 * buffers with hipMalloc per call; synchronous on hip_stream.  Errors:
 * DR_ERR_INVALID_ARG (ranges above, n_batches = 0, null outputs),
 * DR_ERR_DEVICE. */
dr_status dr_mixture_run(const dr_mixture_desc* m, const dr_params* p, uint64_t seed, uint32_t frame,
                         uint32_t n_steps, uint32_t n_batches, double* batch_accum, uint64_t* batch_tours,
                         double* k0_out, double* p_lambda_out, void* hip_stream);

/* One evolve step at global step index `step` with killing constant k0 (> 0)
 * from the host state x, score (d x N planar floats) and killed (N, 0/1),
 * all updated in place (score only for surviving chains); p_out and w_out
 * (host, N) receive p at the new state and the splat weight (time units).
 * Synchronous; allocates with hipMalloc per call.  Errors as
 * dr_mixture_run, and a killed entry other than 0/1. */
dr_status dr_mixture_step(const dr_mixture_desc* m, const dr_params* p, uint64_t seed, uint64_t step, double k0,
                          float* x, float* score, uint32_t* killed, float* p_out, float* w_out, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* DR_H */
