/*
 * ps.h -- free-space Poisson solver by FFT convolution on one MI355X (gfx950).
 *
 * The operation is the potential solve of the paper's benchmark (section 3:
 * the convolution method for potential fields on nested grids; section 1
 * names the FFT as the performance-critical GPU operation).  For a density
 * rho sampled on an N^3 cell-centred grid of spacing dx it computes
 *
 *     phi[i] = G * dx^3 * sum_{j in [0,N)^3} K(i - j) * rho[j],
 *     K(d) = -1 / (dx |d|) for d != 0,   K(0) = -self_coeff / dx,
 *
 * by zero-padding rho to P = 2N per axis, a forward real-to-complex 3D FFT,
 * a pointwise product with the pre-transformed kernel, an inverse FFT and a
 * crop back to [0,N)^3.  Supported N: 8 m for m = 1 .. 64 with no prime
 * factor of m above 5, i.e. P = 2N = 2^a 3^b 5^c with a >= 4 and
 * 16 <= P <= 1024 (N = 8, 16, 24, 32, 40, 48, 64, 72, 80, 96, 120, 128,
 * 144, 160, 192, 200, 216, 240, 256, 288, 320, 360, 384, 400, 432, 480,
 * 512).
 *
 * Memory.  Every pointer passed to the library is a device pointer the
 * caller owns (e.g. torch.Tensor.data_ptr()).  rho and phi are dense
 * C-ordered [z][y][x] arrays (x fastest) of N^3 elements: double for PS_F64
 * and PS_F64_PLAIN, float for PS_F32, PS_F32_SPLIT and PS_F32_PLAIN; they
 * must be aligned to their element size and must not overlap.  The library
 * never allocates device memory: a plan's tables, transformed kernel and
 * intermediates live in one caller-provided workspace of
 * ps_plan_workspace_bytes() bytes, 256-byte aligned, bound to the plan by
 * ps_green_build() and used by every later solve with that plan.
 *
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  Solves
 * are enqueued asynchronously and do not synchronise the host; they make no
 * allocation and no host-to-device copy, so they can be captured into a HIP
 * graph.  A plan (its workspace) serves one solve at a time: two solves with
 * one plan must be ordered on one stream.  Results are bitwise reproducible
 * for a given plan.
 *
 * Errors.  Every call returns a ps_status and never aborts.  Arguments are
 * checked before any HIP call; ps_last_error() gives a thread-local detail
 * string for the last failing call on this thread.
 */
#ifndef PS_H_
#define PS_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ps_plan_s *ps_plan;

typedef enum {
    PS_OK = 0,
    PS_ERR_INVALID = -1,     /* bad argument: NULL, misaligned, overlapping, out of range */
    PS_ERR_UNSUPPORTED = -2, /* size or precision not supported */
    PS_ERR_NOT_READY = -3,   /* solve before a successful ps_green_build */
    PS_ERR_DEVICE = -4,      /* a HIP call failed (no device, launch failure, ...) */
    PS_ERR_CAPTURE = -5      /* called under stream capture where it cannot be */
} ps_status;

typedef enum {
    PS_F64 = 0,       /* pruned, fused pipeline in double */
    PS_F32 = 1,       /* pruned, fused pipeline in float; kernel and twiddles built in double, rounded once */
    PS_F32_SPLIT = 2, /* as PS_F32, radix-16 DFTs on bf16 matrix cores (v_mfma_f32_32x32x16_bf16) with split
                         operands and fp32 accumulation */
    PS_F64_PLAIN = 3, /* the plain method in double: padded grid, full 3D R2C, product, full C2R, crop */
    PS_F32_PLAIN = 4  /* the plain method in float */
} ps_precision;

typedef struct {
    int n;                  /* cells per side */
    int p;                  /* padded length 2n */
    int h;                  /* half-spectrum length n + 1 */
    int precision;          /* ps_precision */
    double dx;              /* cell size */
    size_t workspace_bytes; /* as ps_plan_workspace_bytes */
    size_t ghat_bytes;      /* bytes of the stored kernel spectrum (real octant) */
    int ready;              /* 1 after a successful ps_green_build */
    int radices[8];         /* forward radix plan, 0-terminated */
    size_t t1_offset;       /* byte offset in the workspace of T1 and T4 (pruned plans; 0 otherwise) */
    size_t t2_offset;       /* byte offset in the workspace of T2 (pruned plans; 0 otherwise) */
    size_t t3_offset;       /* byte offset in the workspace of T3 (pruned plans; 0 otherwise) */
    int variant[5];         /* kernel variant of each pruned pass (see ps_plan_set_variant) */
    int split_terms;        /* PS_F32_SPLIT: split-bf16 product terms per DFT-16 (6 or 3); else 0 */
    double dy, dz;          /* cell spacings along y and z (dx unless set by ps_plan_set_spacing) */
    int nx, ny, nz;         /* cells along x, y, z (all n for a cube; n, p, h and radices describe x) */
    int z_tile;             /* pruned plans: pencils per z-pass workgroup, 0 = full tile, 1 = half (ps_plan_set_variant pass 6) */
} ps_plan_info;

/* Create a plan for an n^3 grid of spacing dx (> 0) in the given precision:
 * one mesh level of the convolution method whose potential solve the paper
 * benchmarks (section 3).  The plan is an opaque host object and every
 * device buffer it later uses is the caller's, passed by raw address (the
 * C-bound, caller-owned convention of section 2.2.2 and appendix A).
 * Host work only (radix plan, twiddle tables in double then rounded once to
 * the plan's type, workspace layout); no HIP call.  tune_cache may name a
 * tuning file written by ps_autotune (its choice for this length and
 * precision is applied; a missing file or entry keeps the defaults), or be
 * NULL.  On success *out owns a
 * host object to release with ps_plan_destroy. */
ps_status ps_plan_create(ps_plan *out, int n, double dx, ps_precision prec, const char *tune_cache);

/* A plan for a box of nx x ny x nz cells (arrays [z][y][x], x fastest) of
 * spacings dx, dy, dz (> 0): the same solve on a mesh that is not a cube,
 * phi[i] = G dx dy dz sum_j K(i - j) rho[j] over the box, with each axis
 * zero-padded to twice its own length (the paper's mesh levels are cubes of
 * N^3 cells, section 3; this widens them).  K is the kernel of
 * ps_plan_set_spacing.  Each of nx, ny, nz must be a supported n (else
 * PS_ERR_UNSUPPORTED).  Equal lengths give exactly the plan of
 * ps_plan_create (with ps_plan_set_spacing); unequal lengths run the
 * pruned pipeline's one-tile-per-workgroup kernels for each axis length
 * (PS_F64, PS_F32, PS_F32_SPLIT; the PLAIN precisions are for cubes,
 * PS_ERR_UNSUPPORTED) and ignore tune_cache.  Host work only, no HIP call;
 * every other entry point takes the plan as it takes a cube's, with arrays
 * of nx ny nz reals. */
ps_status ps_plan_create_box(ps_plan *out, int nx, int ny, int nz, double dx, double dy, double dz,
                             ps_precision prec, const char *tune_cache);

/* Bytes of device workspace the plan needs (transformed kernel, tables,
 * intermediates, and the scratch of ps_green_build). */
ps_status ps_plan_workspace_bytes(ps_plan p, size_t *bytes);

/* Plan facts; see ps_plan_info. */
ps_status ps_plan_query(ps_plan p, ps_plan_info *info);

/* Build the transformed kernel in double precision on the GPU into the
 * caller's workspace and bind that workspace to the plan (the
 * pre-transformed Green's function of the convolution method, section 3;
 * the paper does not print the kernel, whose values are fixed by the
 * definition at the top of this file): uploads the
 * twiddle tables, generates K_pad (self cell -self_coeff/dx), transforms it,
 * scales by G dx^3 / P^3 and stores the real octant in the plan's type.
 * Synchronises `stream`.  Must not be called under stream capture
 * (PS_ERR_CAPTURE).  May be called again (new G or workspace). */
ps_status ps_green_build(ps_plan p, void *d_workspace, double G, double self_coeff, void *stream);

/* One solve: phi = potential of rho, enqueued on `stream` (the convolution
 * solve of one mesh level, section 3, whose FFTs section 1 names as the
 * performance-critical GPU work).  rho and phi are device addresses the
 * caller owns (section 2.2.2, appendix A).  Errors: PS_ERR_INVALID for NULL,
 * misaligned or overlapping arrays, PS_ERR_NOT_READY before ps_green_build,
 * PS_ERR_DEVICE if a launch fails; nothing is enqueued on error. */
ps_status ps_solve(ps_plan p, const void *d_rho, void *d_phi, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): ps_solve with
 * the solve's intermediates in the library's static device scratch instead
 * of the plan's workspace.  The scratch is one file-scope device array of
 * 128 MiB per GPU (held until the process ends), enough for the pruned
 * intermediates up to n = 144 in single precision and n = 96 in double;
 * larger plans return PS_ERR_UNSUPPORTED, PLAIN plans PS_ERR_UNSUPPORTED.
 * The plan must be built (its transformed kernel and tables stay in its
 * workspace).  The call allocates nothing and makes no host-to-device copy:
 * it enqueues the same kernels as ps_solve, so results equal ps_solve's
 * bitwise, and it can be captured into a HIP graph.  Every call on one GPU
 * shares that GPU's scratch, and each solve overwrites all of it that it
 * reads, so nothing needs clearing; calls that overlap in time on one GPU
 * (other streams, other host threads) race on the scratch and must be
 * ordered by the caller. */
ps_status ps_solve_static(ps_plan p, const void *d_rho, void *d_phi, void *stream);

/* Bytes of caller-owned device staging memory that ps_solve_host needs for
 * this plan: two input and two output slots of n^3 reals (256-byte aligned).
 * Host only, no HIP call. */
ps_status ps_host_stage_bytes(ps_plan p, size_t *bytes);

/* count solves with one plan on host-resident densities: rho[i] -> phi[i],
 * host pointers to n^3 reals in the layout of ps_solve.  The host <-> device
 * copies the paper's section 2.2.1 measures (pinned against pageable host
 * memory) are staged through d_stage (at least ps_host_stage_bytes, 256-byte
 * aligned, two slots per direction) and run on two copy streams that the
 * plan creates (default priority) and keeps until it is destroyed: the
 * upload of solve i + 1 and the download of solve i - 1 overlap solve i,
 * which runs on `stream`.  Overlap needs pinned host memory (hipHostMalloc,
 * torch pin_memory); with pageable memory the runtime stages each copy and
 * little overlaps.  Everything is ordered after earlier work on `stream`
 * and `stream` resumes after the last download; the call returns before the
 * copies complete, so the host arrays must stay valid until `stream` is
 * synchronised.  A plan runs one such sequence at a time.  Not under stream
 * capture (PS_ERR_CAPTURE). */
ps_status ps_solve_host(ps_plan p, const void *const *h_rho, void *const *h_phi, int count, void *d_stage,
                        size_t stage_bytes, void *stream);

/* count (1..1024) independent solves enqueued on `stream`: several mesh
 * levels (or time steps) on one GPU, where the paper gives each nested level
 * its own GPU and names splitting one GPU among levels as an option it did
 * not pursue (section 3).  Members are
 * grouped by length and kernel variant; each pass is one launch per group,
 * over the group's members (grid z), with the same kernels ps_solve uses, so
 * a member's result equals ps_solve's for its plan bitwise.  The groups of a
 * pass run side by side: the first on `stream`, the others on streams that
 * plans[0] creates (default priority) and keeps until it is destroyed,
 * forked from and joined back into `stream` with events, so the batch is
 * ordered on `stream` as a whole.  All plans must
 * share one pruned precision (PS_F64, PS_F32 or PS_F32_SPLIT); each plan
 * appears at most once and must be built; rho[i] and phi[i] follow the
 * layout of ps_solve, and no output may overlap another array of the batch.
 * The first call with a given list of plans, arrays and kernel variants
 * uploads the members' buffer records into plans[0]'s workspace and
 * synchronises `stream`, so it must not be under stream capture
 * (PS_ERR_CAPTURE); later calls with the same list upload nothing, do not
 * synchronise and can be captured into a HIP graph.  The same plan must not
 * lead two batches in flight at once.  A captured batch reads the records
 * from plans[0]'s workspace each time the graph runs: once plans[0] has led
 * a different list, call the captured list once more outside capture (which
 * uploads its records again) before replaying that graph. */
ps_status ps_solve_batched(const ps_plan *plans, int count, const void *const *d_rho, void *const *d_phi,
                           void *stream);

/* Choose the kernel variant of one pass of a pruned plan (host only, no HIP
 * call).  Passes 0, 1, 3, 4: variant 0 = radix-16-based plan, 1 = two-stage
 * plan, radix 32, 24 or 16 first (n = 72, 144, 160, 192, 200, 216, 240,
 * 256, 288, 320, 360, 384, 400, 432, 480 and 512 only); passes 1 and 3 (the
 * y passes) also
 * take 2 and 3, the same plans run by persistent workgroups that load the
 * next tile while transforming the current one, and 4 and 5, the plans of 0
 * and 1 with half as many pencils per workgroup (8 in float, 4 in double:
 * 64-byte output rows, half the LDS), and 6 and 7, the plans of 0 and 1
 * with every stage exchange through half the LDS in two rounds (twice the
 * workgroups resident per compute unit, the full tile's 128-byte rows;
 * PS_F64 and PS_F32 cubes with n >= 256 only, PS_ERR_UNSUPPORTED
 * otherwise); passes 0 and 4 (the x
 * passes) also take 2 and 3 (8 rows of a z-plane per workgroup instead of
 * 16) and 4 and 5 (32 rows, where the LDS holds them; PS_ERR_UNSUPPORTED
 * otherwise), the family again in the low bit.  Pass 2 (the fused z pass): 0 =
 * workgroup-synchronised pencils, 1 = wavefront-owned pencils, 2 =
 * wavefront-owned pencils on the two-stage plan (where it exists; else as
 * 1), 3 = persistent workgroups that load the next tile while
 * transforming the current one (two-stage plan where it exists, else
 * radix-16-based), 4 = persistent on the radix-16-based plan with fewer
 * pencils per wavefront, 5 = wavefront-owned pencils on the two-stage plan
 * whose stage exchanges pass through half the LDS in two rounds (twice as
 * many pencils resident per compute unit): PS_F64 and PS_F32 cubes with
 * n >= 256 only (PS_ERR_UNSUPPORTED otherwise).  Boxes (ps_plan_create_box with unequal lengths)
 * run the one-tile-per-workgroup variants only: y passes 0 and 1, z pass 0,
 * 1 and 2 (PS_ERR_UNSUPPORTED otherwise); the two-stage plan follows
 * the length of the axis the pass transforms.  Every variant computes the
 * same result to rounding.  PS_F32_SPLIT plans keep the radix-16-based plan
 * (no variant 1 of passes 0, 1, 3, 4, no z variant 2); for them "pass" 5 sets the
 * number of split-bf16 product terms per DFT-16: 6 (three pieces per
 * operand, all piece products of order <= 2; the default) or 3 (two pieces,
 * order <= 1).  "Pass" 6 sets the z pass's tile, for every precision and
 * for boxes: 0 = 16 pencils per workgroup in float, 8 in double (128-byte
 * rows of the z pass's output), 1 = half as many (64-byte rows, half the LDS
 * per workgroup, so that two or more workgroups share a compute unit). */
ps_status ps_plan_set_variant(ps_plan p, int pass, int variant);

/* Cells of spacings dx (the plan's), dy, dz along x, y, z instead of cubes
 * (host only, no HIP call; the plan must be built again with
 * ps_green_build before its next solve, else PS_ERR_NOT_READY).  The solve
 * becomes phi[i] = G dx dy dz sum_j K(i - j) rho[j] with
 * K(d) = -1 / |(d_x dx, d_y dy, d_z dz)| for d != 0 and, for a cell that is
 * not a cube, K(0) = -(self_coeff / C) * A, where A is the average of 1/|r|
 * over the dx x dy x dz cell centred on its centre (closed form) and
 * C = 3 ln(2 + sqrt 3) - pi/2 = 2.38008 is that average over a unit cube
 * (the paper's cells are cubes; this extends its self-cell value to boxes so
 * that a cube gives K(0) = -self_coeff/dx exactly).  dy, dz must be positive
 * and finite (PS_ERR_INVALID). */
ps_status ps_plan_set_spacing(ps_plan p, double dy, double dz);

/* Time every variant of every pass of a built pruned plan on its own
 * workspace (contents are overwritten; the z pass at both tile widths),
 * keep the fastest per pass and, if
 * cache_path is not NULL, record the choice there for ps_plan_create (a text
 * file, one line per length and precision).  Synchronises `stream`; not
 * under stream capture. */
ps_status ps_autotune(ps_plan p, void *stream, const char *cache_path);

/* Release the host object (the workspace stays the caller's). NULL is a no-op. */
void ps_plan_destroy(ps_plan p);

/* Static description of a status code. */
const char *ps_status_str(ps_status s);

/* Detail of the last failing call on this thread ("" if none). */
const char *ps_last_error(void);

/* Measurement aid, not a step of the method: a plain device copy of `bytes`
 * from d_src to d_dst on `stream` (16-byte items, one per thread, in
 * 256-thread workgroups).  Its rate is the achievable HBM bandwidth against
 * which the pass kernels are read.  d_src, d_dst and bytes must be multiples
 * of 16 and the arrays must not overlap (PS_ERR_INVALID). */
ps_status ps_stream_copy(const void *d_src, void *d_dst, size_t bytes, void *stream);

/* Test hook: run a single pass of the pruned pipeline of a built plan on
 * caller arrays (in != out), in the layouts the pipeline uses between passes
 * (H = n + 1, P = 2n, HP = H rounded up to a multiple of 16; complex =
 * interleaved re, im of the plan's type; for a box read n^3 as nz ny nx,
 * H as nx + 1, the y extent of T1 and T4 as ny, the ky extent of T2 and T3
 * as 2 ny, and the z extent as nz):
 *   pass 0  x R2C   in rho[z][y][x] (n^3 real)  -> out T1[kx][z][y]  (H n n complex)
 *   pass 1  y fwd   in T1                       -> out T2[kx][ky][z] (H P n complex)
 *   pass 2  z conv  in T2 -> forward z FFT, product with the kernel, inverse, crop
 *                                               -> out T3[kx][z][ky] (H n P complex)
 *   pass 3  y inv   in T3                       -> out T4[z][y][kx]  (n n HP complex, kx < H used)
 *   pass 4  x C2R   in T4                       -> out phi[z][y][x]
 * Not for PLAIN precisions (PS_ERR_UNSUPPORTED). */
ps_status ps_debug_pass(ps_plan p, int pass, const void *d_in, void *d_out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PS_H_ */
