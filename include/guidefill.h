/*
 * guidefill.h -- C ABI of the MI355X (gfx950) shell-fill library.
 *
 * The library fills the inpainting domain D_h of an image shell by shell
 * (Hocking, MacKenzie, Schoenlieb, "Guidefill", arXiv 1611.05319, Sec. 3,
 * Algorithm 1): at shell k every pixel of the active boundary of D^(k) that is
 * ready receives the normalised weighted average of the readable points of its
 * neighbourhood, with the weights of eqn:weight
 *     w(x, y) = exp(-mu^2 / (2 eps^2) (g_perp(x) . (y - x))^2) / |y - x|,
 * over the rotated ball of ghost pixels (Sec. 3.1, 3.3; bilinear extension
 * eqn:bilinearDef) or the lattice ball; ready is "has a readable point" (onion
 * order) or confidence > c (eqn:confidence, eqn:ready, Sec. 3.4).  Only the
 * pixels of the tracked active front get lanes (Sec. 3.5, "with tracking"), or
 * every pixel gets a lane in every shell ("without tracking").
 *
 * Conventions shared by every entry point
 *   - All array pointers are DEVICE pointers owned by the caller; the library
 *     allocates no memory.  `stream` is a hipStream_t (NULL: default stream).
 *     Calls are asynchronous on `stream`; argument errors are reported
 *     synchronously, device-side findings (label errors, unfilled pixels) in
 *     the stats array after the stream is synchronised.
 *   - Images are B x H x W x C, interleaved channels (HWC per frame), frames
 *     contiguous; element type GF_F32 (binary32) or GF_F16 (binary16).  In
 *     either case the ghost geometry, readable tests, weights and weighted
 *     sums are FP64 and each ghost point's bilinear value is interpolated in
 *     FP32 from the stored colours; results are rounded once to the storage
 *     type.  1 <= C <= 4.
 *   - label: B x H x W uint8, 0 = readable, 1 = inpaint (D_h), 2 = bystander
 *     (B_h, neither filled nor read, Sec. 2.1).  Other values are reported
 *     as label errors and treated as bystanders.
 *   - guide: B x H x W x 2 binary32 (gx, gy), x along columns, y along rows;
 *     read on label-1 pixels only; not normalised (|g| scales the weights).
 *   - shell: B x H x W int32 map: -1 readable, -2 bystander, k >= 0 filled in
 *     shell k, -3 never filled (input colour kept).
 *   - Frames are independent; one call fills all of them.
 *   - Calls that share a workspace must not overlap in time.
 *   - Workspaces: device memory, 256-byte aligned, owned by the caller, zeroed
 *     before their first use; afterwards the library keeps them consistent
 *     (each launch starts with a handshake on a per-workspace epoch number
 *     and join-word set that the library draws on the host for every call,
 *     so a call captured into a graph must not be replayed).
 *   - Each call is one persistent kernel launch: an ordinary (not
 *     cooperative) launch of as many workgroups as the device holds at once.
 *     The workgroups resident at start-up take part and any others leave at
 *     once (stats[GF_STAT_WORKGROUPS] reports how many took part), so work
 *     running concurrently on the device slows a call but cannot deadlock it.
 */
#ifndef GUIDEFILL_H
#define GUIDEFILL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GF_OK = 0,
    GF_EINVAL = -1,     /* bad argument (null pointer, size, parameter, workspace too small) */
    GF_EDEVICE = -2,    /* a HIP call failed (launch, occupancy query, ...) */
    GF_EUNSUPPORTED = -3 /* valid request outside what the library supports */
} gf_status;

typedef enum { GF_F32 = 0, GF_F16 = 1 } gf_dtype;

typedef enum {
    GF_ENGINE_TILED = 0, /* tile windows staged in LDS run pass_shells shells between grid syncs */
    GF_ENGINE_FRONT = 1  /* one grid sync per shell; the front kept as one global list */
} gf_engine;

typedef struct {
    double eps;          /* radius of the ball in pixels, 1 <= eps <= 9 (Sec. 3.1) */
    double mu;           /* anisotropy of the weights, mu > 0 (eqn:weight) */
    double c;            /* < 0: onion order; >= 0: smart order threshold (eqn:ready) */
    int32_t ghost;       /* 1: rotated ball with ghost pixels; 0: lattice ball */
    int32_t tracking;    /* 1: lanes for the tracked front only; 0: one lane per pixel per shell */
    int32_t max_shells;  /* 0: run until no pixel is ready; n > 0: stop after n shells */
    int32_t engine;      /* gf_engine */
    int32_t group;       /* lanes per pixel: 8, 16, 32 or 64; 0 = the smallest with at most
                            4 ball offsets per lane */
    int32_t blocks_per_cu; /* persistent workgroups per compute unit: 0 (auto) or 1..8 */
    int32_t tile_w, tile_h; /* tiled engine: tile interior in pixels, 0 = auto (<= 256) */
    int32_t pass_shells;    /* tiled engine: shells per grid sync, 0 = auto (<= 32); the halo
                               pass_shells * ceil(eps) may not exceed tile_w or tile_h */
    int32_t tile_threads;   /* tiled engine: threads per workgroup, 0 (768), 256, 512, 768, 1024;
                               must be 0 with GF_ENGINE_FRONT */
    double c2;              /* < 0: no data term; >= 0: the data term of eqn:ready2 (Sec. 3.4),
                               ready also requires |g(x)| > c2, until the first shell in which
                               that leaves no pixel ready; that shell and the later ones use
                               eqn:ready (or onion order) alone.  The switch is per frame:
                               c2 >= 0 needs B == 1 (else GF_EUNSUPPORTED) */
} gf_params;

/* Layout of the int32 stats array written by gf_fill / gf_fill_batched
 * (device memory, 8 + 4 * B entries): */
enum {
    GF_STAT_SHELLS = 0,      /* number of shells that filled at least one pixel (K) */
    GF_STAT_FILLED = 1,      /* pixels filled, all frames */
    GF_STAT_HOLE = 2,        /* label-1 pixels, all frames */
    GF_STAT_MAX_FRONT = 3,   /* largest active front (lanes requested in one shell; the
                                tiled engine counts as for front_hist below) */
    GF_STAT_LABEL_ERR = 4,   /* label values outside {0, 1, 2} */
    GF_STAT_ORDER_TRUNC = 5, /* 1 if shell_offsets was too short for K + 1 entries */
    GF_STAT_SYNC_TIMEOUT = 6,/* 1 if a grid barrier gave up waiting (never expected; the
                                results are then invalid) */
    GF_STAT_WORKGROUPS = 7,  /* workgroups that took part in the persistent launch (those
                                resident at start-up; normally the whole launched grid) */
    GF_STAT_FRAME0 = 8,      /* then per frame f at 8 + 4 f: K_f, filled_f, hole_f, 0 */
    GF_STAT_PER_FRAME = 4
};

/*
 * Bytes of workspace gf_fill_batched needs for B frames of H x W (front lists,
 * control words).  The workspace is device memory, 256-byte aligned, zeroed
 * before its first use (see the conventions above).
 */
size_t gf_workspace_size(int B, int H, int W, int C, gf_dtype dt, const gf_params *p);

/*
 * Fill B frames (Algorithm 1, all shells, one persistent launch).
 *   img_in      B*H*W*C of dt, read only.
 *   img_out     B*H*W*C of dt.  May equal img_in (in place: only filled
 *               pixels are written); otherwise every pixel is written (the
 *               input colour where nothing is filled).
 *   label, guide, shell_out: as above; shell_out is required.
 *   stats       int32[8 + 4*B], required.
 *   order_out   nullable; int32[B*H*W]: frame*H*W + pixel of every filled
 *               pixel, grouped by shell;
 *               needs engine GF_ENGINE_FRONT (else GF_EUNSUPPORTED).
 *   shell_offsets nullable (required with order_out); int32[kcap]: entry k is
 *               the start of shell k in order_out, entry K its end.  If
 *               K + 1 > kcap the fill still completes and
 *               stats[GF_STAT_ORDER_TRUNC] is set.
 *   front_hist  nullable; int32[kcap]: active front size of each shell (the
 *               tiled engine counts the active pixels of the tiles it visits;
 *               pixels waiting in tiles whose neighbourhood did not change are
 *               not recounted).
 *   workspace   >= gf_workspace_size(...) bytes.
 * Returns GF_OK or GF_EINVAL / GF_EUNSUPPORTED / GF_EDEVICE.
 */
gf_status gf_fill_batched(const void *img_in, void *img_out, int B, int H, int W, int C,
                          gf_dtype dt, const uint8_t *label, const float *guide,
                          const gf_params *p, int32_t *shell_out, int32_t *stats,
                          int32_t *order_out, int32_t *shell_offsets, int32_t *front_hist,
                          int kcap, void *workspace, size_t ws_bytes, void *stream);

/*
 * gf_fill_batched for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, hosts that forbid hipMalloc.  Same
 * arguments, results and errors as gf_fill_batched, without the workspace:
 * the call uses the library's own scratch, a 16 MiB (GF_SCRATCH_BYTES) array
 * that each device holds from the time it loads the library until the
 * process ends, and calls no allocating routine.  A request whose workspace
 * (gf_workspace_size) exceeds the scratch returns GF_EINVAL with the sizes in
 * gf_last_error: at most about one 1920 x 1080 frame with GF_ENGINE_FRONT,
 * about 200 000 tiles (90 such frames at the default tile) with
 * GF_ENGINE_TILED.  Every call on a device shares that device's scratch and
 * leaves its contents behind (each launch re-initialises what it reads):
 * calls that overlap in time on one device race, whatever their streams, and
 * must be serialised by the caller.
 */
#define GF_SCRATCH_BYTES ((size_t)16 << 20)
gf_status gf_fill_batched_noalloc(const void *img_in, void *img_out, int B, int H, int W, int C,
                                  gf_dtype dt, const uint8_t *label, const float *guide,
                                  const gf_params *p, int32_t *shell_out, int32_t *stats,
                                  int32_t *order_out, int32_t *shell_offsets, int32_t *front_hist,
                                  int kcap, void *stream);

/* One frame: gf_fill_batched with B = 1. */
gf_status gf_fill(const void *img_in, void *img_out, int H, int W, int C, gf_dtype dt,
                  const uint8_t *label, const float *guide, const gf_params *p,
                  int32_t *shell_out, int32_t *stats, void *workspace, size_t ws_bytes,
                  void *stream);

/*
 * Reverse-mode derivative of a completed fill (an extension beyond the paper; the
 * fill is linear in the known colours, Algorithm 1).  One persistent launch:
 * the filled pixels are grouped by shell from the shell map (a counting sort
 * inside the launch), then the shells are replayed from the last to the
 * first, the ghost geometry, readable sets and weights recomputed from the
 * shell map instead of stored.  Any engine's forward can precede it.
 *   grad_out    B*H*W*C binary32: dL/d img_out.
 *   img_out     the forward's output (dt); shell: its shell map.
 *   label       not read (the shell map carries the labels' roles); may be NULL.
 *   guide       the forward's guide.
 *   K           shells to replay: the forward's stats[GF_STAT_SHELLS], or -1
 *               to take max(shell) + 1 from the map on the device (no host
 *               synchronisation).  Pixels with shell >= K are treated as never
 *               filled.  -1 <= K <= H * W.
 *   grad_img    B*H*W*C binary32: dL/d img_in (readable and bystander pixels
 *               and never-filled hole pixels pass grad_out through plus what
 *               the fill propagates to them; filled hole pixels get 0).  May
 *               equal grad_out.
 *   grad_guide  B*H*W*2 binary32: dL/d guide on filled pixels, 0 elsewhere.
 *   p           the forward's parameters (eps, mu, ghost are used; the launch
 *               shape is the adjoint's own: the narrowest lane group that holds
 *               the ball, two workgroups per CU).
 *   workspace   >= gf_backward_workspace_size(...) bytes, 256-byte aligned,
 *               zeroed before its first use (as for the forward).
 * Returns GF_OK or GF_EINVAL / GF_EUNSUPPORTED / GF_EDEVICE.
 */
gf_status gf_fill_backward(const float *grad_out, const void *img_out, int B, int H, int W, int C,
                           gf_dtype dt, const uint8_t *label, const float *guide,
                           const int32_t *shell, int K, const gf_params *p, float *grad_img,
                           float *grad_guide, void *workspace, size_t ws_bytes, void *stream);

/* Bytes of workspace gf_fill_backward needs. */
size_t gf_backward_workspace_size(int B, int H, int W, int C, gf_dtype dt, const gf_params *p);

/*
 * Tile geometry the tiled engine would use for these parameters on the
 * current device: out6 = {tile_w, tile_h, pass_shells, halo, LDS bytes of the
 * window, lanes per pixel}.  Returns GF_EINVAL if no window fits.
 */
gf_status gf_tile_geometry(int H, int W, int C, gf_dtype dt, const gf_params *p, int32_t *out6);

/*
 * Coherence-transport comparison mode (Sec. 3.2, eqn:modStructureTensor):
 * the fill of Algorithm 1 in which, before every shell, each front pixel x
 * (label 1 with a known in-frame 8-neighbour) takes as its guide the
 * coherence direction of the modified structure tensor of the pixels known
 * at that shell (label 0 and the pixels filled so far):
 *   v = (g_sigma * (1_K u)) / (g_sigma * 1_K),
 *   J = (g_rho * (1_K sum_c grad v_c (x) grad v_c)) / (g_rho * 1_K),
 *   g(x) = tanh((lambda+ - lambda-) / Lambda) v-  (0 where no known pixel
 *   lies within the rho window),
 * Gaussians of variance sigma^2 and rho^2 truncated to |dx|, |dy| <= floor(2 s),
 * grad v by central differences (one-sided at the frame edge).  This is the
 * direction estimate the paper shows to kink lines (its Sec. 3.2 example);
 * Guidefill itself uses splines (gf_guide_field).  With p->ghost = 0 the
 * neighbourhood is coherence transport's lattice ball.  The tensor and g are
 * computed in FP64 from the stored colours; the fill as in gf_fill_batched.
 *   img_in / img_out, label, shell_out: as for gf_fill_batched (img_out may
 *               alias img_in); stats: int32[8 + 4*B] device array in the
 *               gf_fill_batched layout (K, filled, hole, largest front,
 *               label errors, per-frame K, filled, hole).
 *   sigma, rho  the two scales (> 0; the paper's example takes 2 and 4;
 *               sigma <= 8, rho <= 16).  lambda: Lambda > 0 (1e-5 in the
 *               paper).
 *   guide_used  nullable, device float32 B*H*W*2: the guide each filled
 *               pixel was filled with (0 elsewhere); sign as computed
 *               (gx > 0, or gx == 0 and gy > 0).
 *   p           as for gf_fill_batched; p->max_shells bounds the shells;
 *               p->c2 must be < 0 (GF_EUNSUPPORTED otherwise); each shell is
 *               one fill launch, on the tiled engine with one shell per pass
 *               unless p->pass_shells is set.
 * Workspace: gf_coherence_workspace_size bytes, zeroed before first use.
 * Unlike the other fills this call is synchronous: it enqueues the shells in
 * batches of 4 and reads their counts back to the host to decide whether to
 * go on (one stream synchronisation per batch; a shell enqueued after the
 * fill has finished or stalled changes nothing), and returns when the fill
 * has finished.
 */
size_t gf_coherence_workspace_size(int B, int H, int W, int C, gf_dtype dt, const gf_params *p);

gf_status gf_fill_coherence(const void *img_in, void *img_out, int B, int H, int W, int C,
                            gf_dtype dt, const uint8_t *label, const gf_params *p,
                            double sigma, double rho, double lambda, int32_t *shell_out,
                            int32_t *stats, float *guide_used, void *workspace, size_t ws_bytes,
                            void *stream);

/*
 * Guide field (Sec. 3.2), the fill's input g built on the device: for every
 * inpaint pixel x (label 1) the spline nearest to x and
 *     g(x) = g_Gamma exp(-d(x, Gamma)^2 / (2 eta^2)),
 * 0 where d(x, Gamma) > cutoff (the paper takes eta = 3 px and cutoff = 3 eta)
 * or the frame has no spline, and 0 on every other pixel.  Splines are
 * polylines: each segment carries its spline's direction g_Gamma (a straight
 * spline is one segment; a sampled curve may give each segment the local
 * tangent); the nearest spline is the one holding the nearest segment, equal
 * distances keeping the first.  Pixel (i, j) sits at (i, j), i the column.
 * Distances and the choice of spline are FP64; g is rounded to binary32.
 *   label    B*H*W uint8 (device).
 *   seg      device float32, nseg * 6: x0, y0, x1, y1, gx, gy per segment
 *            (may be NULL when every frame has none).
 *   seg_off  device int32[B + 1]: frame b's segments are seg_off[b] ..
 *            seg_off[b + 1] - 1 (non-decreasing, within seg).
 *   guide    device float32, B*H*W*2 output (gx, gy), every pixel written.
 * Returns GF_OK or GF_EINVAL (bad size, eta <= 0, cutoff < 0, null
 * pointer) / GF_EDEVICE; asynchronous on `stream`.
 */
gf_status gf_guide_field(int B, int H, int W, const uint8_t *label, const float *seg,
                         const int32_t *seg_off, double eta, double cutoff, float *guide,
                         void *stream);

/* Text for a status code (static storage). */
const char *gf_status_string(gf_status s);

/* Last HIP error text recorded by this thread (static thread-local storage). */
const char *gf_last_error(void);

/* ABI version: 2. */
int gf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GUIDEFILL_H */
