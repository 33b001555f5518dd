/*
 * nst.h -- C ABI of the localized style-transfer loss+gradient library (libnst.so)
 *
 * Method: Galerne, Raad, Lezama, Morel, "Scaling Painting Style Transfer".
 *   Energy (Eq. 1-3):   E(x) = sum_l w_l || G_l(x) - G_l(s) ||_F^2 + alpha || F(x) - F(c) ||^2
 *   Gram (Sec. 3.1):    G_l = V_l^T V_l / n_p^l, V_l the n_p^l x C_l post-ReLU features of
 *                       conv k_1 (style layers), n_p^l the whole-image feature-pixel count
 *   Feature gradients:  Table 1 (Gram row and MSE row)
 *   Localized passes:   Sec. 4.1 (blocks with margin) and Algorithm 1 (Step 1 global
 *                       statistics block by block, Step 2 per-block backward that keeps the
 *                       inner part of the gradient)
 *
 * Conventions shared by every entry point
 *   - Images are device pointers to float32, planar C x H x W (C = 3), row-major.
 *   - Gram matrices are device pointers to float64: the style layers in network order,
 *     each C_l x C_l row-major, concatenated, already divided by n_p^l of the image they
 *     were computed on.
 *   - Feature maps are device pointers to float32, h x w x C (channels fastest), where
 *     h = floor(H / s), w = floor(W / s) and s is the layer's cumulative pooling stride.
 *   - The caller owns every input and output buffer.  The context owns only its packed
 *     copy of the network weights.  Scratch memory is a caller-provided device workspace
 *     sized with nst_workspace_bytes(); the run calls allocate nothing.
 *   - All device work is enqueued on `stream` (a hipStream_t; NULL is the null stream).
 *     Calls return after enqueueing, except that a non-NULL host `energy` output makes
 *     the call wait for the stream to copy the energies back.
 *   - Every call validates its arguments before launching anything; on a validation
 *     error no output is touched.  A HIP runtime failure returns NST_EHIP and leaves the
 *     outputs undefined.  Nothing aborts or throws across the ABI.
 *   - A context is not thread-safe: use one context per host thread / stream.
 *   - Tile plan (block T, margin m): see nst_plan().  Results equal the whole-image ones
 *     (up to rounding) when m >= nst_min_halo(); smaller margins are accepted unless
 *     NST_STRICT_HALO is set, so that the margin-too-small seams can be reproduced.
 */
#ifndef NST_H
#define NST_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NST_ABI_VERSION 2
#define NST_MAX_CONV 16
#define NST_MAX_STYLE 8

typedef struct nst_ctx nst_ctx;

typedef enum {
  NST_OK = 0,
  NST_EINVAL = -1,      /* NULL pointer, bad enum/flag, unsupported network shape       */
  NST_ESHAPE = -2,      /* H, W, T < 1, m < 0, or an image too large for 32-bit indexing */
  NST_EHALO = -3,       /* m < nst_min_halo() under NST_STRICT_HALO                      */
  NST_ENOMEM = -4,      /* nst_create could not allocate the packed weights              */
  NST_EHIP = -5,        /* a HIP runtime call failed                                      */
  NST_ECAPACITY = -6,   /* nst_plan: output array too small (needed count is returned)  */
  NST_EWORKSPACE = -7,  /* workspace smaller than nst_workspace_bytes(..., tile_batch=1), or
                           than the every-tile size under NST_RESIDENT                     */
  NST_ENONFINITE = -8   /* NST_CHECK_FINITE: an input holds a NaN or an infinity          */
} nst_status;

typedef enum { NST_FP32 = 0, NST_BF16 = 1 } nst_precision;

enum {
  NST_STEP1 = 1,        /* Algorithm 1 Step 1: global Grams of x (+ energies)            */
  NST_STEP2 = 2,        /* Algorithm 1 Step 2: gradient from given Grams of x            */
  NST_BOTH = 3,
  NST_STRICT_HALO = 4,  /* reject m < nst_min_halo()                                      */
  NST_CHECK_FINITE = 8, /* check x, content_feats, target_grams (and grams_x when read),
                           w_style and alpha for NaN / infinity before any other work;
                           costs one pass over the inputs and a host wait               */
  NST_RESIDENT = 16     /* keep every tile's activations from Step 1 to Step 2 of the same
                           call instead of recomputing them (needs the every-tile
                           workspace of nst_workspace_bytes; same results, bit for bit)  */
};

/* A VGG-style feature network: n_conv 3x3 convs (zero padding 1, stride 1), each followed
 * by ReLU, some followed by a 2x2 stride-2 floor-mode pool (max, or average where
 * pool_avg says so: the average-pooling variant of the network used for texture synthesis
 * by the work the paper builds on).  Style layers and the content layer name convs whose
 * post-ReLU (pre-pool) output is used.  Supported shapes:
 * c_in[0] == 3; c_in[i] == c_out[i-1]; c_out[i] == 64 or a multiple of 128; no style layer
 * is followed by a pool below the deepest used conv; convs after the deepest style/content
 * layer are ignored. */
typedef struct {
  int n_conv;
  int c_in[NST_MAX_CONV];
  int c_out[NST_MAX_CONV];
  unsigned pool_after;            /* bit i set: max pool after conv i                    */
  int n_style;
  int style_conv[NST_MAX_STYLE];  /* increasing conv indices                              */
  int content_conv;               /* conv index, or -1 (no content term)                  */
  unsigned pool_avg;              /* bit i set: the pool after conv i averages (bits outside
                                     pool_after are an error)                            */
} nst_net_desc;

/* One block of the plan.  Image-pixel coordinates, half-open. */
typedef struct {
  int by0, by1, bx0, bx1;         /* the block (inner part) this tile owns                 */
  int ey0, ey1, ex0, ex1;         /* its window: block + margin, aligned, clipped          */
  int own[NST_MAX_CONV][4];       /* owned feature rows/cols (r0, r1, c0, c1) of each conv */
} nst_tile;

int nst_abi_version(void);
const char *nst_strerror(int status);

/* Fill `out` with the VGG-19 prefix conv1_1..conv5_1 (tiny != 0: conv1_1..conv3_1).
 * Style layers relu{1..5}_1 (tiny: relu1_1, relu2_1, relu3_1); content relu4_2
 * (tiny: relu2_2) or none when with_content == 0.  Sec. 3.1 names these layers. */
int nst_net_vgg19(nst_net_desc *out, int tiny, int with_content);

/* Smallest margin that makes the tiled Grams and gradient exact: the widest receptive
 * field, max_i (a_i + b_i), where feature row q of conv i depends on input rows
 * [s_i q - a_i, s_i q + b_i] (Sec. 4.1: margin must cover the receptive field).
 * Returns a negative nst_status on an invalid descriptor.  Host only. */
int nst_min_halo(const nst_net_desc *net);

/* The tile plan (Sec. 4.1, Algorithm 1).  Blocks: row-major grid, rows [i T, min((i+1) T, H)).
 * Window: [S floor((b0 - m) / S), S ceil((b1 + m) / S)) clipped to the image, S = product of
 * the pooling factors.  Owned feature rows of conv i (stride s): [ceil(b0/s), min(ceil(b1/s),
 * floor(H/s))); columns likewise.  Writes min(cap, count) tiles to `out` (may be NULL when
 * cap == 0) and the count to *n_tiles; returns NST_ECAPACITY if cap < count.  Host only. */
int nst_plan(const nst_net_desc *net, int H, int W, int T, int m,
             nst_tile *out, int cap, int *n_tiles);

/* Device workspace needed to process `tile_batch` tiles of the plan at once with the given
 * precision; the run calls use the largest batch that fits in what they are given, so
 * memory is one tile batch's activations plus the Grams (Algorithm 1: Step 2 recomputes
 * each tile's forward).  tile_batch >= the plan's tile count gives the every-tile size
 * that NST_RESIDENT needs.  Host only. */
int nst_workspace_bytes(const nst_net_desc *net, int precision, int H, int W, int T, int m,
                        int tile_batch, size_t *bytes);

/* Create a context on the current HIP device.  w[i]: host float32 [c_out][c_in][3][3];
 * b[i]: host float32 [c_out] or NULL for zero bias.  Packs device copies. */
int nst_create(const nst_net_desc *net, const float *const *w, const float *const *b,
               int precision, nst_ctx **out);
void nst_destroy(nst_ctx *ctx);

/* Global style Grams of image s (3 x H x W), accumulated tile by tile like Step 1 of
 * Algorithm 1 (its Require line takes the style statistics from such a pass).  grams: device
 * float64 output, sum_l C_l^2 values. */
int nst_style_grams(nst_ctx *ctx, const float *s, int H, int W, int T, int m, double *grams,
                    void *ws, size_t ws_bytes, void *stream);

/* Style statistics of image s for the augmented style loss (Sec. 3.2, Eq. 5; Algorithm 1
 * Require): the Grams as nst_style_grams and, when means != NULL, the spatial mean of
 * each channel of each style layer, mean(V_l(s)), accumulated block by block like the
 * Grams (FP32 per 2048-pixel chunk, FP64 across chunks and blocks, fixed order).
 * means: device float64, sum_l C_l values, style layers in network order. */
int nst_style_stats(nst_ctx *ctx, const float *s, int H, int W, int T, int m, double *grams,
                    double *means, void *ws, size_t ws_bytes, void *stream);

/* Post-ReLU features of conv `conv` for image img, computed block by block and written to
 * the whole-image map feats (device float32, h x w x C_conv).  With conv == content_conv
 * this is the content-feature input of Algorithm 1. */
int nst_layer_feats(nst_ctx *ctx, const float *img, int H, int W, int T, int m, int conv,
                    float *feats, void *ws, size_t ws_bytes, void *stream);

/* Content features V^{Lc}(c) (Algorithm 1 Require) = nst_layer_feats at content_conv. */
int nst_content_feats(nst_ctx *ctx, const float *c, int H, int W, int T, int m, float *feats,
                      void *ws, size_t ws_bytes, void *stream);

/* Algorithm 1 on x (3 x H x W).
 *   target_grams : device float64, Grams of the style image (nst_style_grams layout)
 *   content_feats: device float32 content features of the content image at H x W, or NULL
 *                  iff alpha == 0 or the network has no content layer
 *   w_style      : host float64 [n_style], the w_l of Eq. 3
 *   flags        : NST_STEP1 | NST_STEP2 (| NST_STRICT_HALO | NST_CHECK_FINITE | NST_RESIDENT)
 *   grams_x      : device float64; written by Step 1; read by Step 2 when Step 1 is not
 *                  requested (the autograd backward reuses the forward's Grams)
 *   energy       : host float64 [2 + n_style] = {E, E_content, E_style_l...} or NULL.
 *                  E_content is summed over owned content features of whichever passes ran.
 *   grad         : device float32 3 x H x W, dE/dx, written when NST_STEP2 is set.
 * Memory: one tile batch's activations plus the Grams (every tile's under NST_RESIDENT);
 * nothing whole-image besides the inputs and outputs.
 * Errors: NST_EINVAL (NULL pointer, unknown flag, content_feats NULL with alpha != 0 and a
 * content layer), NST_ESHAPE, NST_EHALO, NST_EWORKSPACE, NST_ENONFINITE (only under
 * NST_CHECK_FINITE; nothing is written), NST_EHIP. */
int nst_loss_grad(nst_ctx *ctx, const float *x, int H, int W, const double *target_grams,
                  const float *content_feats, const double *w_style, double alpha, int T,
                  int m, int flags, double *grams_x, double *energy, float *grad, void *ws,
                  size_t ws_bytes, void *stream);

/* The augmented style loss (Sec. 3.2, Eq. 5): each style layer's term becomes
 *   w_l ||G_l(x) - G_l(s)||_F^2 + w'_l ||mean_l(x) - mean_l(s)||^2 + w''_l ||std_l(x) - std_l(s)||^2
 * with per-channel spatial mean and standard deviation, std = (diag(G) - mean^2)^(1/2)
 * (Algorithm 1 Step 1; a negative radicand counts as 0).  Feature gradients: Table 1 rows
 * 3 and 4; on a channel whose std is 0 the std row is taken as 0. */
typedef struct {
  const double *w_mean;         /* host [n_style]: w'_l                                        */
  const double *w_std;          /* host [n_style]: w''_l                                       */
  const double *target_means;   /* device float64 [sum_l C_l]: mean_l(s) (nst_style_stats); the
                                   target std comes from it and the target Gram's diagonal    */
  double *means_x;              /* device float64 [sum_l C_l]: mean_l(x), written by Step 1,
                                   read by a call that runs Step 2 alone                       */
} nst_mean_std;

/* nst_loss_grad with the augmented style loss; ms == NULL is nst_loss_grad itself.
 * energy[2 + l] is layer l's whole augmented term.  Errors as nst_loss_grad, and
 * NST_EINVAL when a pointer of *ms is NULL. */
int nst_loss_grad_ms(nst_ctx *ctx, const float *x, int H, int W, const double *target_grams,
                     const float *content_feats, const double *w_style, double alpha,
                     const nst_mean_std *ms, int T, int m, int flags, double *grams_x,
                     double *energy, float *grad, void *ws, size_t ws_bytes, void *stream);

/* ---- Allocation-free variant, for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc) ----
 * nst_loss_grad with the workspace replaced by a static device array of
 * nst_scratch_bytes() (256 MiB) that the library holds on each GPU it runs on until the
 * process ends (its address is looked up once per device by nst_create).  The call
 * allocates and frees nothing; it uses the largest tile batch that fits in the array and
 * returns NST_EWORKSPACE, before any launch, when even one tile's activations do not fit
 * (e.g. BF16 tiles of 512 px with margin 155 fit, tiles of 1024 px do not).  Every call on
 * a GPU shares that GPU's array: calls that overlap on one GPU (several streams, several
 * threads) race and must be serialized by the caller.  Arguments, outputs and errors
 * otherwise as nst_loss_grad. */
size_t nst_scratch_bytes(void);
int nst_loss_grad_noalloc(nst_ctx *ctx, const float *x, int H, int W, const double *target_grams,
                          const float *content_feats, const double *w_style, double alpha, int T,
                          int m, int flags, double *grams_x, double *energy, float *grad,
                          void *stream);

/* ---- Profiling (instrumentation of the entry points above; not part of the method) ----
 * While enabled, every kernel the run calls enqueue is bracketed by two HIP events on the
 * caller's stream.  nst_profile_read() waits for those events and returns, per kernel
 * instantiation (its demangled name, as profilers list it), the launch count, the summed
 * event time, and the summed algorithmic work of those launches: FLOPs = 2 x (output
 * pixels) x (output channels) x (multiply-adds per output) with no padding counted, and
 * bytes = minimal HBM traffic (each operand read once, each result written once).
 * Recording adds ~2 event records per launch; it neither reorders nor synchronizes work. */
typedef struct {
  char name[160];
  int launches;
  double ms;
  double flops;
  double bytes;
} nst_kstat;

/* enable != 0: clear previous records and start recording; enable == 0: stop. */
int nst_profile(nst_ctx *ctx, int enable);
/* Aggregate the records (synchronizing on their events), write min(cap, count) entries
 * sorted by decreasing time, set *n to the count, and clear the records. */
int nst_profile_read(nst_ctx *ctx, nst_kstat *out, int cap, int *n);

#ifdef __cplusplus
}
#endif
#endif /* NST_H */
