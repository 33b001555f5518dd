// Internal interface between the host scheduler (nst_api.cpp) and the gfx950 kernels
// (kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stddef.h>

namespace nst {

// Tiles processed by one launch.  Per-tile geometry travels by value in the kernel
// arguments, so a launch needs no device-side descriptor table.
constexpr int kMaxBatch = 32;

// Owned pixels per Gram partial (fixed-order FP32 chunk, then FP64 across chunks).
constexpr int kGramChunk = 2048;
// Owned pixels per content-energy partial.
constexpr int kContentBlockPx = 64;

struct Batch {
  int n;                       // tiles in this launch
  int h[kMaxBatch];            // window rows at this layer
  int w[kMaxBatch];            // window cols at this layer
  int a0[kMaxBatch], a1[kMaxBatch], a2[kMaxBatch], a3[kMaxBatch];  // region (rows a0..a1, cols a2..a3), window-local
  int gy[kMaxBatch], gx[kMaxBatch];   // window origin in whole-image coordinates of this layer
  int slot[kMaxBatch];         // workspace slot of the tile
  int pfx[kMaxBatch + 1];      // prefix sum of work blocks per tile
};

enum InMode { IN_NHWC = 0, IN_IMAGE = 1, IN_NONE = 2 };
enum EpiMode { EPI_FWD = 0, EPI_BWD = 1, EPI_STITCH = 2 };

struct ConvArgs {
  // segment 0: 3x3 taps over `in` (NHWC, cin channels) or an im2col of the image
  const void *in;
  long long in_ss;             // slot stride, elements
  int cin;
  const void *wp;              // packed B operand [cin/CK][taps][cout_pad][CK]
  // segment 1 (optional): centre tap over in2 (NHWC, cin2 channels) with wp2 [cin2/CK][1][cout_pad][CK]
  const void *in2;
  long long in2_ss;
  int cin2;
  const void *wp2;
  // output (EPI_FWD: may be null when only the pooled output is wanted)
  void *out;
  long long out_ss;
  void *pool;                  // EPI_FWD: optional 2x2 pooled output (floor mode), NHWC
  long long pool_ss;
  int pool_avg;                // that pool averages the four stored values (else: first maximum)
  int cout;                    // real output channels
  int cout_pad;                // padded N of the packed operands
  const float *bias;           // EPI_FWD: bias; EPI_BWD (optional): per-channel constant added
                               // to the adjoint before the mask (mean/std seeds)
  const void *mask;            // EPI_BWD: keep where mask > 0 (post-ReLU activation, cout channels)
  long long mask_ss;
  float *rc;                   // content difference relu(acc) - F_c, fp32, cout channels
  long long rc_ss;
  const float *fc;             // EPI_FWD with rc: whole-image content features (h x w x cout)
  int fc_w;
  float two_alpha;             // EPI_BWD with rc
  const float *img;            // IN_IMAGE: 3 x img_h x img_w
  float *grad;                 // EPI_STITCH: 3 x img_h x img_w
  int img_h, img_w;
};

// precision: 0 = fp32, 1 = bf16
int ck_of(int precision);
size_t elem_size(int precision);

// Conv / data-gradient / residual launches (implicit GEMM on MFMA).
hipError_t launch_conv(int precision, int in_mode, int epi, const ConvArgs &a, const Batch &g,
                       hipStream_t s);
int conv_block_px(int precision, int in_mode, int epi, int cout);   // pixels per work block
// Demangled name of the kernel instantiation launch_conv would pick (as profilers list it).
const char *conv_kernel_name(int precision, int in_mode, int epi, const ConvArgs &a);
int conv_block_rows(int precision, int in_mode, int epi, int cout); // patch rows
int conv_block_cols(int precision, int in_mode, int epi, int cout); // patch columns

// avg: the pool averaged (a quarter of dP to each input) instead of taking the first maximum
hipError_t launch_pool_bwd(int precision, const void *dp, long long dp_ss, const void *act,
                           long long act_ss, const float *rc, long long rc_ss, float two_alpha,
                           void *dz, long long dz_ss, int C, bool avg, const Batch &g, hipStream_t s);
hipError_t launch_gram(int precision, const void *act, long long act_ss, int C, const Batch &g,
                       float *part, long long part_ss, hipStream_t s);
hipError_t launch_gram_tile_reduce(const float *part, long long part_ss, int C, const Batch &g,
                                   double *tilesum, hipStream_t s);
hipError_t launch_gram_accum(const double *tilesum, int n_tiles, int C, double *gacc,
                             hipStream_t s);
// csum[c] += sum of channel c over the owned region of each tile of g (chunks of kGramChunk
// pixels, FP32 per chunk, FP64 per tile, added in tile order); part: per-slot scratch of
// (chunks x C) floats
hipError_t launch_chan_sums(int precision, const void *act, long long act_ss, int C, const Batch &g,
                            float *part, long long part_ss, double *csum, hipStream_t s);
hipError_t launch_content_partial(const float *rc, long long rc_ss, int C, const Batch &g,
                                  double *part, long long part_ss, hipStream_t s);
hipError_t launch_content_accum(const double *part, long long part_ss, const Batch &g,
                                double *acc, hipStream_t s);
hipError_t launch_stitch_feats(int precision, const void *act, long long act_ss, int C,
                               const Batch &g, float *feats, int feats_w, hipStream_t s);
hipError_t launch_fill_f64(double *p, size_t n, double v, hipStream_t s);
hipError_t launch_fill_f32(float *p, size_t n, float v, hipStream_t s);
hipError_t launch_fill_u32(unsigned *p, size_t n, unsigned v, hipStream_t s);
// *count += number of NaN / infinite elements of p[0..n)
hipError_t launch_count_nonfinite_f32(const float *p, size_t n, unsigned *count, hipStream_t s);
hipError_t launch_count_nonfinite_f64(const double *p, size_t n, unsigned *count, hipStream_t s);
// g[e] = gacc[e] / n_p for one style layer (the Sec. 3.1 normalization)
hipError_t launch_gram_normalize(const double *gacc, double *g, size_t n, double n_p,
                                 hipStream_t s);

struct StyleTermsArgs {
  int n_style;
  int C[8];
  long long off[8];            // element offset of layer l in the concatenated Gram arrays
  long long dt_off[8];         // element offset of layer l in the packed residual operand
  double w[8];
  double inv_np[8];
  // augmented style loss (Eq. 5), when mx != nullptr
  const double *mx, *mt;       // channel means of x and of the style image, concatenated
  long long moff[8];           // offset of layer l in the concatenated means
  double w1[8], w2[8];         // w'_l (mean) and w''_l (std)
  float *msb;                  // out: per-channel constant of the mean/std seeds
};
// Energy terms w_l ||G_l - Ghat_l||^2 into e_style[l] and the packed residual operand
// (2 w_l / n_p)(D + D^T) in compute precision.
hipError_t launch_style_terms(int precision, const double *g, const double *gt,
                              const StyleTermsArgs &a, void *dt, double *e_style, hipStream_t s);
// energy[0] = alpha * ec + sum e_style; energy[1] = alpha * ec; energy[2 + l] = e_style[l]
hipError_t launch_energy_total(const double *ec, const double *e_style, int n_style,
                               double alpha, double *energy, hipStream_t s);

// Device scratch of the allocation-free entry point: a static device array of kScratchBytes.
constexpr size_t kScratchBytes = (size_t)256 << 20;
// Look up (once per device; that device must be current) the address of the device's copy.
hipError_t scratch_init(int device);
// The address scratch_init stored for `device`, or nullptr.
void *scratch_ptr(int device);

}  // namespace nst
