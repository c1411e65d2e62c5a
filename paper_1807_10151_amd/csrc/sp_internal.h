// Internal declarations of libsuppcg: device-side structs, kernel launchers
// and the canonical chord-weight evaluation shared by the projector and the
// backprojector.  Not part of the public ABI (see include/suppcg.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/suppcg.h"

namespace sp {

// Zero columns kept on each side of every padded image row and sinogram row.
// Candidate indices are clamped into [-PAD, len + PAD) and the pad holds
// zeros, so a clamped candidate contributes exactly 0.
constexpr int PAD = 4;
constexpr int BLOCK = 256;

// Per-angle constants, in pixel units (coordinates divided by the pixel size).
// The chord weight is evaluated in float64 from float64 cos/sin: rounding the
// angle to float32 alone would move a ray by ~1e-5 pixel at radius 256.
struct alignas(16) AngleDev {
    double c, s;      // cos(theta), sin(theta)
    double einv;      // e * inv with e = (|c| + |s|) / 2
    double inv;       // 1 / min(|c|, |s|)   (0 for axis-parallel angles)
    double wmax;      // 1 / max(|c|, |s|): the largest chord, the factor of u
    double slope;     // forward walk: minor index per major step
    double kb;        // backprojection: -s0/ds - hb + 1 + PAD, hb = e/ds + margin (selection only)
    double dc;        // backprojection: ds (1 - hb), the offset s_k - t of a pixel's first
                      // candidate bin when its window index kf is an integer
    double cids, sids;  // backprojection: c / ds and s / ds (oblique window index)
    float hw;         // forward walk: half-width of the nonzero band on the minor axis + margin
    int32_t row;      // sinogram row of this angle (the table is sorted by class)
    int32_t flags;    // bit0 axis-parallel, bit1 walk columns (|s| > |c|)
    int32_t nc;       // forward candidates per major step
    int32_t nb;       // backprojection candidate bins
    int32_t pad_;
};
constexpr int ANG_AXIS = 1;
constexpr int ANG_HORIZ = 2;

struct GeomDev {
    int rows, cols, nA, nB;
    double xoff, yoff;  // (cols-1)/2, (rows-1)/2
    double ds, s0;      // bin spacing and position of bin 0, pixel units
    double inv_ds;
    double pixel;       // weights are in pixel units; outputs are scaled by this
    int pitchX;         // cols + 2 PAD: row pitch of the padded image copy
    int pitchXT;        // rows + 2 PAD: row pitch of the padded transposed copy
    int pitchB;         // nB + 2 PAD: row pitch of the padded sinogram
    int nbmax;          // max backprojection candidates over the angles
    int parts;          // parts each ray's step range is split into by R (1: whole rays)
    int bp_px;          // pixels per lane of R^T (2 or 4, see backproject_px)
    int cls[5];         // angle-table class boundaries: vertical, horizontal,
                        // vertical axis, horizontal axis
    int nwaves;         // waves of R's wave table (see WaveDev)
    int nwg;            // R's ray workgroups, four waves each: ceil(nwaves / 4)
};

// One wave of R: 64 rays, one per lane, of one angle class.  Kinds (`tail`):
//  WAVE_BLOCK: WAVE_ANGLES consecutive angles by WAVE_BINS consecutive bins:
//    lane l takes angle a0 + l / WAVE_BINS and bin k0 + l % WAVE_BINS, while
//    that angle lies before aend (a wave of 64 consecutive bins of one angle
//    would walk the union of rays whose image extents differ more);
//  WAVE_TAIL: the last r = nB % WAVE_BINS bins of consecutive angles of one
//    class, packed: the class's tail rays, angle by angle, form a stream, and
//    lane l takes its entry k0 + l, i.e. angle a0 + (k0 + l) / r and bin
//    nB - r + (k0 + l) % r, while that angle lies before aend;
//  WAVE_ROW: 64 consecutive bins of one angle (lane l: angle a0, bin k0 + l),
//    for the axis-parallel classes (one or two angles).
// Angles are indices of the class-sorted table.
constexpr int WAVE_BINS = 16;
constexpr int WAVE_ANGLES = 4;
enum WaveKind : int32_t { WAVE_BLOCK = 0, WAVE_TAIL = 1, WAVE_ROW = 2 };
struct WaveDev {
    int32_t a0, k0, aend, tail;
};

// Device-resident solver state.  Written only by single-workgroup kernels
// (scalar, decide), read by every solver kernel.
struct Scalars {
    double f;         // f of the last residual computed
    double pth;       // p^T h of the carried (p, h)
    double beta;
    double alpha;
    double lam;       // accepted S_TV step divided by ||t_bar||
    double tv_new;    // TV of the accepted trial
    double eps;
    double a, gamma;  // S_TV parameters
    double f0;        // f(x_0)
    double alpha0;    // alpha of the initial step
    int32_t ell;      // l of Algorithm 1
    int32_t k;        // k of Algorithm 3
    int32_t halt;     // 0: running; else the SP_* status that stopped the run
    int32_t exhausted;
    int32_t iter;     // index of the current loop body
    int32_t inner;    // index of the current S_TV inner step
    int32_t K;
    int32_t max_trials;
    int32_t max_iter;
    int32_t replay;   // 1: accept after replay[iter*K+inner] trials
    int32_t first;    // 1 while computing the initial direction (beta = 0)
    int32_t gate_learned;   // 1: the learned preconditioner runs
    int32_t gate_ramp;      // 1: the Fourier preconditioner runs (fallback)
    int32_t fallbacks;      // loop bodies in which the learned M was rejected
    int32_t pad_;
};

struct TraceDev {
    double* f_half;
    double* tv_half;
    double* alpha;
    double* beta;
    double* s_norm;
    int32_t* ell;
    int32_t* trials;
    const int32_t* replay;
    int32_t cap;
};

// Scalar steps a kernel runs in its workgroup (0, 0) after its own work, in
// place of separate single-workgroup launches: the S_TV step norm from the
// partials ps (when ps != nullptr), then f from the partials pf (when
// pf != nullptr).  Inactive when sc == nullptr.
struct ScalarRide {
    Scalars* sc = nullptr;
    TraceDev tr{};
    const double* pf = nullptr;
    int nf = 0;
    const double* ps = nullptr;
    int ns = 0;
};

// Canonical evaluation of the weight of pixel centre (xj, yi) for ray sk: the
// backprojector's weight for every angle and the projector's for
// axis-parallel angles (oblique rays are split band by band, see ray_split,
// which gives the same lengths to rounding).  Projection of the pixel centre
// on the ray normal:
//   |c| >= |s|:  t = fma(xj, c, yi * s)      |s| > |c|:  t = fma(yi, s, xj * c)
// (the product outside the fma is the one a forward walk shares between
// candidates); offset d = sk - t.  The chord length through the pixel is
// w = wmax * u with the normalised trapezoid
//   u = clamp((e - |d|) / min(|c|, |s|), 0, 1) = clamp(fma(-|d|, inv, einv), 0, 1),
// which compiles to one float64 fma with the output clamp; the per-angle
// factor wmax is applied once to a sum over u-weighted values.  For
// axis-parallel angles wmax = 1 and u is 1 inside the pixel's column, 1/2 on
// its edge and 0 outside.
template <bool AXIS>
__host__ __device__ inline double chord_u(double d, double einv, double inv) {
    const double ad = fabs(d);
    if (AXIS) return ad < 0.5 ? 1.0 : (ad == 0.5 ? 0.5 : 0.0);
    return fmin(fmax(fma(-ad, inv, einv), 0.0), 1.0);
}

__host__ __device__ inline double bin_pos(double k, const GeomDev& G) { return fma(k, G.ds, G.s0); }

// ---- allocation-free entry point (noalloc.hip) ---------------------------------
// Bytes of the static per-GPU scratch array and the largest angle count the
// allocation-free backprojection accepts (its host staging is sized for it).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(32) << 20;
constexpr int NOALLOC_MAX_ANGLES = 8192;
// Device address of the scratch array on `device` (looked up once per device,
// with that device current); the result of that lookup.
hipError_t noalloc_scratch(int device, void** ptr);

// ---- kernel launchers (all enqueue on `st`) ----------------------------------
// projector.hip
// The padded copies of the image (xp, xTp) are float64 widenings of the
// float32 image or of the solvers' float64 vectors: the forward gathers then
// feed the float64 FMAs without a conversion per candidate.  The padded
// sinogram of R p (yp) is float32, that of the residual float64.
void launch_prep(hipStream_t st, const GeomDev& G, const float* x, double* xp, double* xTp,
                 const int* halt);
void launch_prep(hipStream_t st, const GeomDev& G, const double* x, double* xp, double* xTp,
                 const int* halt);
// With G.parts > 1, seg (parts * nA * nB float64) receives the per-part sums
// before they are combined.  outp / outpd: float32 / float64 padded sinograms
// (nullable); the residual's float64 values feed R^T without a float32
// rounding (its cancellation in R^T r amplifies that rounding).  waves: the
// device copy of R's wave table (project_waves); ord: the device copy of
// project_order(G, ...), the ray workgroup each launched workgroup runs.
// With dq (nA x nB float64, b == nullptr) the partials are those of
// (R x)^T dq, and wout (nA x nB float64, nullable) receives R x unrounded.
void launch_project(hipStream_t st, const GeomDev& G, const AngleDev* ang, const WaveDev* waves,
                    const double* xp, const double* xTp, const float* b, float* out, int out_pitch,
                    float* outp, double* outpd, double* partials, double* seg, const int* ord,
                    const int* halt, const double* dq = nullptr, double* wout = nullptr);
// Padded copy of y for R^T with each row scaled by its angle's wmax.
void launch_pad_sino(hipStream_t st, const GeomDev& G, const AngleDev* ang, const float* y,
                     float* yp);
// ride: scalar steps workgroup (0, 0) runs after its tile (see ScalarRide).
void launch_backproject(hipStream_t st, const GeomDev& G, const AngleDev* ang, const float* yp,
                        float* out, const double* dotv, double* partials, const int* halt,
                        const ScalarRide& ride = ScalarRide{});
void launch_backproject(hipStream_t st, const GeomDev& G, const AngleDev* ang, const double* yp,
                        float* out, const double* dotv, double* partials, const int* halt,
                        const ScalarRide& ride = ScalarRide{});

// R^T's workgroup: a tile of BP_TILE rows by 8 PX columns, BP_SPLIT waves each
// over a share of the angles; dot-product partials per BP_TILE x BP_TW sub-tile.
constexpr int BP_TILE = 8;
constexpr int BP_TW = 16;
constexpr int BP_SPLIT = 4;

// ---- host geometry (geometry.cpp) ------------------------------------------------
// cos/sin of angle index a, exact at multiples of pi/4.
void angle_cos_sin(const sp_geometry& g, int a, double& co, double& si);
// Chord and selection constants of angle a.
AngleDev angle_entry(const sp_geometry& g, int a, double ds, double s0, double margin);
// 0 vertical oblique, 1 horizontal oblique, 2 vertical axis, 3 horizontal axis.
int angle_class(const AngleDev& A);
// Device geometry and the class-sorted angle table (n_angles entries written
// to tab) of a validated geometry, for a device of n_cu compute units;
// allocates nothing.  SP_ERR_ARG with a message in err for geometries the
// kernels do not support.
int build_geometry_into(const sp_geometry* g, int n_cu, GeomDev& G, AngleDev* tab, char* err,
                        size_t errlen);
// Bin positions of the padded bin range: t[PAD + k] = s_k, k = -PAD .. nB + PAD - 1.
void bin_sk_fill(const GeomDev& G, double* t);
// R's wave table: its size and its entries (G.nwaves of them; see WaveDev):
// the oblique classes' four-angle by 16-bin blocks, 64-bin chunk by chunk,
// then their packed tail waves, then the axis-parallel classes' 64-bin waves.
int project_wave_count(const GeomDev& G);
// Writes the entries when out != nullptr; returns their number.
int project_waves(const GeomDev& G, WaveDev* out);
// Steps a wave of R walks: the union of its lanes' nonempty step ranges.
long wave_steps(const GeomDev& G, const AngleDev* tab, const WaveDev& W);
// Dispatch order of R's ray workgroups (G.nwg entries, a permutation):
// workgroups by decreasing step count, with every other band of n_cu entries
// reversed so the first workgroups of each compute unit sum to about the same
// work.  Only the order of the work changes; every sum and its partials index
// stay the same.
std::vector<int32_t> project_order(const GeomDev& G, const AngleDev* tab, const WaveDev* waves,
                                   int n_cu);
// Parts R splits each ray's step range into, chosen from the geometry and the
// device's wave slots (both the single-slice and the batched solver use it,
// so their sums agree).
int project_parts(int rows, int cols, int nwaves, int resident_waves);
// Combine workgroups (G.parts > 1): one angle by one 256-bin chunk each.
int project_comb_blocks(const GeomDev& G);
// Number of float64 f partials R's residual form writes: one per combine
// workgroup when the rays are split in parts, else one per ray workgroup.
int project_blocks(const GeomDev& G);
// Number of R^T's float64 dot partials: one per 8 x 16 pixel sub-tile.
// R^T workgroups (8 x 8 px pixel tiles) for px pixels per lane.
int backproject_tiles(const GeomDev& G, int px);
// Pixels per lane R^T uses for an image: 4 when that grid still fills half
// the device's wave slots, else 2.  The result does not depend on it.
int backproject_px(int rows, int cols, int resident_waves);

// fft.hip
struct FFTPlan {
    int P, logP, SP, rows, cols, CB;
    double2* S;           // [rows][SP] complex float64 scratch
    const double2* tw;    // [P/2] twiddles exp(-2 pi i k / P)
};
// With G, z is also written to R's padded copies xp / xTp of geometry G (as
// launch_prep of z would write them).
void launch_precond(hipStream_t st, const FFTPlan& F, double mu, double rho, const float* g,
                    float* z, const float* dotv, double* partials, const int* halt,
                    const int* run = nullptr, const GeomDev* G = nullptr, double* xp = nullptr,
                    double* xTp = nullptr);
int precond_dot_blocks(const FFTPlan& F);
// Dynamic LDS of an FFT workgroup holding ncol length-P transforms (plus the
// twiddle table when it fits).
size_t fft_lds_bytes(int P, int ncol);

// tv.hip (images y, x_{k+1/2} and x_k in float64; t_bar float32)
// t_bar and its ||.||^2 partials: tv_blocks of them for an S_TV call's first
// inner step (later = false), tv_grad_blocks for later ones.
void launch_tv_grad(hipStream_t st, int rows, int cols, const double* y, float* tb, double* partials,
                    const int* halt, bool later = false);
int tv_blocks(int rows, int cols);
// Workgroups (and partials) of the t_bar launches after an S_TV call's first
// inner step (k_tv_grad with later, k_tv_apply_grad: the ||t_bar||^2 partials)
// and of the trials launch (the trial partials).
int tv_grad_blocks(int rows, int cols);
int tv_tpx_blocks(int rows, int cols);
void launch_tv_trials(hipStream_t st, int rows, int cols, const double* y, const float* tb,
                      const double* gpart, int ngpart, Scalars* sc, int J, double* tpart,
                      const int* halt);
void launch_tv_decide(hipStream_t st, int rows, int cols, const double* y, const float* tb,
                      const double* gpart, int ngpart, const double* tpart, int ntpart, int J,
                      Scalars* sc, TraceDev tr, int32_t* trials_out, const int* halt);
void launch_tv_apply(hipStream_t st, int n, const double* src, double* dst, const float* tb,
                     const Scalars* sc, const double* xk, double* partials, const int* halt);
void launch_tv_value(hipStream_t st, int rows, int cols, const double* y, double* partials,
                     const int* halt);
// dst = src + lam tb_in, then tb_out = t_bar(dst) and its ||.||^2 partials
// (k_tv_apply followed by k_tv_grad, bit for bit); no overlap between dst and
// src or between tb_out and tb_in.
// The last update with R's padded copies of dst (prep's xp, xTp layout):
// dst = src + lam tb, or dst = src with tb == nullptr; with xk the partials of
// ||dst - xk||^2, one per 32 x 32 tile (tv_prep_tiles of them).
int tv_prep_tiles(int rows, int cols);
void launch_tv_apply_prep(hipStream_t st, const GeomDev& G, const double* src, double* dst,
                          const float* tb, const Scalars* sc, const double* xk, double* partials,
                          double* xp, double* xTp, const int* halt);
void launch_tv_apply_grad(hipStream_t st, int rows, int cols, const double* src, double* dst,
                          const float* tb_in, float* tb_out, const Scalars* sc, double* partials,
                          const int* halt);

// cg.hip (p, x and x_{k+1/2} in float64; g, z, h float32)
int vec_blocks(int n);
void launch_dot(hipStream_t st, int n, const float* a, const float* b, double* partials,
                const int* halt);
// Forms with the beta / alpha scalar step folded in (ops OP_BETA, OP_ALPHA or
// OP_ALPHA0 of launch_scalar): one launch instead of two, same values.
// p <- -z + beta p (partials of g^T p) and q <- -w + beta q over the m rays
// (partials of q^T q, vec_blocks(m) of them), with the beta step (OP_BETA,
// (R z)^T q from the ndot partials pdot) folded in; pq_blocks(n, m) workgroups.
int pq_blocks(int n, int m);
void launch_update_pq_beta(hipStream_t st, int n, int m, const float* z, double* p, const float* g,
                           const double* w, double* q, Scalars* sc, TraceDev tr, const double* pdot,
                           int ndot, double* pgp, double* pqq);
void launch_update_x_alpha(hipStream_t st, int n, const double* xh, const double* p, double* x,
                           Scalars* sc, TraceDev tr, const double* pph, int nph, const double* pgp,
                           int ngp, int op);
void launch_copy(hipStream_t st, int n, const float* src, float* dst, const int* halt);
void launch_copy(hipStream_t st, int n, const double* src, double* dst, const int* halt);
// dst = src widened to float64 (src == nullptr: zeros); dst = src rounded to float32
void launch_widen(hipStream_t st, int n, const float* src, double* dst);
void launch_narrow(hipStream_t st, int n, const double* src, float* dst);
void launch_snap(hipStream_t st, int n, const float* src, float* dst, int count, const Scalars* sc);
void launch_reduce(hipStream_t st, const double* partials, int np, double* out);
// x = xh if the run stopped on a breakdown after its initial step; *k_out = k
// (nullable): the end of a solve that does not return to the host.
void launch_finish(hipStream_t st, int n, const double* xh, double* x, const Scalars* sc,
                   int32_t* k_out);

// quality.hip (selective error, Section 4.2): partials hold 2 * vec_blocks(n)
// doubles.  First form: SE of a float32 image to *dst.  Second form: SE of the
// float64 iterate to dst_body[sc->iter - 1] (when dst_body is set and that
// entry is below cap) or to *dst; nothing when *halt is set.
void launch_se(hipStream_t st, int rows, int cols, double pixel, double ah, double av,
               const float* x, const float* ref, double C, double* partials, double* dst);
void launch_se(hipStream_t st, int rows, int cols, double pixel, double ah, double av,
               const double* x, const float* ref, double C, double* partials, double* dst,
               double* dst_body, int cap, const Scalars* sc, const int* halt);

// stored.hip (R and R^T as sliced ELLPACK, 64 rows a slice).  Rows come in
// nseg segments of lseg rows (R: angles of nB rays; R^T: image rows of cols
// pixels), each split into spseg = ceil(lseg / 64) slices.  nat: the angle
// table in natural order.  count: nonzeros per row (pixels: R^T's rows, else
// R's) into len; slice sizes: size[s] = 128 * the longest row of slice s
// rounded up to a multiple of 4 (words: column indices and weights); scan:
// out[0] = 0, out[r + 1] = cnt[0] + ... + cnt[r] (sums: scan_blocks(n) int64
// of scratch); fill: the entries of every row at its slice offset sp in ent
// (placement of sp_stored.h; R's near-horizontal rays with transposed pixel
// indices).
struct SellShape {
    int64_t nseg, lseg, spseg;
};
int scan_blocks(int64_t n);
void launch_scan(hipStream_t st, const int32_t* cnt, int64_t n, int64_t* out, int64_t* sums);
void launch_stored_count(hipStream_t st, const GeomDev& G, const AngleDev* nat, bool pixels,
                         int32_t* len);
void launch_slice_sizes(hipStream_t st, const int32_t* len, const SellShape& S, int32_t* size);
void launch_stored_fill(hipStream_t st, const GeomDev& G, const SellShape& S, const AngleDev* nat,
                        bool pixels, const int64_t* sp, const int32_t* len, int32_t* ent);
// y[r] = sum over row r of val * x[col] (float64 sum in a fixed order); the
// segments with segT[seg] = 1 gather from xT (segT nullable: none)
void launch_sell_spmv(hipStream_t st, const SellShape& S, const int64_t* sp, const int32_t* len,
                      const int32_t* ent, const float* x, const float* xT, const uint8_t* segT, float* y);
// xT = x transposed (x: rows x cols)
void launch_transpose(hipStream_t st, int rows, int cols, const float* x, float* xT);

// art.hip (ART / SupART / BlobART, Section 3.4).  Blob basis: generalised
// Kaiser-Bessel blobs (order 2, alpha 10.4, radius 2 pixels) on the pixel
// centres; cproj = a sqrt(2 pi / alpha) / I_2(alpha) scales the projection;
// stencil[di + 2][dj + 2] = b(|(di, dj)|), the image of a unit coefficient;
// tab: the device copy of the projection's table (sp_blob.h: ntab + 1
// entries over [0, a], inv_h = ntab / a), set by the caller.
constexpr double BLOB_RADIUS = 2.0;
constexpr double BLOB_ALPHA = 10.4;
struct BlobDev {
    double a, alpha, cproj;
    double stencil[5][5];
    const double2* tab;
    int ntab;
    double inv_h;
};
BlobDev blob_constants();
// norms: ||R_i||^2 of every ray (blob nullable: pixel basis); init: x = mu /
// divisor (or x0 when given), u = 0 (partials: vec_blocks(m) doubles, sum_b:
// one double); sweep: one cycle through the rays, angle by angle and phase
// by phase (nat_h: the HOST angle table in natural order), skipped when
// *halt is set; synth: img = the blob image of the coefficients c.
void launch_art_norms(hipStream_t st, const GeomDev& G, const AngleDev* nat, const BlobDev* blob, double* nrm2);
void launch_art_init(hipStream_t st, const GeomDev& G, const float* b, const float* x0, double divisor,
                     double* partials, double* sum_b, double* x, double* u);
void launch_art_sweep(hipStream_t st, const GeomDev& G, const AngleDev* nat_h, const BlobDev* blob,
                      const double* nrm2, const float* b, double* x, double* u, double r, double lam,
                      const int* halt);
void launch_blob_synth(hipStream_t st, int rows, int cols, const BlobDev& B, const double* c, double* img,
                       const int* halt);

// learned.hip (learned preconditioner C^T diag(softplus(d)) C)
void lp_conv_mid(hipStream_t st, bool trans, int B, int H, int W, const float* in, float* out,
                 const float* Wl, const float* scale, float* out2, const int* halt, const int* run);
void lp_conv_in(hipStream_t st, int B, int H, int W, const float* in, const int32_t* idx, int nsrc,
                float* out, const float* W1, const int* halt, const int* run);
void lp_conv_out(hipStream_t st, int B, int H, int W, const float* in, float* out, const float* W1,
                 const int* halt, const int* run);
void lp_gather(hipStream_t st, int B, int HW, const float* src, const int32_t* idx, int nsrc, float* dst);
void lp_scale(hipStream_t st, long npix, const float* in, const float* scale, float* out);
void lp_softplus(hipStream_t st, const float* d, float* sp_out, float* sg_out);
void lp_loss(hipStream_t st, int B, int H, int W, int margin, const float* z, const float* v,
             const int32_t* idx, int nsrc, float* e0, double* lpart);
int lp_wgrad_blocks(int B, int H, int W);
void lp_wgrad(hipStream_t st, int fi, int B, int H, int W, const float* G, const float* X, float* partial);
int lp_reduce_chunks(int nb);
void lp_reduce(hipStream_t st, int nb, int nout, const float* pa, bool accumulate, float* out,
               double* tmp);
int lp_gd_blocks();
void lp_gd(hipStream_t st, long npix, const float* E, const float* A, double* part, const float* sg,
           float* gd);
void lp_adam(hipStream_t st, int n, float* theta, float* m, float* v, const float* g, double lr,
             double b1, double b2, double eps, int step);

// ---- batched solve: many slices advance through one launch per stage --------
// Every stage kernel has a batched form that walks a table of work items
// (slice << ITEM_SHIFT | linear virtual block) with a grid-stride loop: a grid
// of one workgroup per item is the flat form, a smaller grid the persistent
// form.  A slice's virtual block runs the same body, with the same partial
// indices, as the single-slice launch, so results are bitwise identical.
constexpr int ITEM_SHIFT = 20;
constexpr uint32_t ITEM_MASK = (1u << ITEM_SHIFT) - 1u;
constexpr int MAX_BATCH = 4096;

struct SliceDev {
    GeomDev G;
    FFTPlan F;
    const AngleDev* ang;
    const WaveDev* pwave;   // R's wave table
    const float* b;
    const float* x0;   // nullable: zero start
    double *xh, *x, *p;  // iterate, x_{k+1/2} and search direction (float64)
    float *g, *z, *tb;
    double *q, *w;      // R p and R z, nA x nB (float64)
    double *xp, *xTp;   // float64 padded copies
    double* rpd;        // float64 padded sinogram (residual)
    double* seg;        // R's per-part ray sums, [parts][nA][nB] (G.parts > 1)
    const int* pord;    // R's ray-workgroup order (project_order)
    double *pf, *pgp, *pqq, *ptg, *ptt, *pts;   // pf: f, then (R z)^T q
    Scalars* sc;
    TraceDev tr;
    int n, m, nf, ngp, nqq, ntv, ntg, ntt, nsn;   // m = nA nB rays; ntg / ntt: t_bar / trial partials; nsn: ||s_k|| tiles
};

// Stage selectors of the batched kernels.
enum BatchVec : int { BV_XH = 0, BV_X = 1, BV_P = 2, BV_Z = 3 };   // BV_Z: the float32 z
enum BatchStage : int {
    BS_PREP = 0, BS_PROJECT, BS_BACKPROJECT, BS_ROWS, BS_COLS, BS_TV, BS_VEC, BS_SLICE, BS_PROJ_COMB,
    BS_PQ, BS_TVT, BS_TVG, BS_COUNT
};
struct ItemTable {
    const uint32_t* items;
    int n;
    int grid;   // workgroups launched: n (flat) or fewer (persistent)
};

// Runs fn(slice, virtual block) for the items of this workgroup; the barrier
// after each item keeps LDS reuse ordered.  ITEM_NONE entries pad the queues
// of the XCD-grouped order and are skipped.
constexpr uint32_t ITEM_NONE = 0xFFFFFFFFu;
template <class Fn>
__device__ __forceinline__ void for_items(const ItemTable& t, Fn&& fn) {
    for (int w = blockIdx.x; w < t.n; w += gridDim.x) {
        const uint32_t it = t.items[w];
        if (it != ITEM_NONE) fn((int)(it >> ITEM_SHIFT), (int)(it & ITEM_MASK));
        __syncthreads();
    }
}

// Pointers read from a slice descriptor are generic (flat) to the compiler,
// which would access them with flat instructions.  gmem re-types one as global
// memory; cmem re-types a table that no kernel writes as constant memory, so
// that wave-uniform reads of it become scalar loads.
template <class T>
__device__ __forceinline__ T* gmem(T* p) {
    return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}
template <class T>
__device__ __forceinline__ const T* cmem(const T* p) {
    return (const T*)(__attribute__((address_space(4))) const T*)(uintptr_t)p;
}

__device__ __forceinline__ double* batch_vec(const SliceDev& S, int which) {
    return gmem(which == BV_XH ? S.xh : (which == BV_X ? S.x : S.p));
}

// projector.hip
void launch_prep_b(hipStream_t st, const SliceDev* sl, ItemTable t, int which);
// residual: rpd = R xh - b with the f partials in pf; else w = R z (from the
// prepared z) with the (R z)^T q partials in pf.
void launch_project_b(hipStream_t st, const SliceDev* sl, ItemTable t, ItemTable tc, bool residual);
// px: pixels per lane of every slice in the launch (their G.bp_px).
void launch_backproject_b(hipStream_t st, const SliceDev* sl, ItemTable t, int nbmax, int px);
// fft.hip (z = M g)
void launch_precond_b(hipStream_t st, const SliceDev* sl, ItemTable rows, ItemTable cols,
                      size_t lds_rows, size_t lds_cols, double mu, double rho);
// tv.hip
void launch_tv_grad_b(hipStream_t st, const SliceDev* sl, ItemTable t, int src);
void launch_tv_trials_b(hipStream_t st, const SliceDev* sl, ItemTable t, int src);
void launch_tv_decide_b(hipStream_t st, const SliceDev* sl, ItemTable t, int src);
void launch_tv_apply_b(hipStream_t st, const SliceDev* sl, ItemTable t, int src, bool snorm);
// BS_PREP items: x_{k+1/2} with R's padded copies (see launch_tv_apply_prep).
void launch_tv_apply_prep_b(hipStream_t st, const SliceDev* sl, ItemTable t, int src, bool copy,
                            bool snorm);
// cg.hip
void launch_init_b(hipStream_t st, const SliceDev* sl, ItemTable t);   // xh = x = x0 (or 0)
void launch_update_pq_b(hipStream_t st, const SliceDev* sl, ItemTable t);   // BS_PQ items
void launch_update_x_b(hipStream_t st, const SliceDev* sl, ItemTable t);
void launch_copy_gz_b(hipStream_t st, const SliceDev* sl, ItemTable t);   // M = I: z = g
void launch_scalar_b(hipStream_t st, const SliceDev* sl, ItemTable t, int op);

enum ScalarOp : int {
    OP_F = 0,        // f = sum(pa); trace / non-finite check
    OP_F0 = 1,       // f(x_0) at initialisation
    OP_BETA = 2,     // beta = sum(pa) / pth (0 on the first direction)
    OP_ALPHA = 3,    // pth = sum(pa); alpha = -sum(pb) / pth; k++, iter++
    OP_ALPHA0 = 4,   // same for the initial step (k = 1)
    OP_SNORM = 5,    // ||s_k|| into the trace
    OP_LCHECK = 6,   // learned M accepted iff g^T z = sum(pa) > 0 and finite; else fall back
    OP_EPS = 7,      // Algorithm 3's loop test at the top of a body: halt if f <= eps (eps > 0)
    OP_NEXT = 8,     // ART / SupART: the body has formed its iterate; k++, iter++
};
void launch_scalar(hipStream_t st, int op, Scalars* sc, TraceDev tr, const double* pa, int na,
                   const double* pb, int nb);

}  // namespace sp
