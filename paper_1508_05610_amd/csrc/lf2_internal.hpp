// lf2_internal.hpp -- argument blocks and launch entry points shared by the
// host plan code and the kernel translation units (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lf2_batch_items.hpp"
#include "lf2_gen.hpp"

namespace lf2 {

constexpr int kMaxBins = 4096;  // LDS histogram limit of the fused binning epilogue

// Epilogue of a strided pass (applies to the last axis, k space, ncomp = 1).
enum : int {
    EPI_STORE = 1,    // write the transformed column back
    EPI_PK = 2,       // accumulate w|F|^2 per bin after the forward transform
    EPI_POISSON = 4,  // scale by -1/(N k^2) (FP64) and run the backward transform
    EPI_PK_AFTER = 8, // accumulate after the Poisson scale instead (spectrum of phi)
    EPI_TSTORE = 16,  // store in the c2c (k_z, k_x, k_y) order (k_strided_t)
    EPI_TLOAD = 32    // load from the c2c (k_z, k_x, k_y) order (k_strided_t)
};

// Description of mode (kx, ky, kz) -> tables, for the fused epilogues.
struct ModeTables {
    int nxk;               // k-space extent of dimension 0 (Nh or N0)
    int n0;                // real-space N0 (weight rule)
    int n1;                // N1
    int half;              // 1: r2c half spectrum weights, 0: c2c
    const double *k2[3];   // per-axis k^2 contributions (FP64), NULL if unused
    const int64_t *q[3];   // per-axis integer (nt L / N)^2
    const int64_t *thresh; // nbins + 1 bin thresholds: smallest q of bin b
    int nbins;
    double qmax;
    double scale_n;        // Poisson: factor 1/N applied with -1/k^2
    uint32_t qz_unit;      // (lcm / N2)^2: q[2][i] = qz_unit * min(i, N2 - i)^2
    uint32_t qx_unit, qy_unit;  // the same for dimensions 0 and 1
    int walk1;             // 1: one step of |n_z| never crosses two bin thresholds
    double k2z_unit;       // continuous k^2: (2 pi / (N2 dx))^2, so k2[2][i] =
                           // k2z_unit * min(i, N2 - i)^2; 0: read k2[2]
    double k2x_unit, k2y_unit;  // the same for dimensions 0 and 1 (when k2z_unit > 0)
};

struct XArgs {
    const void *in;
    void *out;
    int64_t nrows;        // N1 * N2
    int n1;               // rows per plane
    // element offsets: base(y, z) = off + z * plane + y * row (units of the
    // array's element: float for real arrays, complex for complex arrays)
    int64_t in_off, in_row, in_plane;
    int64_t out_off, out_row, out_plane;
    const void *tw;       // FFT twiddles, length L (forward sign)
    const void *tw_post;  // r2c/c2r: exp(-2 pi i k / N0), k = 0..N0/2
    double *sumsq;        // optional per-block FP64 sum of squares of the real input
                          // ([gridDim.x], r2c forward only)
};

struct SArgs {
    const void *in;
    void *out;
    int64_t stride;      // elements between points of a column
    int64_t ncols_inner; // C
    int64_t outer;       // elements between outer column groups
    int64_t ncols;       // total columns (O * C)
    int epi;             // EPI_* flags
    int xcd_chunk;       // tiles per XCD chunk (set by the launcher)
    int hcopies;         // binning: LDS histograms per block, 1 (all waves add into
                         // one) or one per wave (fixed-order sums: reproducible)
    const void *tw;      // twiddles, length L
    ModeTables mt;
    double *partial;     // [gridDim.x][nbins + 1]
    // the transposed side of k_strided_t: column f = (y, x, c) of the
    // natural order, point z, sits at ((y n0 + x) n2 + z) nc + c
    int64_t t_n0, t_n2, t_nc;
};

// Kernel launchers (return hipSuccess or the launch error).  `len` is the
// transform length along the pass axis; nc the number of components.
bool x_supported(int len, int nc);
bool s_supported(int len);
hipError_t launch_x_r2c(int m, int nc, const XArgs &a, hipStream_t s);
hipError_t launch_x_c2r(int m, int nc, const XArgs &a, hipStream_t s);
hipError_t launch_x_c2c(int len, int nc, int sign, const XArgs &a, hipStream_t s);
// c2c x pass of 64-point one-component rows with the stage exchange across
// lanes (eight lanes per row) instead of LDS: DPP moves (dpp) or
// ds_bpermute.
hipError_t launch_x_c2c_shfl(int sign, bool dpp, const XArgs &a, hipStream_t s);
// variant bit 0: STileW (wide tiles, plain passes of s_wide_supported
// lengths) instead of STile (narrow, any pass); bit 2: the register tile
// (k_strided_r: 32 x Q decomposition, plain passes of s_reg_supported
// lengths; not with bit 0); bit 1: nontemporal global loads and stores
// (plain passes).  EPI_TSTORE / EPI_TLOAD in a.epi select
// STileT (z pass to / from the paper's c2c k-space order) whatever the
// variant.  chunk: consecutive tiles per XCD in the tile
// order (16 by default).
hipError_t launch_strided(int len, int sign, const SArgs &a, int grid_cap, hipStream_t s,
                          int *grid_used, int variant = 0, int chunk = 16);
bool s_wide_supported(int len);
bool s_reg_supported(int len);
// The fused Poisson pass (EPI_POISSON, any P(k) flags) with the tile in
// registers (k_fused_r): 512-point lines.  launch_strided selects it with
// variant bit 3 on such passes.
bool fused_reg_supported(int len);
// Whether that tile's LDS holds the binning tables of nbins bins (0: no
// binning) beside it; where it does not, the LDS-staged tile runs.
bool fused_reg_fits(int len, int nbins);
hipError_t launch_fused_reg(int len, const SArgs &a, size_t shm, int grid_cap, hipStream_t s,
                            int *grid_used);
hipError_t launch_strided_reg(int len, int sign, const SArgs &a, int grid_cap, hipStream_t s,
                              int *grid_used, int chunk, bool ntm);
// LDS histogram copies of a fused last-axis tile of length len binning into
// nbins bins, when the block's LDS is `budget` bytes: one per wave if they
// fit with the tile, else one.  0 if len has no compiled fused tile.
int epi_hist_copies(int len, int nbins, size_t budget);

// Run-time-schedule kernels (lf2_kgen.hip): LDS bytes of an x tile of RB
// rows and of a strided tile of B columns (nbins > 0: with the binning
// tables), and their launchers.  mode 0: c2c with `sign`, 1: r2c forward,
// 2: c2r backward.
size_t gx_lds_bytes(int M, int NC, int RB);
size_t gs_lds_bytes(int L, int B, int nbins);
hipError_t launch_gx(int mode, int sign, const XArgs &a, const GSched &sc, int m, int nc, int rb,
                     hipStream_t s);
hipError_t launch_gs(int sign, const SArgs &a, const GSched &sc, int len, int b, int grid_cap,
                     hipStream_t s, int *grid_used);

// Field operations (lf2_kfield.hip).
hipError_t launch_update_halo(void *field, const int64_t n[3], int64_t h, int64_t site_words,
                              hipStream_t s);
hipError_t launch_gradient(const float *in, float *out, const int64_t n[3], int64_t h, int nc,
                           double dx, hipStream_t s);

// Setup and reduction kernels (FP64).
hipError_t launch_twiddles(void *tw, int len, hipStream_t s);
hipError_t launch_k2_table(double *dst, int n, int count, double dx, int discrete, hipStream_t s);
hipError_t launch_q_table(int64_t *dst, int n, int count, int64_t lfac, hipStream_t s);
hipError_t launch_thresholds(int64_t *dst, int nbins, int64_t qmax, hipStream_t s);
hipError_t launch_shell_partials(const ModeTables &mt, int n1, int n2, double lscale,
                                 double *partial_cnt, double *partial_k, int grid,
                                 hipStream_t s);
// out[b] = sum_g partial[g * width + b] in a fixed order, b < width.
hipError_t launch_reduce_cols(const double *partial, int64_t grid, int width, double *out,
                              hipStream_t s);
// the same for two arrays in one launch (width2 = 0: the second is unused)
hipError_t launch_reduce_cols2(const double *partial1, int64_t grid1, int width1, double *out1,
                               const double *partial2, int64_t grid2, int width2, double *out2,
                               hipStream_t s);
hipError_t launch_pk_kspace(const void *F, int n1, int n2, int64_t sx, int64_t sy, int64_t sz,
                            const ModeTables &mt, double *partial, int grid, hipStream_t s);
hipError_t launch_pk_finalize(const double *S, int nbins, const double *count, const double *sumk,
                              double norm, double vscale, double kscale, double *pk,
                              double *kmean, double *count_out, double *parseval,
                              const double *sumsq, double inv_n, hipStream_t s);

int x_rows_per_block(int len, int nc);
int s_cols_per_block(int len);

// ---------------------------------------------------------------- batches
// Passes BP_* of a batched solve and the work-item order: lf2_batch_items.hpp.

struct BatchField {
    XArgs xf, xi;
    SArgs yf, z, yi;
    int m, l1, l2;           // x, y, z line lengths
    int ntiles[BP_COUNT];
    int nbins;               // 0: no binning
    double *partial;         // [ntiles[BP_Z]][nbins + 1]
    const double *count;     // shell table of the lattice
    const double *sumk;
    double norm, kscale;     // dx^3 / N, 2 pi / (L dx)
    double *pk, *kmean, *count_out;  // caller's device arrays (nullable)
};

struct BatchItem {
    int field, tile;
};

constexpr int kBatchMaxBins = 511;
bool batch_len_supported(int len);
int batch_x_rows(int m);
// Persistent batch kernel: x tiles of batch_px_rows(m) rows; one launch of
// `grid` blocks runs every item of the nq queues of `items` (ordered and
// laid out as batch_items makes them; qstart / qcount and ctl have nq + 1
// entries, the last queue empty).  local = 1: a block serves queue
// xq[XCC id] (16 entries); 0: every block serves queue 0.
int batch_px_rows(int m);
size_t batch_persistent_lds();  // LDS bytes of a persistent block
hipError_t batch_persistent_launch(const BatchField *fields, const QItem *items,
                                   const uint32_t *qstart, const uint32_t *qcount, int nq,
                                   const int32_t *xq, QCtl *ctl, uint32_t *done, int ndone,
                                   uint32_t spin_limit, int local, int grid, hipStream_t s);
// XCC (XCD) id of each of n blocks, into out[n].
hipError_t launch_xcc_probe(int32_t *out, int n, hipStream_t s);
// One grouped launch: items of pass `pass` whose line length is `len`.
// k2cont: 1 for the continuous k^2 (computed from |n_z| in the z pass), 0
// for the discrete one (its table).
hipError_t batch_group_launch(int pass, int len, const BatchField *fields,
                              const BatchItem *items, int nitems, int nbins, int k2cont,
                              hipStream_t s);
hipError_t batch_finalize_launch(const BatchField *fields, int nfields, hipStream_t s);

}  // namespace lf2
