/*
 * ssart.h -- symmetric-split SART for mirror-symmetric tomographic systems,
 * on AMD Instinct MI355X (gfx950).
 *
 * The method (Alikhanov et al., arXiv:1902.10559, Section 2): when the scan
 * positions are pairwise symmetric about the OZ axis and voxels are numbered
 * by the vertical-snake rule, the system matrix A (M x N) of eq. (1), A f = p,
 * satisfies eq. (2), w[i,j] = w[M-i+1, N-j+1].  Then A folds into two
 * independent (M/2) x (N/2) systems (3) and (4), A(1) f(1) = p(1) and
 * A(2) f(2) = p(2), with
 *     w1[i,j] = w[i,j] - w[M-i+1,j],   w2[i,j] = w[i,j] + w[M-i+1,j],
 *     p1[i]   = p[i]   - p[M-i+1],     p2[i]   = p[i]   + p[M-i+1],
 * and the solution of (1) is recombined from f(1), f(2) by Theorem 1, eq. (5):
 *     f[j] = (f2[j] + f1[j]) / 2,   f[N-j+1] = (f2[j] - f1[j]) / 2.
 * The paper solves the halves with SART (its refs. [001], [003]); this library
 * runs simultaneous SART on both halves at once on one GPU.
 *
 * Index convention at this interface: 0-based.  Ray i pairs with ray M-1-i,
 * voxel j with voxel N-1-j; m = M/2, n = N/2.
 *
 * Conventions for every call:
 *   - Return value: SS_OK (0) on success; > 0 is a warning and the results
 *     are valid; < 0 is an error, and then no output has been written (for
 *     the asynchronous device calls: no work has been enqueued).  The text of
 *     the last error on the calling thread is returned by ss_last_error().
 *   - Arrays of length 0 (an empty matrix, nnz = 0) may be NULL.
 *   - "device" pointers are caller-owned device memory of the current HIP
 *     device; the library never frees caller memory, and device calls never
 *     allocate device memory (scratch comes from caller workspaces, except
 *     for ss_fold_noalloc's fixed per-device array).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Device calls only enqueue work on it, except where a call says that it
 *     synchronises.
 *   - Calls are reentrant; the only shared state is the thread-local error
 *     text, an internal cache of instantiated HIP graphs (mutex-guarded) and
 *     ss_fold_noalloc's per-device scratch array (see there).
 */
#ifndef SSART_H
#define SSART_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ss_status;
enum {
  SS_OK = 0,
  SS_NOT_CONVERGED = 1,   /* warning: a solve reached max_iter above tol    */
  SS_E_ARG = -1,          /* NULL pointer, bad size, bad option             */
  SS_E_ODD = -2,          /* M, N or nx odd: the fold needs even sizes      */
  SS_E_ASYM = -3,         /* A violates eq. (2) (bitwise, pattern included) */
  SS_E_SHAPE = -4,        /* arrays inconsistent (unsorted, out of range,
                             CSR and CSC holding different entries)         */
  SS_E_NONFINITE = -5,    /* NaN or Inf in A or p                           */
  SS_E_NOMEM = -6,        /* host allocation failed                         */
  SS_E_HIP = -7,          /* a HIP runtime call failed                      */
  SS_E_WORKSPACE = -8     /* workspace too small                            */
};

/* storage type of matrix values */
enum { SS_F32 = 0, SS_BF16 = 1, SS_F16 = 2 };

const char* ss_last_error(void);
const char* ss_version(void);

/* ------------------------------------------------------------------------
 * Geometry and the system matrix A of eq. (1)  (host; setup, not timed)
 * ---------------------------------------------------------------------- */

/* A 2D slice of nx x nz square voxels of side `pitch` (mm), centred on OZ in
 * x, bottom face at z = 0.  Voxel (column c, row r), c = 0 at the most
 * negative x and r = 0 at the top, has the vertical-snake index
 *     j = c*nz + (c even ? r : nz-1-r),
 * so that its mirror (nx-1-c, r) has index N-1-j (needs nx even).  This is
 * the paper's numbering rule of Section 2 (Fig. 1). */
typedef struct {
  int32_t nx, nz;
  double pitch;
} ss_grid;

/* K point sources (src_x ascending, src_x[K-1-k] == -src_x[k] bitwise,
 * src_z[K-1-k] == src_z[k]) and B detector bins at height det_z (bin_x
 * ascending, bin_x[B-1-b] == -bin_x[b] bitwise): positions pairwise
 * symmetric about OZ as Section 2 requires.  Ray i = k*B + b runs from source
 * k to the centre of bin b, so ray M-1-i is the mirror of ray i. */
typedef struct {
  int32_t K;
  const double* src_x;
  const double* src_z;
  int32_t B;
  const double* bin_x;
  double det_z;
} ss_geometry;

/* Host CSR + CSC copy of A (M = K*B rows, N = nx*nz columns); columns ascend
 * within a row and rows within a column.  Arrays are owned by the library
 * and released by ss_matrix_free. */
typedef struct {
  int64_t M, N, nnz;
  int64_t* row_ptr;   /* M+1 */
  int32_t* col_idx;   /* nnz */
  float* val;         /* nnz */
  int64_t* col_ptr;   /* N+1 */
  int32_t* row_idx;   /* nnz */
  float* val_t;       /* nnz */
} ss_matrix;

/* Builds A for the scan: w[i,j] = length (mm) of ray i inside voxel j by
 * Siddon's method (FP64 plane-crossing parameters, segments <= 1e-9 mm
 * dropped), rounded to FP32.  Mirror-exact inputs give an A that satisfies
 * eq. (2) bitwise.  `nthreads` <= 0 uses all hardware threads.
 * Errors: SS_E_ARG (NULL, non-positive sizes, pitch <= 0), SS_E_ODD (nx, K or
 * B odd), SS_E_ASYM (sources or bins not mirror-exact), SS_E_NOMEM. */
ss_status ss_build_system(const ss_grid* grid, const ss_geometry* geom,
                          int32_t nthreads, ss_matrix* out);
void ss_matrix_free(ss_matrix* A);

/* snake[r*nx + c] = vertical-snake index of voxel (c, r), for all nx*nz
 * voxels (host array of nx*nz entries, caller-owned).  Section 2, Fig. 1. */
ss_status ss_snake_order(const ss_grid* grid, int64_t* snake);

/* A polar grid (the closing example's tomographic gamma scanning of a
 * cylindrical container, Fig. 4): a disk of radius `radius` (mm) centred on
 * the origin of the slice plane, cut into `rings` rings of equal width and
 * `sectors` (even) sectors of equal angle whose boundaries include the
 * symmetry axis OZ.  On either side of OZ a voxel is (ring r from the
 * centre, sector h counted from +z by the angle atan2(|x|, z)); on the side
 * x < 0 it has index j = r*(sectors/2) + h and its mirror (x > 0) has N-1-j,
 * N = rings*sectors: the renumbering that makes eq. (2) hold (Fig. 4b). */
typedef struct {
  int32_t rings, sectors;
  double radius;
} ss_polar_grid;

/* A parallel-beam scan: K view angles phi (radians, ascending inside
 * (-pi/2, pi/2), phi[K-1-k] == -phi[k] bitwise; 0 = rays along -z) and B
 * lateral offsets (mm, ascending, offset[B-1-b] == -offset[b] bitwise).  Ray
 * i = k*B + b is the line {offset[b] (cos phi, sin phi) + u (sin phi,
 * -cos phi)}, so ray M-1-i is the mirror of ray i. */
typedef struct {
  int32_t K;
  const double* phi;
  int32_t B;
  const double* offset;
} ss_parallel_scan;

/* Builds A for a polar grid and a parallel scan: w[i,j] = length (mm) of ray
 * i inside voxel j, from the ray's crossings with the ring circles and the
 * sector-boundary lines (FP64; segments <= 1e-9 mm dropped; a voxel crossed
 * twice gets the sum, in order along the ray), rounded to FP32.  A
 * satisfies eq. (2) bitwise.  `nthreads` <= 0 uses all hardware threads.
 * Errors: SS_E_ARG (NULL, non-positive sizes or radius, views or offsets not
 * ascending, a view outside (-pi/2, pi/2)), SS_E_ODD (sectors, K or B odd),
 * SS_E_ASYM (views or offsets not mirror-exact), SS_E_NOMEM. */
ss_status ss_build_polar_system(const ss_polar_grid* grid, const ss_parallel_scan* scan,
                                int32_t nthreads, ss_matrix* out);

/* ------------------------------------------------------------------------
 * Device-side A, the fold into systems (3)-(4), and the solver's system
 * ---------------------------------------------------------------------- */

/* A in device memory (caller-owned), CSR and CSC as in ss_matrix. */
typedef struct {
  int64_t M, N, nnz;
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const float* val;
  const int64_t* col_ptr;
  const int32_t* row_idx;
  const float* val_t;
} ss_matrix_dev;

/* One linear system as the SART solver consumes it, all arrays device memory
 * owned by the caller.
 *   nvals = 2: the folded pair (A(1), A(2)) of systems (3) and (4), stored on
 *              ONE shared sparsity pattern (the union of the positions of
 *              w[i,j] and w[M-1-i,j]; A(1) keeps its cancelled entries as
 *              +0.0).  Per entry the two values are interleaved: val[2k] is
 *              A(1)'s, val[2k+1] is A(2)'s; likewise p[2i] = p1[i],
 *              p[2i+1] = p2[i], and images are interleaved (f1[j], f2[j]).
 *   nvals = 1: a single system (the unsplit A, the baseline).
 * m x n: system size; nnz: stored pattern entries.
 * wdtype: SS_F32, SS_BF16 or SS_F16 storage of val/val_t (FP32 arithmetic).
 * row_ptr (m+1), col_idx (nnz), val (nvals*nnz): CSR, columns ascending.
 * col_ptr (n+1), row_idx (nnz), val_t (nvals*nnz): CSC of the same entries.
 * p (nvals*m): right-hand side.
 * inv_row (m), inv_col (n): FP32 reciprocals of the FP64 row and column sums
 *   of A (which equal those of A(2)), 0 where a sum is 0; SART normalises
 *   both halves with them.
 * Stream layout: the solver reads col_idx/val and row_idx/val_t in chunks
 * of SS_CHUNK entries, so each of these four arrays must start on a 16-byte
 * boundary and have room for ss_stream_len(nnz) entries (nnz rounded up to
 * a multiple of SS_CHUNK, plus SS_CHUNK: the interleaved order's last loads
 * reach up to SS_CHUNK - 1 entries past the last line); entries past nnz are
 * read and ignored, never written.  The same holds for A's arrays when a system aliases them
 * (ss_unsplit).
 * row_lanes, col_lanes: order of the entries within each row (column).
 *   0: ascending, the CSR/CSC convention.  L > 0: the interleaved order of
 *   the solver's stream form for groups of L lanes: a line of n entries is
 *   cut into blocks of SS_CHUNK*L entries (the last one r < SS_CHUNK*L
 *   long), and entry e of a block, with lane g = e mod L and q = r / L,
 *   sits at g*q + min(g, r mod L) + e / L within it.  ss_fold writes that
 *   order when the caller sets these fields; ss_sart_* then read the lines
 *   in place with rows_per_wave = 64/row_lanes (cols_per_wave =
 *   64/col_lanes).  row_lanes is 0, 8, 16, 32 or 64, col_lanes 0, 4, 8, 16,
 *   32 or 64 (else SS_E_ARG).  ss_unsplit, ss_subsets_build, ss_ossart_*
 *   and ss_normal_* need 0 (else SS_E_ARG). */
typedef struct {
  int64_t m, n, nnz;
  int32_t nvals;
  int32_t wdtype;
  int64_t* row_ptr;
  int32_t* col_idx;
  void* val;
  int64_t* col_ptr;
  int32_t* row_idx;
  void* val_t;
  float* p;
  float* inv_row;
  float* inv_col;
  int32_t row_lanes;
  int32_t col_lanes;
} ss_system;

/* Entries per aligned chunk of the solver's index and value streams. */
#define SS_CHUNK 4

/* Capacity, in entries, that the index and value arrays of a system with nnz
 * stored entries must have: nnz rounded up to a multiple of SS_CHUNK, plus
 * SS_CHUNK (0 for nnz <= 0). */
int64_t ss_stream_len(int64_t nnz);

/* Bytes of workspace ss_fold_size and ss_fold need for an M x N matrix. */
ss_status ss_fold_workspace_bytes(int64_t M, int64_t N, size_t* bytes);

/* Validates A (and p, if not NULL) and returns the size of the shared pattern
 * of A(1)/A(2) in *nnz_half.  Checks: M, N even (SS_E_ODD); rows and columns
 * sorted and in range, and CSR and CSC holding the same entries (SS_E_SHAPE);
 * eq. (2) bitwise for every stored entry of both copies (SS_E_ASYM); finite
 * values (SS_E_NONFINITE).  SYNCHRONISES the stream once. */
ss_status ss_fold_size(const ss_matrix_dev* A, const float* p, void* workspace,
                       size_t workspace_bytes, int64_t* nnz_half,
                       void* stream);

/* ss_fold_size for `count` matrices at once: every check pass is one
 * launch over the line pairs of all matrices (the lane groups of the fold's
 * counting pass, one partial record per block, no atomics), then one record
 * per matrix.  A[k]: host array of device matrix descriptors; p: host array
 * of device right-hand sides (or NULL; an entry may be NULL); nnz_half:
 * host, count entries.  Returns the first failing matrix's error (its index
 * in the message), and then writes nothing to nnz_half.  `workspace`: device
 * scratch of ss_fold_batch_workspace_bytes(A, count) bytes.  SYNCHRONISES
 * the stream once. */
ss_status ss_fold_size_batch(const ss_matrix_dev* A, const float* const* p, int32_t count,
                             void* workspace, size_t workspace_bytes, int64_t* nnz_half,
                             void* stream);

/* The fold of Section 2: fills `out` (nvals = 2, m = M/2, n = N/2, nnz =
 * *nnz_half from ss_fold_size, wdtype chosen by the caller; every array
 * allocated by the caller with the sizes listed at ss_system).  Values are
 * one correctly rounded FP32 subtraction/addition per entry, then rounded to
 * nearest-even for BF16/FP16 storage; p1/p2 likewise in FP32; inv_row/inv_col
 * from FP64 sums of A's FP32 entries.  A must have passed ss_fold_size.
 * Each output line is written in the order out->row_lanes (rows) and
 * out->col_lanes (columns) select (see ss_system; 0: ascending).
 * `workspace`: device scratch of ss_fold_workspace_bytes(M, N) bytes (its
 * contents on entry do not matter).  Asynchronous. */
ss_status ss_fold(const ss_matrix_dev* A, const float* p, ss_system* out,
                  void* workspace, size_t workspace_bytes, void* stream);

/* ss_fold with no workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation).  Same arguments, checks and results as ss_fold
 * (bit for bit).  Its only scratch, the per-tile sums of the offset scans,
 * lives in a 32 KiB array that the library holds in each device's memory
 * until the process ends, located once per device on the first call there.
 * It calls no allocating routine.  Limit: M/2 and N/2 at most 4095*4096 - 1
 * (larger: SS_E_ARG, nothing enqueued).  Every call on one device shares
 * that device's array, so calls that overlap on one device (other streams,
 * other threads) race: serialise them.  Asynchronous. */
ss_status ss_fold_noalloc(const ss_matrix_dev* A, const float* p, ss_system* out, void* stream);

/* ss_fold for `count` matrices at once (Section 2 applied to each): every
 * phase (union sizes, offsets, fill; rows, then columns) is one launch over
 * the lines of all matrices.  A[k] (host array of descriptors of device
 * matrices) must have passed ss_fold_size; p[k] (host array of device
 * pointers); out[k] as for ss_fold, all with the same wdtype.  The results
 * equal `count` calls of ss_fold bit for bit.  `workspace`: device scratch
 * of ss_fold_batch_workspace_bytes(A, count) bytes.  Asynchronous. */
ss_status ss_fold_batch_workspace_bytes(const ss_matrix_dev* A, int32_t count,
                                        size_t* bytes);
ss_status ss_fold_batch(const ss_matrix_dev* A, const float* const* p,
                        ss_system* out, int32_t count, void* workspace,
                        size_t workspace_bytes, void* stream);

/* The unsplit baseline: fills a single system (nvals = 1, m = M, n = N) for
 * A itself.  The caller sets out->m, n, nnz, nvals = 1, wdtype and every
 * pointer; row_ptr/col_idx/col_ptr/row_idx may alias A's arrays, and val/
 * val_t may alias A's when wdtype = SS_F32 (otherwise they receive the
 * rounded values).  Writes p (copy unless aliased), inv_row, inv_col.
 * Asynchronous. */
ss_status ss_unsplit(const ss_matrix_dev* A, const float* p, ss_system* out,
                     void* stream);

/* ------------------------------------------------------------------------
 * SART on one or many systems (the paper's solver, refs. [001], [003])
 * ---------------------------------------------------------------------- */

/* Simultaneous SART, every ray in every iteration:
 *     f <- f + lambda * V^-1 A^T W^-1 (p - A f)
 * applied to every half of every system (for nvals = 2 this is SART on (3)
 * and (4) with the sums of A; recombined by eq. (5) it is SART on (1)).
 * Options:
 *   lambda       relaxation, 0 < lambda < 2 (ref. [003])
 *   max_iter     update cap (>= 0)
 *   tol          stop at the first k with rel_res(f^k) <= tol (<= 0: never)
 *   check_every  iterations between host checks for early exit when tol > 0
 *   use_graph    1: replay the iterations as an instantiated HIP graph
 *   rows_per_wave  forward projection rows per 64-lane wavefront: 1,2,4,8
 *                  (0 = choose from the row-length statistics)
 *   cols_per_wave  back projection columns per wavefront: 1,2,4,8,16 (0 =
 *                  choose)
 *   xcd_remap    1: give each of the 8 XCDs a contiguous range of rows or
 *                columns (the hardware deals workgroups round-robin)
 *   zero_start   1: start from f^0 = 0 (the solver clears f itself);
 *                0: start from the image the caller passes
 *   unroll       entries each lane has in flight per pass: 4 or 8 (0 = 4)
 *   nonneg       1: project every updated image onto f >= 0 (each voxel
 *                of the full image clamped at 0; on the folded pair the
 *                equivalent map of each pair (f1, f2) with eq. (5), which
 *                keeps f2 >= |f1|)
 *   chunked      stream form per kernel, bit 0 forward, bit 1 back
 *                projection: 0 = entry-wise (lanes of a group hold adjacent
 *                entries), 1 = aligned chunks of SS_CHUNK entries per lane
 *                (fewer, wider loads; gathers spread over more cache lines);
 *                bit 2 forward, bit 3 back projection (taking precedence
 *                over bits 0 and 1): interleaved, i.e. the solver first
 *                copies the line lists into its workspace in an order where
 *                each lane reads SS_CHUNK entries with one load and a gather
 *                still has adjacent lanes on adjacent entries; the sums run
 *                in the entry-wise order, so results equal the entry-wise
 *                form's bitwise.  Needs entries of at least 4 bytes (not a
 *                single system with 16-bit values: SS_E_ARG) and workspace
 *                for the copies (ss_sart_workspace_bytes counts it); the copy
 *                is made on every solve.  A system stored in that order
 *                (row_lanes / col_lanes nonzero) is read in place with the
 *                interleaved form whatever these bits say, and fixes
 *                rows_per_wave (cols_per_wave) to 64 / its lanes
 *   persistent   1: size the grid to the resident capacity and let each block
 *                loop over tiles (prefetching the next one); 0: one block
 *                per tile
 *   staged       bit 0: band-staged forward projection.  The columns are
 *                cut into bands of band_width consecutive indices; a copy of
 *                the row streams is laid out band by band (each row's
 *                entries in a band form a segment, padded with zero entries
 *                to whole chunks of SS_CHUNK; 16-bit column indices within
 *                the band), made in the workspace on every solve.  A band's
 *                chunks are cut into work tiles of about tile_entries; a
 *                block loads one band of the image into shared memory and
 *                its wavefronts stream the band's tiles, one chunk per lane,
 *                summing each segment with a segmented scan across the
 *                lanes; a second
 *                kernel adds each row's segment sums in band order and
 *                forms the residual.  A row whose columns do not strictly
 *                ascend inside [0, n) gets no segments (it adds nothing to
 *                the forward projection).  Bit 1: tile-staged back
 *                projection.  Columns are taken in tiles of tile_cols; per
 *                tile the distinct rows its entries touch are found once per
 *                solve and each entry's row is rewritten as its rank among
 *                them (16 bits); the block copies those rows of z into
 *                shared memory and sums from there (a tile touching more
 *                than 4096 rows, or rows in more than 128 runs, keeps global
 *                gathers).  Needs lines in ascending order (row_lanes /
 *                col_lanes 0), 16-byte aligned images, nnz < 2^31, and for
 *                bit 1 m <= 2^17.  With bit 1, cols_per_wave counts columns
 *                per wavefront of an 8-wavefront block; rows_per_wave,
 *                `chunked` and `persistent` do not apply to the staged
 *                kernels; `unroll` 8 has the band kernel keep three
 *                windows of loads per wavefront in flight (4: two); the
 *                staged back projection takes two chunks per lane and pass
 *                with 8 or more columns per wavefront, else one.  The sums
 *                run in another order than the unstaged kernels' (equal to
 *                FP32 rounding), always the same one.
 *   band_width   voxels per forward band: a power of two from 1024 to 16384
 *                with band_width * nvals * 4 + 16384 * nvals <= 65536 bytes
 *                of shared memory (0 = 4096)
 *   tile_cols    columns per back-projection tile: a power of two from 64 to
 *                8192 (0 = 1024)
 *   tile_entries  padded entries per forward work tile: a multiple of 256
 *                from 1024 to 65536 (0 = 2048)
 *   residual_every  ordered subsets only (ss_ossart_solve; here 0 or 1): the
 *                residual of the pass-start image, a full forward sweep, is
 *                taken on passes k with k % residual_every == 0 and at
 *                k = max_iter only (0 or 1: every pass); tol is then tested
 *                on those passes, and res_hist[k] is written for them only
 * rel_res(f^k) = ||p - A f^k|| / ||p||, from the halves as
 *   sqrt((||r1||^2 + ||r2||^2) / (||p1||^2 + ||p2||^2)), FP64. */
typedef struct {
  float lambda;
  int32_t max_iter;
  double tol;
  int32_t check_every;
  int32_t use_graph;
  int32_t rows_per_wave;
  int32_t cols_per_wave;
  int32_t xcd_remap;
  int32_t zero_start;
  int32_t unroll;
  int32_t persistent;
  int32_t chunked;
  int32_t nonneg;
  int32_t staged;
  int32_t band_width;
  int32_t tile_cols;
  int32_t tile_entries;
  int32_t residual_every;
} ss_sart_opts;

/* Workspace bytes for solving `nsys` systems together with these options
 * (with the interleaved stream form on systems stored in ascending order,
 * this includes the copies of their streams). */
ss_status ss_sart_workspace_bytes(const ss_system* sys, int32_t nsys,
                                  const ss_sart_opts* opts, size_t* bytes);

/* Solves nsys independent systems in the same launches.
 *   f[s]        device, nvals*n floats: start image on entry (interleaved
 *               halves: zeros, or ss_image_fold of a start; ignored with
 *               zero_start), final iterate on return.
 *   res_hist[s] device, max_iter+1 doubles: res_hist[s][k] = rel_res(f^k)
 *               for k = 0 .. iters[s]; entries after that are not written.
 *   iters       host, nsys ints, or NULL: updates applied per system.
 * With tol <= 0 and iters == NULL the call is asynchronous; otherwise it
 * synchronises the stream (every check_every iterations when tol > 0, and
 * once at the end to read iters).  Returns SS_NOT_CONVERGED if tol > 0 and a
 * system ended at max_iter above tol. */
ss_status ss_sart_solve(const ss_system* sys, int32_t nsys, float* const* f,
                        double* const* res_hist, const ss_sart_opts* opts,
                        int32_t* iters, void* workspace,
                        size_t workspace_bytes, void* stream);

/* Times the two solver kernels over `reps` launches each on `stream` with
 * HIP events and returns their mean durations in milliseconds: the forward
 * projection + residual kernel and the back projection + update kernel.
 * The images f are used as scratch (their contents change). Synchronises. */
ss_status ss_sart_time_kernels(const ss_system* sys, int32_t nsys,
                               float* const* f, const ss_sart_opts* opts,
                               int32_t reps, double* fp_ms, double* bp_ms,
                               void* workspace, size_t workspace_bytes,
                               void* stream);

/* As ss_sart_time_kernels, per launch of an iteration: ms[0] the forward
 * projection kernel (with staged bit 0: the band kernel), ms[1] the residual
 * kernel of the band-staged form (0 otherwise), ms[2] the back projection;
 * mean milliseconds over `reps` iterations, each launch stamped by its own
 * dispatch.  ms: host, 3 doubles.  The images f are used as scratch.
 * Synchronises. */
ss_status ss_sart_time_phases(const ss_system* sys, int32_t nsys, float* const* f,
                              const ss_sart_opts* opts, int32_t reps, double* ms,
                              void* workspace, size_t workspace_bytes, void* stream);

/* The sizes of the staged forms that a solve with these options builds
 * (this call builds them in the workspace, as a solve does; the images f are
 * used as scratch): info[0] forward segments over all systems (a row's
 * entries in one band), info[1] forward work tiles, info[2] back-projection
 * tiles, info[3] of those staged in shared memory, info[4] rows of z those
 * stage in all.  Zero for a form not selected.  opts->staged must be
 * nonzero.  info: host, 5 int64.  Synchronises. */
ss_status ss_sart_staged_info(const ss_system* sys, int32_t nsys, float* const* f,
                              const ss_sart_opts* opts, int64_t* info, void* workspace,
                              size_t workspace_bytes, void* stream);

/* Picks rows_per_wave, cols_per_wave, unroll, persistent, chunked and xcd_remap by
 * timing every candidate (ss_sart_time_kernels) and writes them into
 * *opts.  The interleaved forms are candidates only when workspace_bytes
 * holds their copies; their per-solve copy time, spread over opts->max_iter
 * iterations, is added to their kernel times.  Results are cached per (nvals, wdtype, shape statistics).
 * The images f are used as scratch.  Synchronises. */
ss_status ss_sart_autotune(const ss_system* sys, int32_t nsys, float* const* f,
                           ss_sart_opts* opts, void* workspace,
                           size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Ordered-subset SART (the paper's ref. [004] applied to SART, ref. [001])
 * with subsets that the fold preserves
 * ---------------------------------------------------------------------- */

/* The subsets of one folded pair.  A subset of rays closed under the ray
 * mirror i -> M-1-i (the rays of sources k and K-1-k of the symmetric scan)
 * folds onto a block of rows; with rays ordered source-major, subset s of S
 * is the folded rows [s m/S, (s+1) m/S), and S must divide m.
 *   col_sub      device, (S+1)*n ints, subset-major: column j's entries
 *                in subset s are col_ptr[j] + col_sub[s*n+j] .. col_ptr[j] +
 *                col_sub[(s+1)*n+j] - 1 (rows ascend, so they are
 *                contiguous)
 *   inv_col_sub  device, S*n floats: FP32 reciprocal of the FP64 sum of
 *                A(2) over column j's entries in subset s (0 for a zero
 *                sum); it equals A's column sum over the mirror-closed
 *                subset.
 *   col_ptr_os, row_idx_os, val_t_os  a subset-major copy of the CSC: the
 *                entries of column j in subset s are positions
 *                col_ptr_os[s*n+j] .. col_ptr_os[s*n+j+1]-1 (device,
 *                S*n+1 int64); row_idx_os (int32) and val_t_os (FP32
 *                pairs) have room for ss_stream_len(nnz) entries and are
 *                16-byte aligned.  A subset's back projection then streams
 *                1/S of the entries. */
typedef struct {
  int32_t S;
  int32_t* col_sub;
  float* inv_col_sub;
  int64_t* col_ptr_os;
  int32_t* row_idx_os;
  void* val_t_os;
} ss_subsets;

/* Fills every array of `sub` (caller-allocated) for a folded FP32 pair
 * (nvals = 2, wdtype = SS_F32).  SYNCHRONISES the stream once (the
 * subset-major offsets are scanned on the host). */
ss_status ss_subsets_build(const ss_system* sys, ss_subsets* sub, void* stream);

/* Workspace bytes for ss_ossart_solve on these systems. */
ss_status ss_ossart_workspace_bytes(const ss_system* sys, const ss_subsets* sub,
                                    int32_t nsys, const ss_sart_opts* opts,
                                    size_t* bytes);

/* Ordered-subset SART on nsys folded pairs (all with the same S): one pass
 * applies, for s = 0 .. S-1, f <- f + lambda V_s^-1 A_s^T W^-1 (p_s - A_s f)
 * to both halves, V_s the subset column sums; recombined by eq. (5) the
 * iterates are ordered-subset SART on A with the mirror-closed subsets.
 * Options as for ss_sart_solve, with max_iter counting passes and
 * cols_per_wave up to 64 (a subset sees 1/S of each column); `persistent`
 * is ignored, `staged` must be 0, and `chunked` takes bits 0 and 1 as there
 * and bit 2 (the interleaved forward form: the workspace holds a copy of
 * every system's rows in the interleaved order, made on every solve;
 * results equal the entry-wise form's bit for bit), not bit 3 (SS_E_ARG).  res_hist[s][k] = rel_res of the image after k passes, for
 * k = 0 .. passes[s] (max_iter + 1 doubles); passes (host, or NULL)
 * receives the passes applied.  A pass evaluates the residual of its
 * starting image (one extra forward projection of every row) on every
 * residual_every-th pass (every pass by default).  Returns
 * SS_NOT_CONVERGED as ss_sart_solve does. */
ss_status ss_ossart_solve(const ss_system* sys, const ss_subsets* sub,
                          int32_t nsys, float* const* f,
                          double* const* res_hist, const ss_sart_opts* opts,
                          int32_t* passes, void* workspace,
                          size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * The direct path: normal equations (Theorem 2)
 * ---------------------------------------------------------------------- */

/* Workspace bytes for ss_normal_solve: about nvals*n*n doubles (the dense
 * normal matrices, lower triangles used; both halves are factored together:
 * 2 (N/2)^2 = N^2/2 for the split pair against N^2 for A), plus O(n).  Errors:
 * SS_E_ARG for a NULL argument, a system that is not FP32 with nvals 1 or
 * 2, or n > 2^17. */
ss_status ss_normal_workspace_bytes(const ss_system* sys, size_t* bytes);

/* Solves the normal equations A(k)^T A(k) f(k) = A(k)^T p(k) of each half of
 * a folded FP32 pair (nvals = 2) by Cholesky factorisation in FP64 and
 * writes their recombination by eq. (5), which by Theorem 2 is the normal
 * pseudo-solution of (1) (the least-squares solution when A has full column
 * rank); for nvals = 1 the same solve on A itself.  f: device, 2n doubles
 * (nvals = 2) or n doubles; workspace: device, at least the bytes
 * ss_normal_workspace_bytes returns, owned by the caller and overwritten.
 * B is formed from both the CSR and the CSC of `sys`, and p; inv_row and
 * inv_col are not read.  Errors: those of ss_normal_workspace_bytes;
 * SS_E_WORKSPACE if the workspace is too small; SS_E_SHAPE if a normal
 * matrix is not positive definite (A, or A(1) or A(2), lacks full column
 * rank: a zero or negative pivot; f then holds no solution).  Part of the
 * factorisation runs on a second stream that the library creates once per
 * device (default priority), ordered against `stream` by events; calls on
 * one device are serialised by a lock held for the whole call.
 * SYNCHRONISES the stream once. */
ss_status ss_normal_solve(const ss_system* sys, double* f, void* workspace,
                          size_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Images
 * ---------------------------------------------------------------------- */

/* Theorem 1, eq. (5): f (N = 2n floats) from the interleaved halves f12 (n
 * pairs): f[j] = (f2[j] + f1[j]) / 2, f[N-1-j] = (f2[j] - f1[j]) / 2, FP32.
 * Asynchronous. */
ss_status ss_recombine(const float* f12, int64_t n, float* f, void* stream);

/* ss_recombine for `count` images: f12[k], f[k] device pointers (host
 * arrays), n[k] pairs each (host array).  Asynchronous. */
ss_status ss_recombine_batch(const float* const* f12, const int64_t* n,
                             float* const* f, int32_t count, void* stream);

/* Inverse of eq. (5) (the transform in the proof of Theorem 1): f12 from f,
 * f1[j] = f[j] - f[N-1-j], f2[j] = f[j] + f[N-1-j], FP32.  Asynchronous. */
ss_status ss_image_fold(const float* f, int64_t N, float* f12, void* stream);

/* Forward projection q = A f of eq. (1) (device, FP32 accumulation): q has M
 * entries, f has N.  Asynchronous. */
ss_status ss_project(const ss_matrix_dev* A, const float* f, float* q,
                     void* stream);


/* ------------------------------------------------------------------------
 * Learned initialiser: the kernels of a small convolutional network that
 * maps an early split-SART image to a later one (used to start SART closer
 * to its limit).  Not part of the paper's method; SART itself stays the
 * arbiter (a learned start is only kept if its residual is lower).
 * Tensors are NHWC; activations BF16 (stored as uint16 bit patterns),
 * gradients that accumulate FP32.  3x3 convolutions, stride 1, one pixel of
 * zero padding.  FP32 master weights are laid out [O][3][3][C].  All calls
 * are asynchronous and allocate nothing.
 * ---------------------------------------------------------------------- */

/* fold of the right-hand side only: p12[2i] = p[i] - p[M-1-i],
 * p12[2i+1] = p[i] + p[M-1-i] (Section 2), for systems that share a folded
 * matrix and differ in p. */
ss_status ss_fold_rhs(const float* p, int64_t M, float* p12, void* stream);

/* BF16 forward weights [O][9][Cp] and the flipped, transposed copy
 * [C][9][Op] (w_bwd[c][t][o] = w[o][8-t][c]) that computes the input
 * gradient as a forward convolution; Cp, Op = C, O rounded up to 8 with
 * zero padding. */
ss_status ss_nn_prep_weights(const float* w, int32_t O, int32_t C, void* w_fwd, void* w_bwd, void* stream);

/* y = act(bias + conv3x3(x, w)), x (N,H,W,C) BF16, w [O][9][Cp] BF16, bias FP32
 * or NULL, relu 0/1, y (N,H,W,O) BF16 (y_f32 = 0) or FP32 (y_f32 = 1).
 * FP32 accumulation on the matrix cores.  N*H <= 65535. */
ss_status ss_nn_conv3x3(const void* x, int32_t N, int32_t H, int32_t W, int32_t C, const void* w,
                        const float* bias, int32_t O, int32_t relu, void* y, int32_t y_f32, void* stream);

/* gw [O][3][3][C] += sum over pixels of gy (x) shifted x; gb [O] += sum of gy
 * (gb may be NULL; with gb, O <= 256).  x (N,H,W,C), gy (N,H,W,O), both
 * BF16.  Partial sums per range of pixels go to `workspace` (device, at
 * least ss_nn_wgrad_workspace_bytes) and are added in a fixed order, so the
 * gradients are bitwise the same on every run. */
ss_status ss_nn_wgrad_workspace_bytes(int32_t N, int32_t H, int32_t W, int32_t C, int32_t O, size_t* bytes);
ss_status ss_nn_conv3x3_wgrad(const void* x, const void* gy, int32_t N, int32_t H, int32_t W, int32_t C,
                              int32_t O, float* gw, float* gb, void* workspace, size_t workspace_bytes,
                              void* stream);

/* out = BF16(g * [y > 0]) for the ReLU output y (BF16), or BF16(g) if y is
 * NULL. */
ss_status ss_nn_relu_mask(const float* g, const void* y, int64_t n, void* out, void* stream);

/* 2x2 average pool of x (N,H,W,C) into y (N,H/2,W/2,C), BF16; and its
 * gradient gx (N,H,W,C) (+)= gy/4, FP32. */
ss_status ss_nn_pool2(const void* x, int32_t N, int32_t H, int32_t W, int32_t C, void* y, void* stream);
ss_status ss_nn_pool2_grad(const float* gy, int32_t N, int32_t H, int32_t W, int32_t C, float* gx,
                           int32_t accumulate, void* stream);

/* Channel-slice copies for skip connections: y[..., coff:coff+C] of a
 * (N,Hy,Wy,Ctot) map = x, nearest-upsampled 2x when up = 1 (x is then
 * (N,Hy/2,Wy/2,C)); and the gradient of that slice back into gx (N,Hx,Wx,C),
 * summed over each 2x2 block when up = 1. */
ss_status ss_nn_to_slice(const void* x, int32_t N, int32_t Hy, int32_t Wy, int32_t C, int32_t up, void* y,
                         int32_t Ctot, int32_t coff, void* stream);
ss_status ss_nn_from_slice(const float* gy, int32_t N, int32_t Hx, int32_t Wx, int32_t C, int32_t up,
                           int32_t Ctot, int32_t coff, float* gx, int32_t accumulate, void* stream);

/* out = x + r; with target: g = 2 (out - target) / n (g may be NULL) and,
 * with loss, *loss += mean squared error (FP64; per-block partials in
 * `workspace`, at least ss_nn_mse_workspace_bytes(n), added in block order,
 * so the loss is the same on every run; workspace may be NULL without
 * loss). */
ss_status ss_nn_mse_workspace_bytes(int64_t n, size_t* bytes);
ss_status ss_nn_residual_mse(const float* r, const float* x, const float* target, int64_t n, float* out,
                             float* g, double* loss, void* workspace, size_t workspace_bytes, void* stream);

ss_status ss_nn_to_bf16(const float* x, int64_t n, void* y, void* stream);

/* Adam step (bias-corrected) on FP32 weights; step counts from 1. */
ss_status ss_nn_adam(float* w, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                     float eps, int32_t step, void* stream);

/* Vertical-snake vectors (nimg images of nx*nz voxels) to images (N,nz,nx,1)
 * in FP32 and/or BF16 (to_image = 1), or images (FP32) back to snake order
 * (to_image = 0, dst32). */
ss_status ss_nn_snake_image(const float* src, int64_t nimg, int32_t nx, int32_t nz, int32_t to_image,
                            float* dst32, void* dst16, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SSART_H */
