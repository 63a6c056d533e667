// Solver state shared by solve.hip (multigrid, CG) and smoother.hip (learned
// smoother): per-depth colour-ordered SELL matrices, transfers, smoother
// weights and work vectors.
#pragma once

#include <map>
#include <vector>

#include "internal.hpp"

namespace camfe {

constexpr int SBLK = 256;     // threads per block of the vector kernels
constexpr int SL = 64;        // SELL slice height = wavefront width
constexpr int KMAXS = 4;      // right-hand sides per pass
// eps of eps * Id added to the unit-diagonal-scaled coarsest matrix when a
// call does not say (the learned-smoother calls): large enough that FP32
// rounding of a singular system's restricted residual along its null space
// (~1e-7) is not amplified past O(0.1), and without effect on regular systems
constexpr double DEFAULT_COARSE_EPS = 1e-6;

// position of entry (r, c), r <= c, in the packed upper triangle (row by
// row) of a symmetric W x W cell-block inverse
template <int W>
__host__ __device__ constexpr int bpk(int r, int c) { return r * W - r * (r - 1) / 2 + c - r; }

struct GLevel {
  int d = 0;
  size_t n = 0;
  int ncol = 8;
  int tile = 0;               // colour-sweep tile (sell_kernels.hpp tile_sw / tile_mu), chosen by the autotuner
  std::vector<int> coff;      // colour c owns internal rows [coff[c], coff[c+1])
  std::vector<int> cslice;    // colour c owns slices [cslice[c], cslice[c+1])
  std::vector<long long> cnnz;  // nonzeros of the rows of each colour
  long long nnz = 0, pnnz = 0;  // matrix nonzeros; prolongation entries into this depth
  DArr<int> perm, iperm;      // internal -> canonical, canonical -> internal
  size_t nslices = 0, snnz = 0;
  DArr<int> sl_ptr;           // slice offsets into the value arrays (nslices + 1)
  DArr<int> sl_row0;          // first internal row of each slice
  DArr<int> sl_rows;          // rows in each slice (<= 64)
  DArr<int4> sl_meta;         // {sl_ptr[s], sl_ptr[s + 1], sl_row0[s], sl_rows[s] | flags} per slice
  DArr<int> scol;
  // 16-bit column codes (colour << 13 | offset) and 8 bases per slice, for
  // the slices flagged C16 in sl_meta (sell_kernels.hpp); ns16 of them
  DArr<uint16_t> scol16;
  DArr<int> sbase;
  long long ns16 = 0;
  DArr<double> sval64, invd64;
  DArr<float> sval32, invd32;
  // relaxation weights omega_i / A_ii (internal order), set for smoothers 1 and 2
  DArr<double> winvd64;
  DArr<float> winvd32;
  // transfers in internal numbering (P: rows at d, cols at d-1; R = P^T)
  DArr<int> Pptr, Pcol, Rptr, Rcol;
  DArr<double> Pw64, Rw64;
  DArr<float> Pw32, Rw32;
  // work vectors, n x KMAXS row-major (t: Jacobi ping-pong)
  DArr<double> x64, b64, r64, t64;
  DArr<float> x32, b32, r32, t32;
  // cell-block Schwarz smoother: blocks of at most 8 and of 9..16 functions
  // (internal rows, -1 padding), their symmetric inverses (packed upper
  // triangles, W (W + 1) / 2 values each) and
  // weights 1 / (largest number of blocks holding one of their functions)
  // (the inverses of the unit-diagonal-scaled blocks; bs = 1 / sqrt(A_ii))
  long long nb8 = 0, nb16 = 0;
  // blocks of each class ordered by the colour of their cell (coordinate
  // parities): colour k owns blocks [bc8[k], bc8[k + 1]) and [bc16[k], bc16[k + 1])
  long long bc8[9] = {0}, bc16[9] = {0};
  // automatic damping of the block corrections at this depth: 4 / (3 lambda)
  // (at most 1), lambda a power-iteration estimate of the largest eigenvalue
  // of sum_B w_B R_B^T A_B^-1 R_B A
  double block_lambda = 0, block_omega = 0;
  DArr<int> bidx8, bidx16;
  DArr<double> binv8_64, binv16_64, bw8_64, bw16_64, bs64;
  DArr<float> binv8_32, binv16_32, bw8_32, bw16_32, bs32;
  // batched solver only: meshes whose coarsest depth sits at this level and is
  // solved directly: first row of each, cumulative row counts (ncb + 1) and
  // the offset of each one's dense FP64 inverse in cb_a64
  int ncb = 0;
  long long cb_rows = 0;
  DArr<int> cb_rowoff, cb_cum;
  DArr<long long> cb_aoff;
  DArr<double> cb_a64;
  // batched solver only: the full slice records (sl_meta then holds a gated
  // copy in which the slices of members that stopped iterating are empty),
  // and the member of each slice, of each SBLK-row block and of each direct block
  DArr<int4> sl_meta_all;
  DArr<int> slmem, blkmem, cbmem;
};

struct SolverState {
  camfe_ctx ctx = nullptr;
  double t = 0;
  int precision = 0;
  int gamma = 1;             // coarse cycles per depth: 1 V-cycle, 2 W-cycle (set per solve)
  int nu_coarse = 0;         // sweeps each way below the finest depth (0: as at the finest; set per solve)
  int smoother = 0;          // 0 multicolour Gauss-Seidel, 1 Jacobi (constant omega), 2 learned Jacobi,
                             // 3 cell-block Schwarz
  bool blocks_ready = false; // cell blocks built for this state (t, coarse_eps)
  double block_omega = 0;    // damping of the cell-block corrections (0: each depth's automatic value)
  long long block_colour_min = 0;  // depths with at least this many blocks relax them colour by colour
  int wkind = 0;             // smoother whose weights winvd holds (0: none)
  int wsweep = 0;            // sweep those weights are for: 0 Jacobi, 1 multicolour SOR
  double omega = 0;          // constant omega of smoother 1
  const void* model = nullptr;  // learned model whose weights winvd holds
  double coarse_eps = 0;
  int D = 0, d0 = 0;
  std::vector<GLevel> lev;   // index = depth
  bool direct = false;
  int n0 = 0;
  DArr<double> Ainv64;       // coarsest inverse, FP64 in both precisions
  // outer iteration vectors (finest, internal order, n x KMAXS row-major)
  DArr<double> X, R, Z, P, Q, B;
  DArr<double> sc;           // device scalars: [0..K) rz, [K..2K) pq, [2K..3K) rr, [3K..4K) rz_new, [4K..5K) bb,
                             // [5K..6K) beta
  DArr<double> part, part2;  // per-block partial sums of the reductions (two live at once in a CG step)
  double setup_seconds = 0;
  // batched solver: nmesh meshes side by side at every level (rows mesh-major,
  // each mesh's rows padded to whole SBLK-row blocks); bmesh: mesh of each
  // finest-level block, bstart: first block of each mesh (nmesh + 1)
  bool batch = false;
  int nmesh = 0;
  DArr<int> bmesh, bstart;
  DArr<int> mact;            // batched: 1 while the member still iterates (read by the gated kernels)
  // captured iterations (one graph per right-hand-side count / precision / sweeps / method / smoother)
  hipStream_t cap = nullptr;
  std::map<long long, hipGraphExec_t> graphs;
  void drop_graphs() {
    for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
    graphs.clear();
  }
  ~SolverState() {
    drop_graphs();
    if (cap) (void)hipStreamDestroy(cap);
  }
};

// smoother.hip: Jacobi weights for smoother 1 (constant) or 2 (learned model)
void set_smoother_weights(camfe_sys s, SolverState* S, int smoother, double omega, const void* model);
// block.hip: cell blocks and their inverses at every depth of S (degree 1)
void build_cell_blocks(camfe_sys s, SolverState* S);

}  // namespace camfe
