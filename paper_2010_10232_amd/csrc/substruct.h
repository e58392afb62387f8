// Exact solver of the deflation matrix E = Z^T A Z (section 3) on a variable-k
// level by substructuring: one level of nested dissection of the control-point
// grid, the interiors eliminated exactly, the separator Schur complement dense.
#pragma once

#include <functional>

#include "hh_internal.h"

namespace hh {

// One symmetric matrix of a batch stored as packed upper-triangle tiles
// (128 x 128, row order of the tile grid, each tile row-major, zero-padded).
// Its local index r maps to the vector entry map[map0 + r].
struct SymMat {
    int n;        // order
    int tile0;    // first tile in the packed array
    int row0;     // first tile row in the batch (reduce grid)
    int map0;     // first entry of its index map
};

// y[map[..]] = A x[map[..]] for every matrix of the batch (also y2 if set), in
// two launches: the tile products (partial sums per tile, rowpart / colpart:
// tiles x 128 complex) and their reduction per tile row.
void launch_symv_batch_tiles(const SymMat* mats_dev, int nmat, long long tiles, int rows, const double* P,
                             const int* map, const cx<double>* x, cx<double>* rowpart, cx<double>* colpart,
                             hipStream_t s);
void launch_symv_batch_reduce(const SymMat* mats_dev, int nmat, int rows, const int* map,
                              const cx<double>* rowpart, const cx<double>* colpart, cx<double>* y, cx<double>* y2,
                              hipStream_t s);
// algorithmic bytes of one tile launch (every stored tile once, its partial
// sums written, the mapped inputs)
double symv_batch_tile_bytes(long long tiles);

// Cuts tried at set-up (cheapest first) until one passes the check; refinement
// steps allowed for the best one.
constexpr int kSubCandidates = 4;
constexpr double kSubCheckTol = 1e-12;
constexpr int kSubMaxRefine = 3;

struct SubstructE {
    int n1 = 0, n2 = 0, px = 0, py = 0;
    int bx = 0, by = 0, nsub = 0;   // subdomains per direction, total
    long long nS = 0, nI = 0;       // separator / interior unknowns
    int nd_max = 0, h_max = 0;      // largest subdomain interior / halo
    long long sub_tiles = 0, S_tiles = 0;
    int sub_rows = 0, S_rows = 0;
    DevBuf subP, subMats;           // packed inverses of the subdomain blocks E_dd
    DevBuf SP, SMats;               // packed inverse of the Schur complement S
    DevBuf map;                     // int32: interiors (subdomain-major), then separators
    DevBuf xhat, xt;                // level vectors, zero off the interior / separator entries
    DevBuf rvec;                    // level residual
    DevBuf rowpart, colpart;
    double check0 = -1.0;           // ||c - E y|| / ||c||, y one pass of the block solve (random c)
    double self_check = -1.0;       // the same after the refinement steps below
    int refine = 0;                 // refinement steps y += pass(c - E y) per application
    DevBuf rr, dd;                  // refinement residual and correction
    // bytes streamed by one application (tiles once each, vectors)
    double bytes_per_apply() const;
};

// Partitions (subdomains per direction) that fit the set-up bounds, fewest
// stored tiles first, at most max_count; empty if no cut into at least two
// subdomains fits.  px, py: coupling half-width in index space per direction
// (the degree; 0 for the trivial direction of 1D problems).
std::vector<std::pair<int, int>> substruct_partitions(int n1, int n2, int px, int py, int max_count);

// Entries of E by row: calls f(J, value) for the nonzeros of row I (duplicates
// allowed; they are summed).
using RowVisitor = std::function<void(long long I, const std::function<void(long long, double)>& f)>;

// Builds the factors (host assembly, rocSOLVER LU inverses and rocBLAS
// products of the dense blocks at setup).
void substruct_build(SubstructE& E, int n1, int n2, int px, int py, int bx, int by, const RowVisitor& row,
                     hipStream_t s);

}  // namespace hh
