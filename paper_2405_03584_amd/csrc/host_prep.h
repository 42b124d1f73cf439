// Host-side preparation of QP data: validation, CSR transposition and value
// rounding.  No HIP calls: everything here runs before the first device call.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "qpgpu.h"

namespace qpg {

// CSR with int32 offsets (nnz < 2^31), as stored on the device.
struct HostCsr {
    int32_t rows = 0, cols = 0;
    std::vector<int32_t> ptr;   // rows + 1
    std::vector<int32_t> col;   // nnz
    std::vector<double> val;    // nnz
    int64_t nnz() const { return static_cast<int64_t>(col.size()); }
};

// Returns "" when the CSR is well formed, else the reason.
std::string check_csr(const qp_csr* M, const char* name, int32_t expect_cols);

// Copy a validated qp_csr into int32-offset storage.
HostCsr to_host_csr(const qp_csr* M);

// CSR of the transpose by a counting sort over columns: row j of the result
// lists the rows i of M with M_ij != 0 in increasing i (stable, deterministic).
HostCsr transpose(const HostCsr& M);

// Line format of a dose matrix whose rows come in groups of R consecutive
// rows sharing one column list (a line of R voxels; every spot covering the
// line touches all R rows).  Column ids are stored once per line; values are
// slot-major with the R rows of a slot contiguous:
//   row R*l + r, slot k of line l  ->  val[(ptr[l] + k) * R + r], column col[ptr[l] + k].
// The transpose is a per-spot list of (line, slot) pairs in increasing line
// order, so J^T reads the same value array.
// Slots of a line come in groups of this many (the line's list padded with
// repeats of its last column and zero values), so that a lane can load a
// group of its row's low-precision values at once (4 BF16 or 2 FP32 values
// in 8 bytes).
constexpr int32_t kLineSlotAlign = 4;

struct LineFormat {
    int32_t R = 64, lines = 0, cols = 0;
    std::vector<int32_t> ptr;      // lines + 1
    std::vector<int32_t> col;      // sum of line lengths (padded to kLineSlotAlign)
    std::vector<double> val;       // nnz, slot-major
    std::vector<int32_t> sptr;     // cols + 1
    std::vector<int32_t> sline;    // per spot: lines covered
    std::vector<int32_t> sslot;    // per spot: slot index ptr[l] + k
};

// Line format of M: lines of R consecutive rows (the last one padded with
// empty rows), each storing the union of its rows' column lists (padded to a
// multiple of kLineSlotAlign slots), slot-major, with zeros where a row lacks
// a column.  The per-spot lists name only real slots.  True (and fills lf)
// when the union slots times R number at most max_fill * nnz(M) (1 when every
// line's rows share one list, as in the 64-voxel bands); false leaves lf
// untouched.
bool build_line_format(const HostCsr& M, int32_t R, LineFormat& lf, double max_fill = 2.0);

// Nonzero-balanced blocks of consecutive rows of a CSR matrix (row pointers
// ptr, rows + 1 entries): block b holds rows out[2b] .. out[2b+2] - 1 and
// nonzeros out[2b+1] .. out[2b+3] - 1 (out holds 2(blocks + 1) entries, pairs of
// first row and first nonzero).  Rows join a block while it keeps at most
// max_nnz nonzeros and max_rows rows; a row longer than max_nnz forms a block
// of its own.  Every row falls in exactly one block; rows == 0 gives no block.
void build_row_blocks(const std::vector<int32_t>& ptr, int32_t rows, int32_t max_nnz, int32_t max_rows,
                      std::vector<int32_t>& out);

// Round-to-nearest-even conversions (IEEE 754 binary32 / bfloat16 formats).
uint32_t f64_to_f32_bits(double v);
uint16_t f64_to_bf16_bits(double v);
double bf16_bits_to_f64(uint16_t b);

// Full validation of a qp_create call; "" when valid.
std::string validate_problem(const qp_hessian* H, const qp_csr* J, const double* W,
                             const qp_csr* A, const qp_range* b, const qp_range* bounds,
                             const qp_settings* s);

std::string validate_settings(const qp_settings* s);

// Validation of the objective terms (gamma, p, U, w) for n variables; "" when valid.
std::string validate_hessian(const qp_hessian* H, int32_t n);

}  // namespace qpg
