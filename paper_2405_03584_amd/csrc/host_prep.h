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

// Round-to-nearest-even conversions (IEEE 754 binary32 / bfloat16 formats).
uint32_t f64_to_f32_bits(double v);
uint16_t f64_to_bf16_bits(double v);
double bf16_bits_to_f64(uint16_t b);

// Full validation of a qp_create call; "" when valid.
std::string validate_problem(const qp_hessian* H, const qp_csr* J, const double* W,
                             const qp_csr* A, const qp_range* b, const qp_range* bounds,
                             const qp_settings* s);

std::string validate_settings(const qp_settings* s);

}  // namespace qpg
