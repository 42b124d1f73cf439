// C entry points over the host preparation code, for CPU tests (no HIP).
#include <cstring>

#include "host_prep.h"

using namespace qpg;

static HostCsr make(int rows, int cols, const int* ptr, const int* col, const double* val) {
    HostCsr h;
    h.rows = rows;
    h.cols = cols;
    h.ptr.assign(ptr, ptr + rows + 1);
    h.col.assign(col, col + ptr[rows]);
    h.val.assign(val, val + ptr[rows]);
    return h;
}

extern "C" {

void hp_transpose(int rows, int cols, const int* ptr, const int* col, const double* val, int* optr, int* ocol,
                  double* oval) {
    HostCsr t = transpose(make(rows, cols, ptr, col, val));
    std::memcpy(optr, t.ptr.data(), sizeof(int) * t.ptr.size());
    std::memcpy(ocol, t.col.data(), sizeof(int) * t.col.size());
    std::memcpy(oval, t.val.data(), sizeof(double) * t.val.size());
}

void hp_bf16(const double* in, unsigned short* out, long n) {
    for (long i = 0; i < n; ++i) out[i] = f64_to_bf16_bits(in[i]);
}

// returns 1 and fills the outputs when the line format applies (0 when it
// does not, -1 when its slots exceed cap_slots); lval holds nslots * R values
int hp_line_format(int rows, int cols, const int* ptr, const int* col, const double* val, int R, double max_fill,
                   int cap_slots, int* lptr, int* lcol, double* lval, int* sptr, int* sline, int* sslot,
                   int* nslots) {
    LineFormat lf;
    if (!build_line_format(make(rows, cols, ptr, col, val), R, lf, max_fill)) return 0;
    *nslots = int(lf.col.size());
    if (*nslots > cap_slots) return -1;
    std::memcpy(lptr, lf.ptr.data(), sizeof(int) * lf.ptr.size());
    std::memcpy(lcol, lf.col.data(), sizeof(int) * lf.col.size());
    std::memcpy(lval, lf.val.data(), sizeof(double) * lf.val.size());
    std::memcpy(sptr, lf.sptr.data(), sizeof(int) * lf.sptr.size());
    std::memcpy(sline, lf.sline.data(), sizeof(int) * lf.sline.size());
    std::memcpy(sslot, lf.sslot.data(), sizeof(int) * lf.sslot.size());
    return 1;
}

// blocks of rows (pairs of first row and first nonzero, blocks + 1 pairs);
// returns the block count, or -1 when it exceeds cap_blocks
int hp_row_blocks(int rows, const int* ptr, int max_nnz, int max_rows, int cap_blocks, int* out) {
    std::vector<int32_t> p(ptr, ptr + rows + 1), o;
    build_row_blocks(p, rows, max_nnz, max_rows, o);
    const int nb = int(o.size() / 2) - 1;
    if (nb > cap_blocks) return -1;
    std::memcpy(out, o.data(), sizeof(int) * o.size());
    return nb;
}
}
