// Shared host-side definitions of the stmg library: error handling, sparse
// matrices, complex scalars.
#pragma once

#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/stmg.h"

namespace stmg {

// Internal failures are thrown as StmgError and turned into ABI codes at the
// extern "C" boundary.
struct StmgError : std::runtime_error {
  int code;
  StmgError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string &msg) { throw StmgError(code, msg); }
#define STMG_REQUIRE(cond, code, msg) \
  do {                                \
    if (!(cond)) ::stmg::fail(code, msg); \
  } while (0)

// Allocation point for failure injection (stmg_debug_fail_alloc): counts
// the library's device buffers and large host arrays and throws STMG_ENOMEM
// at the armed one, before the allocation is made.
void alloc_point(const char *what);

// Compressed sparse rows with 64-bit row pointers.
struct Csr {
  int32_t n_rows = 0, n_cols = 0;
  std::vector<int64_t> ptr;   // [n_rows + 1]
  std::vector<int32_t> col;   // [nnz], ascending within a row
  std::vector<double> val;    // [nnz]
  int64_t nnz() const { return ptr.empty() ? 0 : ptr.back(); }
};

// Transpose (pattern and values).
Csr csr_transpose(const Csr &A);
// C = A * B (rows of A, SPA accumulation; explicit zeros from cancellation kept).
Csr csr_multiply(const Csr &A, const Csr &B);
// Two products with a shared union pattern: (P^T A P, P^T B P).
void csr_galerkin_pair(const Csr &P, const Csr &A, const Csr &B, Csr &Ac, Csr &Bc);
// Symmetric permutation B = A(p, p) with p[new] = old; rows re-sorted.
Csr csr_permute_sym(const Csr &A, const std::vector<int32_t> &perm_new_to_old);
// Value of A(i, j) or 0.
double csr_get(const Csr &A, int32_t i, int32_t j);

struct cplx {
  double re, im;
};

double wall_time();

}  // namespace stmg
