// Host-side preparation for the implicit-inverse effective-resistance sweep.
//
// Everything here runs on the CPU before the device sweep: graph ingest and
// grounding (Section II-A), fill-reducing nested-dissection ordering
// (Definition 1, Lemma 2), symbolic analysis of the factor (Lemma 1,
// Definition 2) and the numeric L D L^T factorization (Algorithm 8, step 1).
#pragma once

#include <chrono>
#include <cstdint>
#include <string>
#include <vector>

namespace peers {

enum Status : int {
  OK = 0,
  E_INVALID_ARG = -1,
  E_NODE_RANGE = -2,
  E_WEIGHT = -3,
  E_DISCONNECTED = -4,
  E_NOT_SPD = -5,
  E_HOST_OOM = -6,
  E_OVER_BUDGET = -7,
  E_HIP = -8,
  E_BUSY = -9,
  E_CANCELLED = -10,
  E_TIMEOUT = -11,
  E_UNSUPPORTED = -12,
  E_INTERNAL = -99,
};

void set_error(const std::string& msg);
const char* last_error();

inline double now_s() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

// Symmetric sparse pattern (no diagonal) with values, CSR over reduced ids.
struct SymCsr {
  int32_t n = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> idx;
  std::vector<double> val;  // off-diagonal entries of L_r (negative sums of conductances)
};

struct Ingested {
  int64_t n = 0, m = 0;
  int32_t ground = 0;
  int32_t N = 0;               // n - 1 rows of L_r
  SymCsr A;                    // off-diagonal part of L_r
  std::vector<double> gnd;     // conductance from each node to the ground (its row sum in L_r; compensated sums)
  int64_t self_loops = 0;
};

Status ingest(int64_t n, int64_t m, const int32_t* eu, const int32_t* ev, const double* w,
              int32_t ground, Ingested& out);

// Nested-dissection elimination order over reduced ids (order[new] = reduced id).
// coords: optional N x 3 row-major array in reduced-id order.
void nd_order_coords(const SymCsr& A, const double* coords, int leaf, std::vector<int32_t>& order);
void nd_order_graph(const SymCsr& A, int leaf, std::vector<int32_t>& order);

struct Symbolic {
  int32_t N = 0;
  std::vector<int32_t> perm;    // perm[new] = reduced id
  std::vector<int32_t> iperm;   // iperm[reduced id] = new
  std::vector<int32_t> parent;  // elimination tree, -1 at roots; postordered
  std::vector<int64_t> colptr;  // strict-lower pattern of L, CSC, rows ascending
  std::vector<int32_t> rowidx;
  std::vector<int32_t> snptr;   // fundamental supernodes
  std::vector<int32_t> depth;   // root depth 1
  std::vector<int32_t> first;   // smallest index of subtree(j)
  int32_t height = 0;
  int32_t max_sn_width = 0;
  double f_sweep = 0;           // sum over L_ki != 0 of depth(k)
};

// Elimination tree of the permuted pattern (Liu's algorithm with path compression).
void etree_of(const SymCsr& A, const std::vector<int32_t>& perm, const std::vector<int32_t>& iperm,
              std::vector<int32_t>& parent);
Status symbolic_analyze(const SymCsr& A, const std::vector<int32_t>& order, Symbolic& S);

struct Numeric {
  std::vector<double> Lx;  // unit-lower L, aligned with Symbolic::rowidx
  std::vector<double> D;   // pivots
};

// gnd: per reduced id, the conductance to the ground; every pivot is formed
// from it and the off-diagonal entries (no cancellation, see numeric.cpp).
Status ldlt_numeric(const SymCsr& A, const std::vector<double>& gnd, const Symbolic& S, int threads,
                    Numeric& F);

// Simple fork-join helper: runs fn(i) for i in [0, n) over `threads` workers.
template <class Fn>
void parallel_for(int64_t n, int threads, Fn&& fn);

int default_threads();

}  // namespace peers

#include "parallel.inl"
