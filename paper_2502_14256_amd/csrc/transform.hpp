// Pass-based FWHT / FFTBR / IFFTBR engine for gfx950.
//
// A length-2^m transform is split over the bits of the element index: a
// "row" pass transforms the low a0 bits (contiguous tiles), then "column"
// passes transform higher bit groups (tiles of 2^a strided rows x W
// contiguous columns).  Inside a pass, a workgroup holds its tile in LDS and
// every thread keeps E = 16 elements in registers; radix-2^g stages run in
// registers and bit groups are exchanged through LDS.
//
// FFTBR (Sec. 5.2: decimation-in-time FFT without the input bit reversal)
// factors over the index bits: transform the low bits first; before the
// group of bits [s, s+g) apply the twiddle W_{2^{s+g}}^{k R_g(c)}, where k is
// the (already transformed, natural-order) low index and c the group digit,
// then transform the group.  IFFTBR runs the same steps backwards with
// conjugate twiddles.  The FWHT is the same schedule without twiddles
// (H_m is the Kronecker power of H_1).  All passes are unnormalised; the
// caller folds n^-1/2 or 1/n into one multiply.
#pragma once

#include "common.hpp"

namespace ldk {

enum PassMode { PM_FWD = 0, PM_INV = 1, PM_SOLVE = 2, PM_MATVEC = 3 };

struct PassGeom {
    int b0;    // index bit where this pass's axis starts
    int a;     // axis bits (tile rows 2^a)
    int logW;  // tile width (contiguous columns) log2, logW <= b0
    int logE;  // registers per thread log2 (g), logE <= a
};

struct Plan {
    int m;
    int P;  // number of passes (0 when m == 0)
    PassGeom pass[4];
};

// log_tile: log2 of the elements per workgroup tile (LDS budget).
Plan make_plan(int m, int log_tile);
int log_tile_for(int kind, int dtype);

struct PassArgs {
    const void *src;
    void *dst;
    int64_t src_row;  // elements between consecutive batch rows in src
    int64_t dst_row;  // elements between consecutive batch rows in dst
    int64_t rows;     // batch rows
    int m;
    PassGeom g;
    const double *lam;  // eigenvalues [rows / nrhs][2^m] (solve / matvec), FP64
    int nrhs;
    int global_tw;    // apply the inter-pass FFT twiddle (column passes)
    double sigma2;
    double scale;     // solve: scale / (lambda + sigma2); matvec: scale * lambda;
                      // fwd / inv: multiplies the stored values
};

// kind: LDK_LATTICE (complex FFTBR) or LDK_DNET_B2 (real FWHT).
// dtype: working precision of the pass.
// src_real: rows of src are real (promoted to complex) -- lattice only.
// dst_real: keep only the real part when storing -- lattice only.
// src_f32: src holds floats widened to the FP64 working type (PM_FWD only).
int launch_pass(int kind, int dtype, int mode, bool src_real, bool dst_real, const PassArgs &a,
                hipStream_t s, bool src_f32 = false);

}  // namespace ldk
