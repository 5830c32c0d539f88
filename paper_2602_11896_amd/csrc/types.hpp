// Plain-old-data records shared by the host plan and the HIP kernels.
// Every record is built on the host, copied once into the plan's device arena,
// and read by the kernels; none holds a pointer (only element offsets).
#pragma once
#include <cstdint>

namespace jtfs {

// A band-limited Fourier filter on an L-point grid: bins lo, lo+1, ..., lo+len-1
// (modulo L) hold the non-negligible values, stored contiguously at `off` floats into
// the plan's band-value array. Filters are real in the Fourier domain (Gaussian
// spectra), so one float per bin.
struct Band {
  int32_t L;
  int32_t lo;
  int32_t len;
  int32_t pad_;
  int64_t off;
};

// One row of a batched 1-D transform stage. Field meaning depends on the stage
// (documented next to each stage in kernels_time.hip).
struct RowJob {
  int64_t src;     // element offset of the input
  int64_t dst;     // element offset of the output
  int64_t aux;     // stage-specific second input offset
  int32_t band;    // band index (gather stages) or -1
  int32_t src_len; // length of the input grid
  int32_t n;       // transform length (power of two)
  int32_t shift;   // Fourier subsampling exponent: the fold averages 2^shift blocks
  int32_t t0, t1;  // adjoint gathers: first and end segment (built from a term range)
  Band b;          // copy of bands[band] (zeros without one), so that a row's loads
                   // wait for one record, not two in a chain
};

// A workgroup's share of a single-pass transform stage: `count` consecutive rows of
// length 2^log2n starting at job `job0` (count * 2^log2n <= 4096).
struct RowTask {
  int32_t job0, count, log2n, pad_;
};

// One workgroup of a two-pass (four-step) transform: its row job, log2 of the row length,
// its column block (pass 1) or row block (pass 2), and the row's scratch offset.
struct SplitTask {
  int32_t job, log2n, blk, log2A;   // log2A: the split point n = A B of this row
  int64_t scr;
  RowJob j;                         // copy of jobs[job]
};

// One term of a multi-term adjoint gather: out[m] += band[m] * src[m mod src_len]
// for bins m of the output grid inside the band.
struct GatherTerm {
  int64_t src;
  int32_t band;
  int32_t src_len;
};

// One term of an adjoint-gather segment, self-contained (a gather reads it in one step):
// the source row and its length, and the band's placement (first bin lo on a grid of L
// bins, len values at offset off of the band values).
struct SegTerm {
  int64_t src;
  int64_t off;
  int32_t lo, len, L, src_len;
};

// A second-order group (one n2 with K >= 1 rows), frequential stage bookkeeping.
struct FreqGroup {
  int64_t y2;       // complex offset of the K x L2 stack in the Y2 region
  int64_t phiT;     // float offset of phi_T at level j2 (time domain, L2 values)
  int64_t part;     // float offset of this group's pooled partial sums
  int64_t dP;       // float offset of this group's pooled-gradient rows
  int64_t dYpart;   // complex offset of this group's dY2 partials (RS x K x L2)
  int64_t psum;     // float offset of the chunk sums (R_pad x nF) in the psum region, or -1
                    // (windowed groups: the pooling kernel sums their partials itself)
  int32_t K, L2, j2, s_t;   // s_t = log2 T - j2 (time pooling stride exponent)
  int32_t TC, n_tc;         // t-chunk length of the forward and number of chunks
  int32_t RS, rt_per_split; // backward row splits and row tiles per split
  int32_t n_tb;             // backward 64-column t-blocks
  int32_t rt_fwd;           // forward row tiles per row split (row-tile-loop forward kernel)
  int32_t halo;             // phi_T support: |phi_T[d]| <= 1e-9 max beyond circular distance halo
  int32_t fw;               // > 0: each forward chunk pools into a window of fw frames (see plan)
  int32_t nsub;             // row-tile-loop forward: sub-chunks of TC / nsub times per workgroup
  int32_t n_t;              // unaveraged second order: kept times on the L2 grid
  int64_t u2;               // unaveraged second order: offset of |V| (R_pad x n_t floats) and
                            // of dV (R_pad x n_t complex) in their regions
  int32_t t_lo, pad2_;      // unaveraged second order: first kept time on the L2 grid
  int32_t lt0, nlt;         // live row tiles (rows meeting [0, K)): live_rt[lt0 .. lt0 + nlt)
};

// Forward frequential work item: rows [rb*64, rb*64+64) x columns [tc*TC, (tc+1)*TC).
struct FwdItem {
  int32_t grp, rb, tc, pad_;
};

// Backward frequential work item: columns [tb*64, tb*64+64), row tiles of split rs.
struct BwdItem {
  int32_t grp, tb, rs, pad_;
};

// A frequential filter g as laid out in the row space of the W matrix.
struct FrFilter {
  int32_t row0;     // first row of g in W (multiple of 16)
  int32_t M;        // N_fr / 2^k_g rows carrying data
  int32_t k;        // k_g
  int32_t lowpass;  // 1 for phi_F
  int64_t phiF;     // float offset of phi_F at level k_g (time domain, M values)
  int32_t spin, pad_;
  int64_t taps;     // float offset of g's N_fr complex taps at level 0 (re, im pairs)
};

}  // namespace jtfs
