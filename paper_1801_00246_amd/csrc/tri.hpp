// Compile-time layout of the degree-N nodal triangle shared by all kernels.
//
// Node order: lattice (i, j), j = 0..N rows away from face 0, i = 0..N-j
// along it.  Face f joins vertices f and (f+1)%3 (face 0: s = -1,
// face 1: r + s = 0, face 2: r = -1); its Nfp = N+1 nodes are listed
// counter-clockwise.  Two counter-clockwise neighbours traverse a shared edge
// in opposite directions, so node k of one face meets node N-k of the other.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace ipdg {

// Compile-time loop: calls f(std::integral_constant<int, I>) for I in [B, E),
// so node and face tables can be evaluated as constant expressions.
template <int B, int E, typename F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(static_cast<F&&>(f));
  }
}

template <int N>
struct Tri {
  static constexpr int Np = (N + 1) * (N + 2) / 2;
  static constexpr int Nfp = N + 1;

  __host__ __device__ static constexpr int id(int i, int j) { return j * (N + 1) - (j * (j - 1)) / 2 + i; }
  __host__ __device__ static constexpr int lat_j(int n) {
    int j = 0;
    while (n >= N + 1 - j) { n -= N + 1 - j; ++j; }
    return j;
  }
  __host__ __device__ static constexpr int lat_i(int n) {
    int j = 0;
    while (n >= N + 1 - j) { n -= N + 1 - j; ++j; }
    return n;
  }
  // node id of position k on face f
  __host__ __device__ static constexpr int fm(int f, int k) {
    return f == 0 ? id(k, 0) : (f == 1 ? id(N - k, k) : id(0, N - k));
  }
  // position of node n on face f, or -1
  __host__ __device__ static constexpr int fpos(int f, int n) {
    for (int k = 0; k <= N; ++k)
      if (fm(f, k) == n) return k;
    return -1;
  }
  // Node of the unrotated triangle that sits at node n of the frame whose
  // vertex 0 is vertex k (barycentric lattice a'_m = a_{(m+k)%3}).  Face k of
  // the triangle is face 0 of that frame.
  __host__ __device__ static constexpr int rot(int k, int n) {
    const int ip = lat_i(n), jp = lat_j(n), a0 = N - ip - jp;
    return k == 0 ? n : (k == 1 ? id(a0, ip) : id(jp, a0));
  }
};

// Offsets of the reference operators in one contiguous table per degree.
//   Dr, Ds           reference derivative matrices
//   Krr, Krs, Kss    M Dr Dr, M (Dr Ds + Ds Dr), M Ds Ds  (volume term)
//   QR, QS           M Dr LIFT, M Ds LIFT  (Np x 3 Nfp, lifted-jump volume term)
//   M, Minv          mass matrix and its inverse
//   LIFT             M^{-1} E  (Np x 3 Nfp)
//   M1D              face mass on [-1, 1]
//   NBR              [j][d][m]: entry (m, j) of D_r (d = 0) or D_s (d = 1)
//                    for the face-0 rows m = 0..N, stored column by column
//                    (the neighbour phase streams over j)
template <int N>
struct OpsLayout {
  static constexpr int Np = Tri<N>::Np, Nfp = Tri<N>::Nfp;
  static constexpr int Dr = 0;
  static constexpr int Ds = Dr + Np * Np;
  static constexpr int Krr = Ds + Np * Np;
  static constexpr int Krs = Krr + Np * Np;
  static constexpr int Kss = Krs + Np * Np;
  static constexpr int M = Kss + Np * Np;
  static constexpr int Minv = M + Np * Np;
  static constexpr int QR = Minv + Np * Np;
  static constexpr int QS = QR + Np * 3 * Nfp;
  static constexpr int LIFT = QS + Np * 3 * Nfp;
  static constexpr int M1D = LIFT + Np * 3 * Nfp;
  static constexpr int NBR = M1D + Nfp * Nfp;
  // ROW: per output row i, the contiguous operator stream of the row phase:
  //   Krr_i | Krs_i | Kss_i (Np each) | QR_i | QS_i | E_i (3 Nfp each) | M_i
  // with E = M LIFT (the face mass scattered to face-node rows).
  static constexpr int RowLen = 4 * Np + 9 * Nfp;
  static constexpr int ROW = NBR + 2 * Nfp * Np;
  static constexpr int total = ROW + Np * RowLen;
};

inline int ops_total(int N) {
  const int Np = (N + 1) * (N + 2) / 2, Nfp = N + 1;
  return 7 * Np * Np + 3 * Np * 3 * Nfp + Nfp * Nfp + 2 * Nfp * Np + Np * (4 * Np + 9 * Nfp);
}

// Operator streams of the cooperative kernel (three waves per tile of 64
// elements: wave f takes face f, then a third of the output rows), appended
// after the OpsLayout tables.  All entries a wave reads in one phase are
// contiguous in the order it reads them.
//   FD  [f][j][k][d]      D_r (d = 0), D_s (d = 1) at node k of face f,
//                         column j (own normal derivative, streamed over j)
//   LF  [f2][p][f][k]     LIFT rows at the nodes of face f2
//   per wave w, rows [row_begin(w), row_begin(w+1)), nr rows:
//     CV [j][i][t]        K_rr, K_rs, K_ss (t = 0, 1, 2), column by column
//     CM [j][i]           M
//     CQ [f][k][i][t]     M D_r LIFT, M D_s LIFT (t = 0, 1)
template <int N>
struct CoopLayout {
  static constexpr int Np = Tri<N>::Np, Nfp = Tri<N>::Nfp;
  static constexpr int kWaves = 3;
  __host__ __device__ static constexpr int row_begin(int w) { return (w * Np + kWaves - 1) / kWaves; }
  __host__ __device__ static constexpr int nrows(int w) { return row_begin(w + 1) - row_begin(w); }
  static constexpr int kMaxRows = (Np + kWaves - 1) / kWaves;
  static constexpr int FD = OpsLayout<N>::total;
  static constexpr int LF = FD + 3 * Np * Nfp * 2;
  static constexpr int W0 = LF + 9 * Nfp * Nfp;
  __host__ __device__ static constexpr int wave_len(int w) { return nrows(w) * (4 * Np + 6 * Nfp); }
  __host__ __device__ static constexpr int CV(int w) {
    int o = W0;
    for (int v = 0; v < w; ++v) o += wave_len(v);
    return o;
  }
  __host__ __device__ static constexpr int CM(int w) { return CV(w) + 3 * Np * nrows(w); }
  __host__ __device__ static constexpr int CQ(int w) { return CM(w) + Np * nrows(w); }
  static constexpr int total = W0 + Np * (4 * Np + 6 * Nfp);
};

// Matrix-core form of the cooperative kernel's row phase: the output rows of
// a tile are 16 x 16 blocks (16 rows x 16 elements) computed by
// 16 x 16 x 4 matrix multiply-accumulates.  The operators are stored as the
// A operands of those instructions, one 64-value block per (operator, row
// block rb, column block kb) in lane order: lane l holds entry
// (16 rb + l % 16, 4 kb + l / 16), zero outside the matrix.  Operators:
// volume t = 0..3: K_rr, K_rs, K_ss, M (Np columns); face q = 0..2:
// M D_r LIFT, M D_s LIFT, -M LIFT (3 Nfp columns).  Appended after
// CoopLayout.
template <int N>
struct MfmaLayout {
  static constexpr int Np = Tri<N>::Np, Nfp = Tri<N>::Nfp;
  static constexpr int RB = (Np + 15) / 16;        // row blocks of 16
  static constexpr int KBV = (Np + 3) / 4;         // column blocks of the volume operators
  static constexpr int KBF = (3 * Nfp + 3) / 4;    // column blocks of the face operators
  static constexpr int BASE = CoopLayout<N>::total;
  __host__ __device__ static constexpr int vol(int t, int rb, int kb) { return BASE + ((t * RB + rb) * KBV + kb) * 64; }
  __host__ __device__ static constexpr int face(int q, int rb, int kb) {
    return BASE + 4 * RB * KBV * 64 + ((q * RB + rb) * KBF + kb) * 64;
  }
  static constexpr int total = BASE + 64 * RB * (4 * KBV + 3 * KBF);
};

// Length of the whole per-degree table (OpsLayout, CoopLayout, MfmaLayout).
inline int ops_table_len(int N) {
  const int Np = (N + 1) * (N + 2) / 2, Nfp = N + 1;
  const int RB = (Np + 15) / 16, KBV = (Np + 3) / 4, KBF = (3 * Nfp + 3) / 4;
  return ops_total(N) + 3 * Np * Nfp * 2 + 9 * Nfp * Nfp + Np * (4 * Np + 6 * Nfp) +
         64 * RB * (4 * KBV + 3 * KBF);
}

}  // namespace ipdg
