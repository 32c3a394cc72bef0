// Sizes, K-slot maps and fragment offsets of the BF16x3 component-group
// stage kernel for order N, shared by the device kernel and the host code
// that lays out its operator fragments and material.  No HIP dependencies.
//
// MFMA shape: 16x16x32 bf16.  Rows of a contraction are operator rows (nodes
// or quadrature points), columns are the 16 elements of a tile, K runs over
// the operator's input index.  Lane l = 16 g + e holds column e and the K
// slots 8 g + j (j < 8) of the B operand, and rows 4 g + j (j < 4) of each
// 16-row accumulator tile.  The K order of every contraction is a permutation
// chosen so that each lane feeds the slots it holds from data it already has:
//
//  [Dr|Ds|Dt|LIFT], K step s < SN:  slots j < 6 are the three reference
//      directions d = j % 3 of node m = g + 4 (2 s + j / 3); slots 6, 7 are
//      face node jf = g + 4 (2 s + j - 6);
//  K step s >= SN: face node jf = g + 4 (2 SN + 8 (s - SN) + j);
//  V_q, K step s: node 16 (2 s + j / 4) + 4 g + j % 4 (the accumulator rows
//      of node tiles 2 s and 2 s + 1);
//  P_q, K step c: quadrature point 32 c + 16 (j / 4) + 4 g + j % 4 (the
//      accumulator rows of quadrature tiles 2 c and 2 c + 1).
// Slots whose node, face node or point lies beyond the element's count carry
// a zero operator entry.
#pragma once

namespace dgb {

// Row of a 16-row accumulator tile held in item j (of 4) by the lanes of
// group g = lane / 16: the f32 and bf16 16x16 products place rows 4 g + j
// there, v_mfma_f64_16x16x4f64 places rows 4 j + g (measured on gfx950).
constexpr int acc_row(bool f64, int g, int j) { return f64 ? 4 * j + g : 4 * g + j; }

template <int N>
struct BOrd {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int NF4 = 4 * Nfp;
  static constexpr int Nq = (N + 1) * (N + 1) * (N + 1);
  static constexpr int RT = (Np + 15) / 16;         // 16-row node tiles
  static constexpr int NPG = (Np + 3) / 4;          // nodes per lane group
  static constexpr int SN = (NPG + 1) / 2;          // K steps carrying nodes
  static constexpr int FPG = (NF4 + 3) / 4;         // face nodes per lane group
  static constexpr int SF = FPG > 2 * SN ? (FPG - 2 * SN + 7) / 8 : 0;
  static constexpr int SVL = SN + SF;               // K steps of [Dr|Ds|Dt|LIFT]
  static constexpr int QT = (Nq + 15) / 16;         // 16-row quadrature tiles
  static constexpr int QC = (QT + 1) / 2;           // K steps of P_q (32 points each)
  static constexpr int SVQ = (RT + 1) / 2;          // K steps of V_q
  // fragments of 64 lanes x 8 bf16; hi and lo of one (tile, step) adjacent
  static constexpr int NFV = RT * SVL * 2;
  static constexpr int NFQ = QT * SVQ * 2;
  static constexpr int NFP = RT * QC * 2;
  static constexpr int OFF_V = 0, OFF_Q = NFV, OFF_P = NFV + NFQ;
  static constexpr int NFRAG = NFV + NFQ + NFP;
  // blocked material: floats per (element tile, field)
  static constexpr int MATS = QC * 2 * 64 * 4;
};

}  // namespace dgb

namespace dgb {

// Sizes and fragment offsets of the BF16x3 stage for orders 5-7, which
// works on one element per workgroup with the nine fields (or output
// components) as the MFMA columns.  Operator fragments are in plain K order:
// fragment (t, s) holds, for lane l, rows 16 t + l % 16 and K slots
// 32 s + 8 (l / 16) + j (j < 8) of the operator, hi and lo adjacent.
template <int N>
struct EOrd {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int NF4 = 4 * Nfp;
  static constexpr int Nq = (N + 1) * (N + 1) * (N + 1);
  static constexpr int RT = (Np + 15) / 16;         // node row tiles
  static constexpr int KN = (Np + 31) / 32;         // K steps over nodes
  static constexpr int KF = (NF4 + 31) / 32;        // K steps over face nodes
  static constexpr int KQ = (Nq + 31) / 32;         // K steps over quadrature points
  static constexpr int QT = 2 * KQ;                 // quadrature row tiles
  static constexpr int OFF_D = 0;                              // [3][RT][KN]
  static constexpr int OFF_L = OFF_D + 2 * 3 * RT * KN;        // [RT][KF]
  static constexpr int OFF_V = OFF_L + 2 * RT * KF;            // V_q [QT][KN]
  static constexpr int OFF_P = OFF_V + 2 * QT * KN;            // P_q [RT][KQ]
  static constexpr int NFRAG = OFF_P + 2 * RT * KQ;
};

}  // namespace dgb

namespace dgb {

// Sizes and fragment offsets of the FP32 matrix-core stage (orders 1-4,
// v_mfma_f32_16x16x4_f32): the tiling of BOrd, with FP32 operator
// fragments.  Lane l = 16 g + e supplies K slot g of each 4-slot step.
//  [Dr|Ds|Dt|LIFT], step s < 3 NB (NB = ceil(Np / 4) node blocks): node
//      4 (s / 3) + g in reference direction s % 3; step s >= 3 NB: face
//      node 4 (s - 3 NB) + g;
//  V_q, quadrature tile u, step (t, j): node 16 t + acc_row(g, j) (node tile
//      t's accumulator row; 4 g + j in FP32, 4 j + g in FP64);
//  P_q, node tile t, step (u, j): quadrature point 16 u + acc_row(g, j).
// Fragments hold four consecutive steps per lane (one float4): vol
// [RT][SV4][64][4], V_q [QT][RT][64][4], P_q [RT][QT][64][4]; lane l of
// tile t has operator row 16 t + l % 16.  Slots beyond the counts are zero.
template <int N>
struct FOrd {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int NF4 = 4 * Nfp;
  static constexpr int Nq = (N + 1) * (N + 1) * (N + 1);
  static constexpr int RT = (Np + 15) / 16;
  static constexpr int QT = (Nq + 15) / 16;
  static constexpr int QC = (QT + 1) / 2;
  static constexpr int NB = (Np + 3) / 4;
  static constexpr int SV = 3 * NB + (NF4 + 3) / 4;   // steps of [Dr|Ds|Dt|LIFT]
  static constexpr int SV4 = (SV + 3) / 4;
  static constexpr int OFF_V = 0;                                  // in float4 units
  static constexpr int OFF_Q = OFF_V + RT * SV4 * 64;
  static constexpr int OFF_P = OFF_Q + QT * RT * 64;
  static constexpr int NF4S = OFF_P + RT * QT * 64;                // float4 count
};

}  // namespace dgb

namespace dgb {

// FP32 operator fragments of the orders 5-7 stage (v_mfma_f32_16x16x4_f32,
// one element per workgroup, fields as the MFMA columns).  A K group is 16
// operator columns: fragment (t, s) holds, for lane l, the float4 of rows
// 16 t + l % 16 and columns 16 s + 4 j + l / 16 (j < 4), so that component
// j is the A operand of the group's j-th 16x16x4 product.  Row tiles as in
// EOrd; offsets in float4 units per 64 lanes.
template <int N>
struct EFOrd {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int NF4 = 4 * Nfp;
  static constexpr int Nq = (N + 1) * (N + 1) * (N + 1);
  static constexpr int RT = (Np + 15) / 16;         // node row tiles
  static constexpr int QT = 2 * ((Nq + 31) / 32);   // quadrature row tiles (as EOrd)
  static constexpr int KN = (Np + 15) / 16;         // K groups over nodes
  static constexpr int KF = (NF4 + 15) / 16;        // K groups over face nodes
  static constexpr int KQ = (Nq + 15) / 16;         // K groups over quadrature points
  static constexpr int OFF_D = 0;                   // [3][RT][KN]
  static constexpr int OFF_L = OFF_D + 3 * RT * KN; // [RT][KF]
  static constexpr int OFF_V = OFF_L + RT * KF;     // V_q [QT][KN]
  static constexpr int OFF_P = OFF_V + QT * KN;     // P_q [RT][KQ]
  static constexpr int NFRAG = OFF_P + RT * KQ;
};

}  // namespace dgb

namespace dgt {

// Sizes, FP32 operator fragments and LDS use of the tiled discrete-adjoint
// kernel of order N (orders 1-4, v_mfma_f32_16x16x4_f32).  The 16 elements
// of a tile are the MFMA columns; lane l = 16 g + e holds column e, supplies
// K slot g of every 4-slot step and holds rows 4 g + j (j < 4) of each
// 16-row accumulator tile.  Fragment groups are one float4 per lane (four
// steps, or the three reference directions of one step), [group][64][4];
// for lane l, r = l % 16 and k = l / 16:
//   D   (t, s), item d < 3: D_d[16 t + r][4 s + k]   (item 3 zero)
//   L   (t, s4), item i:    LIFT[16 t + r][4 (4 s4 + i) + k]
//   V   (u, t), item j:     V_q[16 u + r][16 t + 4 k + j]
//   P   (u, t), item j:     P_q[16 t + 4 k + j][16 u + r]     (P_q^T)
//   VT  (u, t), item j:     V_q[16 u + 4 k + j][16 t + r]     (V_q^T)
//   DT  (t, s), item d < 3: D_d[4 s + k][16 t + r]            (D_d^T)
//   LT  (f, t), item j:     LIFT[16 t + 4 k + j][16 f + r]    (LIFT^T)
// t: node tiles, u: quadrature tiles, f: face-node tiles.  The node index
// 16 t + 4 k + j of V, P and LT (and the point index of VT) is the row that
// lane group k holds in item j of an accumulator tile, so those products
// take their B operand straight from the previous product's accumulators.
// Entries beyond Np, Nq or 4 Nfp are zero.
template <int N>
struct AOrd {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int NF4 = 4 * Nfp;
  static constexpr int Nq = (N + 1) * (N + 1) * (N + 1);
  static constexpr int RT = (Np + 15) / 16;    // node tiles
  static constexpr int QT = (Nq + 15) / 16;    // quadrature tiles
  static constexpr int FT = (NF4 + 15) / 16;   // face-node tiles
  static constexpr int KN = (Np + 3) / 4;      // 4-slot steps over the nodes
  static constexpr int KF = (NF4 + 3) / 4;     // 4-slot steps over the face nodes
  static constexpr int KF4 = (KF + 3) / 4;
  static constexpr int G_D = 0;
  static constexpr int G_L = G_D + RT * KN;
  static constexpr int G_V = G_L + RT * KF4;
  static constexpr int G_P = G_V + QT * RT;
  static constexpr int G_VT = G_P + QT * RT;
  static constexpr int G_DT = G_VT + QT * RT;
  static constexpr int G_LT = G_DT + RT * KN;
  // With R y and l read from memory (adj_tile<N, true>), the nodes of the
  // last node tile, when they fit one 4-slot step (VLAST <= 4: orders 1, 3
  // and 4), go in a single step, lane group k holding node 16 (RT - 1) + k:
  //   VX  (u), item 0:      V_q[16 u + r][16 (RT - 1) + k]
  //            item 1:      P_q[16 (RT - 1) + k][16 u + r]   (items 2, 3 zero)
  static constexpr int VLAST = Np - 16 * (RT - 1);
  static constexpr bool PACK = VLAST <= 4;
  static constexpr int G_VX = G_LT + FT * RT;
  static constexpr int NG = G_VX + (PACK ? QT : 0);   // fragment groups
  // LDS, in floats: the stage input y (later mu = W^T l) [9][4 KN][CS]; the
  // face fluxes [9][4 KF][CS], later the two partial stress sums of the
  // gradient, double [2][16 QT][16]; rows of CS = 17 floats (16 elements,
  // padded so that row-wise and column-wise accesses spread over the banks)
  static constexpr int CS = 17;
  static constexpr int LY = 9 * 4 * KN * CS;
  static constexpr int LF = 9 * 4 * KF * CS;
  static constexpr int LG = 2 * 2 * 16 * QT * 16;
  static constexpr int LU = LF > LG ? LF : LG;
  static constexpr int USED = (LY + LU) * 4;
  // padded as the stage kernels are: the workgroups one CU holds never use
  // more than 128 KiB of LDS together
  static constexpr int FLOOR =
      USED <= 43690 ? 40976 : USED <= 65536 ? 54630 : USED <= 81920 ? 81936 : 0;
  static constexpr int BYTES = USED > FLOOR ? USED : FLOOR;
};

}  // namespace dgt
