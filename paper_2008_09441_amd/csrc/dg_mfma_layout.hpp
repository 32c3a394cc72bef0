// Padded sizes and fragment counts of the BF16x3 matrix-core stage for
// order N (shared by the device kernel and the host code that lays out its
// operator fragments and material).  No HIP dependencies.
#pragma once

namespace dgm {

template <int N>
struct MOrd {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int NF4 = 4 * Nfp;
  static constexpr int Nq = (N + 1) * (N + 1) * (N + 1);
  static constexpr int MT = (Np + 15) / 16;        // 16-row tiles of nodes
  static constexpr int CV = (Np + 7) / 8;          // 8-row chunks per derivative section
  static constexpr int CF = (NF4 + 7) / 8;         // 8-row chunks of face nodes
  static constexpr int NCH = 3 * CV + CF;
  static constexpr int KVB = (NCH + 3) / 4;        // K blocks of [Dr|Ds|Dt|LIFT]
  static constexpr int QT = (Nq + 15) / 16;        // 16-row tiles of quadrature points
  static constexpr int QP = 16 * QT;
  static constexpr int KQB = (MT + 1) / 2;         // K blocks of V_q
  static constexpr int PKB = (QT + 1) / 2;         // K blocks of P_q
  static constexpr int NFV = MT * KVB * 2;
  static constexpr int NFQ = QT * KQB * 2;
  static constexpr int NFP = MT * PKB * 2;
  static constexpr int NFRAG = NFV + NFQ + NFP;
  static constexpr int OFF_V = 0, OFF_Q = NFV, OFF_P = NFV + NFQ;
};

}  // namespace dgm
