// Host-side layout of the BF16x3 matrix-core stage: operator fragments in
// MFMA lane order and the blocked material array.  No HIP dependencies.
#pragma once
#include <cstdint>
#include <vector>

#include "dg_host.hpp"

namespace dgh {

// orders with a BF16x3 matrix-core stage kernel (1-4: 16-element tiles,
// blocked material; 5-7: one element per workgroup, material in [K][Nq]
// order)
bool mfma_supported(int N);

// hi/lo bf16 bit patterns of the [Dr|Ds|Dt|LIFT], V_q and P_q fragments in
// the K-slot order of the matrix-core stage kernel of order N, [NFRAG][64
// lanes][8]
std::vector<uint16_t> mfma_fragments(const RefElement& re);

// FP32 operator fragments of the FP32 matrix-core stage: orders 1-4 in the
// layout of FOrd ([NF4S][4] floats), orders 5-7 in that of EFOrd
// ([NFRAG][64 lanes][4] floats)
std::vector<float> mfma_fragments_f32(const RefElement& re);

// FP64 operator fragments of the FP64 matrix-core stage: orders 1-4 in the
// layout of FOrd ([NF4S][4] doubles), orders 5-7 in that of EFOrd
// ([NFRAG][64 lanes][4] doubles)
std::vector<double> mfma_fragments_f64(const RefElement& re);

// FP32 operator fragments of the tiled adjoint kernel of orders 1-4 (the
// layout of dgt::AOrd, [NG][64 lanes][4] floats); empty at higher orders
std::vector<float> adj_fragments_f32(const RefElement& re);

// Transposed operator pack (the generic adjoint kernels): DrT | DsT | DtT [Np][NpP], LIFTT [4 Nfp][NpP],
// VqT [Np][QP], PqT [QP][NpP] (transposed, zero padded; NpP = 4 ceil(Np/4),
// QP = 32 ceil(Nq/32)).
std::vector<double> col_operators(const RefElement& re);

// 1/rho, lam, mu at [K][Nq] -> blocked by 16-element tile in the lane order
// of the kernel's quadrature phase, [ceil(K/16)][3][MATS] (zero padded);
// f64: the accumulator row order of the FP64 product (acc_row)
std::vector<double> mfma_material(int N, int64_t K, const double* irho, const double* lam,
                                  const double* mu, bool f64 = false);

// fragment count and blocked-material floats per (tile, field) of order N
int mfma_frag_count(int N);
// float4 count of the FP32 fragments of order N (1-7)
int mfma_f32_frag_count(int N);
int mfma_mats(int N);

// index in the blocked material array of field f (0 1/rho, 1 lam, 2 mu) at
// quadrature point p of element k
size_t mfma_material_index(int N, int64_t k, int p, int f);

}  // namespace dgh
