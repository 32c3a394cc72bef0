// Host-side FP64 precompute for the nodal DG elastic-wave operator on
// tetrahedra: reference element (nodes, orthonormal basis, derivative, LIFT,
// quadrature interpolation/projection matrices), periodic face connectivity
// and affine geometric factors.  No HIP calls: this part also runs in a
// host-only context.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace dgh {

inline int num_nodes(int N) { return (N + 1) * (N + 2) * (N + 3) / 6; }
inline int num_face_nodes(int N) { return (N + 1) * (N + 2) / 2; }
inline int num_quad(int N) { return (N + 1) * (N + 1) * (N + 1); }

// Reference tetrahedron with vertices (-1,-1,-1), (1,-1,-1), (-1,1,-1),
// (-1,-1,1).  Faces: 0: t=-1, 1: s=-1, 2: r+s+t=-1, 3: r=-1.  All matrices
// are dense row-major FP64.
struct RefElement {
  int N = 0, Np = 0, Nfp = 0, Nq = 0;
  std::vector<double> r, s, t;          // nodes [Np]
  std::vector<double> Dr, Ds, Dt;       // [Np][Np]
  std::vector<double> LIFT;             // [Np][4*Nfp], columns face-major
  std::vector<double> Vq;               // [Nq][Np]
  std::vector<double> Pq;               // [Np][Nq]
  std::vector<double> rq, sq, tq, wq;   // quadrature points/weights [Nq]
  std::vector<int> Fmask;               // [4][Nfp] volume node of face node
  std::vector<double> Minv;             // [Np][Np]
  std::vector<double> V;                // Vandermonde [Np][Np]: V[i][m] = psi_m(node i)
  // barycentric coordinates of each face node w.r.t. the face's three
  // vertices (in face-vertex order), [4][Nfp][3]
  std::vector<double> fbary;
};

// Builds the reference element of order N (1 <= N <= 8).  Returns false and
// sets err on failure.
bool build_ref_element(int N, RefElement& re, std::string& err);

// Periodic tetrahedral mesh connectivity and geometry.
struct MeshData {
  int64_t K = 0;
  std::vector<double> geo;     // [K][9]   d(r,s,t)_i / d(x,y,z)_j
  std::vector<double> fgeo;    // [K][4][4] (nx, ny, nz, Fscale)
  std::vector<double> J;       // [K]
  std::vector<int32_t> EToE;   // [K][4]
  std::vector<uint8_t> EToF;   // [K][4]
  std::vector<uint8_t> EToP;   // [K][4] trace pattern id
  std::vector<int32_t> pat;    // [npat][Nfp] neighbour volume node per own face node
  int npat = 0;
  std::vector<double> vx;      // [K][4][3] vertices as given
  double period[3] = {0.0, 0.0, 0.0};
};

// vxyz: per-element vertex coordinates [K][4][3]; period: box lengths [3]
// (all > 0).  Vertex order defines the affine map; each element must have
// positive orientation.  Every face must match exactly one face of the
// periodic mesh.
bool build_mesh(const RefElement& re, int64_t K, const double* vxyz,
                const double* period, MeshData& m, std::string& err);

// Flat index nb * Np + vP of the neighbour volume node that each face node
// of each element is paired with, [K][4 Nfp] (requires K Np < 2^31).
std::vector<int32_t> neighbour_nodes(const RefElement& re, const MeshData& m);

// Tables of the adjoint's flux transpose: for every face node, the
// neighbour's face node that reads it (flat nb * 4 Nfp + j', [K][4 Nfp]),
// and for every volume node the face nodes on it ([Np][3], -1 padded).
// Returns false with err set when the face tables are inconsistent.
bool adjoint_face_tables(const RefElement& re, const MeshData& m, std::vector<int32_t>& nbface,
                         std::vector<int32_t>& invf, std::string& err);

// Processing order of the tiles of `tile` consecutive elements, for a launch
// whose workgroups are dealt to `parts` caches (XCDs) in contiguous ranges
// of launch positions: the tiles are sorted into `parts` slabs along the
// axis of largest extent of their centroids, and each slab is swept along
// its own longest remaining axis.  Coordinates are bucketed by the typical
// element size, ties keep the element order.  Face neighbours then run
// close together in time on one cache.  Returns the tile of each position.
std::vector<int32_t> tile_order(const MeshData& m, int tile, int parts);

// Orthonormal basis psi[Np] at the reference point (r, s, t) [HW08, Ch. 10].
void basis_at(const RefElement& re, double r, double s, double t, double* psi);

// Element containing the physical point x (any periodic image) and its
// reference coordinates: the first element whose barycentric coordinates
// are all >= -1e-12.  Returns false if there is none.
bool locate_point(const RefElement& re, const MeshData& m, const double* x, int64_t& k,
                  double* rst);

// Physical coordinates of the nodes [K][Np][3] or quadrature points
// [K][Nq][3].
void node_coords(const RefElement& re, const MeshData& m, double* out);
void quad_coords(const RefElement& re, const MeshData& m, double* out);

}  // namespace dgh
