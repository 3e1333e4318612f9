// Host-side finite-element assembly of the operators the step kernel uses.
#pragma once
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "mmsd.h"

namespace mmsd {

constexpr double kMu0 = 4e-7 * 3.14159265358979323846;

struct MatLine {
  double Js, K1, A, u[3];
};

// Operators of one mesh in internal units (nm, mu0 Ms^2 nm^3, Ms).
struct Assembly {
  int64_t n_nodes = 0;
  int N = 0;                     // magnetic nodes
  int Nt = 0;                    // free potential nodes (magnetic ones first)
  double Js = 0, Ms = 0, mu0Ms2 = 0;
  double c_an = 0;               // sum_e V_e K1_e / (mu0 Ms^2)
  double vol = 0;                // sum_i V_i
  std::vector<int> mag_global;   // [N] global id of magnetic node i (ascending)
  std::vector<int> pot_global;   // [Nt] global id of potential row p
  // magnet CSR (rows and columns are magnetic nodes)
  std::vector<int> mrp, mci;
  std::vector<double> K;         // 2 K_ij / V_i
  std::vector<double> D1[3];     // sum_e V_e/4 grad(phi_i)|_e
  std::vector<double> D2[3];     // sum_e V_e/4 grad(phi_j)|_e / V_i
  std::vector<double> Q[6];      // 2 Q_i / V_i (xx yy zz xy xz yz)
  std::vector<double> V;         // lumped nodal volume
  // potential CSR over free nodes
  std::vector<int> lrp, lci;
  std::vector<double> L, invd;
  // kept for re-assembly of the material-dependent values
  std::vector<int> mtet;         // [Em*4] magnetic-node indices of magnetic tets
  std::vector<double> mgeo;      // [Em*13] V_e, grad[4][3]
  std::vector<int> mregion;      // [Em]
  std::vector<int> mnode_tets_ptr, mnode_tets;   // magnetic node -> (tet, vertex) pairs
  std::map<int, MatLine> mats;
};

struct PatternSizes {
  int64_t N, nnzM, Nt, nnzL;
  int64_t nnzLs;   // entries of the sliced (64-row) copy of the potential matrix, padding included
};

// Entries of the 64-row sliced layout of a CSR pattern: each slice of 64
// consecutive rows is padded to its longest row.
int64_t sliced_entries(const std::vector<int>& rp);

// Validate the mesh and count rows and nonzeros (no values).
int pattern_sizes(const mmsd_mesh* mesh, PatternSizes* out, std::string* err);

// Full assembly.  Returns an MMSD_* status.
int assemble(const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats, Assembly* out,
             std::string* err);

// Recompute K, Q and c_an from a.mats (after a material change); with
// operators false only Js, Ms, mu0 Ms^2 and c_an.
int assemble_material_values(Assembly* a, std::string* err, bool operators = true);

// The combinatorial half of the assembly, for the device-side assembly of
// the values: numbering, the magnetic tets with their node adjacency, both
// sparsity patterns, every mesh node's tet adjacency, and per-region
// material factors.  The rows, columns and summation orders are those of
// assemble(), so the device sums the same terms in the same order.
struct AssemblyStructure {
  int64_t E = 0;                 // mesh tets
  int N = 0, Nt = 0;
  std::vector<int> mag_global, pot_global;
  std::vector<int> pot_of;       // [n_nodes] potential row of a mesh node, -1 if none
  std::vector<int> mtet;         // [Em*4] magnetic-node ids of magnetic tet k
  std::vector<int> mtet_mesh;    // [Em] mesh tet of magnetic tet k
  std::vector<int> mregion;      // [Em]
  std::vector<int> mnode_tets_ptr, mnode_tets;   // magnetic node -> (magnetic tet, vertex)
  std::vector<int> mrp, mci, lrp, lci;
  std::vector<int> tptr, tlst;   // mesh node -> (mesh tet, vertex), all tets (when Nt > 0)
  // per region id r (dense, 0..max region): [8r] A / (mu0 Ms^2 nm^2),
  // [8r+1] K1, [8r+2..8r+7] products of the unit easy axis (xx yy zz xy xz yz)
  std::vector<double> reg;
  double Js = 0, mu0Ms2 = 0;
};

// Validates the mesh and the materials (as assemble() does, except that the
// geometry checks, degenerate tets and tets outside the shell, are left to
// the caller) and builds the structure.  With with_patterns false it stops
// after the numbering, the magnetic tets and the material table (the
// adjacency and pattern vectors stay empty: the device builds them).
// Returns an MMSD_* status.
int assemble_structure(const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats, AssemblyStructure* out,
                       std::string* err, bool with_patterns = true);

// The host side of a problem whose operators were assembled on the device:
// numbering, materials, the magnetic tets with their geometry (for later
// material changes), the lumped volumes V (the device's, copied back), their
// total and the anisotropy constant.  Consumes S's numbering and tet lists.
// The operator arrays (K, D1, D2, Q, L, invd) stay empty.
int assemble_host_side(const mmsd_mesh* mesh, const mmsd_material* mats, int n_mats, AssemblyStructure* S,
                       std::vector<double>&& V, Assembly* A, std::string* err);

// The magnetic node -> (magnetic tet, vertex) lists that a material change
// re-assembles from, built if absent (problems assembled on the device).
void ensure_magnet_adjacency(Assembly* A);

}  // namespace mmsd
