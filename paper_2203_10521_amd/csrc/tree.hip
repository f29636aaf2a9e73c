// Top-down OBB tree of covariance boxes: the comparison baseline of the
// paper's quality study (Sec. 5, Fig. 6, against OBB-tree style builders).
// Every node's box is the area-weighted covariance box of its triangles
// (obbv_fit); a node's triangles are then cut into `branching` equal-count
// parts in the order of their centroids' projections on the longest axis of
// the node's box (for branching 2: the median split).  The fits of a level are
// one device call; the ordering and cut run on the host.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "common.h"

namespace obbv {
int fit_impl(const obbv_mesh* mesh, const int32_t* tri_cluster, int32_t n_clusters, obbv_box* out_boxes,
             double* out_eigvals, hipStream_t st);
}

using namespace obbv;

static int obbv_build_obb_tree_body(const obbv_mesh* mesh, int32_t levels, int32_t branching, float* out_boxes,
                                   int32_t* out_parent, int32_t* out_tri_node, void* stream);
extern "C" int obbv_build_obb_tree(const obbv_mesh* mesh, int32_t levels, int32_t branching, float* out_boxes,
                                   int32_t* out_parent, int32_t* out_tri_node, void* stream) {
  return obbv::guarded([&] { return obbv_build_obb_tree_body(mesh, levels, branching, out_boxes, out_parent, out_tri_node, stream); });
}
static int obbv_build_obb_tree_body(const obbv_mesh* mesh, int32_t levels, int32_t branching, float* out_boxes,
                                   int32_t* out_parent, int32_t* out_tri_node, void* stream) {
  clear_error();
  OBBV_ARG(mesh != nullptr, "mesh is NULL");
  OBBV_ARG(levels >= 1 && levels <= 12, "levels must be in [1, 12]");
  OBBV_ARG(branching >= 2 && branching <= 64, "branching must be in [2, 64]");
  OBBV_ARG(mesh->n_triangles > 0 && mesh->triangles && mesh->vertices && mesh->n_vertices > 0, "empty mesh");
  int64_t n_nodes = 0, width = 1;
  for (int l = 0; l < levels; ++l, width *= branching) n_nodes += width;
  OBBV_ARG(n_nodes < (1 << 24), "too many nodes");
  hipStream_t s = (hipStream_t)stream;
  const int nt = mesh->n_triangles, nv = mesh->n_vertices;
  std::vector<float> V((size_t)nv * 3);
  std::vector<int32_t> F((size_t)nt * 3);
  OBBV_HIP(hipMemcpyAsync(V.data(), mesh->vertices, V.size() * 4, hipMemcpyDeviceToHost, s));
  OBBV_HIP(hipMemcpyAsync(F.data(), mesh->triangles, F.size() * 4, hipMemcpyDeviceToHost, s));
  OBBV_HIP(hipStreamSynchronize(s));
  for (int32_t x : F) OBBV_ARG(x >= 0 && x < nv, "triangle index out of range");
  // centroids (float64 of the float32 vertices)
  std::vector<double> cen((size_t)nt * 3);
  for (int t = 0; t < nt; ++t)
    for (int d = 0; d < 3; ++d)
      cen[3 * (size_t)t + d] = (((double)V[3 * F[3 * t] + d] + (double)V[3 * F[3 * t + 1] + d]) +
                                (double)V[3 * F[3 * t + 2] + d]) /
                               3.0;
  int32_t* d_cluster = nullptr;
  obbv_box* d_boxes = nullptr;
  const int64_t max_width = width / branching;
  if (hipMalloc(&d_cluster, 4 * (size_t)nt) != hipSuccess ||
      hipMalloc(&d_boxes, sizeof(obbv_box) * (size_t)max_width) != hipSuccess) {
    (void)hipGetLastError();
    if (d_cluster) (void)hipFree(d_cluster);
    set_error("hipMalloc failed for the tree build");
    return OBBV_ERR_OOM;
  }
  std::vector<int32_t> cluster((size_t)nt, 0), next((size_t)nt), order((size_t)nt);
  std::vector<obbv_box> B;
  std::vector<double> proj((size_t)nt);
  int rc = OBBV_OK;
  int64_t base = 0;
  int64_t n = 1;
  for (int l = 0; l < levels && rc == OBBV_OK; ++l, n *= branching) {
    B.resize((size_t)n);
    if (hipMemcpyAsync(d_cluster, cluster.data(), 4 * (size_t)nt, hipMemcpyHostToDevice, s) != hipSuccess) {
      rc = OBBV_ERR_HIP;
      break;
    }
    rc = fit_impl(mesh, d_cluster, (int32_t)n, d_boxes, nullptr, s);
    if (rc != OBBV_OK) break;
    if (hipMemcpyAsync(B.data(), d_boxes, sizeof(obbv_box) * (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      rc = OBBV_ERR_HIP;
      break;
    }
    for (int64_t j = 0; j < n; ++j) {
      const int64_t g = base + j;
      if (out_boxes) {
        std::memcpy(out_boxes + 15 * g, B[j].center, 12);
        std::memcpy(out_boxes + 15 * g + 3, B[j].axes, 36);
        std::memcpy(out_boxes + 15 * g + 12, B[j].half, 12);
      }
      if (out_parent) out_parent[g] = l == 0 ? -1 : (int32_t)(base - n / branching + j / branching);
    }
    if (out_tri_node)
      for (int t = 0; t < nt; ++t) out_tri_node[(int64_t)l * nt + t] = (int32_t)(base + cluster[t]);
    base += n;
    if (l + 1 == levels) break;
    // cut every node along the longest axis of its box into equal-count parts
    for (int t = 0; t < nt; ++t) {
      const obbv_box& b = B[cluster[t]];
      const int k = b.half[0] >= b.half[1] ? (b.half[0] >= b.half[2] ? 0 : 2) : (b.half[1] >= b.half[2] ? 1 : 2);
      const float* e = b.axes + 3 * k;
      proj[t] = (cen[3 * (size_t)t] * e[0] + cen[3 * (size_t)t + 1] * e[1]) + cen[3 * (size_t)t + 2] * e[2];
    }
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
      if (cluster[x] != cluster[y]) return cluster[x] < cluster[y];
      if (proj[x] != proj[y]) return proj[x] < proj[y];
      return x < y;
    });
    std::vector<int64_t> count((size_t)n, 0), start((size_t)n, 0);
    for (int t = 0; t < nt; ++t) ++count[cluster[t]];
    for (int64_t j = 1; j < n; ++j) start[j] = start[j - 1] + count[j - 1];
    for (int i = 0; i < nt; ++i) {
      const int32_t t = order[i];
      const int64_t c = cluster[t];
      const int64_t rank = i - start[c];
      const int64_t part = std::min<int64_t>(rank * branching / std::max<int64_t>(count[c], 1), branching - 1);
      next[t] = (int32_t)(c * branching + part);
    }
    cluster.swap(next);
  }
  (void)hipFree(d_cluster);
  (void)hipFree(d_boxes);
  return rc;
}
