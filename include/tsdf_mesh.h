/*
 * tsdf_mesh.h -- C ABI of marching-cubes meshing of a libtsdf.so volume (gfx950).
 *
 * The paper's meshing engine extracts a triangle mesh from the fused volume
 * with the Marching-Cubes algorithm of Lorensen and Cline (Sec. 4, meshing
 * engine; Sec. 6, createMeshingEngine), without further detail.  Readings:
 *   - a cell is every voxel cube whose 8 corner voxels (in its block or the
 *     neighbouring blocks in +x, +y, +z) are observed (weight > 0); a corner
 *     is inside when its stored SDF is negative (the raycast's F < 0);
 *   - a vertex sits on each active cell edge at the zero crossing of the
 *     linear interpolation t = F0 / (F0 - F1) from the edge's lower corner,
 *     F = s / 32767; its world position is the voxel coordinates times the
 *     voxel size (lattice points at p v);
 *   - the case table is derived from the cube's faces: on each face the active
 *     edges pair into segments (on an ambiguous face each inside corner is cut
 *     off by its own segment), the segments close into loops, each loop is
 *     oriented so that its normal points from inside to outside corners
 *     (towards free space) and is fanned from its smallest edge index.  The
 *     face rule depends only on the face, so the mesh is closed wherever every
 *     cell is observed.
 * Corner c of a cell is at (c & 1, c >> 1 & 1, c >> 2 & 1); edge 4 a + k runs
 * along axis a from the k-th corner (ascending) whose bit a is 0.  An edge's
 * key packs its lower corner's global voxel coordinates and axis:
 * ((x + 2^19) << 42) | ((y + 2^19) << 22) | ((z + 2^19) << 2) | axis.
 *
 * Conventions as in tsdf.h.
 */
#ifndef TSDF_MESH_H
#define TSDF_MESH_H

#include "tsdf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Device bytes of the meshing workspace for a volume of these parameters
 * (per-chunk triangle counts and offsets; 0 if the parameters are invalid). */
size_t tf_mesh_workspace_bytes(const tf_params *p);

/* Mesh every block with device data.  Triangles are ordered by hash entry
 * index, then cell (z, then y, then x within a block is not promised: the
 * order is fixed but internal), so two calls on the same volume give the same
 * arrays.  d_vertices: max_triangles x 9 floats (three world-space vertices,
 * x y z each, wound counter-clockwise seen from free space), or NULL;
 * d_edge_keys: max_triangles x 3 int64 (the keys of the vertices' edges), or
 * NULL; triangles beyond max_triangles are counted but not written.
 * *d_count (device uint64) receives the total number of triangles.
 * d_workspace: tf_mesh_workspace_bytes() bytes, 8-byte aligned.  Enqueue-only.
 * TF_E_INVAL for a NULL context, count or workspace, or misaligned buffers;
 * TF_E_SPACE for a short workspace.  A submap of a batched map (tf_multi_submap)
 * is meshed in its own coordinates. */
int tf_mesh(tf_ctx *ctx, float *d_vertices, int64_t *d_edge_keys, uint64_t max_triangles, uint64_t *d_count,
            void *d_workspace, size_t workspace_bytes, tf_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* TSDF_MESH_H */
