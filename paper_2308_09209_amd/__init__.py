"""MI355X-native per-frame video stitching path (pre-warp, 3D-M colour transfer,
pyramidal flow, local warp + blend, online colour balancing)."""
