"""MI355X-native batched ray-cast renderer (depth, segmentation, triangle id and
hit points for pinhole cameras and rotating LiDARs against per-environment
triangle meshes).

Importing the package loads nothing native; ``paper_2503_01471_amd.rc`` loads
the HIP library on first use and raises if it is missing.
"""
__all__ = ["scenes", "rc"]
