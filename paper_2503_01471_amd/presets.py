"""Sensor presets and user-defined projection models.

Sec. III-D ships idealised configurations of several real sensors (Ouster
OS-0, OS-1, OS-2 and OS-Dome LiDARs, an Intel RealSense D455 and Luxonis
Oak-D / Oak-D Pro W depth cameras, an ST VL53L5CX multi-zone ToF sensor) and
lets users add sensors with their own projection models, such as a dome
LiDAR.  The paper prints no parameters; the nominal figures below (fields of
view, resolutions, ranges, stereo baselines) are this library's choice,
rounded from the public product descriptions, and every one can be
overridden.  Each function returns a ``SensorDesc`` for
``rc_sensor_add`` (through ``Renderer``): pinhole cameras measure depth;
LiDARs and ToF zones measure range along unit directions.

Projection models beyond the pinhole and the spinning LiDAR are expressed
as direction tables (``RC_TABLE``): any set of unit directions in the sensor
frame (x forward, y left, z up), cast from the sensor origin.
"""
from __future__ import annotations

import math

import numpy as np

from .scenes import DEG, LIDAR, SensorDesc, pinhole, table_sensor

__all__ = ["ouster_os0", "ouster_os1", "ouster_os2", "ouster_dome", "realsense_d455", "oak_d", "oak_d_pro_w",
           "vl53l5cx", "dome_lidar", "tof_grid", "PRESETS", "STEREO_BASELINE"]


def _spinning(azimuths, channels, vfov_deg, near, far, vmin_deg=None):
    lo = -0.5 * vfov_deg if vmin_deg is None else vmin_deg
    return SensorDesc(LIDAR, azimuths, channels, vmin=lo * DEG, vmax=(lo + vfov_deg) * DEG, hmin=-math.pi,
                      hmax=math.pi, near=near, far=far)


def ouster_os0(channels: int = 128, azimuths: int = 1024, near: float = 0.3, far: float = 50.0) -> SensorDesc:
    """Ultra-wide spinning LiDAR: 90 degrees vertical (+-45), 360 horizontal."""
    return _spinning(azimuths, channels, 90.0, near, far)


def ouster_os1(channels: int = 128, azimuths: int = 1024, near: float = 0.3, far: float = 120.0) -> SensorDesc:
    """Mid-range spinning LiDAR: 45 degrees vertical (+-22.5)."""
    return _spinning(azimuths, channels, 45.0, near, far)


def ouster_os2(channels: int = 128, azimuths: int = 1024, near: float = 1.0, far: float = 240.0) -> SensorDesc:
    """Long-range spinning LiDAR: 22.5 degrees vertical (+-11.25)."""
    return _spinning(azimuths, channels, 22.5, near, far)


def ouster_dome(channels: int = 128, azimuths: int = 1024, near: float = 0.3, far: float = 20.0) -> SensorDesc:
    """Hemispherical dome LiDAR: channels from the zenith (90 degrees) down to
    the horizon (0), 360 degrees around."""
    return _spinning(azimuths, channels, 90.0, near, far, vmin_deg=0.0)


def dome_lidar(rings: int, per_ring: int, near: float, far: float, max_polar_deg: float = 90.0) -> SensorDesc:
    """User-defined dome model as a direction table: ``rings`` rings of equal
    polar-angle spacing around the sensor's +z axis (ring 0 at the pole),
    ``per_ring`` beams each; the pole ring holds one repeated direction."""
    dirs = np.empty((rings, per_ring, 3))
    for i in range(rings):
        th = max_polar_deg * DEG * i / max(rings - 1, 1)
        ph = 2 * math.pi * np.arange(per_ring) / per_ring
        dirs[i, :, 0] = math.sin(th) * np.cos(ph)
        dirs[i, :, 1] = math.sin(th) * np.sin(ph)
        dirs[i, :, 2] = math.cos(th)
    return table_sensor(dirs.reshape(-1, 3), per_ring, rings, near, far)


def tof_grid(nx: int, ny: int, hfov_deg: float, vfov_deg: float, near: float, far: float) -> SensorDesc:
    """Multi-zone time-of-flight sensor: an nx x ny grid of zone centres
    evenly spaced in angle over the field of view, looking along +x; each
    zone reports range (unit directions, table model).  Row 0 is the top."""
    az = (0.5 * hfov_deg - (np.arange(nx) + 0.5) * hfov_deg / nx) * DEG  # left (+y) to right
    el = (0.5 * vfov_deg - (np.arange(ny) + 0.5) * vfov_deg / ny) * DEG  # top to bottom
    E, A = np.meshgrid(el, az, indexing="ij")
    dirs = np.stack([np.cos(E) * np.cos(A), np.cos(E) * np.sin(A), np.sin(E)], -1)
    return table_sensor(dirs.reshape(-1, 3), nx, ny, near, far)


def vl53l5cx(near: float = 0.02, far: float = 4.0) -> SensorDesc:
    """8 x 8-zone ToF ranging sensor, 45 x 45 degree field of view."""
    return tof_grid(8, 8, 45.0, 45.0, near, far)


def realsense_d455(width: int = 1280, height: int = 720, near: float = 0.4, far: float = 20.0) -> SensorDesc:
    """Stereo depth camera, 87 degrees horizontal field of view."""
    return pinhole(width, height, 87.0, near, far)


def oak_d(width: int = 1280, height: int = 800, near: float = 0.2, far: float = 20.0) -> SensorDesc:
    """Stereo depth camera, 72 degrees horizontal field of view."""
    return pinhole(width, height, 72.0, near, far)


def oak_d_pro_w(width: int = 1280, height: int = 800, near: float = 0.2, far: float = 20.0) -> SensorDesc:
    """Wide stereo depth camera, 108 degrees horizontal field of view."""
    return pinhole(width, height, 108.0, near, far)


# Distance between the two cameras of the stereo presets (metres, along the
# sensor's y axis), for stereo-shadow rendering.
STEREO_BASELINE = {"realsense_d455": 0.095, "oak_d": 0.075, "oak_d_pro_w": 0.075}

PRESETS = {f.__name__: f for f in (ouster_os0, ouster_os1, ouster_os2, ouster_dome, realsense_d455, oak_d,
                                   oak_d_pro_w, vl53l5cx)}
