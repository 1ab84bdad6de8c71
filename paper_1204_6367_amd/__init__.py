"""MI355X-native Monte Carlo projection step of gDRR (arXiv:1204.6367).

`workloads` builds seeded synthetic inputs; `api` binds the HIP library
libgdrr.so (include/gdrr.h); `build` compiles it for gfx950."""
__version__ = "0.1.0"

_API = ("DeviceVolume", "DevicePhysics", "DeviceSource", "Batch", "JobSpec", "GdrrProject", "project",
        "trace", "majorant", "upload", "geometry_struct")


def __getattr__(name):
    if name in _API:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
