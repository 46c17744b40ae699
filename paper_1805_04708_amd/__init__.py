"""MI355X-native state-vector gate application (De Raedt et al., Sec. 2-4).

``jq``         ctypes binding of the C ABI in ``include/jq.h`` (libjq.so)
``workloads``  seeded synthetic circuits
``build``      hipcc build of libjq.so for gfx950
"""
