"""MI355X-native Newton-iteration hot path of a fully implicit water/oil/polymer
reservoir simulator (after Zhong et al., arXiv 1807.05298).

``inputs`` draws seeded synthetic cases; ``polyflood`` is the thin ctypes
binding over the HIP library ``libpolyflood.so`` (C ABI in
``include/polyflood.h``)."""
