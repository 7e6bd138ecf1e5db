"""MI355X-native engine for the all-pairs posterior stage of QuickProbs 2.

``binding`` is the ctypes binding of the C ABI (``include/qp.h``, library
``libqp.so`` built by ``build``); ``workload`` generates the seeded synthetic
families.  Import ``binding`` explicitly: it loads the gfx950 library and
raises if it is missing.
"""
__all__ = ["binding", "workload", "build"]
