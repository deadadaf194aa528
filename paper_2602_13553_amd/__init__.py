"""MI355X-native ring-polymer PIMD hot path (BAOAB + PILE-L) behind a C ABI.

``paper_2602_13553_amd.pimd`` is the Python binding of ``libpimd.so``;
``paper_2602_13553_amd.inputs`` builds seeded synthetic workloads.
"""
__version__ = "0.1.0"
