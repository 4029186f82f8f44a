"""MI355X-native hash-blocked TSDF fusion (allocate + integrate) behind a C ABI.

``paper_2608_08287_amd.tsdf`` is the Python binding of ``libtsdf.so``;
``paper_2608_08287_amd.scenes`` makes seeded synthetic depth inputs.
"""
