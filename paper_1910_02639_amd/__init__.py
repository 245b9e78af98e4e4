"""MI355X-native b-tree neighbour search (arXiv 1910.02639).

The compute path lives in the HIP library ``libbtree.so`` (``csrc/``), behind
the C ABI declared in ``include/btree.h``.  ``paper_1910_02639_amd.btree`` is
the thin Python binding (argument marshalling only); ``workloads`` holds the
seeded synthetic input generators.  Importing the package loads nothing:
the library is opened on first use of the binding.
"""
__all__ = ["btree", "workloads"]
