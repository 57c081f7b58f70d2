"""Batch transaction engine for MI355X (gfx950): concurrency control over a device-resident table.

The compute path is the C-ABI library ``libcc.so`` built from ``csrc/``; the
Python binding in ``binding`` only marshals arguments to it.  Importing this
package loads nothing native; ``binding`` does, and fails loudly if the
library is missing.
"""
__all__ = ["workload", "binding"]
