"""MI355X-native EPTV fan-beam CT reconstruction (hot path in HIP for gfx950).

``paper_1009_2288_amd.eptv`` is the binding of the C-ABI library ``libeptv.so``;
``paper_1009_2288_amd.synth`` generates seeded synthetic inputs.  Importing the
package loads neither: the binding is loaded on first use of ``eptv``.
"""
__all__ = ["eptv", "synth"]
