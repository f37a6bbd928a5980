"""capred: confidence-aware particle human prediction on MI355X (gfx950).

The compute path is the C-ABI library ``libcapred.so`` (hand-written HIP);
``paper_2603_01122_amd.capred`` is its thin PyTorch binding.  Importing this
package does not load the library; importing ``capred`` does, and fails
loudly when it is missing.
"""
__all__ = ["capred", "scenes"]
