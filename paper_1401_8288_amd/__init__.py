"""MI355X X-stage correlator: the cross-multiply-accumulate of an FX correlator.

Importing the package loads nothing native.  `paper_1401_8288_amd.xcorr` is the
binding to the HIP library; `synth` draws seeded synthetic inputs; `perfmodel`
holds the paper's sizing equations.
"""
__version__ = "0.1.0"
