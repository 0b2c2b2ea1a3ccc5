"""MI355X-native Schwarz waveform relaxation for the 1-D Schroedinger equation
(Besse & Xing, arXiv 1503.02564).

Importing the package has no side effects; the HIP library is loaded on first
use by :mod:`paper_1503_02564_amd.swr`.
"""
