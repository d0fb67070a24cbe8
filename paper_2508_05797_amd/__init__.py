"""MI355X-native chunk-boundary finding for hashless CDC (RAM, AE, MAXP).

``binding`` exposes the C ABI of libcdc.so (``chunk``, ``chunk_batch``...);
``datagen`` draws the seeded synthetic inputs.  Importing the package loads
nothing; the library is loaded on first use and must have been built.
"""
