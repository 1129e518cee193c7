"""Seeded synthetic inputs shared by the library's tests/benchmark and the
oracle.  Input data only (meshes, emissivities, temperatures, request
streams); no view-factor or radiosity arithmetic lives here."""
