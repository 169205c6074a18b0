// STL mesh files (host code only).  The paper takes parts as STEP/STL
// geometry (Sections 1 and 3.1); this reader turns an STL file into the
// indexed FP32 mesh every other call takes.
//
// Binary STL: an 80-byte header, a little-endian uint32 facet count, then 50
// bytes per facet (normal, three vertices as 12 little-endian FP32 values, a
// 16-bit attribute).  A file is binary when its size is exactly 84 + 50 x the
// count; otherwise it is read as ASCII: "solid", then per facet "facet
// [normal nx ny nz] outer loop", three "vertex x y z", "endloop endfacet",
// and "endsolid".  ASCII numbers are parsed to the nearest FP64 value and
// then rounded to FP32.
//
// Vertices are welded: equal FP32 coordinates (-0 taken as +0) share one
// index, numbered in order of first appearance.  Facets keep file order and
// vertex order; stored facet normals are ignored (the winding orients the
// face).  Non-finite coordinates are an error.
#include <cerrno>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/hra.h"

struct hra_stl {
    std::vector<float> verts;     // [n][3]
    std::vector<int32_t> tris;    // [m][3]
};

namespace {

thread_local std::string g_stl_err;

hra_status stl_fail(const std::string &msg) {
    g_stl_err = msg;
    return HRA_ERR_INVALID_ARG;
}

struct Key {
    uint32_t x, y, z;
    bool operator==(const Key &o) const { return x == o.x && y == o.y && z == o.z; }
};

struct KeyHash {
    size_t operator()(const Key &k) const {
        uint64_t h = k.x * 0x9E3779B97F4A7C15ull;
        h ^= (h >> 29) + k.y * 0xBF58476D1CE4E5B9ull;
        h ^= (h >> 31) + k.z * 0x94D049BB133111EBull;
        return (size_t)(h ^ (h >> 32));
    }
};

uint32_t bits_of(float f) {
    if (f == 0.0f) f = 0.0f;   // -0 -> +0
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}

class Welder {
  public:
    explicit Welder(hra_stl *m) : m_(m) {}
    // index of (x, y, z), adding it if new; false for a non-finite coordinate
    bool add(float x, float y, float z, int32_t *idx) {
        if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z)) return false;
        const Key k{bits_of(x), bits_of(y), bits_of(z)};
        auto it = map_.find(k);
        if (it != map_.end()) {
            *idx = it->second;
            return true;
        }
        if (m_->verts.size() / 3 >= (size_t)INT32_MAX) return false;
        const int32_t i = (int32_t)(m_->verts.size() / 3);
        map_.emplace(k, i);
        float c[3] = {x, y, z};
        for (float &f : c)
            if (f == 0.0f) f = 0.0f;
        m_->verts.insert(m_->verts.end(), c, c + 3);
        *idx = i;
        return true;
    }

  private:
    hra_stl *m_;
    std::unordered_map<Key, int32_t, KeyHash> map_;
};

uint32_t le32(const unsigned char *p) { return (uint32_t)p[0] | (uint32_t)p[1] << 8 | (uint32_t)p[2] << 16 | (uint32_t)p[3] << 24; }

float lef(const unsigned char *p) {
    const uint32_t u = le32(p);
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

hra_status read_binary(const std::vector<unsigned char> &buf, uint32_t count, hra_stl *m) {
    Welder w(m);
    m->tris.reserve((size_t)count * 3);
    const unsigned char *p = buf.data() + 84;
    for (uint32_t f = 0; f < count; ++f, p += 50) {
        for (int k = 0; k < 3; ++k) {
            const unsigned char *q = p + 12 + 12 * k;
            int32_t idx;
            if (!w.add(lef(q), lef(q + 4), lef(q + 8), &idx))
                return stl_fail("facet " + std::to_string(f) + ": non-finite coordinate or too many vertices");
            m->tris.push_back(idx);
        }
    }
    return HRA_OK;
}

// ASCII tokenizer over the whole file.
class Tokens {
  public:
    explicit Tokens(const std::vector<unsigned char> &b) : s_((const char *)b.data()), n_(b.size()) {}
    bool next(std::string *t) {
        while (i_ < n_ && (s_[i_] == ' ' || s_[i_] == '\t' || s_[i_] == '\r' || s_[i_] == '\n')) ++i_;
        if (i_ >= n_) return false;
        size_t j = i_;
        while (j < n_ && !(s_[j] == ' ' || s_[j] == '\t' || s_[j] == '\r' || s_[j] == '\n')) ++j;
        t->assign(s_ + i_, j - i_);
        i_ = j;
        return true;
    }
    // rest of the current line (the solid's name)
    void skip_line() {
        while (i_ < n_ && s_[i_] != '\n') ++i_;
    }

  private:
    const char *s_;
    size_t n_, i_ = 0;
};

bool parse_num(const std::string &t, float *out) {
    if (t.empty()) return false;
    errno = 0;
    char *end = nullptr;
    const double d = std::strtod(t.c_str(), &end);
    if (end != t.c_str() + t.size()) return false;
    *out = (float)d;   // nearest FP64, then rounded to FP32
    return true;
}

hra_status read_ascii(const std::vector<unsigned char> &buf, hra_stl *m) {
    Tokens tk(buf);
    std::string t;
    if (!tk.next(&t) || t != "solid") return stl_fail("neither binary STL (size != 84 + 50 x count) nor ASCII (no 'solid')");
    tk.skip_line();
    Welder w(m);
    int64_t facet = 0;
    auto expect = [&](const char *word) { return tk.next(&t) && t == word; };
    for (;;) {
        if (!tk.next(&t)) return stl_fail("ASCII STL: missing 'endsolid'");
        if (t == "endsolid") break;
        if (t != "facet") return stl_fail("ASCII STL: expected 'facet' or 'endsolid', found '" + t + "'");
        if (!tk.next(&t)) return stl_fail("ASCII STL: truncated facet");
        if (t == "normal") {
            float dummy;
            for (int k = 0; k < 3; ++k)
                if (!tk.next(&t) || !parse_num(t, &dummy)) return stl_fail("ASCII STL: bad facet normal");
            if (!expect("outer")) return stl_fail("ASCII STL: expected 'outer loop'");
        } else if (t != "outer") {
            return stl_fail("ASCII STL: expected 'normal' or 'outer', found '" + t + "'");
        }
        if (!expect("loop")) return stl_fail("ASCII STL: expected 'loop'");
        for (int k = 0; k < 3; ++k) {
            float c[3];
            if (!expect("vertex")) return stl_fail("ASCII STL: facet " + std::to_string(facet) + ": expected 'vertex'");
            for (float &x : c)
                if (!tk.next(&t) || !parse_num(t, &x))
                    return stl_fail("ASCII STL: facet " + std::to_string(facet) + ": bad coordinate");
            int32_t idx;
            if (!w.add(c[0], c[1], c[2], &idx))
                return stl_fail("ASCII STL: facet " + std::to_string(facet) + ": non-finite coordinate");
            m->tris.push_back(idx);
        }
        if (!expect("endloop") || !expect("endfacet"))
            return stl_fail("ASCII STL: facet " + std::to_string(facet) + ": expected 'endloop endfacet'");
        ++facet;
    }
    return HRA_OK;
}

}  // namespace

extern "C" {

const char *hra_stl_error(void) { return g_stl_err.c_str(); }

hra_status hra_stl_read(const char *path, hra_stl **out, int64_t *n_verts, int64_t *n_tris) {
    g_stl_err.clear();
    if (!path || !out || !n_verts || !n_tris) return stl_fail("null argument");
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) return stl_fail(std::string("cannot open ") + path);
    std::vector<unsigned char> buf;
    unsigned char chunk[1 << 16];
    size_t got;
    while ((got = std::fread(chunk, 1, sizeof(chunk), f)) > 0) buf.insert(buf.end(), chunk, chunk + got);
    const bool err = std::ferror(f) != 0;
    std::fclose(f);
    if (err) return stl_fail(std::string("read error on ") + path);
    hra_stl *m = new hra_stl();
    hra_status st;
    if (buf.size() >= 84 && buf.size() == 84 + 50 * (uint64_t)le32(buf.data() + 80)) {
        st = read_binary(buf, le32(buf.data() + 80), m);
    } else {
        buf.push_back('\n');
        st = read_ascii(buf, m);
    }
    if (st == HRA_OK && m->tris.empty()) st = stl_fail("no facets");
    if (st != HRA_OK) {
        delete m;
        return st;
    }
    *out = m;
    *n_verts = (int64_t)(m->verts.size() / 3);
    *n_tris = (int64_t)(m->tris.size() / 3);
    return HRA_OK;
}

hra_status hra_stl_copy(const hra_stl *m, float *host_verts, int32_t *host_tris) {
    if (!m || !host_verts || !host_tris) return HRA_ERR_INVALID_ARG;
    std::memcpy(host_verts, m->verts.data(), sizeof(float) * m->verts.size());
    std::memcpy(host_tris, m->tris.data(), sizeof(int32_t) * m->tris.size());
    return HRA_OK;
}

void hra_stl_free(hra_stl *m) { delete m; }

}  // extern "C"
